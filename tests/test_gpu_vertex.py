"""GPU parity of the per-vertex non-rigid stage against the FP64 oracle
(paper Sec. 3.4 energy with vertex positions as unknowns, Sec. 4 non-rigid
solver; the photometric pyramid of Sec. 3.4 as per-step blur kernels).

Bars (written in each test): decisions bit-exact; right-hand side, diagonal
and product element-wise within 1e-5 of their largest entry; solved positions
within 1e-4 of the oracle relative to the oracle's change from the start;
energies within 1e-5 of the start energy.
"""
import math

import numpy as np
import pytest

import synth.sequence as ss
from oracle import vertex as ov

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_1810_02648_amd as cap
    return cap.Context(0)


@pytest.fixture(scope="module")
def seq_small():
    return ss.make_sequence("body_small", 0, n_frames=5, workers=1)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def gpu_frame(ctx, f, start=None, temporal=True, tmpl=None):
    import paper_1810_02648_amd as cap
    if tmpl is None:
        tmpl = cap.VertexTemplate(ctx, dev(f["tri"]), dev(f["rest"]), dev(f["classes"].astype(np.int32)))
    V = dev((f["start"] if start is None else start).astype(np.float32))
    return cap.VertexInputs(tmpl, dev(f["posed"]), dev(f["rgb"]), f["cam"], dev(f["mask"]), dev(f["image"]), V,
                            prev=dev(f["prev"]) if temporal else None, prev2=dev(f["prev2"]) if temporal else None)


def weights_of(f, temporal=True):
    w = dict(f["weights"])
    if not temporal:
        w["w_vel"] = w["w_acc"] = 0.0
    return w


def gpu_params(w, gn, pcg, blur=None, tau=math.inf, outline=True):
    import paper_1810_02648_amd as cap
    return cap.vertex_params(w["w_photo"], w["w_sil"], w["w_smooth"], w["w_edge"], w["w_vel"], w["w_acc"],
                             gn_iters=gn, pcg_iters=pcg, tau_color=tau, exclude_case2=True, outline_only=outline,
                             blur_kernels=blur)


def oracle_problem(f, w, temporal=True, tau=math.inf, outline=True, start=None):
    return ov.VertexProblem(f["rest"], f["posed"], f["tri"], f["rgb"], f["classes"], f["cam"], f["mask"], f["image"],
                            w, start=f["start"] if start is None else start, prev=f["prev"] if temporal else None,
                            prev2=f["prev2"] if temporal else None, tau_c=tau, case2="exclude", outline=outline)


def vertex_flags(P):
    fl = np.zeros(P.nv, np.uint8)
    fl[P.dec["visible"]] |= 1
    fl[P.bnd_idx] |= 2
    return fl


def assert_solution(V_gpu, ref, start, bar=1e-4):
    change = np.linalg.norm(ref["V"] - start.astype(np.float64))
    err = np.linalg.norm(V_gpu.astype(np.float64) - ref["V"])
    print("solution error %.3e of the change %.3e (ratio %.2e)" % (err, change, err / change))
    assert err <= bar * change


def assert_energies(rep, ref, bar=1e-5):
    e0 = ref["energies"][0]["total"]
    assert len(rep["energy"]) == len(ref["energies"])
    for k, e in enumerate(ref["energies"]):
        assert abs(rep["energy"][k] - e["total"]) <= bar * abs(e0), (k, rep["energy"][k], e["total"])


def test_linearisation_and_product_match_the_oracle(ctx, seq_small):
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 3)
    w = weights_of(f)
    P = oracle_problem(f, w)
    A, rhs, e = P.normal_equations(P.start.astype(np.float64))
    fr = gpu_frame(ctx, f)
    p = np.random.default_rng(0).normal(0, 1e-3, (3, P.nv))
    out = cap.vertex_linearize(ctx, fr, gpu_params(w, 3, 4), p=dev(p))
    assert np.array_equal(out["vflags"].cpu().numpy() & 3, vertex_flags(P))
    ref_rhs = rhs.reshape(P.nv, 3).T
    ref_diag = A.diagonal().reshape(P.nv, 3).T
    ref_ap = (A @ p.T.ravel()).reshape(P.nv, 3).T
    for got, ref in ((out["rhs"], ref_rhs), (out["diag"], ref_diag), (out["Ap"], ref_ap)):
        g = got.cpu().numpy()
        assert np.abs(g - ref).max() <= 1e-5 * np.abs(ref).max()
    names = ("photo", "sil", "sil_abs", "smooth", "edge", "vel", "acc")
    for k, n in enumerate(names):
        assert abs(out["energy"][k] - e[n]) <= 1e-6 * e["total"], (n, out["energy"][k], e[n])
    assert torch.equal(fr.V.cpu(), torch.from_numpy(f["start"]))      # the frame's positions are not modified


@pytest.mark.parametrize("temporal", [True, False])
def test_solve_matches_the_oracle_schedule(ctx, seq_small, temporal):
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 4)
    w = weights_of(f, temporal)
    ref = ov.solve(oracle_problem(f, w, temporal), 3, "pcg", 4)
    fr = gpu_frame(ctx, f, temporal=temporal)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 3, 4))
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)
    assert rep["n_visible"] == ref["n_visible"] and rep["n_boundary"] == ref["n_boundary"]
    assert rep["energy"][-1] < 0.7 * rep["energy"][0]


def test_photometric_pyramid_schedule(ctx, seq_small):
    """Three Gauss-Newton steps on I_Gauss of kernels 15, 9, 3 (Sec. 3.4)."""
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 4)
    w = weights_of(f)
    ref = ov.solve(oracle_problem(f, w), 3, "pcg", 4, blur_schedule=(15, 9, 3))
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 3, 4, blur=(15, 9, 3)))
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)


def test_converged_pcg_matches_the_exact_solve(ctx, seq_small):
    """Gauss-Newton with PCG run far enough matches the sparse-Cholesky steps."""
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 4)
    w = weights_of(f)
    ref = ov.solve(oracle_problem(f, w), 2, "chol")
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 2, 1200))      # the oracle's own PCG is within 2e-8 of Cholesky at 1000
    assert_solution(fr.V.cpu().numpy(), ref, f["start"], bar=1e-4)
    assert_energies(rep, ref)


def test_robust_colour_kernel(ctx, seq_small):
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 3)
    w = weights_of(f)
    ref = ov.solve(oracle_problem(f, w, tau=0.05), 2, "pcg", 4)
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 2, 4, tau=0.05))
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)


def test_invalid_arguments_are_rejected_before_any_launch(ctx, seq_small):
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 3)
    w = weights_of(f)
    fr = gpu_frame(ctx, f, temporal=False)
    before = fr.V.clone()
    with pytest.raises(cap.CaptureError) as e:
        cap.vertex_solve(ctx, fr, gpu_params(w, 3, 4))           # velocity and acceleration without prev
    assert e.value.code == -1
    w0 = weights_of(f, False)
    with pytest.raises(cap.CaptureError) as e:
        cap.vertex_solve(ctx, fr, gpu_params(w0, 3, 4, blur=(4, 3, 3)))
    assert e.value.code == -1
    with pytest.raises(cap.CaptureError) as e:
        cap.vertex_solve(ctx, fr, gpu_params(w0, 4, 4, blur=(15, 9, 5, 3)))
    assert e.value.code == -6
    assert torch.equal(fr.V, before)
    with pytest.raises(cap.CaptureError):
        cap.VertexTemplate(ctx, dev(f["tri"]), dev(f["rest"]), dev(np.full(f["rest"].shape[1], 8, np.int32)))


def test_paper_sized_body_frame(ctx):
    """A 20,000-vertex body frame at 1080^2 (the benchmark's shape), 3 GN x 4 PCG."""
    import paper_1810_02648_amd as cap
    seq = ss.make_sequence("body20k", 0, n_frames=4, workers=4)
    f = ss.vertex_frame(seq, 3)
    w = weights_of(f)
    ref = ov.solve(oracle_problem(f, w), 3, "pcg", 4)
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 3, 4))
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)


def test_graph_replay_equals_eager(ctx, seq_small):
    """Solves replayed from a captured HIP graph (one graph, then replays on
    other frames' inputs) are bitwise the eager solves."""
    import paper_1810_02648_amd as cap
    frames = [ss.vertex_frame(seq_small, t) for t in (2, 3, 4, 3)]
    w = weights_of(frames[0])
    prm = gpu_params(w, 3, 4, blur=(15, 9, 3))
    tmpl = gpu_frame(ctx, frames[0]).template
    eager = []
    for f in frames:
        fr = gpu_frame(ctx, f, tmpl=tmpl)
        eager.append((cap.vertex_solve(ctx, fr, prm)["energy"], fr.V.clone()))
    cap.set_graphs(ctx, True)
    try:
        for (e, V), f in zip(eager, frames):
            fr = gpu_frame(ctx, f, tmpl=tmpl)
            rep = cap.vertex_solve(ctx, fr, prm)
            torch.cuda.synchronize()
            assert rep["energy"] == e
            assert torch.equal(fr.V, V)
    finally:
        cap.set_graphs(ctx, False)


def test_vertex_snapping_matches_the_oracle(ctx, seq_small):
    """Snapping after the solve (Sec. 3.4): contour walk on the distance
    transform and the band's Laplacian warp, against the oracle applied to the
    oracle's own solution."""
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 4)
    w = weights_of(f)
    P = oracle_problem(f, w)
    ref = ov.solve(P, 3, "pcg", 4)
    snapped, mask = ov.snap_vertices(P, ref["V"], max_px=3.0, steps=4, rings=2, iters=8)
    fr = gpu_frame(ctx, f)
    prm = gpu_params(w, 3, 4)
    prm.snap_max_px, prm.snap_steps, prm.snap_rings, prm.snap_iters = 3.0, 4, 2, 8
    rep = cap.vertex_solve(ctx, fr, prm)
    got = fr.V.cpu().numpy().astype(np.float64)
    print("snapped %d (oracle %d), max difference %.3e m, largest snap %.3e m"
          % (rep["n_snapped"], mask.sum(), np.abs(got - snapped).max(), np.abs(snapped - ref["V"]).max()))
    assert abs(rep["n_snapped"] - int(mask.sum())) <= 1 and mask.sum() > 20
    assert np.abs(got - snapped).max() <= 1e-4
    assert np.abs(snapped - ref["V"]).max() > 1e-3          # snapping moved something
    assert_energies(rep, ref)                                # the report's energies are those before snapping


def test_body_part_mask_matches_the_oracle(ctx, seq_small):
    """Body-part mask of the silhouette term (Sec. 3.4): the same contour
    vertices lose their residual on both sides (bit-exact), and the solve
    matches the oracle's."""
    import paper_1810_02648_amd as cap
    f = ss.vertex_frame(seq_small, 3)
    w = weights_of(f)
    P = ov.VertexProblem(f["rest"], f["posed"], f["tri"], f["rgb"], f["classes"], f["cam"], f["mask"], f["image"], w,
                         start=f["start"], prev=f["prev"], prev2=f["prev2"], case2="exclude", outline=False,
                         parts=f["parts"], part_dilation=10)
    P0 = oracle_problem(f, w, outline=False)
    assert 0 < P.bnd_idx.size < P0.bnd_idx.size
    tmpl = cap.VertexTemplate(ctx, dev(f["tri"]), dev(f["rest"]), dev(f["classes"].astype(np.int32)),
                              dev(f["parts"].astype(np.int32)))
    fr = gpu_frame(ctx, f, tmpl=tmpl)
    prm = gpu_params(w, 3, 4, outline=False)
    prm.flags |= 8
    prm.part_dilation = 10
    out = cap.vertex_linearize(ctx, fr, prm)
    assert np.array_equal(out["vflags"].cpu().numpy() & 3, vertex_flags(P))
    ref = ov.solve(P, 3, "pcg", 4)
    rep = cap.vertex_solve(ctx, fr, prm)
    assert rep["n_boundary"] == P.bnd_idx.size
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)


def test_empty_silhouette_and_no_regularisers(ctx, seq_small):
    """Edge cases: an empty mask (no image contour: the distance transform is 0,
    so the model's contour vertices carry zero silhouette residuals) and a
    solve with only the data terms and the temporal priors (no one-ring
    terms), both against the oracle."""
    import paper_1810_02648_amd as cap
    f = dict(ss.vertex_frame(seq_small, 3))
    f["mask"] = np.zeros_like(f["mask"])
    w = weights_of(f)
    P = oracle_problem(f, w)
    assert float(P.dt.max()) == 0.0
    ref = ov.solve(P, 2, "pcg", 4)
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w, 2, 4))
    assert rep["n_boundary"] == P.bnd_idx.size and rep["e_sil"] == 0.0
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)
    f = ss.vertex_frame(seq_small, 3)
    w2 = dict(weights_of(f), w_smooth=0.0, w_edge=0.0)
    ref = ov.solve(oracle_problem(f, w2), 2, "pcg", 4)
    fr = gpu_frame(ctx, f)
    rep = cap.vertex_solve(ctx, fr, gpu_params(w2, 2, 4))
    assert rep["e_smooth"] == 0.0 and rep["e_edge"] == 0.0
    assert_solution(fr.V.cpu().numpy(), ref, f["start"])
    assert_energies(rep, ref)
