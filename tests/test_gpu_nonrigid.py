"""GPU parity of the non-rigid stage against the FP64 oracle (through the C ABI).

Bars: integer outputs (graph indices, depth buffer bits, visibility, contour
set, direction signs, distance-transform bits) bit-exact; float outputs
within tolerances derived from float32 arithmetic; solved node parameters
within 1e-4 of the parameter change and energies within 1e-5 of the start
energy (relative), against the oracle run with the same PCG schedule.
"""
import numpy as np
import pytest

import synth
from oracle import graph as og
from oracle import image as oi
from oracle import nonrigid as onr
from oracle import so3

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_1810_02648_amd as cap
    return cap.Context(0)


@pytest.fixture(scope="module")
def frames():
    return {"small0": synth.make_nonrigid_frame("small", 0),
            "small1": synth.make_nonrigid_frame("small", 1),
            "mid": synth.make_nonrigid_frame("small", 2, n_vertices=9001, n_nodes=203, side=517)}


def test_graph_build_matches_oracle(ctx, frames):
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    for name in ("small0", "mid"):
        f = frames[name]
        nn = int(f["n_nodes"]) if name != "mid" else 203
        ref = og.build_graph(f["xyz"], nn)
        g = cap.graph_build(ctx, dev(f["xyz"]), nn)
        assert np.array_equal(g["node_vertex"].cpu().numpy(), ref["node_vertex"]), name
        assert np.array_equal(g["bind_idx"].cpu().numpy(), ref["bind_idx"]), name
        assert np.array_equal(g["edge_dst"].cpu().numpy(), ref["edge_dst"]), name
        assert np.abs(g["bind_w"].cpu().numpy() - ref["bind_w64"]).max() < 2e-6, name


def test_graph_build_many_vertices_per_thread(ctx):
    """Farthest-point sampling on a cloud large enough that the grid is capped
    (256 workgroups, several vertices per thread, a ragged tail), against the
    oracle's sampling, binding and node edges."""
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    rng = np.random.default_rng(17)
    xyz = (rng.standard_normal((3, 70001)) * np.array([[0.3], [0.8], [0.2]])).astype(np.float32)
    ref = og.build_graph(xyz, 301)
    g = cap.graph_build(ctx, dev(xyz), 301)
    assert np.array_equal(g["node_vertex"].cpu().numpy(), ref["node_vertex"])
    assert np.array_equal(g["bind_idx"].cpu().numpy(), ref["bind_idx"])
    assert np.array_equal(g["edge_dst"].cpu().numpy(), ref["edge_dst"])


@pytest.mark.parametrize("nv,nn", [(300, 4), (300, 300), (257, 257)])
def test_graph_build_node_count_limits(ctx, nv, nn):
    """Farthest-point sampling at the smallest node count and with every vertex a
    node (the last selections decided by the lowest-index rule), against the oracle."""
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    rng = np.random.default_rng(nv + nn)
    xyz = rng.standard_normal((3, nv)).astype(np.float32)
    ref = og.build_graph(xyz, nn)
    g = cap.graph_build(ctx, dev(xyz), nn)
    assert np.array_equal(g["node_vertex"].cpu().numpy(), ref["node_vertex"])
    assert np.array_equal(g["bind_idx"].cpu().numpy(), ref["bind_idx"])
    assert np.array_equal(g["edge_dst"].cpu().numpy(), ref["edge_dst"])


@pytest.mark.parametrize("name", ["small0", "small1", "mid"])
def test_frame_decisions_bit_exact(ctx, frames, name):
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = frames[name]
    nn = 64 if name != "mid" else 203
    g = og.build_graph(f["xyz"], nn)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    fr = make_frame(ctx, f, g)
    out = cap.frame_decisions(ctx, fr)
    assert np.array_equal(out["dt"].cpu().numpy().view(np.uint32), P.dt.view(np.uint32))
    assert np.array_equal(out["zbuf"].cpu().numpy().view(np.uint32), P.dec["zbuf"])
    fl = out["vflags"].cpu().numpy()
    assert np.array_equal((fl & 1) != 0, P.dec["visible"])
    assert np.array_equal((fl & 2) != 0, P.dec["boundary"])
    assert np.array_equal((fl & 4) != 0, P.dec["bsign"] < 0)
    assert np.abs(out["blurred"].cpu().numpy() - P.img).max() < 1e-6


def test_distance_transform_edge_cases(ctx, frames):
    """Empty mask (no contour: DT = 0), full mask (contour = image border), one pixel."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = dict(frames["small0"])
    g = og.build_graph(f["xyz"], 64)
    H, W = f["mask"].shape
    cases = [np.zeros((H, W), np.uint8), np.ones((H, W), np.uint8)]
    one = np.zeros((H, W), np.uint8)
    one[H - 1, 7] = 1
    cases.append(one)
    for m in cases:
        f["mask"] = m
        out = cap.frame_decisions(ctx, make_frame(ctx, f, g))
        ref, _ = oi.distance_transform(m)
        assert np.array_equal(out["dt"].cpu().numpy().view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("W", [8, 17, 31, 32, 33, 64, 600, 2048, 4096])
def test_distance_transform_row_widths(ctx, frames, W):
    """Row pass at widths where its anchor pixels coincide (W <= 32: every
    pixel an anchor, the last ones repeated), where the last anchors repeat
    the last pixel (33), where the intervals hold many pixels (600, 2048) and
    at the largest image side (4096, where no integer term may leave 32 bits);
    masks of random blobs with empty rows, bit-exact against the oracle."""
    import dataclasses
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = dict(frames["small0"])
    g = og.build_graph(f["xyz"], 64)
    H = 48
    rng = np.random.default_rng(W)
    m = np.zeros((H, W), np.uint8)
    for _ in range(max(1, W // 40)):
        cy, cx, r = rng.integers(6, H - 6), rng.integers(0, W), rng.integers(1, 6)
        yy, xx = np.mgrid[0:H, 0:W]
        m[(yy - cy) ** 2 + (xx - cx) ** 2 <= r * r] = 1
    m[:5] = 0                                   # rows with no site at all
    f["mask"] = m
    f["image"] = np.zeros((3, H, W), np.float32)
    f["cam"] = dataclasses.replace(f["cam"], width=W, height=H, cx=(W - 1) / 2.0, cy=(H - 1) / 2.0)
    out = cap.frame_decisions(ctx, make_frame(ctx, f, g))
    ref, _ = oi.distance_transform(m)
    assert np.array_equal(out["dt"].cpu().numpy().view(np.uint32), ref.view(np.uint32))


def normal_equations_dense(P, state):
    A, rhs, e = P.normal_equations(state)
    return A, rhs, e


@pytest.mark.parametrize("name,w_vel", [("small0", 0.0), ("mid", 0.0), ("small1", 100.0)])
def test_linearization_and_jtj_product(ctx, frames, name, w_vel):
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame, dev
    f = frames[name]
    nn = 64 if name != "mid" else 203
    g = og.build_graph(f["xyz"], nn)
    rng = np.random.default_rng(11)
    st = onr.apply_update(onr.identity_state(nn), rng.normal(0, 0.02, 6 * nn)).astype(np.float32)
    case2 = "exclude" if w_vel > 0 else "push"
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"], state0=st,
                    w_vel=w_vel, case2=case2)
    A, rhs, e = P.normal_equations(st.astype(np.float64))
    fr = make_frame(ctx, f, g, state=st)
    pvec = rng.normal(size=(6, nn)).astype(np.float32)
    prm = cap.params(*f["weights"], gn_iters=1, pcg_iters=1, w_vel=w_vel, exclude_case2=case2 == "exclude")
    out = cap.linearize(ctx, fr, prm, dev(pvec))
    # node-major (6 per node) vectors of the oracle -> [6][nn]
    rhs_ref = rhs.reshape(nn, 6).T
    diag_ref = A.diagonal().reshape(nn, 6).T
    ap_ref = (A @ pvec.T.reshape(-1).astype(np.float64)).reshape(nn, 6).T
    for got, ref in ((out["rhs"], rhs_ref), (out["diag"], diag_ref), (out["Ap"], ap_ref)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got - ref) <= 2e-5 * np.linalg.norm(ref)
        assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
    ge = out["energy"]
    for got, ref in zip(ge, (e["photo"], e["sil"], e["sil_abs"], e["arap"], e["vel"])):
        assert abs(got - ref) <= 1e-5 * max(e["total"], 1e-12)


def params_of(state):
    st = state.astype(np.float64)
    return so3.log_all(st), st[9:12]


@pytest.mark.parametrize("standard", [False, True])
@pytest.mark.parametrize("name,gn,pcg", [("small0", 5, 10), ("small1", 5, 10), ("mid", 3, 8)])
def test_solve_matches_schedule_matched_oracle(ctx, frames, name, gn, pcg, standard):
    """Both arrangements of the PCG iteration (one launch per iteration in the
    Chronopoulos-Gear form, and the standard recurrence) against the oracle's
    PCG with the same schedule."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = frames[name]
    nn = 64 if name != "mid" else 203
    g = og.build_graph(f["xyz"], nn)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    ref = onr.solve(P, gn, "pcg", pcg)
    fr = make_frame(ctx, f, g)
    rep = cap.nonrigid_solve(ctx, fr, cap.params(*f["weights"], gn_iters=gn, pcg_iters=pcg, pcg_standard=standard))
    assert rep["status"] == 0
    assert rep["n_visible"] == ref["n_visible"] and rep["n_boundary"] == ref["n_boundary"]
    r_gpu, t_gpu = params_of(fr.node_state.cpu().numpy())
    r_ref, t_ref = params_of(ref["state"])
    assert np.linalg.norm(r_gpu - r_ref) <= 1e-4 * max(np.linalg.norm(r_ref), 1e-6)
    assert np.linalg.norm(t_gpu - t_ref) <= 1e-4 * max(np.linalg.norm(t_ref), 1e-6)
    e0 = ref["energies"][0]["total"]
    for k, e in enumerate(ref["energies"]):
        assert abs(rep["energy"][k] - e["total"]) <= 1e-5 * e0, k


@pytest.mark.parametrize("sigma,w_vel,case2,bar", [(0.0, 100.0, "exclude", 1e-4), (0.01, 100.0, "exclude", 1e-4),
                                                   (0.03, 0.0, "exclude", 1e-3), (0.03, 100.0, "exclude", 1e-3)])
def test_velocity_prior_and_case2_exclusion_match_oracle(ctx, frames, sigma, w_vel, case2, bar):
    """Temporal prior anchored at the start geometry, case-2 vertices excluded,
    from the rest state and from perturbed starts (sigma: rad and m per component).

    The first Gauss-Newton step is held to 1e-4 of the parameter change in
    every case (measured: 1.3e-5 from the 0.03 starts, where splitting the
    float32 error showed it to come from the float32 linearisation, which
    enters the right-hand side and J^T J p consistently).  The three-step
    result keeps 1e-4 for starts within 0.01 of the solution.  From the 0.03
    starts the schedule itself amplifies a first-step error of that size to
    1.6e-4 ... 1.3e-3 in FP64 alone (tests/test_oracle_sensitivity.py), so the
    three-step bar there is 1e-3; energies stay within 1e-5 everywhere."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = frames["small1"]
    g = og.build_graph(f["xyz"], 64)
    rng = np.random.default_rng(12)
    st = onr.apply_update(onr.identity_state(64), rng.normal(0, sigma, 384)).astype(np.float32)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"], state0=st,
                    w_vel=w_vel, case2=case2)
    r0, t0 = params_of(st)
    for gn, step_bar in ((1, 1e-4), (3, bar)):
        ref = onr.solve(P, gn, "pcg", 8)
        fr = make_frame(ctx, f, g, state=st)
        rep = cap.nonrigid_solve(ctx, fr, cap.params(*f["weights"], gn_iters=gn, pcg_iters=8, w_vel=w_vel,
                                                     exclude_case2=case2 == "exclude"))
        assert rep["n_boundary"] == ref["n_boundary"]
        r_gpu, t_gpu = params_of(fr.node_state.cpu().numpy())
        r_ref, t_ref = params_of(ref["state"])
        er = np.linalg.norm(r_gpu - r_ref) / max(np.linalg.norm(r_ref - r0), 1e-6)
        et = np.linalg.norm(t_gpu - t_ref) / max(np.linalg.norm(t_ref - t0), 1e-6)
        e0 = ref["energies"][0]["total"]
        print("sigma %g w_vel %g, %d GN: rel r err %.2e, t err %.2e; E gpu %s ref %s" % (
            sigma, w_vel, gn, er, et, rep["energy"], [e["total"] for e in ref["energies"]]), flush=True)
        assert er <= step_bar and et <= step_bar, gn
        for k, e in enumerate(ref["energies"]):
            assert abs(rep["energy"][k] - e["total"]) <= 1e-5 * e0, k
        assert abs(rep["e_vel"] - ref["energies"][-1]["vel"]) <= 1e-5 * e0


def test_batch_equals_single_solves(ctx, frames):
    """An uneven batch in one launch sequence gives each frame's single-solve result."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    prm = cap.params(1.0, 0.1, 10.0, gn_iters=3, pcg_iters=6)
    singles, batch = [], []
    for name, nn in (("small0", 64), ("mid", 203), ("small1", 64)):
        f = frames[name]
        g = og.build_graph(f["xyz"], nn)
        a = make_frame(ctx, f, g)
        b = make_frame(ctx, f, g, tmpl=a.template)
        singles.append((a, cap.nonrigid_solve(ctx, a, prm)))
        batch.append(b)
    reps = cap.batch_solve(ctx, batch, prm)
    for (a, ra), b, rb in zip(singles, batch, reps):
        assert np.array_equal(a.node_state.cpu().numpy(), b.node_state.cpu().numpy())
        assert ra["energy"] == rb["energy"]


def test_large_tile_grid_equals_single_solves(ctx, frames):
    """A batch whose tile grid exceeds what the chip holds at once (16-vertex
    tiles, over 1024 tiles in total) takes the two-pass J^T J p reduction and
    the standard PCG recurrence; its frames equal their single solves with the
    standard recurrence forced (one-pass reduction) bit for bit."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    prm = cap.params(1.0, 0.1, 10.0, gn_iters=2, pcg_iters=5, pcg_standard=True)
    singles, batch = [], []
    for name, nn in (("mid", 203), ("small0", 64), ("mid", 203), ("small1", 64), ("mid", 203)):
        f = frames[name]
        g = og.build_graph(f["xyz"], nn)
        a = make_frame(ctx, f, g, vertices_per_tile=16)
        b = make_frame(ctx, f, g, tmpl=a.template)
        singles.append((a, cap.nonrigid_solve(ctx, a, prm)))
        batch.append(b)
    assert sum(fr.template.n_tiles for fr in batch) > 1024
    assert all(a.template.n_tiles <= 1024 for a, _ in singles)
    reps = cap.batch_solve(ctx, batch, prm)
    for (a, ra), b, rb in zip(singles, batch, reps):
        assert np.array_equal(a.node_state.cpu().numpy(), b.node_state.cpu().numpy())
        assert ra["energy"] == rb["energy"]


def test_wide_batch_equals_single_solves(ctx, frames):
    """A batch with 16384 or more image columns in total takes the
    thread-per-column segment scan of the distance transform (single frames
    take the wave-per-column scan); its frames equal their single solves bit
    for bit."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    prm = cap.params(1.0, 0.1, 10.0, gn_iters=1, pcg_iters=2, pcg_standard=True)   # 32 frames: over 1024 tiles
    f = frames["mid"]
    g = og.build_graph(f["xyz"], 203)
    a = make_frame(ctx, f, g)
    ra = cap.nonrigid_solve(ctx, a, prm)
    batch = [make_frame(ctx, f, g, tmpl=a.template) for _ in range(32)]
    assert sum(fr.camera.width for fr in batch) >= 16384
    reps = cap.batch_solve(ctx, batch, prm)
    for b, rb in zip(batch, reps):
        assert np.array_equal(a.node_state.cpu().numpy(), b.node_state.cpu().numpy())
        assert ra["energy"] == rb["energy"]


def test_graph_replay_matches_eager(ctx, frames):
    """Solves replayed from captured HIP graphs equal the eager launches bit for
    bit, on every replay, with unrelated eager GPU work and synchronisations in
    between, for two launch shapes (a batch of three and a single frame)."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    prm = cap.params(1.0, 0.1, 10.0, gn_iters=3, pcg_iters=6)
    fs = []
    for name, nn in (("small0", 64), ("mid", 203), ("small1", 64)):
        f = frames[name]
        fs.append(make_frame(ctx, f, og.build_graph(f["xyz"], nn)))
    starts = [fr.node_state.clone() for fr in fs]

    def run(batch):
        for fr, st in zip(fs, starts):
            fr.node_state.copy_(st)
        reps = cap.batch_solve(ctx, fs, prm) if batch else [cap.nonrigid_solve(ctx, fs[1], prm)]
        idx = range(3) if batch else [1]
        return [fs[i].node_state.cpu().numpy().copy() for i in idx], [r["energy"] for r in reps]

    eager = {b: run(b) for b in (True, False)}
    cap.set_graphs(ctx, True)
    try:
        for rep in range(3):
            for b in (True, False):
                got = run(b)
                for x, y in zip(got[0], eager[b][0]):
                    assert np.array_equal(x, y), (rep, b)
                assert got[1] == eager[b][1], (rep, b)
                junk = torch.randn(1 << 16, device="cuda")
                float(junk.square().sum())
                torch.cuda.synchronize()
    finally:
        cap.set_graphs(ctx, False)


def test_run_to_run_deterministic(ctx, frames):
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = frames["mid"]
    g = og.build_graph(f["xyz"], 203)
    prm = cap.params(1.0, 0.1, 10.0, gn_iters=2, pcg_iters=5)
    a = make_frame(ctx, f, g)
    b = make_frame(ctx, f, g, tmpl=a.template)
    cap.nonrigid_solve(ctx, a, prm)
    cap.nonrigid_solve(ctx, b, prm)
    assert np.array_equal(a.node_state.cpu().numpy(), b.node_state.cpu().numpy())


def test_degenerate_schedules_and_masks(ctx, frames):
    """pcg_iters = 0 leaves the state; an empty mask switches the silhouette term off;
    a 4-node graph and a small tile size still match the oracle."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = dict(frames["small0"])
    g = og.build_graph(f["xyz"], 64)
    fr = make_frame(ctx, f, g)
    rep = cap.nonrigid_solve(ctx, fr, cap.params(gn_iters=2, pcg_iters=0))
    assert np.array_equal(fr.node_state.cpu().numpy(), np.asarray(fr.node_state.cpu().numpy()))
    st = fr.node_state.cpu().numpy()
    assert np.allclose(st[[0, 4, 8]], 1.0) and np.allclose(st[[1, 2, 3, 5, 6, 7, 9, 10, 11]], 0.0)
    assert rep["energy"][0] == rep["energy"][2]
    f["mask"] = np.zeros_like(f["mask"])
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    ref = onr.solve(P, 2, "pcg", 4)
    fr = make_frame(ctx, f, g)
    rep = cap.nonrigid_solve(ctx, fr, cap.params(gn_iters=2, pcg_iters=4))
    assert rep["e_sil"] == 0.0 and rep["e_sil_abs"] == 0.0
    assert abs(rep["energy"][-1] - ref["energies"][-1]["total"]) <= 1e-5 * ref["energies"][0]["total"]
    # 4 nodes, tiles of 37 vertices (ragged tails everywhere)
    f = frames["small1"]
    g = og.build_graph(f["xyz"], 4)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    ref = onr.solve(P, 3, "pcg", 5)
    fr = make_frame(ctx, f, g, vertices_per_tile=37)
    rep = cap.nonrigid_solve(ctx, fr, cap.params(gn_iters=3, pcg_iters=5))
    r_gpu, t_gpu = params_of(fr.node_state.cpu().numpy())
    r_ref, t_ref = params_of(ref["state"])
    assert np.linalg.norm(r_gpu - r_ref) <= 1e-4 * max(np.linalg.norm(r_ref), 1e-6)
    assert np.linalg.norm(t_gpu - t_ref) <= 1e-4 * max(np.linalg.norm(t_ref), 1e-6)


def test_invalid_arguments_are_rejected(ctx, frames):
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = frames["small0"]
    g = og.build_graph(f["xyz"], 64)
    fr = make_frame(ctx, f, g)
    before = fr.node_state.clone()
    for bad in (cap.params(gn_iters=0), cap.params(gn_iters=33), cap.params(pcg_iters=-1),
                cap.params(w_sil=-1.0), cap.params(w_photo=float("nan"))):
        with pytest.raises(cap.CaptureError) as ei:
            cap.nonrigid_solve(ctx, fr, bad)
        assert ei.value.code == -1
    assert torch.equal(before, fr.node_state)
    with pytest.raises(cap.CaptureError):
        cap.graph_build(ctx, fr.xyz, 3)


def test_tile_size_autotuner_and_tile_independence(ctx, frames):
    """The autotuner returns one of its candidates and leaves the start states
    alone; every tile size reproduces the oracle within the parity bar."""
    import paper_1810_02648_amd as cap
    from gpu_util import dev, device_graph, make_frame
    f = frames["mid"]
    g = og.build_graph(f["xyz"], 203)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    ref = onr.solve(P, 3, "pcg", 8)
    prm = cap.params(*f["weights"], gn_iters=3, pcg_iters=8)
    fr = make_frame(ctx, f, g)
    start = fr.node_state.clone()
    best, times = cap.autotune_tiles(ctx, [dev(f["tri"])], [device_graph(g)], [fr], prm, candidates=(64, 160, 256))
    print("autotune", best, times, flush=True)
    assert best in (64, 160, 256) and all(t > 0 for t in times.values())
    assert torch.equal(fr.node_state, start)
    r_ref, t_ref = params_of(ref["state"])
    for tile in (64, 160, 256):
        fr = make_frame(ctx, f, g, vertices_per_tile=tile)
        rep = cap.nonrigid_solve(ctx, fr, prm)
        r_gpu, t_gpu = params_of(fr.node_state.cpu().numpy())
        assert np.linalg.norm(r_gpu - r_ref) <= 1e-4 * max(np.linalg.norm(r_ref), 1e-6), tile
        assert np.linalg.norm(t_gpu - t_ref) <= 1e-4 * max(np.linalg.norm(t_ref), 1e-6), tile
        assert abs(rep["energy"][-1] - ref["energies"][-1]["total"]) <= 1e-5 * ref["energies"][0]["total"]


def test_large_graph_split_pcg_matches_oracle(ctx):
    """More than 1365 nodes (more (component, node) pairs than one workgroup
    holds in registers): the PCG vector updates run distributed over the tiles
    like every other size; the solve matches the oracle."""
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    f = synth.make_nonrigid_frame("small", 5, n_vertices=12001, n_nodes=1500, side=400)
    g = og.build_graph(f["xyz"], 1500)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    ref = onr.solve(P, 2, "pcg", 6)
    fr = make_frame(ctx, f, g)
    rep = cap.nonrigid_solve(ctx, fr, cap.params(*f["weights"], gn_iters=2, pcg_iters=6))
    r_gpu, t_gpu = params_of(fr.node_state.cpu().numpy())
    r_ref, t_ref = params_of(ref["state"])
    er = np.linalg.norm(r_gpu - r_ref) / max(np.linalg.norm(r_ref), 1e-6)
    et = np.linalg.norm(t_gpu - t_ref) / max(np.linalg.norm(t_ref), 1e-6)
    print("split pcg: rel r err %.2e t err %.2e" % (er, et), flush=True)
    assert er <= 1e-4 and et <= 1e-4
    e0 = ref["energies"][0]["total"]
    for k, e in enumerate(ref["energies"]):
        assert abs(rep["energy"][k] - e["total"]) <= 1e-5 * e0, k
