"""Pins for the per-vertex non-rigid oracle (paper Sec. 3.4 regularisers, Sec. 3.1 Table 1).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own formulas: the printed Table 1, the
topology of a mesh whose neighbourhoods are known, energies that vanish by
invariance, closed-form energies and minimisers, finite differences, and the
chain rule against the (separately pinned) embedded-deformation oracle.
"""
import os

import numpy as np
import pytest

import synth
from oracle import decisions as od
from oracle import graph as og
from oracle import nonrigid as onr
from oracle import so3
from oracle import vertex as ov
from synth.meshes import ellipsoid_icosphere
from synth.render import render_targets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def octahedron():
    xyz = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float).T
    tri = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]).T
    return xyz, tri.astype(np.int32)


@pytest.fixture(scope="module")
def mini():
    """A 162-vertex ellipsoid seen by a 64-pixel camera, rendered after a small deformation."""
    xyz, tri = ellipsoid_icosphere(2, (0.15, 0.5, 0.15), (0.0, 0.0, 2.5))
    cam = synth.Camera.square(64)
    rng = np.random.default_rng(3)
    rgb = rng.uniform(0, 1, (3, xyz.shape[1])).astype(np.float32)
    gt = (xyz + rng.normal(0, 0.005, xyz.shape)).astype(np.float32)
    mask, image = render_targets(gt, tri, rgb, cam)
    classes = rng.integers(1, 8, xyz.shape[1])
    return dict(xyz=xyz, tri=tri, cam=cam, rgb=rgb, mask=mask, image=image, classes=classes, gt=gt)


def problem(m, weights, posed=None, start=None, prev=None, prev2=None, rest=None, **kw):
    rest = m["xyz"] if rest is None else rest
    posed = m["xyz"] if posed is None else posed
    return ov.VertexProblem(rest, posed, m["tri"], m["rgb"], m["classes"], m["cam"], m["mask"], m["image"],
                            weights, start=start, prev=prev, prev2=prev2, **kw)


# ---------------------------------------------------------------- Table 1 and the one-ring
def test_class_weights_are_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_nonrigidity_weights.txt")) if not l.startswith("#")]
    ids = np.array([int(r[0]) for r in rows])
    w = np.array([float(r[1]) for r in rows])
    assert np.array_equal(ov.vertex_weights(ids), w)
    with pytest.raises(ValueError):
        ov.vertex_weights([0])


def test_one_ring_of_octahedron():
    xyz, tri = octahedron()
    nb = ov.one_ring(tri, 6)
    for i in range(6):
        antipode = i ^ 1
        assert sorted(nb[i].tolist()) == [j for j in range(6) if j not in (i, antipode)]


def test_edge_weight_averages_the_two_classes_over_the_degree(mini):
    P = problem(mini, dict(w_smooth=1.0))
    s = ov.CLASS_WEIGHTS[mini["classes"] - 1]
    for e in np.random.default_rng(0).integers(0, P.e_src.size, 20):
        i, j = P.e_src[e], P.e_dst[e]
        deg = sum(1 for a, b in zip(P.e_src, P.e_dst) if a == i)
        assert P.e_w[e] == pytest.approx((s[i] + s[j]) / 2.0 / deg, rel=1e-15)


# ---------------------------------------------------------------- regulariser closed forms
def test_smooth_vanishes_at_posed_and_under_translation(mini):
    rng = np.random.default_rng(1)
    posed = mini["xyz"] + rng.normal(0, 0.01, mini["xyz"].shape)
    P = problem(mini, dict(w_smooth=10.0), posed=posed)
    assert P.energy(posed)["smooth"] < 1e-24
    assert P.energy(posed + np.array([[0.3], [-0.1], [0.2]]))["smooth"] < 1e-20
    _, rhs, _ = P.normal_equations(posed)
    assert np.abs(rhs).max() < 1e-12


def test_smooth_single_vertex_displacement(mini):
    """Moving one vertex k by d changes 2 |N_k| directed edge differences by d:
    E = w |d|^2 sum_{j in N_k} (s_kj / |N_k| + s_jk / |N_j|)."""
    P = problem(mini, dict(w_smooth=3.0))
    s = ov.CLASS_WEIGHTS[mini["classes"] - 1]
    nb = ov.one_ring(mini["tri"], mini["xyz"].shape[1])
    d = np.array([0.01, -0.02, 0.005])
    for k in (0, 17, 100):
        V = mini["xyz"].astype(np.float64).copy()
        V[:, k] += d
        expect = 3.0 * (d @ d) * sum((s[k] + s[j]) / 2 * (1 / len(nb[k]) + 1 / len(nb[j])) for j in nb[k])
        assert P.energy(V)["smooth"] == pytest.approx(expect, rel=1e-12)


def test_edge_vanishes_under_rigid_motion_and_scales_quadratically(mini):
    P = problem(mini, dict(w_edge=2.0))
    rest = mini["xyz"].astype(np.float64)
    R = so3.exp([0.3, -0.2, 0.5])
    assert P.energy(R @ rest + np.array([[0.1], [0.2], [-0.3]]))["edge"] < 1e-22
    s = ov.CLASS_WEIGHTS[mini["classes"] - 1]
    nb = ov.one_ring(mini["tri"], rest.shape[1])
    c = 1.07
    expect = 0.0
    for i in range(rest.shape[1]):
        for j in nb[i]:
            L = np.linalg.norm(rest[:, i] - rest[:, j])
            expect += (s[i] + s[j]) / 2 / len(nb[i]) * ((c - 1.0) * L) ** 2
    assert P.energy(c * rest)["edge"] == pytest.approx(2.0 * expect, rel=1e-10)


def test_temporal_terms_minimiser_is_the_closed_form_translation(mini):
    """With smooth, edge (rigid posed mesh), velocity and acceleration only and
    V^{t-1} = V^S + c1, V^{t-2} = V^S + c2, the minimiser is the translation
    V^S + lam, lam = (w_v c1 + w_a (2 c1 - c2)) / (w_v + w_a): smooth and edge
    vanish for every translation, and the temporal terms are then a 1-D
    least-squares problem per coordinate."""
    rest = mini["xyz"].astype(np.float64)
    posed = so3.exp([0.1, 0.2, -0.1]) @ rest + np.array([[0.02], [0.0], [0.05]])
    c1, c2 = np.array([0.01, -0.02, 0.03]), np.array([0.03, 0.01, -0.02])
    for wv, wa in ((2.0, 0.0), (0.0, 1.5), (0.7, 0.3)):
        w = dict(w_smooth=5.0, w_edge=3.0, w_vel=wv, w_acc=wa)
        P = problem(mini, w, posed=posed, start=posed, prev=posed + c1[:, None], prev2=posed + c2[:, None])
        out = ov.solve(P, 3, "chol")
        lam = (wv * c1 + wa * (2 * c1 - c2)) / (wv + wa)
        assert np.abs(out["V"] - (posed + lam[:, None])).max() < 1e-10


def test_missing_temporal_inputs_are_rejected(mini):
    with pytest.raises(ValueError):
        problem(mini, dict(w_vel=1.0))
    with pytest.raises(ValueError):
        problem(mini, dict(w_acc=1.0), prev=mini["xyz"])


# ---------------------------------------------------------------- derivatives
def test_colour_kernel_prunes_photometric_rows_by_residual_norm(mini):
    """Sec. 3.4 robust colour kernel in the per-vertex oracle: template colours
    set to the blurred image's colour at each vertex plus an offset whose norm
    is 0.49 or 0.51 (spread over the channels).  With tau_c = 0.5 exactly the
    0.49 residuals remain, with their Jacobian rows, and the 0.51 rows vanish;
    with tau_c = inf all remain.  The energy is the offsets' closed form."""
    from oracle import image as oi
    w = dict(w_photo=3.0, w_sil=0.0, w_smooth=0.0, w_edge=0.0, w_vel=0.0, w_acc=0.0)
    V = mini["xyz"].astype(np.float64)
    P0 = problem(mini, w)
    cam = mini["cam"]
    val, _, _ = oi.sample(P0.image(), cam.fx * V[0] / V[2] + cam.cx, cam.fy * V[1] / V[2] + cam.cy)
    rng = np.random.default_rng(8)
    dirs = rng.normal(size=(3, V.shape[1]))
    dirs /= np.linalg.norm(dirs, axis=0)
    small = rng.uniform(size=V.shape[1]) < 0.5
    mag = np.where(small, 0.49, 0.51)
    rgb = val + mag * dirs
    vid = P0.vis_idx[V[2][P0.vis_idx] > 0]
    assert vid.size > 20 and 0 < small[vid].sum() < vid.size
    for tau, expect in ((0.5, 3.0 * 0.49 ** 2 * small[vid].sum()), (np.inf, 3.0 * (mag[vid] ** 2).sum())):
        P = ov.VertexProblem(V, V, mini["tri"], rgb, mini["classes"], cam, mini["mask"], mini["image"], w, tau_c=tau)
        F, b, J, e = P.linearize(V)
        assert e["photo"] == pytest.approx(expect, rel=1e-9), tau
        rows = np.abs(J[: 3 * vid.size]).sum(axis=1).A.ravel().reshape(3, vid.size).sum(axis=0)
        if np.isfinite(tau):
            assert (rows[~small[vid]] == 0).all() and (rows[small[vid]] > 0).all()
            assert (F[: 3 * vid.size].reshape(3, vid.size)[:, ~small[vid]] == 0).all()
        else:
            assert (rows > 0).all()


def test_pyramid_takes_the_levels_in_order_and_touches_only_the_photometric_term(mini):
    """Sec. 3.4 pyramid, one Gauss-Newton step per level (15, 9, 3): the first
    step's energy is the photometric energy on the 15-tap image at the start
    and the final energy the one on the 3-tap image at the result (each
    computed here from the separately pinned blur and sampling); without the
    photometric term the schedule changes nothing, bit for bit."""
    from oracle import image as oi
    rng = np.random.default_rng(21)
    V0 = mini["xyz"].astype(np.float64) + rng.normal(0, 0.003, mini["xyz"].shape)
    cam = mini["cam"]

    def photo(P, V, k):
        vid = P.vis_idx[V[2][P.vis_idx] > 0]
        val, _, _ = oi.sample(oi.blur(mini["image"], k), cam.fx * V[0, vid] / V[2, vid] + cam.cx,
                              cam.fy * V[1, vid] / V[2, vid] + cam.cy)
        return 2.0 * float(((val - mini["rgb"][:, vid].astype(np.float64)) ** 2).sum())

    w = dict(w_photo=2.0, w_sil=0.5, w_smooth=7.0, w_edge=11.0, w_vel=0.0, w_acc=0.0)
    P = problem(mini, w, start=V0.astype(np.float32))
    out = ov.solve(P, 3, "chol", blur_schedule=(15, 9, 3))
    Vs = P.start.astype(np.float64)
    assert out["energies"][0]["photo"] == pytest.approx(photo(P, Vs, 15), rel=1e-12)
    assert out["energies"][-1]["photo"] == pytest.approx(photo(P, out["V"], 3), rel=1e-12)
    assert photo(P, Vs, 15) != pytest.approx(photo(P, Vs, 3), rel=1e-3)     # the levels differ here
    w0 = dict(w, w_photo=0.0)
    P0 = problem(mini, w0, start=V0.astype(np.float32))
    a = ov.solve(P0, 3, "chol", blur_schedule=(15, 9, 3))["V"]
    b = ov.solve(P0, 3, "chol")["V"]
    assert np.array_equal(a, b)


def test_jacobian_matches_central_differences(mini):
    rng = np.random.default_rng(5)
    rest = mini["xyz"].astype(np.float64)
    posed = rest + rng.normal(0, 0.004, rest.shape)
    w = dict(w_photo=2.0, w_sil=0.5, w_smooth=7.0, w_edge=11.0, w_vel=0.3, w_acc=0.2)
    P = problem(mini, w, posed=posed, start=posed.astype(np.float32), prev=posed + 0.003, prev2=posed - 0.002)
    assert P.vis_idx.size > 20 and P.bnd_idx.size > 5
    V = posed + rng.normal(0, 0.002, rest.shape)
    F, b, J, _ = P.linearize(V)
    J = J.toarray()
    h = 1e-6
    for col in rng.choice(J.shape[1], 60, replace=False):
        i, a = divmod(col, 3)
        Vp, Vm = V.copy(), V.copy()
        Vp[a, i] += h
        Vm[a, i] -= h
        fd = (P.linearize(Vp, False)[0] - P.linearize(Vm, False)[0]) / (2 * h)
        assert np.abs(fd - J[:, col]).max() <= 2e-4 * max(1.0, np.abs(J[:, col]).max()), col
    # energy = sum b F^2 per term, and the system's gradient is the energy's
    e = P.energy(V)
    assert e["total"] == pytest.approx(float((b * F * F).sum()), rel=1e-12)


def test_data_rows_agree_with_the_deformation_graph_oracle_by_the_chain_rule(small_frame):
    """At the same decisions, the ED oracle's photometric and silhouette rows are
    the per-vertex rows composed with dV/d(node unknowns)."""
    f = small_frame
    g = og.build_graph(f["xyz"], f["n_nodes"])
    nn = f["n_nodes"]
    rng = np.random.default_rng(2)
    st = onr.identity_state(nn).astype(np.float64)
    for k in range(nn):
        st[:9, k] = (so3.exp(rng.normal(0, 0.02, 3))).ravel()
    st[9:] = rng.normal(0, 0.004, (3, nn))
    st = st.astype(np.float32)
    E = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], (1.3, 0.7, 0.0), state0=st)
    start = np.stack([E.dec["X"], E.dec["Y"], E.dec["Z"]])
    P = ov.VertexProblem(f["xyz"], f["xyz"], f["tri"], f["rgb"], np.full(f["xyz"].shape[1], 2), f["cam"], f["mask"],
                         f["image"], dict(w_sil=1.3, w_photo=0.7), start=start)
    assert np.array_equal(P.vis_idx, E.vis_idx) and np.array_equal(P.bnd_idx, E.bnd_idx)
    V, q = onr.ed_deform(f["xyz"], g, st)
    Fe, be, Je, _ = E.linearize(st)
    Fv, bv, Jv, _ = P.linearize(V)
    nd = 3 * P.vis_idx.size + P.bnd_idx.size           # data rows come first in both
    assert np.allclose(Fe[:nd], Fv[:nd], rtol=0, atol=1e-12)
    assert np.array_equal(be[:nd], bv[:nd])
    # dV/dx: 3N x 6nn
    nv = f["xyz"].shape[1]
    M = np.zeros((3 * nv, 6 * nn))
    for k, blk in onr._vertex_cols(g, q, np.arange(nv)):
        for a in range(3):
            for c in range(6):
                M[3 * np.arange(nv) + a, 6 * k + c] += blk[:, a, c]
    lhs = Je.toarray()[:nd]
    rhs = Jv.toarray()[:nd] @ M
    assert np.abs(lhs - rhs).max() <= 1e-9 * max(1.0, np.abs(lhs).max())


def test_gauss_newton_lowers_the_energy_on_a_body_frame():
    import synth.sequence as ss
    seq = ss.make_sequence("body_small", 0, n_frames=4, workers=1)
    f = ss.vertex_frame(seq, 3)
    P = ov.VertexProblem(f["rest"], f["posed"], f["tri"], f["rgb"], f["classes"], f["cam"], f["mask"], f["image"],
                         f["weights"], start=f["start"], prev=f["prev"], prev2=f["prev2"], case2="exclude",
                         outline=True)
    out = ov.solve(P, 3, "pcg", 4)
    e = [x["total"] for x in out["energies"]]
    assert e[-1] < 0.5 * e[0]
    exact = ov.solve(P, 3, "chol")
    assert exact["energies"][-1]["total"] <= e[-1] * 1.0001


# ---------------------------------------------------------------- vertex snapping (Sec. 3.4)
def test_snapping_lands_contour_vertices_on_the_silhouette_and_warps_the_band(mini):
    """Moved off the silhouette by less than max_px, contour vertices walk back
    onto it (I_DT at the snapped projection below tol); the band's warp is the
    given number of Jacobi sweeps of the mean-value rule; vertices outside the
    band do not move."""
    P = problem(mini, dict(w_sil=1.0), start=mini["gt"])
    V0 = mini["gt"].astype(np.float64)
    rng = np.random.default_rng(8)
    V = V0 + rng.normal(0, 0.002, V0.shape)
    out, snapped = ov.snap_vertices(P, V, max_px=3.0, steps=6, rings=2, iters=8)
    assert snapped.sum() > 10
    cam = mini["cam"]
    from oracle.image import sample
    X, Y, Z = out[:, snapped]
    d, _, _ = sample(P.dt, cam.fx * X / Z + cam.cx, cam.fy * Y / Z + cam.cy)
    assert np.median(d) < 0.1
    assert np.allclose(out[2], V[2])                  # depth is kept
    # band and outside
    nb = ov.one_ring(mini["tri"], V.shape[1])
    ring1 = np.zeros(V.shape[1], bool)
    for i in np.nonzero(snapped)[0]:
        ring1[nb[i]] = True
    ring1 &= ~snapped
    ring2 = np.zeros_like(ring1)
    for i in np.nonzero(ring1)[0]:
        ring2[nb[i]] = True
    ring2 &= ~snapped & ~ring1
    outside = ~(snapped | ring1 | ring2)
    assert np.array_equal(out[:, outside], V[:, outside])
    assert np.abs(out[:, ring1] - V[:, ring1]).max() > 0
    # one sweep: a ring-1 vertex gets the mean of its neighbours' starting displacements
    out1, _ = ov.snap_vertices(P, V, max_px=3.0, steps=6, rings=2, iters=1)
    d_snap = out - V
    i = np.nonzero(ring1)[0][0]
    expect = np.mean([d_snap[:, j] if snapped[j] else np.zeros(3) for j in nb[i]], axis=0)
    assert np.allclose(out1[:, i] - V[:, i], expect, rtol=0, atol=1e-15)


def test_laplacian_warp_converges_to_the_harmonic_interpolant(mini):
    """Many sweeps of the warp reach the harmonic displacement field of the band
    (Dirichlet data: snap displacements, 0 beyond the band), solved directly."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    P = problem(mini, dict(w_sil=1.0), start=mini["gt"])
    V = mini["gt"].astype(np.float64) + np.random.default_rng(9).normal(0, 0.002, mini["gt"].shape)
    out, snapped = ov.snap_vertices(P, V, iters=4000)
    d = out - V
    nb = ov.one_ring(mini["tri"], V.shape[1])
    nv = V.shape[1]
    dist = np.where(snapped, 0, 3)
    for r in (1, 2):
        for i in range(nv):
            if dist[i] > r and any(dist[j] == r - 1 for j in nb[i]):
                dist[i] = r
    band = np.nonzero((dist >= 1) & (dist <= 2))[0]
    idx = {v: k for k, v in enumerate(band)}
    A = sps.lil_matrix((band.size, band.size))
    rhs = np.zeros((band.size, 3))
    for k, i in enumerate(band):
        A[k, k] = 1.0
        for j in nb[i]:
            if j in idx:
                A[k, idx[j]] -= 1.0 / len(nb[i])
            elif snapped[j]:
                rhs[k] += d[:, j] / len(nb[i])
    x = spl.spsolve(A.tocsc(), rhs)
    assert np.abs(x.T - d[:, band]).max() < 1e-9


# ---------------------------------------------------------------- body-part mask (Sec. 3.4)
def test_part_mask_renders_labels_and_dilates_with_torso_precedence():
    """Two labelled squares (torso 0 at left, part 3 at right) with a 4-pixel
    gap: the rendered labels cover exactly each square's pixels; after 3
    growth steps the torso holds the 3 gap pixels next to it (it takes
    precedence where both grow) and part 3 the last one; the background
    grows by 3 pixels."""
    cam = synth.Camera(24, 12, 100.0, 100.0, 0.0, 0.0)
    Z = 2.0
    def square(x0, x1, y0, y1):      # pixel-corner rectangle as two triangles, counter-clockwise on screen
        pts = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
        return [(p[0] * Z / 100.0, p[1] * Z / 100.0, Z) for p in pts]
    P = square(1.5, 6.5, 2.5, 8.5) + square(10.5, 16.5, 2.5, 8.5)
    xyz = np.array(P, np.float32).T
    tri = np.array([[0, 2, 1], [0, 3, 2], [4, 6, 5], [4, 7, 6]], np.int32).T
    from oracle.decisions import frame_decisions_from_positions
    mask = np.zeros((12, 24), np.uint8)
    dec = frame_decisions_from_positions(xyz[0], xyz[1], xyz[2], tri, cam, mask, np.zeros((12, 24), np.float32))
    parts = np.array([0, 0, 0, 0, 3, 3, 3, 3])
    lab0 = ov.part_label_image(dec, tri, parts, cam, dilation=0)
    covered = dec["zbuf"] > 0
    assert np.array_equal(lab0 >= 0, covered)
    assert set(np.unique(lab0[:, :8])) <= {-1, 0} and set(np.unique(lab0[:, 9:])) <= {-1, 3}
    lab = ov.part_label_image(dec, tri, parts, cam, dilation=3)
    cols0 = np.nonzero((lab0 == 0).any(axis=0))[0]
    cols3 = np.nonzero((lab0 == 3).any(axis=0))[0]
    row = 5
    assert (lab[row, cols0.max() + 1:cols0.max() + 4] == 0).all()          # torso grew by 3 into the gap
    gap = cols3.min() - cols0.max() - 1
    assert gap == 4
    assert lab[row, cols3.min()] == 3 and (lab[row, cols3.max() + 1:cols3.max() + 4] == 3).all()
    assert lab[row, cols0.max() + 4] == 3                                   # part 3 grew left into the remaining gap pixel
    # the background grows by exactly 3 pixels around the union
    from scipy.ndimage import binary_dilation
    assert np.array_equal(lab >= 0, binary_dilation(covered, np.ones((3, 3), bool), iterations=3))
