"""Pins for the FP64 oracle: closed forms, invariants, finite differences, brute force.

None of these re-types an oracle formula: each checks the oracle against a
fact fixed by the mathematics (a closed form, an invariant, a finite
difference, a brute-force search, or a library routine solving the same
problem a different way).
"""
import numpy as np
import pytest
from scipy.optimize import least_squares

import synth
from oracle import decisions as od
from oracle import graph as og
from oracle import image as oi
from oracle import nonrigid as onr
from oracle import so3


def rigid_state(graph, xyz, R, t):
    """Node state reproducing the global rigid motion x -> R x + t."""
    g = xyz.astype(np.float64)[:, graph["node_vertex"]]
    nn = g.shape[1]
    st = np.zeros((12, nn))
    st[:9] = np.repeat(R.reshape(9, 1), nn, axis=1)
    st[9:] = (R @ g) + t[:, None] - g
    return st


# ---------------------------------------------------------------- SO(3)
def test_so3_roundtrip_and_orthonormal():
    rng = np.random.default_rng(1)
    for _ in range(50):
        a = rng.normal(size=3)
        w = a / np.linalg.norm(a) * rng.uniform(1e-9, 3.0)   # angle below pi
        R = so3.exp(w)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13
        assert np.allclose(so3.log(R), w, atol=1e-9 * max(1.0, np.linalg.norm(w)))
    # rotation about z by pi/2 maps x to y
    assert np.allclose(so3.exp([0, 0, np.pi / 2]) @ [1, 0, 0], [0, 1, 0], atol=1e-15)


# ---------------------------------------------------------------- ED closed forms
def test_ed_identity_translation_rigid(small_frame):
    f = small_frame
    g = og.build_graph(f["xyz"], 64)
    xyz = f["xyz"].astype(np.float64)
    nn = 64
    V, _ = onr.ed_deform(f["xyz"], g, onr.identity_state(nn))
    assert np.abs(V - xyz).max() < 1e-6          # weights sum to 1 (float32 inputs)
    st = onr.identity_state(nn).astype(np.float64)
    st[9:] = np.array([0.01, -0.02, 0.03])[:, None]
    V, _ = onr.ed_deform(f["xyz"], g, st)
    assert np.abs(V - (xyz + st[9:, :1])).max() < 1e-6
    R = so3.exp([0.1, -0.2, 0.05])
    t = np.array([0.02, 0.0, -0.01])
    V, _ = onr.ed_deform(f["xyz"], g, rigid_state(g, f["xyz"], R, t))
    assert np.abs(V - (R @ xyz + t[:, None])).max() < 1e-6


def test_arap_zero_under_rigid_motion(small_frame):
    f = small_frame
    g = og.build_graph(f["xyz"], 64)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    assert P.energy(onr.identity_state(64))["arap"] == 0.0
    st = rigid_state(g, f["xyz"], so3.exp([0.3, 0.1, -0.2]), np.array([0.1, 0.2, -0.3]))
    assert P.energy(st)["arap"] < 1e-20


# ---------------------------------------------------------------- image sampling
def test_keys_interpolates_samples_and_linear_images():
    rng = np.random.default_rng(2)
    img = rng.uniform(size=(20, 30))
    jj, ii = np.meshgrid(np.arange(20), np.arange(30), indexing="ij")
    val, _, _ = oi.sample(img, ii.ravel().astype(float), jj.ravel().astype(float))
    assert np.allclose(val, img.ravel(), atol=1e-14)
    lin = 0.3 * ii + 0.7 * jj + 0.1
    u = rng.uniform(2, 27, 200)
    v = rng.uniform(2, 17, 200)
    val, gu, gv = oi.sample(lin, u, v)
    assert np.allclose(val, 0.3 * u + 0.7 * v + 0.1, atol=1e-12)
    assert np.allclose(gu, 0.3, atol=1e-12) and np.allclose(gv, 0.7, atol=1e-12)


def test_keys_gradient_matches_finite_difference():
    rng = np.random.default_rng(3)
    img = rng.uniform(size=(16, 16))
    u = rng.uniform(2, 13, 100)
    v = rng.uniform(2, 13, 100)
    _, gu, gv = oi.sample(img, u, v)
    h = 1e-6
    fu = (oi.sample(img, u + h, v)[0] - oi.sample(img, u - h, v)[0]) / (2 * h)
    fv = (oi.sample(img, u, v + h)[0] - oi.sample(img, u, v - h)[0]) / (2 * h)
    assert np.allclose(gu, fu, atol=1e-7) and np.allclose(gv, fv, atol=1e-7)
    gx32, gy32 = oi.keys_gradient_f32(img.astype(np.float32), u.astype(np.float32), v.astype(np.float32))
    _, gu2, gv2 = oi.sample(img.astype(np.float32), u.astype(np.float32), v.astype(np.float32))
    assert np.allclose(gx32, gu2, atol=2e-5) and np.allclose(gy32, gv2, atol=2e-5)


def test_blur_preserves_constants_and_is_normalised():
    w = oi.gaussian_weights(3)
    assert abs(w.sum() - 1.0) < 1e-15 and w[0] == w[2]
    # sigma = 0.8 for k = 3
    assert abs(w[0] / w[1] - np.exp(-1.0 / (2 * 0.64))) < 1e-15
    img = np.full((3, 9, 11), 0.37)
    assert np.allclose(oi.blur(img), 0.37, atol=1e-15)


# ---------------------------------------------------------------- distance transform
def brute_edt(mask):
    c = oi.contour(mask)
    cj, ci = np.nonzero(c)
    H, W = mask.shape
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    if cj.size == 0:
        return np.zeros((H, W), np.float32)
    d2 = ((jj[..., None] - cj) ** 2 + (ii[..., None] - ci) ** 2).min(axis=-1)
    return np.sqrt(d2.astype(np.float32))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_edt_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    H, W = 40, 53
    mask = np.zeros((H, W), np.uint8)
    for _ in range(4):
        cy, cx, r = rng.integers(0, H), rng.integers(0, W), rng.integers(3, 15)
        jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        mask[(jj - cy) ** 2 + (ii - cx) ** 2 <= r * r] = 1
    dt, _ = oi.distance_transform(mask)
    assert np.array_equal(dt, brute_edt(mask))


def test_edt_special_cases():
    mask = np.zeros((30, 40), np.uint8)
    mask[12, 17] = 1                          # single pixel: it is its own contour
    dt, _ = oi.distance_transform(mask)
    jj, ii = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    assert np.array_equal(dt, np.sqrt(((jj - 12) ** 2 + (ii - 17) ** 2).astype(np.float32)))
    mask = np.zeros((30, 40), np.uint8)
    mask[:, :15] = 1                          # half plane: contour is column 14 (and the border)
    dt, _ = oi.distance_transform(mask)
    col = np.abs(np.arange(40) - 14).astype(np.float32)
    assert np.array_equal(dt[:, 15:], np.broadcast_to(col[15:], (30, 25)))
    assert np.array_equal(oi.distance_transform(np.zeros((5, 6), np.uint8))[0], np.zeros((5, 6), np.float32))


# ---------------------------------------------------------------- graph
def test_graph_selection_properties(small_frame):
    xyz = small_frame["xyz"]
    g = og.build_graph(xyz, 64)
    p = xyz.T.astype(np.float64)
    nodes = g["node_vertex"]
    assert nodes[0] == 0 and len(set(nodes.tolist())) == 64
    # farthest-point property at every step (float64 check of the float32 choice)
    for n in range(1, 64):
        prev = p[nodes[:n]]
        mind = ((p[:, None, :] - prev[None]) ** 2).sum(-1).min(axis=1)
        assert mind[nodes[n]] >= mind.max() * (1 - 1e-5)
    # binding: the 4 chosen nodes are the 4 nearest
    gpos = p[nodes]
    d2 = ((p[:, None, :] - gpos[None]) ** 2).sum(-1)
    chosen = np.take_along_axis(d2, g["bind_idx"].T.astype(np.int64), axis=1)
    others = d2.copy()
    np.put_along_axis(others, g["bind_idx"].T.astype(np.int64), np.inf, axis=1)
    assert (chosen.max(axis=1) <= others.min(axis=1) * (1 + 1e-5)).all()
    assert np.allclose(g["bind_w64"].sum(axis=0), 1.0, atol=1e-14)
    assert (np.diff(g["bind_w64"], axis=0) <= 1e-15).all()   # nearer node, larger weight
    # edges: 8 nearest other nodes
    dn = ((gpos[:, None] - gpos[None]) ** 2).sum(-1)
    np.fill_diagonal(dn, np.inf)
    for k in range(64):
        e = g["edge_dst"][:, k]
        assert k not in e
        rest = np.setdiff1d(np.arange(64), np.append(e, k))
        assert dn[k, e].max() <= dn[k, rest].min() * (1 + 1e-5)


# ---------------------------------------------------------------- raster
def test_raster_watertight_and_depth(small_frame):
    f = small_frame
    cam = f["cam"]
    W, H = cam.width, cam.height
    X, Y, Z = (f["xyz"][a] for a in range(3))
    u, v, valid = od.project_f32(X, Y, Z, cam)
    front = np.zeros(H * W, np.int32)
    back = np.zeros(H * W, np.int32)
    zb = np.zeros(H * W, np.uint32)
    for face, flipped, pix, inv in od.triangle_coverage(u, v, Z, valid, f["tri"], W, H):
        # outward CCW faces project clockwise in the y-down image when front-facing
        np.add.at(back if not flipped else front, pix, 1)
        np.maximum.at(zb, pix, inv.view(np.uint32))
    assert front.max() == 1 and back.max() == 1      # no pixel covered twice by one side
    assert np.array_equal(front > 0, back > 0)       # closed convex surface: one of each
    assert np.array_equal(zb.reshape(H, W), od.raster_zbuffer(u, v, Z, valid, f["tri"], W, H))
    # depth of the nearest surface vs the analytic ellipsoid along each pixel ray
    cov = np.nonzero(zb)[0]
    jj, ii = cov // W, cov % W
    d = np.stack([(ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy, np.ones_like(ii, float)])
    a = np.array(synth.workloads.SEMI_AXES)[:, None]
    c = np.array(synth.workloads.CENTRE)[:, None]
    A = ((d / a) ** 2).sum(0)
    B = -2 * ((d * c) / a ** 2).sum(0)
    C = ((c / a) ** 2).sum(0) - 1
    disc = B * B - 4 * A * C
    ok = disc > 0
    s = (-B[ok] - np.sqrt(disc[ok])) / (2 * A[ok])
    zr = 1.0 / zb[cov][ok].view(np.float32)
    assert np.all(zr >= s - 1e-4)                     # polyhedron lies inside the ellipsoid
    assert np.median(zr - s) < 2e-3
    # coverage agrees with the independent target renderer except along the rim
    ref_mask = synth.render_targets(f["xyz"], f["tri"], f["rgb"], cam)[0]
    assert abs(int((zb > 0).sum()) - int(ref_mask.sum())) <= 20


# ---------------------------------------------------------------- Jacobian
def test_jacobian_matches_central_differences(small_frame):
    f = small_frame
    g = og.build_graph(f["xyz"], 64)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    rng = np.random.default_rng(5)
    st = onr.apply_update(onr.identity_state(64), rng.normal(0, 0.01, 384))
    F, b, J, _ = P.linearize(st)
    Jd = J.toarray()
    h = 1e-6
    for col in rng.choice(384, 24, replace=False):
        e = np.zeros(384)
        e[col] = h
        fd = (P.linearize(onr.apply_update(st, e))[0] - P.linearize(onr.apply_update(st, -e))[0]) / (2 * h)
        scale = max(1.0, np.abs(Jd[:, col]).max())
        assert np.abs(fd - Jd[:, col]).max() <= 2e-5 * scale, col


# ---------------------------------------------------------------- tiny brute-force problem
def tiny_problem(sign_free=True):
    xyz, tri = synth.ellipsoid_icosphere(1, synth.workloads.SEMI_AXES, synth.workloads.CENTRE)
    rng = np.random.default_rng(7)
    rgb = rng.uniform(size=(3, xyz.shape[1])).astype(np.float32)
    cam = synth.Camera.square(64)
    gt = synth.workloads.smooth_field(xyz, 4, rng)
    mask, image = synth.render_targets(gt, tri, rgb, cam)
    g = og.build_graph(xyz, 4)
    P = onr.Problem(xyz, tri, rgb, g, cam, mask, image, (1.0, 0.1, 10.0))
    if sign_free:
        P.bsign[:] = 1.0
    return P


def test_normal_equations_match_dense_least_squares():
    P = tiny_problem()
    st = onr.identity_state(4).astype(np.float64)
    A, rhs, _ = P.normal_equations(st)
    delta = onr.solve_cholesky(A, rhs)
    # independent: finite-difference Jacobian of the residual map, then lstsq
    F0 = P.linearize(st)[0]
    h = 1e-7
    Jfd = np.zeros((F0.size, 24))
    for c in range(24):
        e = np.zeros(24)
        e[c] = h
        Jfd[:, c] = (P.linearize(onr.apply_update(st, e))[0] - P.linearize(onr.apply_update(st, -e))[0]) / (2 * h)
    step, *_ = np.linalg.lstsq(Jfd, -F0, rcond=None)
    assert np.allclose(delta, step, rtol=1e-5, atol=1e-8 * np.abs(step).max())


def test_gauss_newton_step_vanishes_at_scipy_minimiser():
    """At a least-squares minimiser found by SciPy (finite-difference Jacobian,
    trust region), the oracle's energy equals SciPy's cost and its analytic
    Gauss-Newton step and gradient vanish."""
    P = tiny_problem()

    def resid(x):
        return P.linearize(onr.apply_update(onr.identity_state(4), x))[0]

    ref = least_squares(resid, np.zeros(24), method="trf", xtol=1e-15, ftol=1e-15, gtol=1e-15)
    st = onr.apply_update(onr.identity_state(4), ref.x)
    A, rhs, e = P.normal_equations(st)
    assert abs(e["total"] - 2 * ref.cost) <= 1e-12 * e["total"]
    assert np.linalg.norm(rhs) <= 1e-6 * np.linalg.norm(P.normal_equations(onr.identity_state(4))[1])
    delta = onr.solve_cholesky(A, rhs)
    assert np.abs(delta).max() < 1e-7


def test_pcg_reaches_the_cholesky_solution():
    P = tiny_problem()
    A, rhs, _ = P.normal_equations(onr.identity_state(4).astype(np.float64))
    x_c = onr.solve_cholesky(A, rhs)
    x_p = onr.solve_pcg(A, rhs, 200)
    assert np.linalg.norm(x_p - x_c) <= 1e-8 * np.linalg.norm(x_c)
    # with n iterations CG is exact in exact arithmetic; on this system it is close
    x_n = onr.solve_pcg(A, rhs, 24)
    assert np.linalg.norm(x_n - x_c) <= 1e-3 * np.linalg.norm(x_c)


# ---------------------------------------------------------------- zero residual / decrease
def test_self_rendered_targets(small_frame):
    f = small_frame
    g = og.build_graph(f["xyz"], 64)
    mask, image = synth.render_targets(f["xyz"], f["tri"], f["rgb"], f["cam"])
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], mask, image, f["weights"])
    e = P.energy(onr.identity_state(64))
    assert e["arap"] == 0.0
    # boundary vertices sit on the rendered contour (within the rim discretisation)
    d, _, _ = oi.sample(P.dt, P.dec["u"][P.bnd_idx].astype(float), P.dec["v"][P.bnd_idx].astype(float))
    assert np.median(d) < 0.75 and d.max() < 2.0
    # constant colour template and image: photometric residual vanishes
    const = np.full_like(f["rgb"], 0.5)
    Pc = onr.Problem(f["xyz"], f["tri"], const, g, f["cam"], mask, np.full_like(image, 0.5), f["weights"])
    assert Pc.energy(onr.identity_state(64))["photo"] < 1e-25


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_energy_decreases_and_recovers(seed):
    f = synth.make_nonrigid_frame("small", seed)
    g = og.build_graph(f["xyz"], 64)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    out = onr.solve(P, 5, "chol")
    E = [e["total"] for e in out["energies"]]
    assert E[1] < E[0] and E[-1] < 0.3 * E[0]
    # monocular: depth is weakly observed, so compare image-plane positions
    V, _ = onr.ed_deform(f["xyz"], g, out["state"])
    cam = f["cam"]

    def proj(p):
        return np.stack([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    gt = proj(f["gt_xyz"].astype(np.float64))
    err0 = np.sqrt(((proj(f["xyz"].astype(np.float64)) - gt) ** 2).sum(0)).mean()
    err1 = np.sqrt(((proj(V) - gt) ** 2).sum(0)).mean()
    assert err1 < err0


# ---------------------------------------------------------------- warm-start network
def test_warmstart_gradients_match_finite_differences():
    from oracle import warmstart as ow
    rng = np.random.default_rng(3)
    nn = 40
    X = rng.normal(size=(nn, ow.NF))
    X[:, 27:] = 0.0
    Y = rng.normal(size=(nn, 6))
    edges = np.full((8, nn), -1, np.int64)
    for k in range(nn):
        nb = rng.choice(np.setdiff1d(np.arange(nn), [k]), size=rng.integers(0, 9), replace=False)
        edges[:nb.size, k] = nb
    P = ow.init_params(1)
    P["W3"] = rng.normal(0, 0.1, P["W3"].shape)
    P["b1"] = rng.normal(0, 0.1, ow.HID)
    y, cache = ow.forward(P, X, edges)
    g = ow.backward(P, cache, y, Y, edges)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = ow.loss(ow.forward(P, X, edges)[0], Y)
            flat[idx] = old - h
            lm = ow.loss(ow.forward(P, X, edges)[0], Y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_neighbour_mean_adjoint():
    """<mean(H), G> == <H, mean^T(G)> for random H, G (the backward pass's message passing)."""
    from oracle import warmstart as ow
    rng = np.random.default_rng(4)
    nn = 30
    edges = rng.integers(-1, nn, size=(8, nn))
    H = rng.normal(size=(nn, 5))
    G = rng.normal(size=(nn, 5))
    M, cnt = ow.neighbour_mean(H, edges)
    assert abs((M * G).sum() - (H * ow.neighbour_mean_transpose(G, edges, cnt)).sum()) < 1e-12


def test_adam_matches_closed_form_first_step():
    """First Adam step moves every parameter by lr * sign(g) (bias-corrected m/sqrt(v))."""
    from oracle import warmstart as ow
    P = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    ow.adam(P, g, st, lr=0.1)
    assert np.allclose(P["w"], [1.0 - 0.1, -2.0 + 0.1, 3.0 - 0.1 * 1e-3 / (1e-3 + 1e-8)], atol=1e-12)
