"""More pins for the FP64 oracle: the parts a plausible mistake could slip
through the first set (velocity rows, visibility and direction signs, binding
weights, the truncated PCG iterate, the robust colour kernel, blur clamping,
warm-start features and targets, the sparse Cholesky).

Each test checks the oracle against something other than itself: a
constructed scene whose answer follows from the geometry, a library routine
solving the same problem another way, a closed form, or central differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy import ndimage
from scipy.sparse.linalg import LinearOperator, cg
from scipy.spatial.transform import Rotation
from scipy.stats import norm

import synth
from oracle import decisions as od
from oracle import graph as og
from oracle import image as oi
from oracle import nonrigid as onr
from oracle import so3
from oracle import warmstart as ow


def perturbed_state(nn, sigma, seed):
    rng = np.random.default_rng(seed)
    return onr.apply_update(onr.identity_state(nn), rng.normal(0, sigma, 6 * nn))


# ---------------------------------------------------------------- velocity rows (Sec. 3.4, E_velocity)
@pytest.fixture(scope="module")
def vel_problem():
    f = synth.make_nonrigid_frame("small", 1)
    g = og.build_graph(f["xyz"], 64)
    st0 = perturbed_state(64, 0.02, 21).astype(np.float32)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"],
                    state0=st0, w_vel=100.0, case2="exclude")
    return f, g, st0, P


def test_velocity_rows_match_central_differences(vel_problem):
    """Every Jacobian column, velocity rows included, against central
    differences of the residual map at a state away from the anchor."""
    f, g, st0, P = vel_problem
    st = onr.apply_update(st0.astype(np.float64), np.random.default_rng(22).normal(0, 0.01, 384))
    F, b, J, e = P.linearize(st)
    assert e["vel"] > 0.0
    nv = f["xyz"].shape[1]
    nvis = int((P.dec["Z"][P.vis_idx] > 0).sum())
    nb = int((P.dec["Z"][P.bnd_idx] > 0).sum())
    v0 = 3 * nvis + nb                      # velocity rows follow the photometric and silhouette rows
    Jv = J.toarray()[v0:v0 + 3 * nv]
    h = 1e-6
    rng = np.random.default_rng(23)
    for col in rng.choice(384, 16, replace=False):
        d = np.zeros(384)
        d[col] = h
        fd = (P.linearize(onr.apply_update(st, d))[0] - P.linearize(onr.apply_update(st, -d))[0]) / (2 * h)
        fdv = fd[v0:v0 + 3 * nv]
        assert np.abs(fdv - Jv[:, col]).max() <= 1e-6 * max(1.0, np.abs(Jv[:, col]).max()), col


def test_velocity_energy_closed_forms(vel_problem):
    """At the start state the carried positions are the anchor (E_velocity = 0
    up to the float32 anchor); moving every node by t moves every vertex by t
    (weights sum to one), so E_velocity = w_vel * N * |t|^2."""
    f, g, st0, P = vel_problem
    nv = f["xyz"].shape[1]
    e0 = P.energy(st0.astype(np.float64))["vel"]
    t = np.array([0.004, -0.007, 0.01])
    d = np.zeros((64, 6))
    d[:, 3:] = t
    e1 = P.energy(onr.apply_update(st0.astype(np.float64), d.ravel()))["vel"]
    closed = 100.0 * nv * float(t @ t)
    assert e0 <= 1e-8 * closed
    assert abs(e1 - closed) <= 1e-4 * closed


# ---------------------------------------------------------------- visibility (Sec. 3.4 photometric term)
def _sphere(level, r, c):
    pts, tri = synth.icosphere(level)
    return (pts * r + np.asarray(c)), tri


def _ray_hits(d, c, r):
    """Distance along unit rays d (n x 3) from the origin to the first hit of
    the spheres (c [n x 3], r [n]) (inf if missed), and the distance from the
    ray line to the centre."""
    b = (d * c).sum(axis=1)
    perp = np.sqrt(np.maximum((c * c).sum(axis=1) - b * b, 0.0))
    disc = r * r - perp * perp
    s = np.where(disc > 0, b - np.sqrt(np.maximum(disc, 0.0)), np.inf)
    return s, perp


def test_visibility_follows_occlusion_geometry():
    """A front sphere partly covering a back sphere: vertices whose ray is
    clearly blocked by the other sphere, or which face away from the camera,
    are hidden; front-facing vertices with a clear ray are visible."""
    cA, rA = np.array([0.0, 0.0, 2.0]), 0.2
    cB, rB = np.array([0.18, 0.05, 2.8]), 0.3
    pa, ta = _sphere(3, rA, cA)
    pb, tb = _sphere(3, rB, cB)
    pts = np.concatenate([pa, pb])
    tri = np.concatenate([ta, tb + pa.shape[0]]).T.astype(np.int32)
    xyz = pts.T.astype(np.float32)
    cam = synth.Camera.square(256)
    X, Y, Z = (xyz[a] for a in range(3))
    mask = np.zeros((256, 256), np.uint8)
    dt, _ = oi.distance_transform(mask)
    dec = od.frame_decisions_from_positions(X, Y, Z, tri, cam, mask, dt)
    p = xyz.T.astype(np.float64)
    dist = np.linalg.norm(p, axis=1)
    d = p / dist[:, None]
    own_c = np.where(np.arange(p.shape[0])[:, None] < pa.shape[0], cA, cB)
    own_r = np.where(np.arange(p.shape[0]) < pa.shape[0], rA, rB)
    facing = np.einsum("ij,ij->i", (p - own_c) / own_r[:, None], d)       # < 0: faces the camera
    oth_c = np.where(np.arange(p.shape[0])[:, None] < pa.shape[0], cB, cA)
    oth_r = np.where(np.arange(p.shape[0]) < pa.shape[0], rB, rA)
    s_hit, perp = _ray_hits(d, oth_c, oth_r)
    px = 4.0 * dist / cam.fx                          # four pixels, in metres at the vertex's depth
    clear_ray = (perp > oth_r + px) | (s_hit > dist)
    blocked = (perp < oth_r - px) & (s_hit < dist - 0.1)
    vis_expected = (facing < -0.3) & clear_ray
    hid_expected = (facing > 0.5) | ((facing < -0.3) & blocked)
    assert vis_expected.sum() > 200 and ((facing < -0.3) & blocked).sum() > 50
    assert dec["visible"][vis_expected].all()
    assert not dec["visible"][hid_expected].any()


# ---------------------------------------------------------------- direction signs (Sec. 3.3, the two cases)
def _disc_mask(side, centre, radius):
    jj, ii = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    return (((ii - centre[0]) ** 2 + (jj - centre[1]) ** 2) <= radius * radius).astype(np.uint8)


@pytest.mark.parametrize("target_radius", [100.0, 12.0])
def test_direction_signs_follow_the_two_cases(target_radius):
    """A sphere whose image is a disc of ~31 px, offset 40 px from the centre
    of a disc-shaped target silhouette.  Inside a 100 px target, z = -grad DT
    points away from the target centre: on the model contour's far side the
    model normal agrees (b = +1), on the near side it opposes z (case 2,
    b = -1).  A 12 px target lies inside the model's image: every contour
    point is outside the image silhouette, so b = +1 throughout."""
    side = 256
    cam = synth.Camera.square(side)
    pts, tri = _sphere(4, 0.15, [40 * 2.5 / cam.fx, 0.0, 2.5])
    xyz = pts.T.astype(np.float32)
    tri = tri.T.astype(np.int32)
    ct = (cam.cx, cam.cy)
    mask = _disc_mask(side, ct if target_radius > 50 else (cam.cx + 40, cam.cy), target_radius)
    dt, _ = oi.distance_transform(mask)
    X, Y, Z = (xyz[a] for a in range(3))
    dec = od.frame_decisions_from_positions(X, Y, Z, tri, cam, mask, dt)
    B = np.nonzero(dec["boundary"])[0]
    assert B.size > 40
    u, v = dec["u"][B].astype(np.float64), dec["v"][B].astype(np.float64)
    cm = np.array([cam.cx + 40.0, cam.cy])
    n2 = np.stack([u - cm[0], v - cm[1]])
    n2 /= np.linalg.norm(n2, axis=0)                                   # model outline normal
    if target_radius > 50:
        z = np.stack([u - ct[0], v - ct[1]])
        z /= np.linalg.norm(z, axis=0)                                 # towards the nearest target contour
        s = (n2 * z).sum(axis=0)
        sure = np.abs(s) > 0.3
        expect = np.where(s < 0, -1, 1)
        assert (expect[sure] == -1).sum() > 10 and (expect[sure] == 1).sum() > 10
        assert np.array_equal(dec["bsign"][B][sure], expect[sure])
    else:
        assert (dec["bsign"][B] == 1).all()


# ---------------------------------------------------------------- binding weights (embedded deformation)
def test_binding_weights_are_normalised_gaussians_of_the_fourth_distance():
    """A vertex at the origin and nodes at distances 1, 2, 3, 4 (and farther):
    the weights are the normal density with sigma = d_4 at d_1..d_4,
    normalised; a tie in distance keeps the lower node index first."""
    dirs = Rotation.from_rotvec([[0.1, 0.2, 0.3], [1.0, -0.5, 0.2], [-0.3, 0.9, 1.1], [2.0, 0.1, -0.4],
                                 [0.5, 0.5, 0.5], [1.5, -1.0, 0.0]]).apply([1.0, 0.0, 0.0])
    dists = np.array([3.0, 1.0, 4.0, 2.0, 8.0, 9.0])
    pts = np.concatenate([np.zeros((1, 3)), dirs * dists[:, None]])
    xyz = pts.T.astype(np.float32)
    nodes = np.arange(1, 7, dtype=np.int32)
    idx, w = og.bind_vertices(xyz, nodes)
    assert list(idx[:, 0]) == [1, 3, 0, 2]                      # node order by distance 1, 2, 3, 4
    dens = norm.pdf([1.0, 2.0, 3.0, 4.0], scale=4.0)
    assert np.allclose(w[:, 0], dens / dens.sum(), rtol=1e-6)
    # equal distances: lower node index first, equal weights
    pts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 5]], np.float64)
    idx, w = og.bind_vertices(pts.T.astype(np.float32), np.arange(1, 6, dtype=np.int32))
    assert list(idx[:, 0]) == [0, 1, 2, 3] and np.allclose(w[:, 0], 0.25, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- truncated PCG (Sec. 4: diagonal preconditioner)
def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T
    D = np.diag(rng.uniform(0.5, 4.0, n))
    return sp.csr_matrix(D @ A @ D), rng.normal(size=n)


def test_pcg_first_iterate_closed_form():
    A, b = _spd(9, 50.0, 1)
    z = b / A.diagonal()
    x1 = (b @ z) / (z @ (A @ z)) * z
    assert np.allclose(onr.solve_pcg(A, b, 1), x1, rtol=1e-13, atol=0)


def test_pcg_iterates_equal_library_cg():
    """The k-th iterate equals SciPy's preconditioned CG after k iterations
    (same preconditioner, start 0, no convergence stop) for every k."""
    A, b = _spd(14, 300.0, 2)
    Minv = LinearOperator(A.shape, matvec=lambda r: r / A.diagonal())
    for k in range(1, 9):
        ref, _ = cg(A, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=k, M=Minv)
        got = onr.solve_pcg(A, b, k)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), k


def test_pcg_is_exact_after_n_iterations():
    """n iterations on a well-conditioned n x n system reach the direct solve."""
    A, b = _spd(12, 10.0, 3)
    x = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(onr.solve_pcg(A, b, 12) - x) <= 1e-10 * np.linalg.norm(x)


def test_pcg_guards():
    """A zero right-hand side stops at once (r.z = 0); a non-positive diagonal
    entry is replaced by 1 in the preconditioner, checked on a first iterate."""
    A, b = _spd(6, 5.0, 4)
    assert not onr.solve_pcg(A, np.zeros(6), 5).any()
    Ad = A.toarray()
    Ad[2, 2] = 0.0
    Ad[0, 0] = -1.0
    A2 = sp.csr_matrix(Ad)
    dg = Ad.diagonal().copy()
    dg[dg <= 0] = 1.0
    z = b / dg
    pap = z @ (Ad @ z)
    if pap > 0:
        assert np.allclose(onr.solve_pcg(A2, b, 1), (b @ z) / pap * z, rtol=1e-13)


# ---------------------------------------------------------------- sparse Cholesky
def test_sparse_cholesky_reconstructs_and_solves():
    f = synth.make_nonrigid_frame("small", 0)
    g = og.build_graph(f["xyz"], 64)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    A, rhs, _ = P.normal_equations(perturbed_state(64, 0.01, 5))
    perm, Lb = onr.sparse_cholesky(A)
    n = A.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    L = np.zeros((n, n))
    for k in range(Lb.shape[0]):                  # lower band storage: Lb[k, j] = L[j + k, j]
        j = np.arange(n - k)
        L[j + k, j] = Lb[k, : n - k]
    Ap = A.toarray()[np.ix_(perm, perm)]
    assert np.abs(L @ L.T - Ap).max() <= 1e-12 * np.abs(Ap).max()
    x = onr.solve_cholesky(A, rhs)
    assert np.linalg.norm(A @ x - rhs) <= 1e-10 * np.linalg.norm(rhs)
    assert np.linalg.norm(x - np.linalg.solve(A.toarray(), rhs)) <= 1e-9 * np.linalg.norm(x)


# ---------------------------------------------------------------- robust colour kernel sigma_c (Sec. 3.4)
def test_colour_kernel_prunes_by_residual_norm():
    """Template colours set to the sampled image colour plus an offset whose
    norm is 0.49 or 0.51 (spread over the three channels): with tau_c = 0.5
    exactly the 0.49 residuals remain, with their full Jacobian rows, and the
    0.51 rows vanish; with tau_c = inf all remain."""
    f = synth.make_nonrigid_frame("small", 0)
    g = og.build_graph(f["xyz"], 64)
    P0 = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"])
    st = onr.identity_state(64).astype(np.float64)
    V, _ = onr.ed_deform(f["xyz"], g, st)
    cam = f["cam"]
    u = cam.fx * V[0] / V[2] + cam.cx
    v = cam.fy * V[1] / V[2] + cam.cy
    val, _, _ = oi.sample(P0.img, u, v)
    rng = np.random.default_rng(8)
    dirs = rng.normal(size=(3, u.size))
    dirs /= np.linalg.norm(dirs, axis=0)
    small = rng.uniform(size=u.size) < 0.5
    mag = np.where(small, 0.49, 0.51)
    rgb = (val + mag * dirs).astype(np.float64)
    vis = P0.vis_idx[V[2][P0.vis_idx] > 0]
    wp = f["weights"][1]
    for tau, expect in ((0.5, wp * (0.49 ** 2) * small[vis].sum()), (np.inf, wp * (mag[vis] ** 2).sum())):
        P = onr.Problem(f["xyz"], f["tri"], rgb, g, cam, f["mask"], f["image"], f["weights"], tau_c=tau)
        F, b, J, e = P.linearize(st)
        assert abs(e["photo"] - expect) <= 1e-9 * expect, tau
        rows = np.abs(J[: 3 * vis.size]).sum(axis=1).A.ravel().reshape(3, vis.size).sum(axis=0)
        if np.isfinite(tau):
            assert (rows[~small[vis]] == 0).all() and (rows[small[vis]] > 0).all()
        else:
            assert (rows > 0).all()


# ---------------------------------------------------------------- blur (Sec. 3.4, I_Gauss)
@pytest.mark.parametrize("k", [3, 9, 15])
def test_blur_equals_library_separable_filter_with_nearest_edges(k):
    rng = np.random.default_rng(k)
    img = rng.uniform(size=(3, 23, 31))
    w = oi.gaussian_weights(k)
    ref = ndimage.correlate1d(ndimage.correlate1d(img, w, axis=2, mode="nearest"), w, axis=1, mode="nearest")
    assert np.abs(oi.blur(img, k) - ref).max() <= 1e-14


def test_blur_of_a_corner_impulse():
    """Impulse in the corner texel: clamp-to-edge folds the missing left/upper
    tap onto the corner, so the 2x2 corner block is (a+b)^2, a(a+b), a(a+b),
    a^2 with the 3-tap weights (a, b, a) of a unit-sum Gaussian with sigma 0.8."""
    img = np.zeros((1, 6, 7))
    img[0, 0, 0] = 1.0
    e = np.exp(-1.0 / (2 * 0.8 ** 2))
    a, b = e / (1 + 2 * e), 1 / (1 + 2 * e)
    out = oi.blur(img, 3)[0]
    assert np.allclose(out[:2, :2], [[(a + b) ** 2, a * (a + b)], [a * (a + b), a * a]], rtol=1e-14)
    assert out[2:].max() == 0.0 and out[:, 2:].max() == 0.0


# ---------------------------------------------------------------- warm-start features and targets
def test_warmstart_features_and_targets_closed_forms():
    rng = np.random.default_rng(9)
    nn = 12
    a = rng.normal(0, 0.3, (nn, 3))
    w = rng.normal(0, 0.05, (nn, 3))
    t2 = rng.normal(0, 0.1, (nn, 3))
    dt = rng.normal(0, 0.01, (nn, 3))
    prev2 = np.zeros((12, nn))
    prev = np.zeros((12, nn))
    for k in range(nn):
        R2 = Rotation.from_rotvec(a[k]).as_matrix()
        prev2[:9, k] = R2.ravel()
        prev[:9, k] = (Rotation.from_rotvec(w[k]).as_matrix() @ R2).ravel()
    prev2[9:] = t2.T
    prev[9:] = (t2 + dt).T
    rhs = np.zeros((6, nn))
    rhs[0] = np.e - 1.0
    rhs[1] = -(np.e ** 2 - 1.0)
    diag = np.full((6, nn), np.e ** 3 - 1.0)
    pos = rng.normal(size=(3, nn))
    X = ow.raw_features(prev, prev2, rhs, diag, pos)
    for k in range(nn):
        assert np.allclose(X[k, 0:3], Rotation.from_matrix(prev[:9, k].reshape(3, 3)).as_rotvec(), atol=1e-12)
    assert np.allclose(X[:, 3:6], (t2 + dt), atol=1e-15)
    assert np.allclose(X[:, 6:9], w, atol=1e-12)
    assert np.allclose(X[:, 9:12], dt, atol=1e-15)
    assert np.allclose(X[:, 12], 1.0) and np.allclose(X[:, 13], -2.0) and not X[:, 14:18].any()
    assert np.allclose(X[:, 18:24], 3.0)
    assert np.allclose(X[:, 24:27].sum(axis=0), 0.0, atol=1e-12)
    assert np.allclose(X[:, 24:27] - X[:1, 24:27], (pos - pos[:, :1]).T, atol=1e-12)
    assert not X[:, 27:].any()
    assert not ow.raw_features(prev, None, rhs, diag, pos)[:, 6:12].any()
    Y = ow.target_update(prev2, prev)
    assert np.allclose(Y, np.concatenate([w, dt], axis=1) / ow.SCALE, atol=1e-10)
