"""Pins for the FP64 pose-stage oracle (skeleton, skinning, pose energy, Gauss-Newton).

Each test checks the oracle against something fixed outside it: numpy's
sin/cos closed form of a rotation, finite differences of its own residual
function, zero-pose and rigid-motion invariants, a brute-force outline test on
the rendered buffer, and exact recovery of a noise-free pose.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import pose as op
from oracle import so3
from synth import body as sb


@pytest.fixture(scope="module")
def small_pose():
    return sb.make_pose_frame(n_vertices=2000, side=320, seed=3, angle_sigma=0.15, px_sigma=0.0, m_sigma=0.0)


def skeleton(frame):
    b = frame["body"]
    return op.Skeleton(b["parents"], b["joints"], sb.NO_DOF)


def test_series_exp_matches_closed_form():
    rng = np.random.default_rng(0)
    for _ in range(200):
        a = rng.normal(size=3)
        th = rng.uniform(0.0, 2.0 * np.pi)
        w = a / np.linalg.norm(a) * th
        ref = Rotation.from_rotvec(w).as_matrix()
        assert np.abs(op.exp_so3(w) - ref).max() < (2e-15 if th < 1.0 else 2e-14)
    assert np.array_equal(op.exp_so3(np.zeros(3)), np.eye(3))


def test_left_jacobian_is_the_exp_derivative():
    """Exp(w + e) Exp(w)^T = Exp(J_l(w) e) to first order."""
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(30):
        w = rng.normal(size=3) * rng.uniform(0.0, 1.5)
        Jl = op.left_jacobian(w)
        R0 = op.exp_so3(w)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            D = (op.exp_so3(w + e) - op.exp_so3(w - e)) @ R0.T / (2 * h)   # = [J_l e_c]x
            col = np.array([D[2, 1], D[0, 2], D[1, 0]])
            assert np.abs(col - Jl[:, c]).max() < 1e-8


def test_fk_zero_pose_and_single_joint_rotation(small_pose):
    sk = skeleton(small_pose)
    pose = np.zeros(sk.nu)
    t = np.array([0.1, -0.2, 0.3])
    pose[sk.it:sk.it + 3] = t
    R, p, _ = sk.fk(pose)
    assert np.allclose(R, np.eye(3)[None], atol=0)
    assert np.allclose(p.T, sk.J + t[:, None], atol=1e-15)
    # rotating the left elbow turns every descendant rigidly about the elbow
    el = sb.JOINTS.index("l_elbow")
    w = np.array([0.2, -0.4, 0.7])
    pose2 = pose.copy()
    pose2[sk.col[el]:sk.col[el] + 3] = w
    R2, p2, _ = sk.fk(pose2)
    Rw = Rotation.from_rotvec(w).as_matrix()
    for j in range(sk.nj):
        if el in sk.anc[j][1:]:
            assert np.allclose(p2[j] - p2[el], Rw @ (p[j] - p[el]), atol=1e-14)
        else:
            assert np.allclose(p2[j], p[j], atol=0)


def test_lbs_zero_pose_is_rest_mesh(small_pose):
    b = small_pose["body"]
    sk = skeleton(small_pose)
    R, p, _ = sk.fk(np.zeros(sk.nu))
    X, Y, Z = op.lbs_f32(b["xyz"], b["bind_idx"], b["bind_w"], sk.J, R, p)
    assert np.abs(np.stack([X, Y, Z]) - b["xyz"]).max() < 2e-6


def test_lbs_matches_the_input_generator(small_pose):
    """The posing used to render the targets (input side, np.sin/np.cos) agrees
    with the oracle's series FK plus float32 skinning."""
    b = small_pose["body"]
    sk = skeleton(small_pose)
    gt = small_pose["gt_pose"].copy()
    gt[sk.itp:] = 0.0
    R, p, _ = sk.fk(gt)
    X, Y, Z = op.lbs_f32(b["xyz"], b["bind_idx"], b["bind_w"], sk.J, R, p)
    assert np.abs(np.stack([X, Y, Z]) - small_pose["posed"]).max() < 1e-5
    assert np.abs(p - small_pose["gt_joints"]).max() < 1e-13


def problem(frame, pose0, weights=(1 / 9, 2500.0, 0.05), case2="exclude"):
    b = frame["body"]
    return op.PoseProblem(skeleton(frame), b["xyz"], b["tri"], b["bind_idx"], b["bind_w"], frame["cam"],
                          frame["mask"], frame["p2d"], frame["p3d"], frame["lam"], weights, pose0, case2=case2)


def start_pose(frame, sigma=0.05, seed=7):
    rng = np.random.default_rng(seed)
    sk = skeleton(frame)
    pose0 = frame["gt_pose"].copy()
    pose0[:sk.it] += rng.normal(0.0, sigma, sk.it)
    pose0[sk.it:sk.it + 3] += rng.normal(0.0, 0.02, 3)
    return pose0


def test_pose_jacobian_matches_central_differences(small_pose):
    P = problem(small_pose, start_pose(small_pose), case2="push")
    assert P.bnd.size > 20 and (P.bsign < 0).any()
    pose = P.pose0 + np.random.default_rng(2).normal(0.0, 0.01, P.skel.nu)
    F0, b, J, _ = P.linearize(pose)
    h = 1e-6
    Jfd = np.zeros_like(J)
    for c in range(P.skel.nu):
        e = np.zeros(P.skel.nu)
        e[c] = h
        Fp = P.linearize(pose + e, need_jacobian=False)[0]
        Fm = P.linearize(pose - e, need_jacobian=False)[0]
        Jfd[:, c] = (Fp - Fm) / (2 * h)
    scale = np.abs(J).max(axis=1, keepdims=True) + 1e-12
    assert np.abs(J - Jfd).max() / np.abs(J).max() < 1e-6
    assert (np.abs(J - Jfd) / scale).max() < 1e-4


def test_energy_terms_are_the_residual_sums(small_pose):
    P = problem(small_pose, start_pose(small_pose), case2="push")
    F, b, _, e = P.linearize(P.pose0, need_jacobian=False)
    nj = P.skel.nj
    assert np.isclose(e["e2d"], (F[:2 * nj] ** 2).sum(), rtol=1e-14)
    assert np.isclose(e["e3d"], (F[2 * nj:5 * nj] ** 2).sum(), rtol=1e-14)
    assert np.isclose(e["sil"], (b[5 * nj:] * F[5 * nj:] ** 2).sum(), rtol=1e-13)
    assert np.isclose(e["sil_abs"], (F[5 * nj:] ** 2).sum(), rtol=1e-13)


def test_outline_filter_matches_brute_force(small_pose):
    P = problem(small_pose, start_pose(small_pose), case2="push")
    d = P.dec
    zb = d["zbuf"]
    H, W = zb.shape
    plain = op.frame_decisions_from_positions(d["X"], d["Y"], d["Z"], small_pose["body"]["tri"], small_pose["cam"],
                                              small_pose["mask"], P.dt, outline=False)["boundary"]
    kept = set(np.nonzero(d["boundary"])[0].tolist())
    assert kept <= set(np.nonzero(plain)[0].tolist())
    for i in np.nonzero(plain)[0]:
        x, y = int(np.rint(d["u"][i])), int(np.rint(d["v"][i]))
        win = [zb[yy, xx] for yy in range(y - 1, y + 2) for xx in range(x - 1, x + 2) if 0 <= yy < H and 0 <= xx < W]
        assert (i in kept) == any(z == 0 for z in win)
    assert len(kept) < plain.sum()          # overlapping parts do produce inner contours


def test_noise_free_recovery(small_pose):
    """Exact detections, no silhouette: Gauss-Newton lands on the true joints."""
    pose0 = start_pose(small_pose, sigma=0.05)
    P = problem(small_pose, pose0, weights=(1 / 9, 2500.0, 0.0))
    out = op.solve(P, 6)
    E = [e["total"] for e in out["energies"]]
    assert E[0] > 100.0 and E[-1] < 1e-8 * E[0]
    _, p, _ = P.skel.fk(out["pose"])
    assert np.abs(p - small_pose["gt_joints"]).max() < 1e-5
    assert np.abs(out["pose"][P.skel.itp:] - small_pose["gt_pose"][P.skel.itp:]).max() < 1e-5


def test_gauss_newton_step_matches_dense_least_squares(small_pose):
    """One step equals the damped normal-equation solution computed by lstsq on
    the stacked system [J; sqrt(mu) I] (all row signs +1)."""
    P = problem(small_pose, start_pose(small_pose), case2="exclude")
    F, b, J, _ = P.linearize(P.pose0)
    assert np.all(b == 1.0)
    mu = 1e-6 * (J * J).sum(axis=0).max()
    Js = np.vstack([J, np.sqrt(mu) * np.eye(J.shape[1])])
    Fs = np.concatenate([F, np.zeros(J.shape[1])])
    step = np.linalg.lstsq(Js, -Fs, rcond=None)[0]
    out = op.solve(P, 1)
    assert np.abs(out["pose"] - P.pose0 - step).max() < 1e-9 * max(1.0, np.abs(step).max())


# ---------------------------------------------------------------- displacement warping (Sec. 3.4)
def _warp_setup():
    from synth import body as sb
    b = sb.make_body(2000)
    skel = op.Skeleton(b["parents"], b["joints"])
    rng = np.random.default_rng(7)
    p0 = np.zeros(skel.nu)
    p0[:skel.it] = rng.normal(0, 0.3, skel.it)
    p1 = p0.copy()
    p1[:skel.it] += rng.normal(0, 0.2, skel.it)
    p1[skel.it:skel.it + 3] += [0.05, -0.02, 0.03]
    d = rng.normal(0, 0.01, b["xyz"].shape)
    S0 = rng.normal(0, 1, b["xyz"].shape)
    S1 = rng.normal(0, 1, b["xyz"].shape)
    return b, skel, p0, p1, d, S0, S1


def test_warp_is_a_plain_carry_when_the_pose_does_not_change():
    b, skel, p0, _, d, S0, S1 = _warp_setup()
    out = op.warp_displacements(skel, b["bind_idx"], b["bind_w"], p0, p0, S0 + d, S0, S1)
    assert np.abs(out - (S1 + d)).max() < 1e-12


def test_warp_under_a_global_rotation_rotates_the_displacement():
    """Every joint turned by the same root rotation G: M_t M_{t-1}^T = G_t G_{t-1}^T."""
    b, skel, _, _, d, S0, S1 = _warp_setup()
    pa, pb = np.zeros(skel.nu), np.zeros(skel.nu)
    wa, wb = np.array([0.2, -0.4, 0.1]), np.array([-0.5, 0.3, 0.7])
    pa[0:3], pb[0:3] = wa, wb                             # joint 0 (the root) carries the global rotation
    Ga, Gb = so3.exp(wa), so3.exp(wb)
    out = op.warp_displacements(skel, b["bind_idx"], b["bind_w"], pa, pb, S0 + d, S0, S1)
    assert np.abs(out - (S1 + Gb @ Ga.T @ d)).max() < 1e-12


def test_warp_with_one_influence_follows_that_joint():
    b, skel, p0, p1, d, S0, S1 = _warp_setup()
    bi = b["bind_idx"].copy()
    bw = np.zeros_like(b["bind_w"])
    bw[0] = 1.0
    R0, _, _ = skel.fk(p0)
    R1, _, _ = skel.fk(p1)
    out = op.warp_displacements(skel, bi, bw, p0, p1, S0 + d, S0, S1)
    j = bi[0]
    expect = S1 + np.einsum("nab,nb->na", R1[j] @ np.transpose(R0[j], (0, 2, 1)), d.T).T
    assert np.abs(out - expect).max() < 1e-12
    # blended rotations are rotations, and the blend of two equal rotations is that rotation
    M = op.blended_rotations(skel, b["bind_idx"], b["bind_w"], p1)
    assert np.abs(np.einsum("nab,ncb->nac", M, M) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(M) - 1).max() < 1e-12


def test_euler_extrapolation_is_exact_for_constant_velocity():
    p2 = np.linspace(-0.3, 0.4, 69)
    v = np.linspace(0.01, -0.02, 69)
    assert np.allclose(op.extrapolate_pose(p2 + v, p2), p2 + 2 * v, rtol=0, atol=1e-15)


def test_temporal_and_limit_rows_match_finite_differences_and_vanish_where_they_should():
    """E_temporal vanishes at the previous joints and E_anatomic inside the
    limits; their Jacobian rows match central differences (Sec. 3.3)."""
    f = sb.make_pose_frame(n_vertices=2000, side=320, seed=3)
    b = f["body"]
    sk = op.Skeleton(b["parents"], b["joints"], sb.NO_DOF)
    rng = np.random.default_rng(4)
    pose = f["gt_pose"].copy()
    pose[:sk.it] += rng.normal(0, 0.1, sk.it)
    _, pj, _ = sk.fk(pose)
    lo, hi = np.full(sk.it, -5.0), np.full(sk.it, 5.0)
    P = op.PoseProblem(sk, b["xyz"], b["tri"], b["bind_idx"], b["bind_w"], f["cam"], f["mask"], f["p2d"], f["p3d"],
                       f["lam"], (0.0, 0.0, 0.0), pose, prev_joints=pj.T, lam_temporal=np.full(sk.nj, 7.0),
                       limits=(lo, hi), l_anat=3.0)
    e = P.energy(pose)
    assert e["temporal"] < 1e-24 and e["anatomic"] == 0.0
    # a translation of the root moves every joint by it: E_temporal = sum_j w_j |d|^2
    d = np.array([0.01, -0.02, 0.03])
    moved = pose.copy()
    moved[sk.it:sk.it + 3] += d
    assert P.energy(moved)["temporal"] == pytest.approx(7.0 * sk.nj * (d @ d), rel=1e-10)
    # one unknown 0.5 over its upper limit and one 0.25 under its lower limit
    out = pose.copy()
    out[4], out[10] = 5.5, -5.25
    assert P.energy(out)["anatomic"] == pytest.approx(3.0 * (0.5 ** 2 + 0.25 ** 2), rel=1e-12)
    F, bb, J, _ = P.linearize(out)
    h = 1e-6
    for c in (0, 4, 10, 20, sk.it, sk.it + 1, sk.it + 4):
        pp, pm = out.copy(), out.copy()
        pp[c] += h
        pm[c] -= h
        fd = (P.linearize(pp, False)[0] - P.linearize(pm, False)[0]) / (2 * h)
        assert np.abs(fd - J[:, c]).max() <= 1e-5 * max(1.0, np.abs(J[:, c]).max()), c
