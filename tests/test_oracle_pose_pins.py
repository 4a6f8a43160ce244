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
