"""GPU parity of the pose stage against the FP64 oracle (through the C ABI).

Bars: decisions (visible set, contour set B on the outline, signs b_i)
bit-exact; the normal equations and energies at a pose within 1e-9 of the
oracle (both sides are FP64, only the summation order differs); solved poses
within 1e-4 of the pose change and energies within 1e-5 of the start energy
(relative), against the oracle run with the same number of steps.
"""
import numpy as np
import pytest

from oracle import pose as op
from synth import body as sb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WEIGHTS = (1.0 / 9.0, 2500.0, 0.05)


@pytest.fixture(scope="module")
def ctx():
    import paper_1810_02648_amd as cap
    return cap.Context(0)


@pytest.fixture(scope="module")
def frames():
    return {"small": sb.make_pose_frame(n_vertices=2000, side=320, seed=3),
            "ragged": sb.make_pose_frame(n_vertices=3001, side=517, seed=4),
            "full": sb.make_pose_frame(n_vertices=5000, side=1080, seed=0)}


def start_pose(f, sigma=0.05, seed=7):
    rng = np.random.default_rng(seed)
    nr = 3 * len(sb.dof_joints())
    pose0 = f["gt_pose"].copy()
    pose0[:nr] += rng.normal(0.0, sigma, nr)
    pose0[nr:nr + 3] += rng.normal(0.0, 0.02, 3)
    return pose0


def body_on_device(ctx, f):
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    b = f["body"]
    has_rot = [j not in sb.NO_DOF for j in range(len(sb.JOINTS))]
    return cap.Body(ctx, dev(b["tri"]), dev(b["xyz"]), dev(b["bind_idx"]), dev(b["bind_w"]), b["parents"],
                    b["joints"], has_rot)


def pose_inputs(body, f, pose):
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    return cap.PoseInputs(body, f["cam"], dev(f["mask"]), dev(f["p2d"], torch.float64), dev(f["p3d"], torch.float64),
                          dev(f["lam"], torch.float64), dev(pose, torch.float64))


def oracle_problem(f, pose0, weights=WEIGHTS, case2="exclude", outline=True):
    b = f["body"]
    sk = op.Skeleton(b["parents"], b["joints"], sb.NO_DOF)
    return op.PoseProblem(sk, b["xyz"], b["tri"], b["bind_idx"], b["bind_w"], f["cam"], f["mask"], f["p2d"],
                          f["p3d"], f["lam"], weights, pose0, case2=case2, outline=outline)


@pytest.mark.parametrize("name,case2,outline", [("small", "exclude", True), ("small", "push", False),
                                                ("ragged", "push", True)])
def test_decisions_and_normal_equations(ctx, frames, name, case2, outline):
    import paper_1810_02648_amd as cap
    f = frames[name]
    pose0 = start_pose(f)
    P = oracle_problem(f, pose0, case2=case2, outline=outline)
    body = body_on_device(ctx, f)
    prm = cap.pose_params(*WEIGHTS, gn_iters=1, exclude_case2=case2 == "exclude", outline_only=outline)
    fr = pose_inputs(body, f, pose0)
    out = cap.pose_linearize(ctx, fr, prm)
    vf = out["vflags"].cpu().numpy()
    print(name, case2, outline, "B", P.bnd.size, flush=True)
    assert np.array_equal((vf & 1) != 0, P.dec["visible"])
    bnd = np.zeros(body.nv, bool)
    bnd[P.bnd] = True
    assert np.array_equal((vf & 2) != 0, bnd)
    neg = np.zeros(body.nv, bool)
    neg[P.bnd[P.bsign < 0]] = True
    assert np.array_equal((vf & 4) != 0, neg)
    assert np.array_equal(fr.pose.cpu().numpy(), pose0)
    F, b, J, e = P.linearize(pose0)
    A = J.T @ J
    rhs = -(J.T @ (b * F))
    S = out["system"].cpu().numpy()
    assert np.abs(S[:, :-1] - A).max() <= 1e-9 * np.abs(A).max()
    assert np.abs(S[:, -1] - rhs).max() <= 1e-9 * np.abs(rhs).max()
    got = out["energy"]
    for k, key in enumerate(("e2d", "e3d", "sil", "sil_abs")):
        assert abs(got[k] - e[key]) <= 1e-10 * max(1.0, abs(e["total"])), (key, got[k], e[key])


@pytest.mark.parametrize("name,gn", [("small", 3), ("ragged", 4), ("full", 3)])
def test_pose_solve_matches_oracle(ctx, frames, name, gn):
    import paper_1810_02648_amd as cap
    f = frames[name]
    pose0 = start_pose(f, seed=11)
    P = oracle_problem(f, pose0)
    ref = op.solve(P, gn)
    body = body_on_device(ctx, f)
    fr = pose_inputs(body, f, pose0)
    rep = cap.pose_solve(ctx, fr, cap.pose_params(*WEIGHTS, gn_iters=gn))
    got = fr.pose.cpu().numpy()
    step = np.linalg.norm(ref["pose"] - pose0)
    err = np.linalg.norm(got - ref["pose"])
    E_ref = [e["total"] for e in ref["energies"]]
    print(name, "pose err %.3e of step %.3e" % (err, step), "E gpu", rep["energy"], "ref", E_ref, flush=True)
    assert rep["status"] == 0 and rep["gn_done"] == gn
    assert rep["n_boundary"] == P.bnd.size and rep["n_visible"] == int(P.dec["visible"].sum())
    assert err <= 1e-4 * max(step, 1e-6)
    for a, r in zip(rep["energy"], E_ref):
        assert abs(a - r) <= 1e-5 * E_ref[0]
    fin = ref["energies"][-1]
    assert abs(rep["e2d"] - fin["e2d"]) <= 1e-5 * E_ref[0]
    assert abs(rep["e_sil_abs"] - fin["sil_abs"]) <= 1e-5 * E_ref[0]


def test_noise_free_recovery_on_device(ctx):
    """Exact detections, no silhouette term: the device solve reaches the true joints."""
    import paper_1810_02648_amd as cap
    f = sb.make_pose_frame(n_vertices=2000, side=320, seed=5, px_sigma=0.0, m_sigma=0.0)
    pose0 = start_pose(f, sigma=0.05, seed=2)
    body = body_on_device(ctx, f)
    fr = pose_inputs(body, f, pose0)
    rep = cap.pose_solve(ctx, fr, cap.pose_params(1.0 / 9.0, 2500.0, 0.0, gn_iters=6))
    assert rep["energy"][-1] < 1e-8 * rep["energy"][0]
    b = f["body"]
    sk = op.Skeleton(b["parents"], b["joints"], sb.NO_DOF)
    _, p, _ = sk.fk(fr.pose.cpu().numpy())
    assert np.abs(p - f["gt_joints"]).max() < 1e-5


def test_pose_errors(ctx, frames):
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    f = frames["small"]
    b = f["body"]
    pose0 = start_pose(f)
    body = body_on_device(ctx, f)
    fr = pose_inputs(body, f, pose0)
    # all weights zero: J^T J = 0, the first pivot is not positive; the pose is restored
    with pytest.raises(cap.CaptureError) as ei:
        cap.pose_solve(ctx, fr, cap.pose_params(0.0, 0.0, 0.0, gn_iters=2))
    assert ei.value.code == -2
    assert np.array_equal(fr.pose.cpu().numpy(), pose0)
    for prm in (cap.pose_params(gn_iters=0), cap.pose_params(l2d=-1.0), cap.pose_params(lsil=float("nan"))):
        with pytest.raises(cap.CaptureError) as ei:
            cap.pose_solve(ctx, fr, prm)
        assert ei.value.code == -1
    bad = cap.pose_params()
    bad.flags = 8
    with pytest.raises(cap.CaptureError):
        cap.pose_solve(ctx, fr, bad)
    has_rot = [j not in sb.NO_DOF for j in range(len(sb.JOINTS))]
    parents = b["parents"].copy()
    parents[3] = 5                        # a parent after its child
    with pytest.raises(cap.CaptureError) as ei:
        cap.Body(ctx, dev(b["tri"]), dev(b["xyz"]), dev(b["bind_idx"]), dev(b["bind_w"]), parents, b["joints"],
                 has_rot)
    assert ei.value.code == -1
    bj = b["bind_idx"].copy()
    bj[0, 7] = len(sb.JOINTS)
    with pytest.raises(cap.CaptureError) as ei:
        cap.Body(ctx, dev(b["tri"]), dev(b["xyz"]), dev(bj), dev(b["bind_w"]), b["parents"], b["joints"], has_rot)
    assert ei.value.code == -1
    assert np.array_equal(fr.pose.cpu().numpy(), pose0)


def test_pose_solve_is_deterministic(ctx, frames):
    import paper_1810_02648_amd as cap
    f = frames["ragged"]
    pose0 = start_pose(f, seed=3)
    body = body_on_device(ctx, f)
    outs = []
    for _ in range(2):
        fr = pose_inputs(body, f, pose0)
        rep = cap.pose_solve(ctx, fr, cap.pose_params(*WEIGHTS, gn_iters=3))
        outs.append((fr.pose.cpu().numpy(), rep["energy"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("name", ["small", "full"])
def test_temporal_and_joint_limit_terms_match_oracle(ctx, frames, name):
    """E_temporal (previous joint positions, per-joint weights) and E_anatomic
    (quadratic barrier outside the limits, Sec. 3.3): normal equations and a
    3-step solve against the oracle; the limits are set so that several
    unknowns start outside them."""
    import paper_1810_02648_amd as cap
    from gpu_util import dev
    f = frames[name]
    b = f["body"]
    sk = op.Skeleton(b["parents"], b["joints"], sb.NO_DOF)
    pose0 = start_pose(f, seed=5)
    prev = start_pose(f, sigma=0.08, seed=9)
    _, pj, _ = sk.fk(prev)
    prevj = np.ascontiguousarray(pj.T)
    lt = 300.0 * sb.TEMPORAL_JOINT_WEIGHTS
    lo = np.full(sk.it, -0.25)
    hi = np.full(sk.it, 0.25)
    lo[:3], hi[:3] = -np.inf, np.inf
    assert ((pose0[:sk.it] > hi) | (pose0[:sk.it] < lo)).sum() >= 3
    P = op.PoseProblem(sk, b["xyz"], b["tri"], b["bind_idx"], b["bind_w"], f["cam"], f["mask"], f["p2d"], f["p3d"],
                       f["lam"], WEIGHTS, pose0, case2="exclude", outline=True, prev_joints=prevj, lam_temporal=lt,
                       limits=(lo, hi), l_anat=1e4)
    body = body_on_device(ctx, f)
    prm = cap.pose_params(*WEIGHTS, gn_iters=3, l_temporal=lt, l_anatomic=1e4, theta_min=lo, theta_max=hi)
    fr = cap.PoseInputs(body, f["cam"], dev(f["mask"]), dev(f["p2d"], torch.float64), dev(f["p3d"], torch.float64),
                        dev(f["lam"], torch.float64), dev(pose0, torch.float64), prev_joints=dev(prevj))
    out = cap.pose_linearize(ctx, fr, prm)
    F, bb, J, e = P.linearize(pose0)
    A = J.T @ (np.abs(bb)[:, None] * J)
    rhs = -(J.T @ (bb * F))
    S = out["system"].cpu().numpy()
    assert np.abs(S[:, :-1] - A).max() <= 1e-9 * np.abs(A).max()
    assert np.abs(S[:, -1] - rhs).max() <= 1e-9 * np.abs(rhs).max()
    for k, key in enumerate(("e2d", "e3d", "sil", "sil_abs", "temporal", "anatomic")):
        assert abs(out["energy"][k] - e[key]) <= 1e-10 * max(1.0, abs(e["total"])), (key, out["energy"][k], e[key])
    assert e["temporal"] > 0 and e["anatomic"] > 0
    ref = op.solve(P, 3)
    rep = cap.pose_solve(ctx, fr, prm)
    got = fr.pose.cpu().numpy()
    step = np.linalg.norm(ref["pose"] - pose0)
    assert np.linalg.norm(got - ref["pose"]) <= 1e-4 * step
    E_ref = [x["total"] for x in ref["energies"]]
    for a, r in zip(rep["energy"], E_ref):
        assert abs(a - r) <= 1e-5 * E_ref[0]
    assert abs(rep["e_temporal"] - ref["energies"][-1]["temporal"]) <= 1e-5 * E_ref[0]
    assert abs(rep["e_anatomic"] - ref["energies"][-1]["anatomic"]) <= 1e-5 * E_ref[0]
