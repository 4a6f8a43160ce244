"""How strongly the non-rigid Gauss-Newton schedule itself amplifies a small
error in its first step (FP64 oracle, CPU).

The GPU's float32 linearisation gives a first step within ~1.3e-5 of the
oracle's (relative to the parameter change) from starts 0.03 rad / 0.03 m
away from the solution.  These checks show that the schedule (Sec. 4:
Gauss-Newton with the Jacobi-preconditioned CG of the normal equations, 3
steps of 8 iterations, decisions frozen for the frame) maps first-step errors
of that size (random, 0.6-2e-5) to 1.6e-4 ... 1.3e-3 at the end in FP64 alone,
while from starts 0.01 away it stays below 1e-4.  The GPU parity test sets its bar for the three-step result
from the far starts accordingly (first step 1e-4, three steps 1e-3); the
near starts keep 1e-4 throughout."""
import numpy as np
import pytest

import synth
from oracle import graph as og
from oracle import nonrigid as onr
from oracle import so3


def _run(P, gn, pcg, pert=0.0, seed=0):
    rng = np.random.default_rng(seed)
    state = P.state0.astype(np.float64)
    for k in range(gn):
        A, rhs, _ = P.normal_equations(state)
        d = onr.solve_pcg(A, rhs, pcg)
        if k == 0 and pert:
            d = d * (1.0 + pert * rng.normal(size=d.size))
        state = onr.apply_update(state, d)
    return state


def _rel(s, ref, s0):
    r, t = so3.log_all(s), s[9:12]
    rr, tr = so3.log_all(ref), ref[9:12]
    r0, t0 = so3.log_all(s0.astype(np.float64)), s0[9:12].astype(np.float64)
    return max(np.linalg.norm(r - rr) / np.linalg.norm(rr - r0), np.linalg.norm(t - tr) / np.linalg.norm(tr - t0))


@pytest.fixture(scope="module")
def frame():
    f = synth.make_nonrigid_frame("small", 1)
    return f, og.build_graph(f["xyz"], 64)


@pytest.mark.parametrize("sigma,w_vel,lo,hi", [(0.03, 0.0, 5e-4, 2e-3), (0.03, 100.0, 5e-4, 2e-3),
                                               (0.01, 100.0, None, 1e-4)])
def test_first_step_error_amplification(frame, sigma, w_vel, lo, hi):
    f, g = frame
    rng = np.random.default_rng(12)
    st = onr.apply_update(onr.identity_state(64), rng.normal(0, sigma, 384)).astype(np.float32)
    P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], f["weights"], state0=st,
                    w_vel=w_vel, case2="exclude")
    ref = _run(P, 3, 8)
    one = _run(P, 1, 8)
    errs = []
    for seed in range(4):
        s1 = _run(P, 1, 8, pert=5e-6, seed=seed)
        assert _rel(s1, one, st) <= 2.5e-5        # a first-step error of the GPU's size (~1e-5)
        errs.append(_rel(_run(P, 3, 8, pert=5e-6, seed=seed), ref, st))
    if lo is not None:
        assert max(errs) >= lo
    if hi is not None:
        assert max(errs) <= hi
