"""Frame-by-frame tracking of a capture sequence with the plain and the learned
warm start, and training of the warm-start network on the plain solves.

Host orchestration only: every solve, feature, training and update step runs
in the library (C ABI); torch holds the device buffers.
"""
import math
import time

import numpy as np
import torch

from . import (FrameInputs, Template, WarmStart, batch_solve, graph_build, nonrigid_solve, nonrigid_solve_warm,
               params, warmstart_features, warmstart_target)

N_PARAMS = 38662


def init_params(seed=0):
    """Seeded initial network parameters in the library's order
    (W1 [128][32], b1, W2 [128][256], b2, W3 [6][256], b3): He-normal hidden
    layers, small output layer, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.normal(0, math.sqrt(2.0 / 32), (128, 32)), np.zeros(128),
             rng.normal(0, math.sqrt(2.0 / 256), (128, 256)), np.zeros(128),
             rng.normal(0, 0.01, (6, 256)), np.zeros(6)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


def identity_state(nn, device="cuda"):
    s = torch.zeros((12, nn), dtype=torch.float32, device=device)
    s[0] = s[4] = s[8] = 1.0
    return s


class DeviceSequence:
    """A synthetic sequence's inputs resident on the device, with its template."""

    def __init__(self, ctx, seq, graph=None, vertices_per_tile=0):
        self.ctx = ctx
        self.seq = seq
        self.xyz = torch.from_numpy(seq["xyz"]).cuda()
        self.posed = [torch.from_numpy(p).cuda() for p in seq["posed"]]
        self.rgb = torch.from_numpy(seq["rgb"]).cuda()
        nn = seq["n_nodes"]
        if graph is None:
            graph = graph_build(ctx, self.xyz, nn)
        self.graph = graph
        self.template = Template(ctx, torch.from_numpy(seq["tri"]).cuda(), graph, vertices_per_tile)
        self.masks = [torch.from_numpy(m).cuda() for m in seq["masks"]]
        self.images = [torch.from_numpy(i).cuda() for i in seq["images"]]
        self.nn = nn
        self.n = len(self.masks)
        self.prm = params(*seq["weights"], gn_iters=seq["gn"], pcg_iters=seq["pcg"], w_vel=seq["w_vel"],
                          exclude_case2=True, outline_only=seq.get("outline", False))

    def frame(self, t, state):
        return FrameInputs(self.template, self.posed[t], self.rgb, self.seq["cam"], self.masks[t], self.images[t],
                           state)


def track_plain(S, start=None):
    """x*_t for every frame: the plain schedule started from x*_{t-1} (rest state for frame 0)."""
    states, reports = [], []
    cur = identity_state(S.nn) if start is None else start.clone()
    for t in range(S.n):
        st = cur.clone()
        reports.append(nonrigid_solve(S.ctx, S.frame(t, st), S.prm))
        states.append(st)
        cur = st
    return states, reports


def training_set(S, states, frames):
    """Features at x*_{t-1} on frame t (with x*_{t-2}) and targets x*_t (-) x*_{t-1}."""
    X, Y = [], []
    for t in frames:
        prev = states[t - 1].clone()
        prev2 = states[t - 2] if t >= 2 else None
        X.append(warmstart_features(S.ctx, S.frame(t, prev), S.prm, prev2))
        Y.append(warmstart_target(S.ctx, states[t - 1], states[t]))
    return X, Y


def train(S, net, X, Y, epochs=40, lr=1e-3, seed=0, log=None):
    """Adam, one frame per step, frames in a seeded shuffled order each epoch."""
    net.fit_scaling(torch.cat(X, dim=0))
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = []
    for ep in range(epochs):
        order = rng.permutation(len(X))
        tot = 0.0
        for i in order:
            tot += net.train_step(S.template, X[i], Y[i], lr=lr, update=True)
        losses.append(tot / len(X))
        if log is not None and (ep % 10 == 0 or ep == epochs - 1):
            log("epoch %d loss %.5f" % (ep, losses[-1]))
    return losses


def evaluate(S, net, states, frames, step_cap=2):
    """Equal-energy comparison on held-out frames.

    For each frame t both methods start from x*_{t-1}: the plain start runs
    the full schedule and its final energy is the target; the learned start
    runs Gauss-Newton until the energy at the start of a step is at or below
    that target, for at most step_cap times the plain schedule's steps (so a
    worse start costs extra steps instead of ending above the target).
    Returns per-frame steps and the wall time of each method over all frames
    (synchronous calls, identical host overhead)."""
    import copy
    prm_l = copy.copy(S.prm)
    prm_l.gn_iters = min(32, step_cap * S.prm.gn_iters)
    targets, plain_steps = [], []
    for t in frames:
        st = states[t - 1].clone()
        rep = nonrigid_solve(S.ctx, S.frame(t, st), S.prm)
        targets.append(rep["energy"][-1])
        plain_steps.append(rep["gn_done"])
    bufs = [states[t - 1].clone() for t in frames]

    def run_plain():
        for b, t in zip(bufs, frames):
            b.copy_(states[t - 1])
            nonrigid_solve(S.ctx, S.frame(t, b), S.prm)

    def run_learned():
        reps = []
        for b, t, e in zip(bufs, frames, targets):
            b.copy_(states[t - 1])
            prev2 = states[t - 2] if t >= 2 else None
            reps.append(nonrigid_solve_warm(S.ctx, S.frame(t, b), prm_l, net, prev2, e))
        return reps

    run_plain()
    run_learned()   # warm up both paths
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps = run_learned()
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    learned_steps = [r["gn_done"] for r in reps]
    reached = [r["energy"][-1] <= e * (1 + 1e-12) + 1e-12 for r, e in zip(reps, targets)]
    return dict(targets=targets, plain_steps=plain_steps, learned_steps=learned_steps, reached=reached,
                used_prediction=[r["warm_start"] == 1 for r in reps], t_plain=t_plain, t_learned=t_learned,
                final_learned=[r["energy"][-1] for r in reps])


__all__ = ["DeviceSequence", "track_plain", "training_set", "train", "evaluate", "init_params", "batch_solve"]
