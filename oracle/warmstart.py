"""Learned warm start for the non-rigid stage, float64 (oracle).

The paper starts each frame's non-rigid solve from the previous frame's
result warped to the new pose (Sec. 3.4, displacement warping) and mentions
learned motion priors as future work (Sec. 6).  The build adds a small
per-node network that predicts the initial node update from the previous
frame's node parameters and per-node statistics of the new frame's
linearisation at that state; plain Gauss-Newton from the previous frame
remains the fallback.

Features per node k (32, zero-padded), at the start state x_{t-1}:
    [0:3]   axis-angle of R_k            [3:6]   t_k
    [6:9]   axis-angle of R_k^{t-1} (R_k^{t-2})^T    [9:12] t_k^{t-1} - t_k^{t-2}
            (zero when there is no frame t-2)
    [12:18] sign(b) log(1 + |b|), b = -J^T B F of node k (dw, dt)
    [18:24] log(1 + d), d = diag(J^T |B| J) of node k
    [24:27] node position minus the mean node position
each then standardised with the training set's mean and standard deviation
(standard deviation floored at 1e-6; padding stays zero).

Network (per node, weights shared):
    h1 = ReLU(W1 x + b1)                       32 -> 128
    m1 = mean of h1 over the node's graph out-neighbours
    h2 = ReLU(W2 [h1; m1] + b2)               256 -> 128
    m2 = mean of h2 over the out-neighbours
    y  = W3 [h2; m2] + b3                     256 -> 6
and the predicted update is y * (0.05, 0.05, 0.05, 0.01, 0.01, 0.01)
(rad, rad, rad, m, m, m).  Loss: mean squared error of y against the
target update divided by the same scale.  Adam (lr 1e-3, betas 0.9, 0.999,
eps 1e-8), one frame per step.
"""
import numpy as np

from . import so3

SCALE = np.array([0.05, 0.05, 0.05, 0.01, 0.01, 0.01])
NF = 32
HID = 128


def raw_features(state_prev, state_prev2, rhs, diag, node_pos):
    """Unstandardised [nn][32] features (see module docstring)."""
    nn = state_prev.shape[1]
    X = np.zeros((nn, NF))
    st = state_prev.astype(np.float64)
    for k in range(nn):
        R = st[:9, k].reshape(3, 3)
        X[k, 0:3] = so3.log(R)
        X[k, 3:6] = st[9:12, k]
        if state_prev2 is not None:
            R2 = state_prev2[:9, k].astype(np.float64).reshape(3, 3)
            X[k, 6:9] = so3.log(R @ R2.T)
            X[k, 9:12] = st[9:12, k] - state_prev2[9:12, k]
    X[:, 12:18] = np.sign(rhs.T) * np.log1p(np.abs(rhs.T))
    X[:, 18:24] = np.log1p(np.maximum(diag.T, 0.0))
    X[:, 24:27] = node_pos.T - node_pos.mean(axis=1)[None, :]
    return X


def target_update(state_prev, state_next):
    """Per-node (dw, dt) with R_next = Exp(dw) R_prev, t_next = t_prev + dt, scaled."""
    nn = state_prev.shape[1]
    Y = np.zeros((nn, 6))
    for k in range(nn):
        R0 = state_prev[:9, k].astype(np.float64).reshape(3, 3)
        R1 = state_next[:9, k].astype(np.float64).reshape(3, 3)
        Y[k, :3] = so3.log(R1 @ R0.T)
        Y[k, 3:] = state_next[9:12, k].astype(np.float64) - state_prev[9:12, k]
    return Y / SCALE


def init_params(seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return dict(W1=rng.normal(0, np.sqrt(2.0 / NF), (HID, NF)), b1=np.zeros(HID),
                W2=rng.normal(0, np.sqrt(2.0 / (2 * HID)), (HID, 2 * HID)), b2=np.zeros(HID),
                W3=rng.normal(0, 0.01, (6, 2 * HID)), b3=np.zeros(6))


def neighbour_mean(H, edge_dst):
    """m_k = mean over valid out-edges (k, l) of H_l (zero for a node without edges)."""
    nn = H.shape[0]
    out = np.zeros_like(H)
    cnt = np.zeros(nn)
    for e in range(edge_dst.shape[0]):
        l = edge_dst[e]
        ok = l >= 0
        out[ok] += H[l[ok]]
        cnt[ok] += 1
    return out / np.maximum(cnt, 1)[:, None], cnt


def neighbour_mean_transpose(G, edge_dst, cnt):
    """Adjoint of neighbour_mean: dH_l += sum over k with l in N(k) of G_k / |N(k)|."""
    out = np.zeros_like(G)
    w = 1.0 / np.maximum(cnt, 1)
    for e in range(edge_dst.shape[0]):
        l = edge_dst[e]
        ok = np.nonzero(l >= 0)[0]
        np.add.at(out, l[ok], G[ok] * w[ok, None])
    return out


def forward(P, X, edge_dst):
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    m1, cnt = neighbour_mean(h1, edge_dst)
    c1 = np.concatenate([h1, m1], axis=1)
    z2 = c1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    m2, _ = neighbour_mean(h2, edge_dst)
    c2 = np.concatenate([h2, m2], axis=1)
    y = c2 @ P["W3"].T + P["b3"]
    return y, dict(X=X, z1=z1, c1=c1, z2=z2, c2=c2, cnt=cnt)


def loss(y, Y):
    return float(((y - Y) ** 2).mean())


def backward(P, cache, y, Y, edge_dst):
    """Gradients of the mean-squared-error loss."""
    n = y.size
    dy = 2.0 * (y - Y) / n
    g = dict(W3=dy.T @ cache["c2"], b3=dy.sum(0))
    dc2 = dy @ P["W3"]
    dh2 = dc2[:, :HID] + neighbour_mean_transpose(dc2[:, HID:], edge_dst, cache["cnt"])
    dz2 = dh2 * (cache["z2"] > 0)
    g["W2"] = dz2.T @ cache["c1"]
    g["b2"] = dz2.sum(0)
    dc1 = dz2 @ P["W2"]
    dh1 = dc1[:, :HID] + neighbour_mean_transpose(dc1[:, HID:], edge_dst, cache["cnt"])
    dz1 = dh1 * (cache["z1"] > 0)
    g["W1"] = dz1.T @ cache["X"]
    g["b1"] = dz1.sum(0)
    return g


def adam(P, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place; `state` holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[:] = b1 * m + (1 - b1) * g[k]
        v[:] = b2 * v + (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[k] -= lr * mh / (np.sqrt(vh) + eps)
