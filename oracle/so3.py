"""Rotation exponential and logarithm (float64).

The node rotations are updated multiplicatively, R <- Exp(dw) R, which is the
left-perturbation reading of the Gauss-Newton step of Sec. 4 (Eq. gaussnewton)
for unknowns living on SO(3).
"""
import numpy as np


def hat(w):
    """Skew matrix [w]x with [w]x v = w x v."""
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp(w):
    """Rodrigues' formula; second-order series for tiny angles."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.sqrt(w @ w))
    K = hat(w)
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / (th * th)) * K @ K


def log(R):
    """Axis-angle vector of a rotation matrix (angle in [0, pi))."""
    R = np.asarray(R, dtype=np.float64)
    c = np.clip((np.trace(R) - 1.0) * 0.5, -1.0, 1.0)
    th = float(np.arccos(c))
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-8:
        return 0.5 * v
    return th / (2.0 * np.sin(th)) * v


def log_all(state):
    """Axis-angle of every node of a [12][n] node-state array (R row-major, t)."""
    n = state.shape[1]
    out = np.zeros((3, n))
    for k in range(n):
        out[:, k] = log(state[:9, k].astype(np.float64).reshape(3, 3))
    return out
