"""Skeletal pose stage, float64 Gauss-Newton (oracle).  Paper Sec. 3.3.

Unknowns: three axis-angle values for each rotating joint, in joint order
(the root first: its rotation is the global R), then the root translation t
(3) and the auxiliary translation t' of the 3D term (3); 69 for the 23-joint
body with 21 rotating joints.  Joint j's local rotation is
Exp(theta_j); global rotations compose down the tree, joint positions follow
the rest offsets:  R_j = R_parent Exp(theta_j),  p_j = p_parent + R_parent (J_j - J_parent),
p_root = J_root + t.  Vertices follow by linear blend skinning,
V_i = sum_s w_is (R_js (v_i - J_js) + p_js) (4 bones per vertex).

Energy (the pose energy's 2D, 3D and silhouette terms):
    E_2D  = lambda_2D sum_j lambda_j ||pi(p_j) - P2D_j||^2
    E_3D  = lambda_3D sum_j ||p_j - (P3D_j + t')||^2
    E_sil = lambda_sil sum_{i in B} b_i I_DT(pi(V_i))^2   (decisions at the start pose,
            B restricted to the rendered model's outline, b_i = -1 rows optional)
Gauss-Newton with (J^T |B| J + mu I) delta = -J^T B F, exact Cholesky solve,
additive update theta <- theta + delta.  mu = 1e-6 * max diag(J^T |B| J): a
fixed, tiny Levenberg-style regularisation (no residual re-evaluation, unlike
Levenberg-Marquardt) so that directions the data leave unobserved (e.g. the
twist of a round limb) keep the system positive definite.

Exp and the derivative use the series sin(x)/x, (1 - cos x)/x^2 and
(x - sin x)/x^3 in x = |w|^2, evaluated by nested Horner steps
S <- 1 - (x / (k (k + 1))) S from k = 2N down (N = 24 terms), so that every
implementation computes the same float64 rotation from the same angles
(valid for angles up to 2 pi).  The derivative of Exp(w) v with respect to w
is -[Exp(w) v]x J_l(w) with the left Jacobian J_l = I + B [w]x + C [w]x^2.
"""
import numpy as np

from .decisions import frame_decisions_from_positions

N_TERMS = 24


def _series(x, first):
    """1 - x/(f (f+1)) (1 - x/((f+2)(f+3)) (...)), N_TERMS factors, innermost first."""
    s = 1.0
    for n in range(N_TERMS, 0, -1):
        k = first + 2 * (n - 1)
        s = 1.0 - (x / float(k * (k + 1))) * s
    return s


def exp_coeffs(w):
    """A = sin(t)/t, B = (1 - cos t)/t^2, C = (t - sin t)/t^3 for t = |w|, x = t^2."""
    x = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]
    A = _series(x, 2)
    B = 0.5 * _series(x, 3)
    C = _series(x, 4) / 6.0
    return x, A, B, C


def _hat(w):
    return [[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]]


def exp_so3(w):
    """Rotation matrix (float64) with the fixed operation order."""
    w = [float(w[0]), float(w[1]), float(w[2])]
    x, A, B, _ = exp_coeffs(w)
    K = _hat(w)
    R = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            kk = w[a] * w[b] - (x if a == b else 0.0)
            R[a, b] = ((1.0 if a == b else 0.0) + A * K[a][b]) + B * kk
    return R


def left_jacobian(w):
    w = [float(w[0]), float(w[1]), float(w[2])]
    x, _, B, C = exp_coeffs(w)
    K = _hat(w)
    Jl = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            kk = w[a] * w[b] - (x if a == b else 0.0)
            Jl[a, b] = ((1.0 if a == b else 0.0) + B * K[a][b]) + C * kk
    return Jl


def _mat(A, B):
    """3x3 product with ((a0 b0 + a1 b1) + a2 b2) sums."""
    out = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            out[i, j] = (A[i, 0] * B[0, j] + A[i, 1] * B[1, j]) + A[i, 2] * B[2, j]
    return out


def _vec(A, v):
    return np.array([(A[i, 0] * v[0] + A[i, 1] * v[1]) + A[i, 2] * v[2] for i in range(3)])


class Skeleton:
    def __init__(self, parents, rest_joints, no_dof=(9, 14)):
        self.parents = np.asarray(parents)
        self.J = np.asarray(rest_joints, dtype=np.float64)        # [3][nj]
        self.nj = self.parents.size
        self.dof = [j for j in range(self.nj) if j not in no_dof]
        self.col = {j: 3 * i for i, j in enumerate(self.dof)}     # first unknown of joint j
        self.it = 3 * len(self.dof)                                # root translation t
        self.itp = self.it + 3                                     # t' of the 3D term
        self.nu = self.it + 6
        anc = []
        for j in range(self.nj):
            a, k = [], j
            while k >= 0:
                a.append(k)
                k = self.parents[k]
            anc.append(a)                                          # j itself first, then up to the root
        self.anc = anc

    def fk(self, pose):
        """Global rotations R [nj][3][3], positions p [nj][3], derivative axes Ax [nj][3][3]."""
        R = np.zeros((self.nj, 3, 3))
        p = np.zeros((self.nj, 3))
        Ax = np.zeros((self.nj, 3, 3))
        J = self.J.T
        for j in range(self.nj):
            par = self.parents[j]
            if j in self.col:
                w = pose[self.col[j]:self.col[j] + 3]
                Rl, Jl = exp_so3(w), left_jacobian(w)
            else:
                Rl, Jl = np.eye(3), np.zeros((3, 3))
            if par < 0:
                R[j] = Rl
                p[j] = J[j] + pose[self.it:self.it + 3]
                Ax[j] = Jl
            else:
                R[j] = _mat(R[par], Rl)
                p[j] = p[par] + _vec(R[par], J[j] - J[par])
                Ax[j] = _mat(R[par], Jl)
        return R, p, Ax


def lbs_f32(xyz, bind_idx, bind_w, Jrest, R, p):
    """Float32 recipe for the start-pose decisions:
    d = v - J_j;  q_a = (R_a0 d0 + R_a1 d1) + R_a2 d2;  y = q + p_j;  acc = acc + w y."""
    F = np.float32
    x = [xyz[a].astype(F) for a in range(3)]
    R32, p32, J32 = R.astype(F), p.astype(F), Jrest.astype(F)
    acc = [np.zeros_like(x[0]) for _ in range(3)]
    for s in range(bind_idx.shape[0]):
        j = bind_idx[s]
        w = bind_w[s].astype(F)
        d = [x[a] - J32[a][j] for a in range(3)]
        for a in range(3):
            q = (R32[j, a, 0] * d[0] + R32[j, a, 1] * d[1]) + R32[j, a, 2] * d[2]
            acc[a] = acc[a] + w * (q + p32[j, a])
    return acc


class PoseProblem:
    """One frame of the pose stage with frozen start-pose decisions."""

    def __init__(self, skel, xyz, tri, bind_idx, bind_w, cam, mask, p2d, p3d, lam, weights, pose0,
                 case2="push", outline=True, prev_joints=None, lam_temporal=None, limits=None, l_anat=0.0):
        """prev_joints [3][nj]: the previous frame's joint positions p^{t-1} and
        lam_temporal [nj]: lambda_temporal * lambda_i per joint (E_temporal,
        Sec. 3.3); limits (theta_min, theta_max) [it] over the rotational
        unknowns (+-inf: none) with weight l_anat (E_anatomic, Sec. 3.3)."""
        from .image import distance_transform
        self.skel, self.xyz, self.tri, self.cam = skel, xyz, tri, cam
        self.prev_joints = None if prev_joints is None else np.asarray(prev_joints, np.float64)
        self.lam_t = None if lam_temporal is None else np.asarray(lam_temporal, np.float64)
        self.limits = None if limits is None else (np.asarray(limits[0], np.float64),
                                                   np.asarray(limits[1], np.float64))
        self.l_anat = float(l_anat)
        self.bind_idx, self.bind_w = bind_idx, bind_w
        self.p2d, self.p3d, self.lam = np.asarray(p2d, np.float64), np.asarray(p3d, np.float64), np.asarray(lam)
        self.l2d, self.l3d, self.lsil = (float(w) for w in weights)
        self.pose0 = np.asarray(pose0, np.float64)
        self.dt, _ = distance_transform(mask)
        R, p, _ = skel.fk(self.pose0)
        X, Y, Z = lbs_f32(xyz, bind_idx, bind_w, skel.J, R, p)
        self.dec = frame_decisions_from_positions(X, Y, Z, tri, cam, mask, self.dt, outline=outline)
        self.bnd = np.nonzero(self.dec["boundary"])[0]
        self.bsign = self.dec["bsign"][self.bnd].astype(np.float64)
        if case2 == "exclude":
            keep = self.bsign > 0
            self.bnd, self.bsign = self.bnd[keep], self.bsign[keep]

    def linearize(self, pose, need_jacobian=True):
        from .image import sample
        sk, cam = self.skel, self.cam
        R, p, Ax = sk.fk(pose)
        rows_F, rows_b, rows_J = [], [], []
        e = dict(e2d=0.0, e3d=0.0, sil=0.0, sil_abs=0.0, temporal=0.0, anatomic=0.0)

        def dpoint(y, chain):
            """d y / d unknowns for a point y carried by the joints in `chain` (j first)."""
            D = np.zeros((3, sk.nu))
            for k in chain:
                if k in sk.col:
                    c = sk.col[k]
                    yk = y - p[k]
                    hat = np.array(_hat(yk))
                    D[:, c:c + 3] = -hat @ Ax[k]
            D[:, sk.it:sk.it + 3] = np.eye(3)
            return D

        for j in range(sk.nj):
            chain = sk.anc[j][1:]        # a joint's position does not depend on its own rotation
            X, Y, Z = p[j]
            u = cam.fx * X / Z + cam.cx
            v = cam.fy * Y / Z + cam.cy
            s = np.sqrt(self.l2d * self.lam[j])
            r = s * np.array([u - self.p2d[0, j], v - self.p2d[1, j]])
            e["e2d"] += float(r @ r)
            rows_F.append(r)
            rows_b.append(np.ones(2))
            if need_jacobian:
                Pj = np.array([[cam.fx / Z, 0, -cam.fx * X / (Z * Z)], [0, cam.fy / Z, -cam.fy * Y / (Z * Z)]])
                rows_J.append(s * Pj @ dpoint(p[j], chain))
        s3 = np.sqrt(self.l3d)
        for j in range(sk.nj):
            chain = sk.anc[j][1:]
            r = s3 * (p[j] - self.p3d[:, j] - pose[sk.itp:sk.itp + 3])
            e["e3d"] += float(r @ r)
            rows_F.append(r)
            rows_b.append(np.ones(3))
            if need_jacobian:
                D = dpoint(p[j], chain)
                D[:, sk.itp:sk.itp + 3] = -np.eye(3)
                rows_J.append(s3 * D)
        # silhouette rows
        if self.bnd.size:
            v = self.xyz.astype(np.float64)
            Vb = np.zeros((3, self.bnd.size))
            Js = []
            for n, i in enumerate(self.bnd):
                D = np.zeros((3, sk.nu))
                for s in range(self.bind_idx.shape[0]):
                    j = self.bind_idx[s, i]
                    w = float(self.bind_w[s, i])
                    y = R[j] @ (v[:, i] - sk.J[:, j]) + p[j]
                    Vb[:, n] += w * y
                    if need_jacobian:
                        D += w * dpoint(y, sk.anc[j])
                Js.append(D)
            X, Y, Z = Vb
            u = cam.fx * X / Z + cam.cx
            vv = cam.fy * Y / Z + cam.cy
            d, du, dv = sample(self.dt, u, vv)
            ss = np.sqrt(self.lsil)
            r = ss * d
            e["sil"] = float((self.bsign * r * r).sum())
            e["sil_abs"] = float((r * r).sum())
            rows_F.append(r)
            rows_b.append(self.bsign)
            if need_jacobian:
                for n in range(self.bnd.size):
                    Pn = np.array([[cam.fx / Z[n], 0, -cam.fx * X[n] / Z[n] ** 2],
                                   [0, cam.fy / Z[n], -cam.fy * Y[n] / Z[n] ** 2]])
                    g = ss * np.array([du[n], dv[n]]) @ Pn
                    rows_J.append((g @ Js[n])[None, :])
        # temporal stabilisation: sqrt(lambda_T lambda_j) (p_j - p_j^{t-1})
        if self.prev_joints is not None:
            for j in range(sk.nj):
                st = np.sqrt(self.lam_t[j])
                r = st * (p[j] - self.prev_joints[:, j])
                e["temporal"] += float(r @ r)
                rows_F.append(r)
                rows_b.append(np.ones(3))
                if need_jacobian:
                    rows_J.append(st * dpoint(p[j], sk.anc[j][1:]))
        # joint limits: quadratic barrier on every rotational unknown outside its range
        if self.limits is not None and self.l_anat > 0:
            lo, hi = self.limits
            th = pose[:sk.it]
            sa = np.sqrt(self.l_anat)
            over, under = th > hi, th < lo
            r = sa * np.where(over, th - hi, np.where(under, lo - th, 0.0))
            e["anatomic"] = float(r @ r)
            rows_F.append(r)
            rows_b.append(np.ones(sk.it))
            if need_jacobian:
                Ja = np.zeros((sk.it, sk.nu))
                Ja[np.arange(sk.it), np.arange(sk.it)] = sa * np.where(over, 1.0, np.where(under, -1.0, 0.0))
                rows_J.append(Ja)
        F = np.concatenate(rows_F)
        b = np.concatenate(rows_b)
        e["total"] = e["e2d"] + e["e3d"] + e["sil"] + e["temporal"] + e["anatomic"]
        Jm = np.concatenate(rows_J, axis=0) if need_jacobian else None
        return F, b, Jm, e

    def energy(self, pose):
        return self.linearize(pose, need_jacobian=False)[3]


def solve(problem, gn_iters):
    pose = problem.pose0.copy()
    energies = []
    for _ in range(gn_iters):
        F, b, J, e = problem.linearize(pose)
        energies.append(e)
        A = J.T @ (np.abs(b)[:, None] * J)
        A[np.diag_indices(A.shape[0])] += 1e-6 * A.diagonal().max()
        rhs = -(J.T @ (b * F))
        L = np.linalg.cholesky(A)
        delta = np.linalg.solve(L.T, np.linalg.solve(L, rhs))
        pose = pose + delta
    energies.append(problem.energy(pose))
    return dict(pose=pose, energies=energies, n_boundary=int(problem.bnd.size),
                n_visible=int(problem.dec["visible"].sum()))


def blended_rotations(skel, bind_idx, bind_w, pose):
    """Per-vertex rotation of dual-quaternion skinning (its rotation part):
    the unit quaternions of the influencing joints' global rotations, each
    flipped into the hemisphere of the first influence's, blended by the
    skinning weights and normalised (Sec. 3.1: the template is rigged with
    dual quaternion skinning).  Returns [nv][3][3] (float64)."""
    from scipy.spatial.transform import Rotation
    R, _, _ = skel.fk(np.asarray(pose, np.float64))
    q = Rotation.from_matrix(R).as_quat()                      # [nj][4] (x, y, z, w), library conversion
    nv = bind_idx.shape[1]
    acc = np.zeros((nv, 4))
    q0 = q[bind_idx[0]]
    for s in range(bind_idx.shape[0]):
        qs = q[bind_idx[s]]
        sign = np.where((qs * q0).sum(axis=1) < 0.0, -1.0, 1.0)
        acc += (bind_w[s].astype(np.float64) * sign)[:, None] * qs
    acc /= np.linalg.norm(acc, axis=1, keepdims=True)
    return Rotation.from_quat(acc).as_matrix()


def warp_displacements(skel, bind_idx, bind_w, pose_prev, pose_cur, V_prev, S_prev, S_cur):
    """Displacement warping (Sec. 3.4): the non-rigid displacement of the
    previous frame d = V^{t-1} - V^{S,t-1} is taken back to the rest pose by
    the inverse of the previous pose's skinning rotation, carried forward by
    the current pose's, and added to the current skinned mesh:
        V^t_start = V^{S,t} + M_t M_{t-1}^T d,  M = blended_rotations(...).
    Arrays [3][nv]; result float64."""
    Mp = blended_rotations(skel, bind_idx, bind_w, pose_prev)
    Mc = blended_rotations(skel, bind_idx, bind_w, pose_cur)
    d = (np.asarray(V_prev, np.float64) - np.asarray(S_prev, np.float64)).T     # [nv][3]
    rest = np.einsum("nba,nb->na", Mp, d)                                       # M_{t-1}^T d
    return np.asarray(S_cur, np.float64) + np.einsum("nab,nb->na", Mc, rest).T


def extrapolate_pose(pose_prev, pose_prev2):
    """Start pose of the next frame (Sec. 3.3): an explicit Euler step in
    joint-angle space from the last two frames' poses, p + (p - p_prev)."""
    p1 = np.asarray(pose_prev, np.float64)
    return p1 + (p1 - np.asarray(pose_prev2, np.float64))

