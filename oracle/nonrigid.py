"""Non-rigid stage on an embedded deformation graph, float64 Gauss-Newton (oracle).

Unknowns: per node k a rotation R_k and translation t_k (state [12][n]:
R row-major, then t).  A vertex moves as
    V_i = sum_k w_ik [R_k (v_i - g_k) + g_k + t_k],   g_k = v_{node_vertex[k]}.
Linearisation uses the left perturbation R_k <- Exp(dw_k) R_k, t_k <- t_k + dt_k,
so the unknown block of node k is (dw_k, dt_k) in R^6 and
    dV_i / d(dw_k) = -w_ik [q_ik]x,  dV_i / d(dt_k) = w_ik I,  q_ik = R_k (v_i - g_k).

Energy (Sec. 3.4, Eq. for E_photo and E_silhouette, with the as-rigid-as-
possible regulariser on graph edges):
    photo:  r_i = sqrt(w_photo) (I_Gauss(pi(V_i)) - C_i) in R^3, i in the visible set;
            the robust kernel sigma_c zeroes the residual (and its Jacobian) when
            ||I_Gauss - C_i||_2 > tau_c (tau_c = inf disables it);
    sil:    r_i = sqrt(w_sil) I_DT(pi(V_i)), i in B, direction weight b_i;
    ARAP:   r_kl = sqrt(w_arap) (R_k (g_l - g_k) + g_k + t_k - g_l - t_l), directed edges.
    velocity (optional, w_vel > 0): r_i = sqrt(w_vel) (V_i - V_i^a) for every vertex,
            the paper's temporal prior (Sec. 3.4, E_velocity) with V^{t-1} carried
            to the current frame by the start state: V^a is the input mesh
            deformed by the start node state (the float32 start positions of
            the decision recipe), i.e. the previous frame's result displaced
            onto the current pose;
With outline=True the contour set keeps only vertices on the outline of the
rendered model (see decisions.frame_decisions_from_positions), for meshes made
of overlapping closed parts.
E = sum b r^2 with b = 1 except the silhouette rows (the paper's energy, which
has negative terms when b_i = -1).  With case2="exclude" the silhouette rows of
b_i = -1 vertices are dropped instead (b = 0): the literal term is unbounded
below and, with decisions frozen for the frame, Gauss-Newton doubles such a
vertex's distance to the contour at every step.  Gauss-Newton (Sec. 4, Eq. gaussnewton)
solves  (J^T |B| J) delta = -J^T B F  with B = diag(b): the system matrix uses
|b| so that it stays positive semi-definite.

Linear solve, two modes:
    'chol': exact solve by a sparse Cholesky factorisation (bandwidth-reducing
            reverse Cuthill-McKee ordering, banded factorisation);
    'pcg':  exactly ``pcg_iters`` Jacobi-preconditioned CG iterations from 0
            (Sec. 4, non-rigid paragraph: diagonal preconditioner), stopping early
            only when p.Ap <= 0 or r.z == 0; a non-positive diagonal entry
            is replaced by 1 in the preconditioner.
"""
import numpy as np
import scipy.sparse as sp

from . import so3
from .image import blur, distance_transform, sample
from .decisions import frame_decisions


def ed_deform(xyz, graph, state):
    """Deformed positions V (float64, [3][nv]) and q_ik ([k][3][nv])."""
    p = xyz.astype(np.float64)
    nodes = graph["node_vertex"]
    g = p[:, nodes]
    st = state.astype(np.float64)
    R = st[:9].reshape(3, 3, -1)
    t = st[9:12]
    bidx, bw = graph["bind_idx"], graph["bind_w"].astype(np.float64)
    V = np.zeros_like(p)
    q = np.zeros((bidx.shape[0], 3, p.shape[1]))
    for j in range(bidx.shape[0]):
        k = bidx[j]
        d = p - g[:, k]
        qj = np.einsum("abn,bn->an", R[:, :, k], d)
        q[j] = qj
        V += bw[j] * (qj + g[:, k] + t[:, k])
    return V, q


def projection_jacobian(V, cam):
    X, Y, Z = V
    P = np.zeros((V.shape[1], 2, 3))
    P[:, 0, 0] = cam.fx / Z
    P[:, 0, 2] = -cam.fx * X / (Z * Z)
    P[:, 1, 1] = cam.fy / Z
    P[:, 1, 2] = -cam.fy * Y / (Z * Z)
    return P


def _vertex_cols(graph, q, vid):
    """Per-vertex 3x(6*nn) Jacobian blocks as (row-local, col, val) triplets source."""
    bidx, bw = graph["bind_idx"], graph["bind_w"].astype(np.float64)
    blocks = []
    for j in range(bidx.shape[0]):
        k = bidx[j, vid]
        w = bw[j, vid]
        qq = q[j][:, vid]
        # -w [q]x  : columns dw_x, dw_y, dw_z
        Mw = np.zeros((vid.size, 3, 3))
        Mw[:, 0, 1] = w * qq[2]
        Mw[:, 0, 2] = -w * qq[1]
        Mw[:, 1, 0] = -w * qq[2]
        Mw[:, 1, 2] = w * qq[0]
        Mw[:, 2, 0] = w * qq[1]
        Mw[:, 2, 1] = -w * qq[0]
        Mt = np.zeros((vid.size, 3, 3))
        Mt[:, 0, 0] = Mt[:, 1, 1] = Mt[:, 2, 2] = w
        blocks.append((k, np.concatenate([Mw, Mt], axis=2)))   # [n][3][6]
    return blocks


class Problem:
    """One non-rigid frame: inputs plus the frozen per-frame decisions."""

    def __init__(self, xyz, tri, rgb, graph, cam, mask, image, weights, tau_c=np.inf,
                 state0=None, w_vel=0.0, case2="push", outline=False):
        self.xyz, self.tri, self.rgb, self.graph, self.cam = xyz, tri, rgb, graph, cam
        self.w_sil, self.w_photo, self.w_arap = (float(w) for w in weights)
        self.tau_c = float(tau_c)
        nn = graph["node_vertex"].size
        if state0 is None:
            state0 = identity_state(nn)
        self.state0 = state0.astype(np.float32)
        self.mask = mask
        self.dt, _ = distance_transform(mask)
        self.img = blur(image, 3)
        self.dec = frame_decisions(xyz, tri, graph, self.state0, cam, mask, self.dt, outline=outline)
        self.vis_idx = np.nonzero(self.dec["visible"])[0]
        self.bnd_idx = np.nonzero(self.dec["boundary"])[0]
        self.bsign = self.dec["bsign"][self.bnd_idx].astype(np.float64)
        if case2 == "exclude":
            keep = self.bsign > 0
            self.bnd_idx, self.bsign = self.bnd_idx[keep], self.bsign[keep]
        self.w_vel = float(w_vel)
        self.anchor = np.stack([self.dec["X"], self.dec["Y"], self.dec["Z"]]).astype(np.float64)
        self.nn = nn
        ed = graph["edge_dst"]
        src = np.repeat(np.arange(nn)[None, :], ed.shape[0], axis=0)
        keep = ed >= 0
        self.e_src, self.e_dst = src[keep], ed[keep]

    # ---- residuals and Jacobian -------------------------------------------
    def linearize(self, state, need_jacobian=True):
        """Residual vector F, row weights b, Jacobian J (csr) and per-term energies."""
        V, q = ed_deform(self.xyz, self.graph, state)
        cam = self.cam
        X, Y, Z = V
        u = cam.fx * X / Z + cam.cx
        v = cam.fy * Y / Z + cam.cy
        P = projection_jacobian(V, cam)
        rows_F, rows_b, trip = [], [], []
        row0 = 0
        e = dict(photo=0.0, sil=0.0, sil_abs=0.0, arap=0.0, vel=0.0)

        # photometric rows
        vid = self.vis_idx
        vid = vid[Z[vid] > 0]
        val, gu, gv = sample(self.img, u[vid], v[vid])            # [3][n]
        res = val - self.rgb[:, vid].astype(np.float64)
        keep = np.sqrt((res * res).sum(axis=0)) <= self.tau_c
        sw = np.sqrt(self.w_photo)
        r_ph = sw * res * keep
        e["photo"] = float((r_ph ** 2).sum())
        if need_jacobian:
            G = np.einsum("cn,nk->cnk", gu, P[vid, 0, :]) + np.einsum("cn,nk->cnk", gv, P[vid, 1, :])
            G *= (sw * keep)[None, :, None]                          # [3][n][3] dr/dV
            blocks = _vertex_cols(self.graph, q, vid)
        for c in range(3):
            nrow = vid.size
            rows_F.append(r_ph[c])
            rows_b.append(np.ones(nrow))
            if need_jacobian:
                rr = row0 + np.arange(nrow)
                for k, M in blocks:
                    vals = np.einsum("nk,nkm->nm", G[c], M)        # [n][6]
                    cols = 6 * k[:, None] + np.arange(6)[None, :]
                    trip.append((np.repeat(rr, 6), cols.ravel(), vals.ravel()))
            row0 += nrow

        # silhouette rows
        vid = self.bnd_idx
        okz = Z[vid] > 0
        vid, bs = vid[okz], self.bsign[okz]
        d, du, dv = sample(self.dt, u[vid], v[vid])
        sw = np.sqrt(self.w_sil)
        r_s = sw * d
        e["sil"] = float((bs * r_s * r_s).sum())
        e["sil_abs"] = float((r_s * r_s).sum())
        rows_F.append(r_s)
        rows_b.append(bs)
        if need_jacobian:
            G = sw * (du[:, None] * P[vid, 0, :] + dv[:, None] * P[vid, 1, :])
            rr = row0 + np.arange(vid.size)
            for k, M in _vertex_cols(self.graph, q, vid):
                vals = np.einsum("nk,nkm->nm", G, M)
                cols = 6 * k[:, None] + np.arange(6)[None, :]
                trip.append((np.repeat(rr, 6), cols.ravel(), vals.ravel()))
        row0 += vid.size

        # velocity rows (all vertices)
        if self.w_vel > 0:
            sw = np.sqrt(self.w_vel)
            r_v = sw * (V - self.anchor)
            e["vel"] = float((r_v ** 2).sum())
            vid = np.arange(V.shape[1])
            if need_jacobian:
                blocks = _vertex_cols(self.graph, q, vid)
            for c in range(3):
                rows_F.append(r_v[c])
                rows_b.append(np.ones(vid.size))
                if need_jacobian:
                    rr = row0 + np.arange(vid.size)
                    for k, M in blocks:
                        vals = sw * M[:, c, :]
                        cols = 6 * k[:, None] + np.arange(6)[None, :]
                        trip.append((np.repeat(rr, 6), cols.ravel(), vals.ravel()))
                row0 += vid.size

        # ARAP rows
        g = self.xyz.astype(np.float64)[:, self.graph["node_vertex"]]
        st = state.astype(np.float64)
        R = st[:9].reshape(3, 3, -1)
        t = st[9:12]
        ks, ls = self.e_src, self.e_dst
        ekl = np.einsum("abn,bn->an", R[:, :, ks], g[:, ls] - g[:, ks])     # [3][ne]
        sw = np.sqrt(self.w_arap)
        r_a = sw * (ekl + g[:, ks] + t[:, ks] - g[:, ls] - t[:, ls])
        e["arap"] = float((r_a ** 2).sum())
        ne = ks.size
        for c in range(3):
            rows_F.append(r_a[c])
            rows_b.append(np.ones(ne))
        if need_jacobian:
            for c in range(3):
                rr = row0 + c * ne + np.arange(ne)
                # d r_c / d dw_k = -sw [e]x row c ; d/d dt_k = sw e_c ; d/d dt_l = -sw e_c
                hat_row = {0: (None, -ekl[2], ekl[1]), 1: (ekl[2], None, -ekl[0]),
                           2: (-ekl[1], ekl[0], None)}[c]
                for m in range(3):
                    if hat_row[m] is not None:
                        trip.append((rr, 6 * ks + m, -sw * hat_row[m]))
                trip.append((rr, 6 * ks + 3 + c, np.full(ne, sw)))
                trip.append((rr, 6 * ls + 3 + c, np.full(ne, -sw)))
            row0 += 3 * ne
        F = np.concatenate(rows_F)
        b = np.concatenate(rows_b)
        e["total"] = e["photo"] + e["sil"] + e["arap"] + e["vel"]
        J = None
        if need_jacobian:
            r = np.concatenate([x[0] for x in trip])
            cidx = np.concatenate([x[1] for x in trip])
            vals = np.concatenate([x[2] for x in trip])
            J = sp.csr_matrix((vals, (r, cidx)), shape=(row0, 6 * self.nn))
        return F, b, J, e

    def energy(self, state):
        return self.linearize(state, need_jacobian=False)[3]

    def normal_equations(self, state):
        F, b, J, e = self.linearize(state)
        A = (J.T @ sp.diags(np.abs(b)) @ J).tocsr()
        rhs = -(J.T @ (b * F))
        return A, rhs, e


def identity_state(nn):
    s = np.zeros((12, nn), dtype=np.float32)
    s[0] = s[4] = s[8] = 1.0
    return s


def sparse_cholesky(A):
    """Sparse Cholesky factorisation A[perm][:, perm] = L L^T of an SPD matrix.

    Ordering: reverse Cuthill-McKee on the sparsity graph, which gathers the
    non-zeros of every row into a band next to the diagonal; all fill-in of the
    factor stays inside that band.  The band is factored by LAPACK's banded
    Cholesky.  Returns (perm, band factor in LAPACK lower band storage).
    """
    from scipy.linalg import cholesky_banded
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    A = sp.csr_matrix(A)
    n = A.shape[0]
    perm = np.asarray(reverse_cuthill_mckee(A, symmetric_mode=True), dtype=np.int64)
    B = A[perm][:, perm].tocoo()
    low = B.row >= B.col
    r, c, v = B.row[low], B.col[low], B.data[low]
    bw = int((r - c).max()) if r.size else 0
    band = np.zeros((bw + 1, n))
    band[r - c, c] = v                 # lower storage: band[i - j, j] = B[i, j]
    return perm, cholesky_banded(band, lower=True)


def solve_cholesky(A, rhs):
    """Exact solve of the normal equations by the sparse Cholesky factorisation."""
    from scipy.linalg import cho_solve_banded
    perm, L = sparse_cholesky(A)
    y = cho_solve_banded((L, True), rhs[perm])
    x = np.empty_like(y)
    x[perm] = y
    return x


def solve_pcg(A, rhs, iters):
    d = A.diagonal().copy()
    d[d <= 0] = 1.0
    minv = 1.0 / d
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = minv * r
    p = z.copy()
    rz = float(r @ z)
    for _ in range(iters):
        if rz == 0.0:
            break
        Ap = A @ p
        pAp = float(p @ Ap)
        if pAp <= 0.0:
            break
        alpha = rz / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        z = minv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x


def apply_update(state, delta):
    """R_k <- Exp(dw_k) R_k, t_k <- t_k + dt_k (float64 state)."""
    st = state.astype(np.float64).copy()
    nn = st.shape[1]
    d = delta.reshape(nn, 6)
    for k in range(nn):
        R = st[:9, k].reshape(3, 3)
        st[:9, k] = (so3.exp(d[k, :3]) @ R).ravel()
        st[9:12, k] += d[k, 3:]
    return st


def solve(problem, gn_iters, mode="chol", pcg_iters=10, start=None):
    """Run the Gauss-Newton schedule; returns state (float64) and energies.

    The schedule starts at ``start`` if given (e.g. a predicted start), else at
    the state the frame's decisions were taken at (problem.state0)."""
    state = (problem.state0 if start is None else start).astype(np.float64)
    energies = []
    for _ in range(gn_iters):
        A, rhs, e = problem.normal_equations(state)
        energies.append(e)
        if mode == "chol":
            delta = solve_cholesky(A, rhs)
        else:
            delta = solve_pcg(A, rhs, pcg_iters)
        state = apply_update(state, delta)
    energies.append(problem.energy(state))
    return dict(state=state, energies=energies, n_visible=int(problem.vis_idx.size),
                n_boundary=int(problem.bnd_idx.size))
