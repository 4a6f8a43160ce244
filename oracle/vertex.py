"""Non-rigid stage with per-vertex unknowns, float64 Gauss-Newton (oracle).

Test infrastructure only (tests, the smoke check and the benchmark's CPU
baseline may use it; the product library never does).

This is the paper's own parameterisation of Stage II (Sec. 3.4): the unknowns
are the vertex positions V in R^{3N}, started from the skinned pose result
V^S (or any start V0 the caller passes, e.g. the displacement-warped start),
and

    E(V) = E_photo + E_silhouette + E_smooth + E_edge + E_velocity + E_acceleration

    photo:   w_photo sum_{i in visible} ||sigma_c(I_Gauss(pi(V_i)) - C_i)||^2
    sil:     w_sil   sum_{i in B} b_i I_DT(pi(V_i))^2
    smooth:  w_smooth sum_i sum_{j in N_i} s_ij/|N_i| ||(V_i - V_j) - (V^S_i - V^S_j)||^2
    edge:    w_edge   sum_i sum_{j in N_i} s_ij/|N_i| (||V_i - V_j|| - ||Vhat_i - Vhat_j||)^2
    velocity:     w_vel sum_i ||V_i - V^{t-1}_i||^2
    acceleration: w_acc sum_i ||V_i - 2 V^{t-1}_i + V^{t-2}_i||^2

(Sec. 3.4, the equations of the dense photometric and silhouette alignment and
of the spatial and temporal regularisers).  I_Gauss is the frame blurred by a
Gaussian of odd kernel size k (``image.blur``); the paper's photometric pyramid
takes one Gauss-Newton step per level with k = 15, 9, 3 (read as three blur
levels at full resolution; ``solve(..., blur_schedule=(15, 9, 3))``).  N_i is the one-ring of vertex i
(the vertices that share a mesh edge with it), Vhat the template's rest pose,
s_ij = (s_i + s_j)/2 with s_i the Table 1 non-rigidity weight of vertex i's
material class (Sec. 3.1).  The robust kernel sigma_c zeroes a vertex's whole
colour residual when ||I_Gauss - C_i||_2 > tau_c (tau_c = inf: off).  The
acceleration term needs V^{t-2}; without it the term is absent.

Decisions (visible set, contour set B, signs b_i) are taken once per frame
at the float32 start positions by the recipe of ``decisions`` (the paper takes
visibility from the skinned mesh after the pose step and updates B after
Stage I).  With per-vertex body-part labels, a contour vertex whose pixel
lies in another part's region of the dilated part mask loses its silhouette
residual (b_i = 0; ``part_label_image``; the mask is rendered from the start
positions, the posed model carried into the frame).  A vertex whose edge vector has zero length contributes no edge-term
derivative (its unit direction is taken as 0).

Gauss-Newton (Sec. 4, Eq. gaussnewton) solves (J^T |B| J) delta = -J^T B F and
sets V <- V + delta; the linear solve is the exact sparse Cholesky of
``nonrigid.solve_cholesky`` or exactly ``pcg_iters`` Jacobi-PCG iterations of
``nonrigid.solve_pcg`` (diagonal preconditioner, Sec. 4 non-rigid paragraph).
"""
import numpy as np
import scipy.sparse as sp

from .decisions import frame_decisions_from_positions, mesh_edges, triangle_coverage
from .image import blur, distance_transform, sample
from .nonrigid import projection_jacobian, solve_cholesky, solve_pcg

# Table 1: non-rigidity weight of each material class (class ids 1..7).
CLASS_WEIGHTS = np.array([1.0, 2.0, 2.5, 3.0, 50.0, 100.0, 200.0])


def vertex_weights(classes):
    """Per-vertex smoothness weight s_i from class ids in 1..7 (Table 1)."""
    c = np.asarray(classes, dtype=np.int64)
    if c.min() < 1 or c.max() > 7:
        raise ValueError("material classes are 1..7")
    return CLASS_WEIGHTS[c - 1]


def one_ring(tri, nv):
    """Sorted neighbour list of every vertex (vertices sharing a mesh edge)."""
    nb = [set() for _ in range(nv)]
    for a, b, _, _ in mesh_edges(tri):
        nb[a].add(b)
        nb[b].add(a)
    return [np.array(sorted(s), dtype=np.int64) for s in nb]


class VertexProblem:
    """One frame of the per-vertex non-rigid stage with its frozen decisions."""

    def __init__(self, rest, posed, tri, rgb, classes, cam, mask, image, weights, start=None,
                 prev=None, prev2=None, tau_c=np.inf, case2="push", outline=False, blur_k=3, parts=None,
                 part_dilation=10):
        """rest: Vhat [3][N]; posed: V^S [3][N]; weights: dict with w_photo, w_sil,
        w_smooth, w_edge, w_vel, w_acc; start: V0 (default V^S); prev, prev2:
        V^{t-1}, V^{t-2} (None: the velocity / acceleration term is absent)."""
        self.rest = rest.astype(np.float64)
        self.posed = posed.astype(np.float64)
        self.tri, self.rgb, self.cam = tri, rgb, cam
        self.nv = rest.shape[1]
        w = dict(w_photo=0.0, w_sil=0.0, w_smooth=0.0, w_edge=0.0, w_vel=0.0, w_acc=0.0)
        w.update(weights)
        self.w = {k: float(v) for k, v in w.items()}
        self.tau_c = float(tau_c)
        self.s = vertex_weights(classes)
        self.nbr = one_ring(tri, self.nv)
        start = self.posed if start is None else start
        self.start = start.astype(np.float32)
        self.prev = None if prev is None else prev.astype(np.float64)
        self.prev2 = None if prev2 is None else prev2.astype(np.float64)
        if self.prev is None and self.w["w_vel"] > 0:
            raise ValueError("velocity term without V^{t-1}")
        if (self.prev is None or self.prev2 is None) and self.w["w_acc"] > 0:
            raise ValueError("acceleration term without V^{t-1} and V^{t-2}")
        self.dt, _ = distance_transform(mask)
        self.image_in = image
        self.blur_k = int(blur_k)
        self._blurred = {}
        X, Y, Z = self.start
        self.dec = frame_decisions_from_positions(X, Y, Z, tri, cam, mask, self.dt, outline=outline)
        self.vis_idx = np.nonzero(self.dec["visible"])[0]
        self.bnd_idx = np.nonzero(self.dec["boundary"])[0]
        self.bsign = self.dec["bsign"][self.bnd_idx].astype(np.float64)
        if case2 == "exclude":
            keep = self.bsign > 0
            self.bnd_idx, self.bsign = self.bnd_idx[keep], self.bsign[keep]
        self.part_image = None
        if parts is not None:
            self.part_image = part_label_image(self.dec, tri, parts, cam, part_dilation)
            px = np.rint(self.dec["u"][self.bnd_idx]).astype(np.int64)
            py = np.rint(self.dec["v"][self.bnd_idx]).astype(np.int64)
            lab = self.part_image[py, px]
            keep = (lab < 0) | (lab == np.asarray(parts)[self.bnd_idx])
            self.bnd_idx, self.bsign = self.bnd_idx[keep], self.bsign[keep]
        # directed edges (i, j), j in N_i, with weight s_ij / |N_i|
        src = np.concatenate([np.full(len(n), i) for i, n in enumerate(self.nbr)]).astype(np.int64)
        dst = np.concatenate(self.nbr).astype(np.int64)
        deg = np.array([len(n) for n in self.nbr], dtype=np.float64)
        self.e_src, self.e_dst = src, dst
        self.e_w = 0.5 * (self.s[src] + self.s[dst]) / deg[src]
        d = self.rest[:, src] - self.rest[:, dst]
        self.e_rest = np.sqrt((d * d).sum(axis=0))

    def image(self, k=None):
        """I_Gauss of the frame with Gaussian kernel size k (default: the problem's)."""
        k = self.blur_k if k is None else int(k)
        if k not in self._blurred:
            self._blurred[k] = blur(self.image_in, k)
        return self._blurred[k]

    def linearize(self, V, need_jacobian=True, blur_k=None):
        """Residuals F, row weights b, Jacobian J (csr, 3N columns), per-term energies;
        the photometric term samples I_Gauss of kernel size blur_k."""
        V = np.asarray(V, dtype=np.float64)
        img = self.image(blur_k)
        cam, nv = self.cam, self.nv
        X, Y, Z = V
        u = cam.fx * X / Z + cam.cx
        v = cam.fy * Y / Z + cam.cy
        P = projection_jacobian(V, cam)
        Fs, bs, trip = [], [], []
        row0 = 0
        e = dict(photo=0.0, sil=0.0, sil_abs=0.0, smooth=0.0, edge=0.0, vel=0.0, acc=0.0)

        def add_block(rows, cols_vertex, M):
            """Rows `rows` (n) get the 1x3 blocks M (n x 3) at columns of the vertices."""
            for a in range(3):
                trip.append((rows, 3 * cols_vertex + a, M[:, a]))

        # photometric rows: 3 per visible vertex
        vid = self.vis_idx[Z[self.vis_idx] > 0]
        val, gu, gv = sample(img, u[vid], v[vid])
        res = val - self.rgb[:, vid].astype(np.float64)
        keep = np.sqrt((res * res).sum(axis=0)) <= self.tau_c
        sw = np.sqrt(self.w["w_photo"])
        r_ph = sw * res * keep
        e["photo"] = float((r_ph ** 2).sum())
        for c in range(3):
            Fs.append(r_ph[c])
            bs.append(np.ones(vid.size))
            if need_jacobian:
                G = (sw * keep)[:, None] * (gu[c][:, None] * P[vid, 0, :] + gv[c][:, None] * P[vid, 1, :])
                add_block(row0 + np.arange(vid.size), vid, G)
            row0 += vid.size

        # silhouette rows: 1 per contour vertex
        vid = self.bnd_idx
        okz = Z[vid] > 0
        vid, bsg = vid[okz], self.bsign[okz]
        d, du, dv = sample(self.dt, u[vid], v[vid])
        sw = np.sqrt(self.w["w_sil"])
        r_s = sw * d
        e["sil"] = float((bsg * r_s * r_s).sum())
        e["sil_abs"] = float((r_s * r_s).sum())
        Fs.append(r_s)
        bs.append(bsg)
        if need_jacobian:
            G = sw * (du[:, None] * P[vid, 0, :] + dv[:, None] * P[vid, 1, :])
            add_block(row0 + np.arange(vid.size), vid, G)
        row0 += vid.size

        # spatial smoothness: 3 rows per directed edge
        i, j = self.e_src, self.e_dst
        ne = i.size
        sw = np.sqrt(self.w["w_smooth"] * self.e_w)
        r_sm = sw * ((V[:, i] - V[:, j]) - (self.posed[:, i] - self.posed[:, j]))
        e["smooth"] = float((r_sm ** 2).sum())
        for c in range(3):
            Fs.append(r_sm[c])
            bs.append(np.ones(ne))
            if need_jacobian:
                rr = row0 + np.arange(ne)
                trip.append((rr, 3 * i + c, sw))
                trip.append((rr, 3 * j + c, -sw))
            row0 += ne

        # edge length: 1 row per directed edge
        dvec = V[:, i] - V[:, j]
        ell = np.sqrt((dvec * dvec).sum(axis=0))
        sw = np.sqrt(self.w["w_edge"] * self.e_w)
        r_ed = sw * (ell - self.e_rest)
        e["edge"] = float((r_ed ** 2).sum())
        Fs.append(r_ed)
        bs.append(np.ones(ne))
        if need_jacobian:
            with np.errstate(invalid="ignore", divide="ignore"):
                unit = np.where(ell > 0, dvec / ell, 0.0)
            rr = row0 + np.arange(ne)
            add_block(rr, i, (sw * unit).T)
            add_block(rr, j, (-sw * unit).T)
        row0 += ne

        # temporal priors: 3 rows per vertex each
        allv = np.arange(nv)
        for name, wkey, target in (("vel", "w_vel", None), ("acc", "w_acc", None)):
            wt = self.w[wkey]
            if wt <= 0:
                continue
            if name == "vel":
                ref = self.prev
            else:
                ref = 2.0 * self.prev - self.prev2
            sw = np.sqrt(wt)
            r_t = sw * (V - ref)
            e[name] = float((r_t ** 2).sum())
            for c in range(3):
                Fs.append(r_t[c])
                bs.append(np.ones(nv))
                if need_jacobian:
                    trip.append((row0 + allv, 3 * allv + c, np.full(nv, sw)))
                row0 += nv

        F = np.concatenate(Fs)
        b = np.concatenate(bs)
        e["total"] = e["photo"] + e["sil"] + e["smooth"] + e["edge"] + e["vel"] + e["acc"]
        J = None
        if need_jacobian:
            r = np.concatenate([t[0] for t in trip])
            cidx = np.concatenate([t[1] for t in trip])
            vals = np.concatenate([np.broadcast_to(t[2], t[0].shape) for t in trip])
            J = sp.csr_matrix((vals, (r, cidx)), shape=(row0, 3 * nv))
        return F, b, J, e

    def energy(self, V, blur_k=None):
        return self.linearize(V, need_jacobian=False, blur_k=blur_k)[3]

    def normal_equations(self, V, blur_k=None):
        """System J^T |B| J, right-hand side -J^T B F (unknowns vertex-major: 3i + a)."""
        F, b, J, e = self.linearize(V, blur_k=blur_k)
        A = (J.T @ sp.diags(np.abs(b)) @ J).tocsr()
        rhs = -(J.T @ (b * F))
        return A, rhs, e


def part_label_image(dec, tri, parts, cam, dilation=10):
    """Body-part mask (Sec. 3.4, dense silhouette alignment): the model at the
    frame's start positions rendered with per-face part labels (a face takes
    its first vertex's label; a pixel the label of the face that sets its
    depth-buffer value, the smallest on ties; -1 for background), then
    `dilation` growth steps over the 3x3 neighbourhood in which label 0 (the
    torso) takes precedence: a pixel becomes torso when a neighbour is torso,
    and a background pixel otherwise takes the smallest label among its
    labelled neighbours.  Returns int [H][W]."""
    W, H = cam.width, cam.height
    zb = dec["zbuf"].reshape(-1)
    lab = np.full(H * W, np.iinfo(np.int64).max, dtype=np.int64)
    parts = np.asarray(parts, dtype=np.int64)
    for f, _, pix, inv in triangle_coverage(dec["u"], dec["v"], dec["Z"], dec["valid"], tri, W, H):
        top = inv.view(np.uint32) == zb[pix]
        np.minimum.at(lab, pix[top], parts[tri[0, f]])
    lab = np.where(lab == np.iinfo(np.int64).max, -1, lab).reshape(H, W)
    for _ in range(dilation):
        pad = np.pad(lab, 1, constant_values=-1)
        nb = [pad[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        nb = np.stack(nb)                                           # [9][H][W], the pixel itself included
        torso = (nb == 0).any(axis=0)
        big = np.iinfo(np.int64).max
        smallest = np.where(nb >= 0, nb, big).min(axis=0)
        new = np.where(torso, 0, np.where(lab >= 0, lab, np.where(smallest < big, smallest, -1)))
        lab = new
    return lab


def solve(problem, gn_iters, mode="chol", pcg_iters=10, start=None, blur_schedule=None):
    """Gauss-Newton schedule from the frame's start (or `start`); V [3][N] float64.

    blur_schedule: Gaussian kernel size of I_Gauss per Gauss-Newton step (the
    photometric pyramid of Sec. 3.4 is (15, 9, 3): one step per level); the
    final energy uses the last step's kernel.  Default: the problem's kernel."""
    V = (problem.start if start is None else start).astype(np.float64).copy()
    ks = [problem.blur_k] * gn_iters if blur_schedule is None else [int(k) for k in blur_schedule]
    if len(ks) != gn_iters:
        raise ValueError("one blur kernel per Gauss-Newton step")
    energies = []
    for g in range(gn_iters):
        A, rhs, e = problem.normal_equations(V, blur_k=ks[g])
        energies.append(e)
        delta = solve_cholesky(A, rhs) if mode == "chol" else solve_pcg(A, rhs, pcg_iters)
        V = V + delta.reshape(problem.nv, 3).T
    energies.append(problem.energy(V, blur_k=ks[-1]))
    return dict(V=V, energies=energies, n_visible=int(problem.vis_idx.size), n_boundary=int(problem.bnd_idx.size))


def snap_vertices(problem, V, max_px=3.0, steps=4, rings=2, iters=8, tol_px=0.05):
    """Vertex snapping (Sec. 3.4) after the non-rigid stage, float64.

    Contour vertices of the frame's set B with b_i = +1 walk on the distance
    transform along its negative gradient: u <- u - I_DT(u) grad/|grad|, at
    most `steps` times, stopping once I_DT(u) <= tol_px or the gradient
    vanishes (|grad| < 1e-6); a vertex whose distance at the start exceeds
    max_px is not snapped.  The snapped pixel is lifted back at the vertex's
    depth: X = (u - cx) Z / fx, Y = (v - cy) Z / fy.  The other vertices within
    `rings` one-ring steps of a snapped vertex follow a Laplacian warp: their
    displacement starts at 0 and takes `iters` Jacobi sweeps
    d_i <- mean_{j in N_i} d_j, with snapped vertices held at their snap
    displacement and vertices farther away held at 0.  Returns (V', snapped
    mask)."""
    V = np.asarray(V, np.float64)
    cam, nv = problem.cam, problem.nv
    disp = np.zeros((3, nv))
    snapped = np.zeros(nv, bool)
    for i, b in zip(problem.bnd_idx, problem.bsign):
        if b < 0:
            continue
        X, Y, Z = V[:, i]
        if Z <= 0:
            continue
        u = cam.fx * X / Z + cam.cx
        v = cam.fy * Y / Z + cam.cy
        d0 = sample(problem.dt, np.array([u]), np.array([v]))[0][0]
        if d0 > max_px:
            continue
        for _ in range(steps):
            d, gu, gv = (a[0] for a in sample(problem.dt, np.array([u]), np.array([v])))
            g = np.hypot(gu, gv)
            if d <= tol_px or g < 1e-6:
                break
            u, v = u - d * gu / g, v - d * gv / g
        disp[:, i] = [(u - cam.cx) * Z / cam.fx - X, (v - cam.cy) * Z / cam.fy - Y, 0.0]
        snapped[i] = True
    # ring distance from the snapped vertices
    dist = np.where(snapped, 0, rings + 1)
    for r in range(1, rings + 1):
        for i in range(nv):
            if dist[i] > r and any(dist[j] == r - 1 for j in problem.nbr[i]):
                dist[i] = r
    band = (dist >= 1) & (dist <= rings)
    for _ in range(iters):
        new = disp.copy()
        for i in np.nonzero(band)[0]:
            new[:, i] = disp[:, problem.nbr[i]].mean(axis=1)
        disp = new
    return V + disp, snapped
