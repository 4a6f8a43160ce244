"""Once-per-frame integer decisions, float32 recipe (oracle).

The paper takes three discrete decisions once per frame from the mesh at the
start of the stage: the visible set by depth buffering (Sec. 3.4,
photometric term), the contour vertex set B (Sec. 3.3 and 3.4, silhouette
terms) and the direction signs b_i (Sec. 3.3, Eq. sillhouette and the two
cases that follow it).  Because they are integers, every implementation must
take them identically; this module states one float32 recipe for them.  Each
arithmetic step below is a single IEEE float32 operation with round-to-
nearest-even, in the order written; no fused multiply-add.

Deformed positions (embedded deformation at the start state)
    for j = 0..3 (binding slot order), with k = bind_idx[j][i], w = bind_w[j][i]:
      d = v_i - g_k;  q_a = (R_a0*d_0 + R_a1*d_1) + R_a2*d_2;  y = (q + g_k) + t_k
      acc = acc + w*y   (acc starts at 0)
Projection (Sec. 3.2, pinhole, world = camera frame)
    u = (fx*X)/Z + cx,  v = (fy*Y)/Z + cy;  pixel (i, j) has its centre at (i, j).
    A vertex is *valid* if Z > 0 and |u|, |v| <= 65536.
Depth buffer
    Valid vertices snap to a 1/256-pixel grid: U = rint(256u), V = rint(256v)
    (int64).  For a triangle with three valid vertices,
    A = (U1-U0)(V2-V0) - (V1-V0)(U2-U0); A == 0 is skipped; A < 0 swaps
    vertices 1 and 2.  Edge e (a->b) in {0: 1->2, 1: 2->0, 2: 0->1} has
    E_e(P) = (Ub-Ua)(Pv-Va) - (Vb-Va)(Pu-Ua) at the pixel centre
    P = (256i, 256j); the pixel is covered iff every E_e > 0, or E_e == 0 on an
    edge that owns its boundary: dV < 0, or dV == 0 and dU > 0 (so a shared
    edge belongs to exactly one of its two triangles).  The inverse depth
    invz = ((E0f*iz0 + E1f*iz1) + E2f*iz2) / Af with iz = 1/Z and E, A converted
    to float32; the buffer keeps the largest invz bit pattern (0 = empty).
Visibility
    valid, (rint u, rint v) inside the image, and either no covered pixel in
    the clipped 3x3 neighbourhood or Z <= 1/invz_min + 0.05 (metres), where
    invz_min is the smallest non-zero buffer entry of that neighbourhood (the
    farthest covered surface: vertices on the silhouette rim sit behind the
    front surface one pixel inwards by up to a few centimetres).
Facing and contour vertices
    c_f = (v1-v0) x (v2-v0) with x = e1y*e2z - e1z*e2y etc.;
    s_f = (v0x*cx + v0y*cy) + v0z*cz; back-facing iff s_f >= 0 (camera at the
    origin).  An edge with two faces is a contour edge iff their facing bits
    differ; an edge with one face iff that face is front-facing.  B = visible
    vertices on a contour edge.
Direction signs b_i (i in B)
    n_i = sum of c_f over incident faces in ascending face order;
    (gx, gy) = float32 cubic-convolution gradient of I_DT at (u, v);
    a = (n_x*Z - n_z*X)*fx,  b = (n_y*Z - n_z*Y)*fy  (the projected normal
    times Z^2 > 0);  s = a*(-gx) + b*(-gy)  (n projected, dotted with z = -grad);
    b_i = -1 iff the vertex lies inside the image silhouette and s < 0, else +1.
    Inside means: the vertex's pixel (rint u, rint v) is foreground in the
    mask and its I_DT value is >= 1.5.  This is the paper's "model points fall
    inside the image silhouette" case; points outside always follow z, and so
    do points in the band within 1.5 px of a contour pixel, where the unsigned
    distance field has a kink and its gradient gives no usable direction.
"""
import numpy as np

from .image import keys_gradient_f32

F32 = np.float32
LIM = F32(65536.0)


def ed_deform_f32(xyz, node_vertex, bind_idx, bind_w, state):
    x = [xyz[a].astype(F32) for a in range(3)]
    g = [x[a][node_vertex] for a in range(3)]
    st = state.astype(F32)
    acc = [np.zeros_like(x[0]) for _ in range(3)]
    for j in range(bind_idx.shape[0]):
        k = bind_idx[j]
        w = bind_w[j].astype(F32)
        d = [x[a] - g[a][k] for a in range(3)]
        for a in range(3):
            q = (st[3 * a + 0][k] * d[0] + st[3 * a + 1][k] * d[1]) + st[3 * a + 2][k] * d[2]
            y = (q + g[a][k]) + st[9 + a][k]
            acc[a] = acc[a] + w * y
    return acc


def project_f32(X, Y, Z, cam):
    fx, fy, cx, cy = (F32(cam.fx), F32(cam.fy), F32(cam.cx), F32(cam.cy))
    with np.errstate(divide="ignore", invalid="ignore"):
        u = (fx * X) / Z + cx
        v = (fy * Y) / Z + cy
    valid = (Z > 0) & (np.abs(u) <= LIM) & (np.abs(v) <= LIM)
    return u, v, valid


def triangle_coverage(u, v, Z, valid, tri, W, H):
    """Yield (face, back_in_screen, pixel indices, invz float32) for every covering triangle."""
    U = np.where(valid, np.rint(u * F32(256)), 0).astype(np.int64)
    V = np.where(valid, np.rint(v * F32(256)), 0).astype(np.int64)
    with np.errstate(divide="ignore"):
        iz = (F32(1.0) / Z).astype(F32)
    for f in range(tri.shape[1]):
        a, b, c = int(tri[0, f]), int(tri[1, f]), int(tri[2, f])
        if not (valid[a] and valid[b] and valid[c]):
            continue
        A = (U[b] - U[a]) * (V[c] - V[a]) - (V[b] - V[a]) * (U[c] - U[a])
        if A == 0:
            continue
        flipped = A < 0
        if flipped:
            b, c = c, b
            A = -A
        pu = [U[a], U[b], U[c]]
        pv = [V[a], V[b], V[c]]
        i0 = max(0, -((-min(pu)) // 256))
        i1 = min(W - 1, max(pu) // 256)
        j0 = max(0, -((-min(pv)) // 256))
        j1 = min(H - 1, max(pv) // 256)
        if i1 < i0 or j1 < j0:
            continue
        jj, ii = np.meshgrid(np.arange(j0, j1 + 1, dtype=np.int64),
                             np.arange(i0, i1 + 1, dtype=np.int64), indexing="ij")
        Pu, Pv = ii * 256, jj * 256
        cover = np.ones(Pu.shape, dtype=bool)
        E = []
        for (sa, sb) in ((1, 2), (2, 0), (0, 1)):
            dU = pu[sb] - pu[sa]
            dV = pv[sb] - pv[sa]
            e = dU * (Pv - pv[sa]) - dV * (Pu - pu[sa])
            owns = (dV < 0) or (dV == 0 and dU > 0)
            cover &= (e > 0) | ((e == 0) & owns)
            E.append(e)
        if not cover.any():
            continue
        e0 = E[0][cover].astype(F32)
        e1 = E[1][cover].astype(F32)
        e2 = E[2][cover].astype(F32)
        inv = ((e0 * iz[a] + e1 * iz[b]) + e2 * iz[c]) / F32(A)
        yield f, flipped, jj[cover] * W + ii[cover], inv.astype(F32)


def raster_zbuffer(u, v, Z, valid, tri, W, H):
    """Inverse-depth buffer (uint32 bit patterns, [H][W]) by the fixed-point recipe."""
    zb = np.zeros(H * W, dtype=np.uint32)
    for _, _, pix, inv in triangle_coverage(u, v, Z, valid, tri, W, H):
        np.maximum.at(zb, pix, inv.view(np.uint32))
    return zb.reshape(H, W)


def mesh_edges(tri):
    """Edge list (a < b) with adjacent faces f0 < f1 (f1 = -1 on a border)."""
    nf = tri.shape[1]
    ea = np.concatenate([tri[0], tri[1], tri[2]]).astype(np.int64)
    eb = np.concatenate([tri[1], tri[2], tri[0]]).astype(np.int64)
    f = np.concatenate([np.arange(nf)] * 3)
    lo, hi = np.minimum(ea, eb), np.maximum(ea, eb)
    order = np.lexsort((f, hi, lo))
    lo, hi, f = lo[order], hi[order], f[order]
    edges = {}
    for a, b, ff in zip(lo.tolist(), hi.tolist(), f.tolist()):
        edges.setdefault((a, b), []).append(ff)
    out = []
    for (a, b), fs in edges.items():
        if len(fs) > 2:
            raise ValueError("mesh is not edge-manifold")
        out.append((a, b, fs[0], fs[1] if len(fs) == 2 else -1))
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def frame_decisions(xyz, tri, graph, state, cam, mask, dt, outline=False):
    """All per-frame decisions of the non-rigid stage (start positions by the ED recipe)."""
    X, Y, Z = ed_deform_f32(xyz, graph["node_vertex"], graph["bind_idx"], graph["bind_w"], state)
    return frame_decisions_from_positions(X, Y, Z, tri, cam, mask, dt, outline=outline)


def frame_decisions_from_positions(X, Y, Z, tri, cam, mask, dt, outline=False):
    """Decisions from float32 start positions: u, v, Z, zbuf, visible, boundary, bsign.

    outline: keep in B only contour vertices on the outline of the rendered
    model, i.e. with an uncovered pixel (zbuf 0) in the 3x3 window around the
    vertex pixel (window clipped to the image).  A mesh made of overlapping
    closed parts has contour edges inside its own silhouette; they have no
    counterpart in the image silhouette's distance transform."""
    W, H = cam.width, cam.height
    u, v, valid = project_f32(X, Y, Z, cam)
    zb = raster_zbuffer(u, v, Z, valid, tri, W, H)

    nv = X.size
    with np.errstate(invalid="ignore"):
        px = np.where(valid, np.rint(u), -1).astype(np.int64)
        py = np.where(valid, np.rint(v), -1).astype(np.int64)
    inside = valid & (px >= 0) & (px < W) & (py >= 0) & (py < H)
    vis = np.zeros(nv, dtype=bool)
    open_ = np.zeros(nv, dtype=bool)
    for i in np.nonzero(inside)[0]:
        y0, y1 = max(0, py[i] - 1), min(H - 1, py[i] + 1)
        x0, x1 = max(0, px[i] - 1), min(W - 1, px[i] + 1)
        blk = zb[y0:y1 + 1, x0:x1 + 1]
        cov = blk[blk > 0]
        open_[i] = cov.size < blk.size
        if cov.size == 0:
            vis[i] = True
        else:
            zfar = F32(1.0) / cov.min().view(np.float32)
            vis[i] = Z[i] <= (zfar + F32(0.05))

    # facing per face
    p = [X, Y, Z]
    t0, t1, t2 = tri[0], tri[1], tri[2]
    e1 = [p[a][t1] - p[a][t0] for a in range(3)]
    e2 = [p[a][t2] - p[a][t0] for a in range(3)]
    c = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    s = (p[0][t0] * c[0] + p[1][t0] * c[1]) + p[2][t0] * c[2]
    back = s >= 0
    edges = mesh_edges(tri)
    cont = np.zeros(nv, dtype=bool)
    for a, b, f0, f1 in edges:
        is_c = (back[f0] != back[f1]) if f1 >= 0 else (not back[f0])
        if is_c:
            cont[a] = True
            cont[b] = True
    bnd = vis & cont
    if outline:
        bnd &= open_

    # vertex normals: incident faces in ascending order
    n = [np.zeros(nv, dtype=F32) for _ in range(3)]
    vid = tri.T.ravel()                      # face-major: every face's corners in turn
    for a in range(3):
        np.add.at(n[a], vid, np.repeat(c[a], 3))   # sequential, list order
    gx, gy = keys_gradient_f32(dt, u[bnd], v[bnd])
    fx, fy = F32(cam.fx), F32(cam.fy)
    aa = (n[0][bnd] * Z[bnd] - n[2][bnd] * X[bnd]) * fx
    bb = (n[1][bnd] * Z[bnd] - n[2][bnd] * Y[bnd]) * fy
    ss = aa * (-gx) + bb * (-gy)
    fg = (mask[py[bnd], px[bnd]] != 0) & (dt[py[bnd], px[bnd]] >= F32(1.5))
    bsign = np.zeros(nv, dtype=np.int8)
    bsign[bnd] = np.where(fg & (ss < 0), -1, 1).astype(np.int8)
    return dict(X=X, Y=Y, Z=Z, u=u, v=v, valid=valid, zbuf=zb, visible=vis,
                contour=cont, boundary=bnd, bsign=bsign, back=back, normal=n)
