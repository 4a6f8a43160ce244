"""Target images rendered from a ground-truth mesh (input generation only).

A plain float64 z-buffered rasteriser: a pixel ``(i, j)`` (column, row) is
sampled at its centre ``(u, v) = (i, j)``; it is covered when the centre lies
inside (or on the boundary of) a projected triangle; the nearest surface wins;
its colour is the perspective-correct interpolation of the vertex colours.
Uncovered pixels are background: mask 0 and colour 0.

This stands in for the paper's foreground segmentation and colour frames
(Sec. 3.2); it is deliberately written independently of the solvers'
visibility raster, which has its own fixed-point rules.
"""
import numpy as np


def _project(xyz, cam):
    X, Y, Z = (xyz[0].astype(np.float64), xyz[1].astype(np.float64), xyz[2].astype(np.float64))
    u = cam.fx * X / Z + cam.cx
    v = cam.fy * Y / Z + cam.cy
    return u, v, Z


def render_targets(xyz, tri, rgb, cam, chunk=60000, boxes=(4, 8, 16, 32)):
    """Render mask (uint8 [H][W]) and colour (float32 [3][H][W]) images."""
    W, H = cam.width, cam.height
    u, v, Z = _project(xyz, cam)
    t0, t1, t2 = tri[0], tri[1], tri[2]
    ok = (Z[t0] > 0) & (Z[t1] > 0) & (Z[t2] > 0)
    best_iz = np.zeros(H * W)
    best_tri = np.full(H * W, -1, dtype=np.int64)
    best_l = np.zeros((H * W, 3))
    nf = tri.shape[1]
    umin = np.minimum(np.minimum(u[t0], u[t1]), u[t2])
    umax = np.maximum(np.maximum(u[t0], u[t1]), u[t2])
    vmin = np.minimum(np.minimum(v[t0], v[t1]), v[t2])
    vmax = np.maximum(np.maximum(v[t0], v[t1]), v[t2])
    i0 = np.clip(np.ceil(umin), 0, W).astype(np.int64)
    i1 = np.clip(np.floor(umax), -1, W - 1).astype(np.int64)
    j0 = np.clip(np.ceil(vmin), 0, H).astype(np.int64)
    j1 = np.clip(np.floor(vmax), -1, H - 1).astype(np.int64)
    nonempty = ok & (i1 >= i0) & (j1 >= j0)
    bw = i1 - i0 + 1
    bh = j1 - j0 + 1
    ext = np.maximum(bw, bh)
    big = np.nonzero(nonempty & (ext > boxes[-1]))[0]

    def merge(pix, iz, f, lam):
        if pix.size == 0:
            return
        order = np.lexsort((-iz, pix))
        pix, iz, f, lam = pix[order], iz[order], f[order], lam[order]
        first = np.ones(pix.size, dtype=bool)
        first[1:] = pix[1:] != pix[:-1]
        pix, iz, f, lam = pix[first], iz[first], f[first], lam[first]
        better = iz > best_iz[pix]
        pix, iz, f, lam = pix[better], iz[better], f[better], lam[better]
        best_iz[pix] = iz
        best_tri[pix] = f
        best_l[pix] = lam

    def candidates(faces, ii, jj):
        a, b, c = t0[faces], t1[faces], t2[faces]
        ua, va, ub, vb, uc, vc = u[a], v[a], u[b], v[b], u[c], v[c]
        area = (ub - ua) * (vc - va) - (vb - va) * (uc - ua)
        e0 = (uc - ub) * (jj - vb) - (vc - vb) * (ii - ub)
        e1 = (ua - uc) * (jj - vc) - (va - vc) * (ii - uc)
        e2 = (ub - ua) * (jj - va) - (vb - va) * (ii - ua)
        s = np.sign(area)
        inside = (area != 0) & (e0 * s >= 0) & (e1 * s >= 0) & (e2 * s >= 0)
        inside &= (ii >= 0) & (ii < W) & (jj >= 0) & (jj < H)
        area = np.where(area == 0, 1.0, area)
        lam = np.stack([e0 / area, e1 / area, e2 / area], axis=-1)
        iz = lam[..., 0] / Z[a] + lam[..., 1] / Z[b] + lam[..., 2] / Z[c]
        return inside, lam, iz

    lo = 0
    for box in boxes:                       # vectorise triangles by bounding-box size class
        cls = np.nonzero(nonempty & (ext > lo) & (ext <= box))[0]
        lo = box
        oi, oj = np.meshgrid(np.arange(box), np.arange(box), indexing="xy")
        oi, oj = oi.ravel(), oj.ravel()
        step = max(1, chunk * 64 // (box * box))
        for s in range(0, cls.size, step):
            faces = cls[s:s + step][:, None]
            ii = (i0[faces] + oi[None, :]).astype(np.float64)
            jj = (j0[faces] + oj[None, :]).astype(np.float64)
            inside, lam, iz = candidates(faces, ii, jj)
            inside &= (oi[None, :] < bw[faces]) & (oj[None, :] < bh[faces])
            fsel = np.broadcast_to(faces, ii.shape)[inside]
            pix = (jj[inside].astype(np.int64) * W + ii[inside].astype(np.int64))
            merge(pix, iz[inside], fsel, lam[inside])
    for f in big:
        jj, ii = np.meshgrid(np.arange(j0[f], j1[f] + 1, dtype=np.float64),
                             np.arange(i0[f], i1[f] + 1, dtype=np.float64), indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
        faces = np.full(ii.shape, f, dtype=np.int64)
        inside, lam, iz = candidates(faces, ii, jj)
        pix = jj[inside].astype(np.int64) * W + ii[inside].astype(np.int64)
        merge(pix, iz[inside], faces[inside], lam[inside])

    cov = best_tri >= 0
    mask = cov.astype(np.uint8).reshape(H, W)
    colour = np.zeros((3, H * W))
    f = best_tri[cov]
    lam = best_l[cov]
    idx = np.stack([t0[f], t1[f], t2[f]], axis=1)
    wz = lam / Z[idx]
    wz /= wz.sum(axis=1, keepdims=True)
    for c in range(3):
        colour[c, cov] = (wz * rgb[c][idx].astype(np.float64)).sum(axis=1)
    return mask, colour.reshape(3, H, W).astype(np.float32)
