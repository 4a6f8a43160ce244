"""Per-frame image preprocessing and image sampling (oracle).

* Contour pixels: foreground pixels with a background 4-neighbour (outside
  the image counts as background).
* Distance transform I_DT (Sec. 3.2, Sec. 3.3 Eq. sillhouette): unsigned
  Euclidean distance, in pixels, from each pixel centre to the nearest contour
  pixel centre.  The value is the correctly rounded float32 square root of the
  exact integer squared distance.  A mask with no contour gives I_DT = 0.
* I_Gauss (Sec. 3.4, photometric term): separable Gaussian blur with kernel
  size 3 (the finest of the paper's three pyramid levels), sigma =
  0.3*((k-1)/2 - 1) + 0.8, clamp-to-edge.
* Sampling I(pi(V)): separable cubic convolution (Keys, a = -0.5) on the 4x4
  texel neighbourhood with clamp-to-edge; the image gradient is the exact
  derivative of that interpolant (C1 continuous across cells).
"""
import numpy as np
from scipy import ndimage

F32 = np.float32


def contour(mask):
    m = mask != 0
    pad = np.pad(m, 1, constant_values=False)
    nb_bg = (~pad[:-2, 1:-1]) | (~pad[2:, 1:-1]) | (~pad[1:-1, :-2]) | (~pad[1:-1, 2:])
    return m & nb_bg


def distance_transform(mask):
    """Exact EDT to the contour; returns (dt float32 [H][W], d2 int64 [H][W])."""
    c = contour(mask)
    H, W = c.shape
    if not c.any():
        return np.zeros((H, W), dtype=F32), np.zeros((H, W), dtype=np.int64)
    # library feature transform: index of the nearest contour pixel
    _, ind = ndimage.distance_transform_edt(~c, return_indices=True)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    d2 = (ind[0] - jj).astype(np.int64) ** 2 + (ind[1] - ii).astype(np.int64) ** 2
    return np.sqrt(d2.astype(F32)), d2


def gaussian_weights(k=3):
    sigma = 0.3 * ((k - 1) * 0.5 - 1.0) + 0.8
    r = (k - 1) // 2
    d = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-d * d / (2.0 * sigma * sigma))
    return w / w.sum()


def blur(rgb, k=3):
    """Separable Gaussian blur of a [C][H][W] image (float64 result)."""
    w = gaussian_weights(k)
    r = (k - 1) // 2
    img = rgb.astype(np.float64)
    C, H, W = img.shape
    out = np.zeros_like(img)
    for d in range(-r, r + 1):           # horizontal pass
        xs = np.clip(np.arange(W) + d, 0, W - 1)
        out += w[d + r] * img[:, :, xs]
    img, out = out, np.zeros_like(img)
    for d in range(-r, r + 1):           # vertical pass
        ys = np.clip(np.arange(H) + d, 0, H - 1)
        out += w[d + r] * img[:, ys, :]
    return out


def keys_weights(f):
    """Cubic-convolution weights and their derivatives for offsets -1..2."""
    f2, f3 = f * f, f * f * f
    w = np.stack([(-f3 + 2 * f2 - f) / 2, (3 * f3 - 5 * f2 + 2) / 2,
                  (-3 * f3 + 4 * f2 + f) / 2, (f3 - f2) / 2])
    d = np.stack([(-3 * f2 + 4 * f - 1) / 2, (9 * f2 - 10 * f) / 2,
                  (-9 * f2 + 8 * f + 1) / 2, (3 * f2 - 2 * f) / 2])
    return w, d


def sample(img, u, v):
    """Cubic-convolution sample of img ([H][W] or [C][H][W]) at (u, v) (float64).

    Returns (value, d/du, d/dv), each shaped [C][n] (or [n] for 2-D input).
    """
    squeeze = img.ndim == 2
    im = img[None] if squeeze else img
    im = im.astype(np.float64)
    C, H, W = im.shape
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    ix = np.floor(u).astype(np.int64)
    iy = np.floor(v).astype(np.int64)
    wx, dx = keys_weights(u - ix)
    wy, dy = keys_weights(v - iy)
    val = np.zeros((C, u.size))
    gu = np.zeros((C, u.size))
    gv = np.zeros((C, u.size))
    for m in range(4):
        yy = np.clip(iy + m - 1, 0, H - 1)
        for n in range(4):
            xx = np.clip(ix + n - 1, 0, W - 1)
            t = im[:, yy, xx]
            val += wy[m] * wx[n] * t
            gu += wy[m] * dx[n] * t
            gv += dy[m] * wx[n] * t
    if squeeze:
        return val[0], gu[0], gv[0]
    return val, gu, gv


def keys_gradient_f32(img, u, v):
    """Float32 gradient of the cubic interpolant, fixed operation order.

    Used only for the silhouette direction decision, which must be taken
    identically by every implementation.  Per axis with f the fractional
    part: f2 = f*f, f3 = f2*f, derivative weights
    d0 = ((4f - 3f2) - 1)/2, d1 = (9f2 - 10f)/2, d2 = ((8f - 9f2) + 1)/2,
    d3 = (3f2 - 2f)/2 and value weights w0 = ((2f2 - f3) - f)/2,
    w1 = ((3f3 - 5f2) + 2)/2, w2 = ((4f2 - 3f3) + f)/2, w3 = (f3 - f2)/2
    (each product and sum rounded to float32, halving last).  Rows are
    accumulated n = 0..3 then combined m = 0..3, starting from 0.
    """
    H, W = img.shape
    u = np.asarray(u, dtype=F32)
    v = np.asarray(v, dtype=F32)
    ix = np.floor(u).astype(np.int64)
    iy = np.floor(v).astype(np.int64)
    fx = (u - ix.astype(F32)).astype(F32)
    fy = (v - iy.astype(F32)).astype(F32)

    def wts(f):
        h = F32(0.5)
        f2 = f * f
        f3 = f2 * f
        w = [((F32(2) * f2 - f3) - f) * h, ((F32(3) * f3 - F32(5) * f2) + F32(2)) * h,
             ((F32(4) * f2 - F32(3) * f3) + f) * h, (f3 - f2) * h]
        d = [((F32(4) * f - F32(3) * f2) - F32(1)) * h, (F32(9) * f2 - F32(10) * f) * h,
             ((F32(8) * f - F32(9) * f2) + F32(1)) * h, (F32(3) * f2 - F32(2) * f) * h]
        return w, d

    wx, dx = wts(fx)
    wy, dy = wts(fy)
    gx = np.zeros(u.shape, dtype=F32)
    gy = np.zeros(u.shape, dtype=F32)
    for m in range(4):
        yy = np.clip(iy + m - 1, 0, H - 1)
        rx = np.zeros(u.shape, dtype=F32)
        rv = np.zeros(u.shape, dtype=F32)
        for n in range(4):
            xx = np.clip(ix + n - 1, 0, W - 1)
            t = img[yy, xx].astype(F32)
            rx = rx + dx[n] * t
            rv = rv + wx[n] * t
        gx = gx + wy[m] * rx
        gy = gy + dy[m] * rv
    return gx, gy
