// Once-per-frame kernels: blurred image, distance transform, depth buffer,
// visibility, contour vertices and direction signs (Sec. 3.2-3.4).  Every
// launch covers a whole batch: blockIdx.y selects the problem, blocks beyond
// the problem's own extent return at once.
#include "device.hpp"

namespace cap {

// ---------------------------------------------------------------- fills
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------- blur
// Separable Gaussian (kernel 3), clamp-to-edge, in one pass: each pixel forms
// the horizontal sums of its three rows (rounded as a horizontal pass would
// store them) and then the vertical sum.
__device__ inline void blur_body(const ProbDev &pr, int bx, float w0, float w1) {
    const int W = pr.W, H = pr.H;
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    int y = i / W, x = i - y * W;
    const size_t plane = size_t(W) * H;
    const int xl = max(x - 1, 0), xr = min(x + 1, W - 1);
    const int rows[3] = {max(y - 1, 0), y, min(y + 1, H - 1)};
    // all 27 taps loaded before any store (the output could alias the input
    // as far as the compiler knows, which would order each channel's loads
    // behind the previous channel's store)
    float v[3][3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const CAP_GLOBAL float *row = pr.image.g() + c * plane + size_t(rows[r]) * W;
            v[c][r][0] = row[xl];
            v[c][r][1] = row[x];
            v[c][r][2] = row[xr];
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float h[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)      // horizontal pass of rows y-1, y, y+1 (clamped)
            h[r] = (w0 * v[c][r][0] + w1 * v[c][r][1]) + w0 * v[c][r][2];
        pr.blurred[c * plane + i] = (w0 * h[0] + w1 * h[1]) + w0 * h[2];
    }
}

// ---------------------------------------------------------------- distance transform
// Contour pixels: foreground with a background 4-neighbour (outside = background).
__device__ inline void contour_body(const ProbDev &pr, int bx) {
    const int W = pr.W, H = pr.H;
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= W * H) return;
    int y = i / W, x = i - y * W;
    const CAP_GLOBAL uint8_t *m = pr.mask.g();
    // the pixel and its four neighbours loaded together (clamped at the border,
    // where the pixel counts as contour anyway), then tested
    const uint8_t mc = m[i], ml = m[x > 0 ? i - 1 : i], mr = m[x < W - 1 ? i + 1 : i];
    const uint8_t mu = m[y > 0 ? i - W : i], md = m[y < H - 1 ? i + W : i];
    const bool border = x == 0 || y == 0 || x == W - 1 || y == H - 1;
    const bool bg = border | (ml == 0) | (mr == 0) | (mu == 0) | (md == 0);
    pr.contour[i] = (mc != 0 && bg) ? 1 : 0;
}

__global__ void k_contour(const ProbDev *__restrict__ P) { contour_body(P[blockIdx.y], blockIdx.x); }

constexpr int kFar = 1 << 20;
constexpr int kSeg = 16;   // rows per column segment

// Phase 1a: per (column, 16-row segment), the first and last contour row.
__device__ inline void dt_seg_body(const ProbDev &pr, int bx) {
    const int W = pr.W, H = pr.H, nseg = (H + kSeg - 1) / kSeg;
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= W * nseg) return;
    const int s = i / W, x = i - s * W;
    int first = kFar, last = -kFar;
    const int y0 = s * kSeg, y1 = min(H, y0 + kSeg);
    // the segment's kSeg rows loaded together (rows past the image re-read
    // its last row and are not counted), then scanned in order
    uint8_t c[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) c[k] = pr.contour[size_t(min(y0 + k, H - 1)) * W + x];
#pragma unroll
    for (int k = 0; k < kSeg; ++k)
        if (y0 + k < y1 && c[k]) { first = min(first, y0 + k); last = y0 + k; }
    pr.seg_first[i] = first;
    pr.seg_last[i] = last;
}

__global__ void k_dt_seg(const ProbDev *__restrict__ P) { dt_seg_body(P[blockIdx.y], blockIdx.x); }

// Phase 1b: per column, the nearest contour row above and below each segment,
// written over seg_last (above) and seg_first (below).  One wave per column,
// a lane per segment (kScanChunks chunks of 64 segments): the rows above are
// an exclusive prefix maximum of the segments' last contour rows (rows grow
// with the segment), the rows below an exclusive suffix minimum of their
// first ones, both formed with lane shuffles.
constexpr int kScanChunks = (kMaxImageSide / kSeg + 63) / 64;

__device__ inline void dt_scan_body(const ProbDev &pr, int bx) {
    const int W = pr.W, H = pr.H, nseg = (H + kSeg - 1) / kSeg;
    const int x = bx * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (x >= W) return;
    int last[kScanChunks], first[kScanChunks];
#pragma unroll
    for (int q = 0; q < kScanChunks; ++q) {
        const int t = q * 64 + lane;
        last[q] = t < nseg ? pr.seg_last[t * W + x] : -kFar;
        first[q] = t < nseg ? pr.seg_first[t * W + x] : kFar;
    }
    int up = -kFar;        // rows above: carried forward over the chunks
#pragma unroll
    for (int q = 0; q < kScanChunks; ++q) {
        int v = last[q];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o);
            if (lane >= o) v = max(v, u);
        }
        const int before = __shfl_up(v, 1);
        const int excl = lane == 0 ? up : max(up, before);
        up = max(up, __shfl(v, 63));
        last[q] = excl;
    }
    int down = kFar;       // rows below: carried backward over the chunks
#pragma unroll
    for (int q = kScanChunks - 1; q >= 0; --q) {
        int v = first[q];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_down(v, o);
            if (lane + o < 64) v = min(v, u);
        }
        const int after = __shfl_down(v, 1);
        const int excl = lane == 63 ? down : min(down, after);
        down = min(down, __shfl(v, 0));
        first[q] = excl;
    }
#pragma unroll
    for (int q = 0; q < kScanChunks; ++q) {
        const int t = q * 64 + lane;
        if (t < nseg) {
            pr.seg_last[t * W + x] = last[q] < 0 ? -kFar : last[q];
            pr.seg_first[t * W + x] = first[q] >= kFar ? 2 * kFar : first[q];
        }
    }
}

// The same with one thread per column (coalesced across columns), in one pass
// down and one up; segments are read kScanBatch at a time into registers, so
// the loads of a batch are in flight together.  Used when the frames have
// enough columns in total to fill the chip.
constexpr int kScanBatch = 16;

__global__ void k_dt_scan_cols(const ProbDev *__restrict__ P) {
    const ProbDev &pr = P[blockIdx.y];
    const int W = pr.W, H = pr.H, nseg = (H + kSeg - 1) / kSeg;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    int carry = -kFar;
    for (int t0 = 0; t0 < nseg; t0 += kScanBatch) {
        int v[kScanBatch];
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) v[u] = t0 + u < nseg ? pr.seg_last[(t0 + u) * W + x] : -kFar;
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            if (t0 + u < nseg) pr.seg_last[(t0 + u) * W + x] = carry;
            if (v[u] >= 0) carry = v[u];
        }
    }
    carry = 2 * kFar;
    for (int t1 = nseg; t1 > 0; t1 -= kScanBatch) {
        int v[kScanBatch];
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) v[u] = t1 - 1 - u >= 0 ? pr.seg_first[(t1 - 1 - u) * W + x] : kFar;
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            if (t1 - 1 - u >= 0) pr.seg_first[(t1 - 1 - u) * W + x] = carry;
            if (v[u] < kFar) carry = v[u];
        }
    }
}

// Phase 1c: per (column, segment), distance in rows to the nearest contour
// pixel of the column (carry from the other segments, then the segment's rows).
__device__ inline void dt_cols_body(const ProbDev &pr, int bx) {
    const int W = pr.W, H = pr.H, nseg = (H + kSeg - 1) / kSeg;
    const int i = bx * blockDim.x + threadIdx.x;
    if (i >= W * nseg) return;
    const int s = i / W, x = i - s * W;
    const int above = pr.seg_last[i], below = pr.seg_first[i];
    const int y0 = s * kSeg, y1 = min(H, y0 + kSeg);
    int d[kSeg];
    uint8_t c[kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {      // loaded together: rows past the image re-read its last row
        c[k] = pr.contour[size_t(min(y0 + k, H - 1)) * W + x];
        if (y0 + k >= y1) c[k] = 0;
    }
    int last = above;
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
        if (c[k]) last = y0 + k;
        d[k] = y0 + k - last;
    }
    int next = below;
#pragma unroll
    for (int k = kSeg - 1; k >= 0; --k) {
        if (c[k]) next = y0 + k;
        const int dd = next - (y0 + k);
        if (y0 + k < y1) pr.colg[size_t(y0 + k) * W + x] = dd < d[k] ? dd : d[k];
    }
}

// Phase 2: per row, D(x) = min over x' of (x - x')^2 + G(x'), G = g^2, exact.
// With H(x') = G(x') + x'^2 the value is x^2 + H(x') - 2 x x'.  The matrix of
// H(x') - 2 x x' over (x, x') is Monge (its cross term is), so the smallest
// minimising column of a pixel never decreases along the row.  kDtAnchors
// anchor pixels (every s-th one and the last) take the minimum over the whole
// row, eight lanes each, and keep their smallest minimising column; every
// other pixel scans only the columns between the minimising columns of the
// anchors on either side of it.  That is at most kDtAnchors W + s (W + kDtAnchors)
// candidates per row, whatever the sites, and each costs a three-operand add
// and a share of a three-operand min (the -2 x x' term steps by -2x along the
// columns).  Integer arithmetic throughout (no term leaves 32 bits for rows up
// to 4096 pixels), so the result is exact.  One 256-thread workgroup per row.
constexpr int kDtAnchors = 32;
constexpr int kDtLanes = 8;                  // lanes per anchor: kDtAnchors x kDtLanes = 256
constexpr int kDtUnroll = 8;

__device__ inline void dt_rows_body(const ProbDev &pr, int y) {
    extern __shared__ int Hs[];
    __shared__ int aq[kDtAnchors];
    const int W = pr.W, H = pr.H;
    if (y >= H) return;
    const int far2 = 1 << 30;
    // the row's column distances staged four per thread per round (loads at
    // clamped columns in flight together, then the LDS stores)
    for (int x0 = threadIdx.x; x0 < W; x0 += 4 * blockDim.x) {
        int g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) g[u] = pr.colg[size_t(y) * W + min(x0 + u * int(blockDim.x), W - 1)];
        __asm__ volatile("" ::"v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]));     // (none moved behind a store)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int x = x0 + u * int(blockDim.x);
            if (x < W) Hs[x] = (g[u] >= kFar ? far2 : g[u] * g[u]) + x * x;
        }
    }
    __syncthreads();
    float *out = pr.dt + size_t(y) * W;
    const int s = max(1, (W - 1 + kDtAnchors - 2) / (kDtAnchors - 1));     // anchor k at min(k s, W - 1)
    {
        const int k = threadIdx.x / kDtLanes, part = threadIdx.x % kDtLanes;
        const int x = min(k * s, W - 1);
        const int m2x = -2 * x;
        int bv = INT_MAX, bq = INT_MAX;      // smallest value, then smallest column, of this lane's columns
        int base = m2x * part;
#pragma unroll 4
        for (int q = part; q < W; q += kDtLanes, base += m2x * kDtLanes) {
            const int v = Hs[q] + base;
            if (v < bv) { bv = v; bq = q; }
        }
#pragma unroll
        for (int o = 1; o < kDtLanes; o <<= 1) {
            const int ov = __shfl_xor(bv, o, kDtLanes), oq = __shfl_xor(bq, o, kDtLanes);
            if (ov < bv || (ov == bv && oq < bq)) { bv = ov; bq = oq; }
        }
        if (part == 0) {
            aq[k] = bq;
            if (k == 0 || x != min((k - 1) * s, W - 1)) {       // once per distinct anchor pixel
                const int best = bv + x * x;
                out[x] = best >= far2 ? 0.0f : sqrtf(float(best));
            }
        }
    }
    __syncthreads();
    // every other pixel: its interval's column range, kDtUnroll reads in flight
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        const int k = x / s;
        if ((x % s == 0 && k < kDtAnchors) || x == W - 1) continue;
        const int a = aq[k], b = aq[k + 1] + 1;
        const int m2x = -2 * x;
        int step[kDtUnroll];                 // -2 x u
#pragma unroll
        for (int u = 0; u < kDtUnroll; ++u) step[u] = m2x * u;
        int base = m2x * a;                  // -2 x q at the block's first column
        int m = far2;                        // m + x^2 >= 2^30: no site in the range
        int q = a;
        for (; q + kDtUnroll <= b; q += kDtUnroll) {
            int v[kDtUnroll];
#pragma unroll
            for (int u = 0; u < kDtUnroll; ++u) v[u] = Hs[q + u] + base + step[u];
#pragma unroll
            for (int u = 0; u < kDtUnroll; u += 2) m = min(m, min(v[u], v[u + 1]));
            base += m2x * kDtUnroll;
        }
        for (; q < b; ++q, base += m2x) m = min(m, Hs[q] + base);
        const int best = m + x * x;
        out[x] = best >= far2 ? 0.0f : sqrtf(float(best));
    }
}

// ---------------------------------------------------------------- start-state geometry
// Embedded deformation at the start state, float32 recipe, then projection
// and 1/256-pixel snapping.  Vertex order.
__device__ inline void deform_start_body(const ProbDev &pr, int bx) {
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nn = T.nn;
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    float v[3] = {pr.xyz[i], pr.xyz[nv + i], pr.xyz[2 * nv + i]};
    // the four bindings and then all of their nodes' data (position: the
    // frame's mesh at the node vertex, set up per frame; R and t) in two
    // rounds of loads, before the arithmetic
    int k[4];
    float w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        k[j] = T.bind_idx[size_t(j) * nv + i];
        w[j] = T.bind_w[size_t(j) * nv + i];
    }
    float g[4][3], S[4][12];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) g[j][a] = pr.gpos[size_t(a) * nn + k[j]];
#pragma unroll
        for (int q = 0; q < 12; ++q) S[j][q] = pr.state[size_t(q) * nn + k[j]];
    }
    float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float d[3] = {v[0] - g[j][0], v[1] - g[j][1], v[2] - g[j][2]};
        for (int a = 0; a < 3; ++a) {
            const float *R = S[j] + 3 * a;
            float q = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
            float yv = (q + g[j][a]) + S[j][9 + a];
            acc[a] = acc[a] + w[j] * yv;
        }
    }
    store_start_vertex(pr, i, acc[0], acc[1], acc[2]);
}

// Fixed-point triangle set-up of the coverage rule: 1/256-pixel vertices,
// counter-clockwise order, pixel box clipped to the image, edge ownership.
struct TriRaster {
    long long U0, V0, U1, V1, U2, V2, dU0, dV0, dU1, dV1, dU2, dV2;
    long long i0, i1, j0, j1;
    bool o0, o1, o2;
    float iz0, iz1, iz2, Af;
};

// The face's vertex data (fixed-point coordinates, depths, validity) held in
// registers, loaded in one round.
struct TriVerts {
    int u[3], v[3];
    float z[3];
    bool valid;
};

__device__ inline TriVerts tri_verts(const ProbDev &pr, int a, int b, int c) {
    const int nv = pr.T.nv;
    const int id[3] = {a, b, c};
    TriVerts t;
    uint8_t ok[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        ok[q] = pr.dvalid[id[q]];
        t.u[q] = pr.dfix[id[q]];
        t.v[q] = pr.dfix[nv + id[q]];
        t.z[q] = pr.dx[2 * nv + id[q]];
    }
    t.valid = (ok[0] != 0) & (ok[1] != 0) & (ok[2] != 0);     // no short circuit: the loads go together
    return t;
}

__device__ inline bool tri_setup_from(const ProbDev &pr, const TriVerts &t, TriRaster &s) {
    if (!t.valid) return false;
    s.U0 = t.u[0]; s.V0 = t.v[0];
    s.U1 = t.u[1]; s.V1 = t.v[1];
    s.U2 = t.u[2]; s.V2 = t.v[2];
    long long A = (s.U1 - s.U0) * (s.V2 - s.V0) - (s.V1 - s.V0) * (s.U2 - s.U0);
    if (A == 0) return false;
    int ib = 1, ic = 2;
    if (A < 0) {
        long long tt;
        tt = s.U1; s.U1 = s.U2; s.U2 = tt;
        tt = s.V1; s.V1 = s.V2; s.V2 = tt;
        ib = 2; ic = 1;
        A = -A;
    }
    s.iz0 = 1.0f / t.z[0];
    s.iz1 = 1.0f / (ib == 1 ? t.z[1] : t.z[2]);
    s.iz2 = 1.0f / (ic == 1 ? t.z[1] : t.z[2]);
    const long long umin = min(s.U0, min(s.U1, s.U2)), umax = max(s.U0, max(s.U1, s.U2));
    const long long vmin = min(s.V0, min(s.V1, s.V2)), vmax = max(s.V0, max(s.V1, s.V2));
    s.i0 = max(0LL, -((-umin) >> 8));
    s.i1 = min((long long)pr.W - 1, umax >> 8);
    s.j0 = max(0LL, -((-vmin) >> 8));
    s.j1 = min((long long)pr.H - 1, vmax >> 8);
    // edges 0: 1->2, 1: 2->0, 2: 0->1 and their boundary ownership
    s.dU0 = s.U2 - s.U1; s.dV0 = s.V2 - s.V1;
    s.dU1 = s.U0 - s.U2; s.dV1 = s.V0 - s.V2;
    s.dU2 = s.U1 - s.U0; s.dV2 = s.V1 - s.V0;
    s.o0 = s.dV0 < 0 || (s.dV0 == 0 && s.dU0 > 0);
    s.o1 = s.dV1 < 0 || (s.dV1 == 0 && s.dU1 > 0);
    s.o2 = s.dV2 < 0 || (s.dV2 == 0 && s.dU2 > 0);
    s.Af = float(A);
    return s.i0 <= s.i1 && s.j0 <= s.j1;
}

__device__ inline bool tri_setup(const ProbDev &pr, int f, TriRaster &s) {
    const TemplateDev &T = pr.T;
    const int nf = T.nf;
    return tri_setup_from(pr, tri_verts(pr, T.tri[f], T.tri[nf + f], T.tri[2 * size_t(nf) + f]), s);
}

// Coverage and inverse depth of pixel (i, j); the buffer keeps the largest bits.
__device__ inline void tri_pixel(const ProbDev &pr, const TriRaster &s, long long i, long long j) {
    const long long Pu = i * 256, Pv = j * 256;
    const long long E0 = s.dU0 * (Pv - s.V1) - s.dV0 * (Pu - s.U1);
    const long long E1 = s.dU1 * (Pv - s.V2) - s.dV1 * (Pu - s.U2);
    const long long E2 = s.dU2 * (Pv - s.V0) - s.dV2 * (Pu - s.U0);
    const bool in = (E0 > 0 || (E0 == 0 && s.o0)) && (E1 > 0 || (E1 == 0 && s.o1)) && (E2 > 0 || (E2 == 0 && s.o2));
    if (!in) return;
    const float inv = ((float(E0) * s.iz0 + float(E1) * s.iz1) + float(E2) * s.iz2) / s.Af;
    __hip_atomic_fetch_max(pr.zbuf.g() + size_t(j) * pr.W + i, __float_as_uint(inv), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Per face: cross product (for normals), then rasterise the inverse depth.
// A face whose pixel box holds more than kRasterSmall pixels is queued for
// the large-face pass instead, so one thread never walks a large box.
__device__ inline void raster_body(const ProbDev &pr, int bx) {
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nf = T.nf;
    int f = bx * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int a = T.tri[f], b = T.tri[nf + f], c = T.tri[2 * size_t(nf) + f];
    // every vertex datum of the face in one round (positions, then the
    // rasterisation data), before the normal is stored
    float p0[3] = {pr.dx[a], pr.dx[nv + a], pr.dx[2 * nv + a]};
    float p1[3] = {pr.dx[b], pr.dx[nv + b], pr.dx[2 * nv + b]};
    float p2[3] = {pr.dx[c], pr.dx[nv + c], pr.dx[2 * nv + c]};
    const TriVerts tv = tri_verts(pr, a, b, c);
    // consumed here so that the coordinate loads are not moved behind the
    // validity test (a round of their own)
    __asm__ volatile("" ::"v"(tv.u[0]), "v"(tv.u[1]), "v"(tv.u[2]), "v"(tv.v[0]), "v"(tv.v[1]), "v"(tv.v[2]));
    float e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    float e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    float cr[3];
    cross3(e1, e2, cr);
    pr.fcross[f] = cr[0];
    pr.fcross[nf + f] = cr[1];
    pr.fcross[2 * size_t(nf) + f] = cr[2];
    TriRaster s;
    if (!tri_setup_from(pr, tv, s)) return;
    if ((s.i1 - s.i0 + 1) * (s.j1 - s.j0 + 1) > kRasterSmall) {
        pr.bigq[__hip_atomic_fetch_add(pr.counts.g() + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)] = f;
        return;
    }
    for (long long j = s.j0; j <= s.j1; ++j)
        for (long long i = s.i0; i <= s.i1; ++i) tri_pixel(pr, s, i, j);
}

// Queued large faces: one workgroup per face at a time, threads over its pixel box.
__device__ inline void raster_big_body(const ProbDev &pr, int bx, int nbx) {
    const int nq = pr.counts[2];
    for (int q = bx; q < nq; q += nbx) {
        TriRaster s;
        if (!tri_setup(pr, pr.bigq[q], s)) continue;
        const long long w = s.i1 - s.i0 + 1, area = w * (s.j1 - s.j0 + 1);
        for (long long k = threadIdx.x; k < area; k += blockDim.x) tri_pixel(pr, s, s.i0 + k % w, s.j0 + k / w);
    }
}

// Body-part labels of the rendered model: the pixels where a face sets the
// depth-buffer value take the smaller of their label and the face's (its
// first vertex's part).  Small faces one per thread; the queued large faces
// (from the depth pass) one workgroup each.
__device__ inline void label_pixel(const ProbDev &pr, const TriRaster &s, long long i, long long j, int lab,
                                   int *__restrict__ img) {
    const long long Pu = i * 256, Pv = j * 256;
    const long long E0 = s.dU0 * (Pv - s.V1) - s.dV0 * (Pu - s.U1);
    const long long E1 = s.dU1 * (Pv - s.V2) - s.dV1 * (Pu - s.U2);
    const long long E2 = s.dU2 * (Pv - s.V0) - s.dV2 * (Pu - s.U0);
    const bool in = (E0 > 0 || (E0 == 0 && s.o0)) && (E1 > 0 || (E1 == 0 && s.o1)) && (E2 > 0 || (E2 == 0 && s.o2));
    if (!in) return;
    const float inv = ((float(E0) * s.iz0 + float(E1) * s.iz1) + float(E2) * s.iz2) / s.Af;
    const size_t q = size_t(j) * pr.W + i;
    if (__float_as_uint(inv) == pr.zbuf[q]) atomicMin(img + q, lab);
}

__global__ void k_part_labels(const ProbDev *__restrict__ P, const int *__restrict__ parts, int *__restrict__ img) {
    const ProbDev &pr = *P;
    const TemplateDev &T = pr.T;
    const int nf = T.nf, f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    TriRaster s;
    if (!tri_setup(pr, f, s)) return;
    if ((s.i1 - s.i0 + 1) * (s.j1 - s.j0 + 1) > kRasterSmall) return;      // queued by the depth pass
    const int lab = parts[T.tri[f]];
    for (long long j = s.j0; j <= s.j1; ++j)
        for (long long i = s.i0; i <= s.i1; ++i) label_pixel(pr, s, i, j, lab, img);
}

__global__ __launch_bounds__(256) void k_part_labels_big(const ProbDev *__restrict__ P, const int *__restrict__ parts,
                                                         int *__restrict__ img) {
    const ProbDev &pr = *P;
    const int nq = pr.counts[2];
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int f = pr.bigq[q];
        TriRaster s;
        if (!tri_setup(pr, f, s)) continue;
        const int lab = parts[pr.T.tri[f]];
        const long long w = s.i1 - s.i0 + 1, area = w * (s.j1 - s.j0 + 1);
        for (long long k = threadIdx.x; k < area; k += blockDim.x) label_pixel(pr, s, s.i0 + k % w, s.j0 + k / w, lab, img);
    }
}

// Per mesh edge: contour edge when its faces' facing differs (a border edge
// when its one face is front-facing); marks both endpoints.
__device__ inline void contour_edges_body(const ProbDev &pr, int bx) {
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nf = T.nf, ne = T.nmedges;
    int e = bx * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int a = T.medge[e], b = T.medge[ne + e], f0 = T.medge[2 * ne + e], f1 = T.medge[3 * ne + e];
    auto back = [&](int f) {
        int v0 = T.tri[f];
        float s = (pr.dx[v0] * pr.fcross[f] + pr.dx[nv + v0] * pr.fcross[nf + f]) +
                  pr.dx[2 * nv + v0] * pr.fcross[2 * size_t(nf) + f];
        return s >= 0.0f;
    };
    // both faces evaluated (a border edge's missing face as face f0 again), so
    // that their loads go together
    __asm__ volatile("" ::"v"(a), "v"(b));     // the endpoints' loads stay with the faces' (not behind the test)
    const bool b0 = back(f0), b1 = back(f1 >= 0 ? f1 : f0);
    bool c = f1 >= 0 ? (b0 != b1) : !b0;
    if (c) {
        pr.vcont[a] = 1;
        pr.vcont[b] = 1;
    }
}

// ---------------------------------------------------------------- per-frame set-up
// Scalars and counters (block 0), the start-state copy and the node positions
// (the frame's mesh at the node vertices, node-major, read by the tile
// kernels), and an empty depth buffer (4 pixels per thread), over nbx blocks.
__device__ inline void frame_init_body(const ProbDev &pr, int bx, int nbx, int gn_iters) {
    const TemplateDev &T = pr.T;
    const int nn = T.nn, tid = bx * blockDim.x + threadIdx.x, nt = nbx * blockDim.x;
    if (bx == 0) {
        for (int i = threadIdx.x; i < kScalars; i += blockDim.x) pr.scal[i] = i == 3 ? double(gn_iters) : 0.0;
        if (threadIdx.x < 3) pr.counts[threadIdx.x] = 0;
    }
    for (int i = tid; i < 12 * nn; i += nt) pr.state0[i] = pr.state[i];
    for (int i = tid; i < 3 * nn; i += nt) {
        const int a = i / nn, k = i - a * nn;
        pr.gpos[i] = pr.xyz[size_t(a) * T.nv + T.node_vertex[k]];
    }
    const size_t hw = size_t(pr.W) * pr.H;
    const size_t i = size_t(tid) * 4;
    for (int q = 0; q < 4; ++q)
        if (i + q < hw) pr.zbuf[i + q] = 0u;
}

// ---------------------------------------------------------------- combined launches
// A frame's preprocessing is two independent chains, the image one (blur;
// contour pixels, column segments, segment scan, column distances, row pass)
// and the geometric one (deformed start, rasterisation, large faces, contour
// edges), joined by the per-vertex decisions.  Steps of the two chains that
// have the same predecessors share a launch: consecutive block ranges of one
// grid run different steps (256 threads each; blockIdx.y = problem), which
// takes a frame from eleven launches to six.  The contour edges run last in
// the row pass's launch, so the vertex and face data they read is fresh in
// cache for the decisions that follow.

// Set-up (nb_init blocks), blur (nb_px), contour pixels (nb_px).
__global__ __launch_bounds__(256) void k_prep_image(const ProbDev *__restrict__ P, int nb_init, int nb_px, int gn_iters,
                                                    float w0, float w1) {
    const ProbDev &pr = P[blockIdx.y];
    const int bx = blockIdx.x;
    if (bx < nb_init)
        frame_init_body(pr, bx, nb_init, gn_iters);
    else if (bx < nb_init + nb_px)
        blur_body(pr, bx - nb_init, w0, w1);
    else
        contour_body(pr, bx - nb_init - nb_px);
}

// Deformed start (nb_v blocks), then the column segments' contour rows.
__global__ __launch_bounds__(256) void k_prep_geom(const ProbDev *__restrict__ P, int nb_v) {
    const ProbDev &pr = P[blockIdx.y];
    const int bx = blockIdx.x;
    if (bx < nb_v)
        deform_start_body(pr, bx);
    else
        dt_seg_body(pr, bx - nb_v);
}

// Rasterisation (nb_f blocks), then (when `scan`) the segment scan, a wave
// per column.
__global__ __launch_bounds__(256) void k_prep_raster(const ProbDev *__restrict__ P, int nb_f, int scan) {
    const ProbDev &pr = P[blockIdx.y];
    const int bx = blockIdx.x;
    if (bx < nb_f)
        raster_body(pr, bx);
    else if (scan)
        dt_scan_body(pr, bx - nb_f);
}

// Large faces (kRasterBigBlocks blocks), then the column distances.
__global__ __launch_bounds__(256) void k_prep_cols(const ProbDev *__restrict__ P) {
    const ProbDev &pr = P[blockIdx.y];
    const int bx = blockIdx.x;
    if (bx < kRasterBigBlocks)
        raster_big_body(pr, bx, kRasterBigBlocks);
    else
        dt_cols_body(pr, bx - kRasterBigBlocks);
}

// Row pass (one block per row of the largest image, nb_rows; dynamic LDS
// dt_rows_lds(largest width)), then the contour edges.
__global__ __launch_bounds__(256) void k_prep_rows(const ProbDev *__restrict__ P, int nb_rows) {
    const ProbDev &pr = P[blockIdx.y];
    const int bx = blockIdx.x;
    if (bx < nb_rows)
        dt_rows_body(pr, bx);
    else
        contour_edges_body(pr, bx - nb_rows);
}

// Per vertex: visibility, contour set and direction sign; writes the flags in
// vertex order and the solver's code byte in plan order.
__global__ void k_decide(const ProbDev *__restrict__ P) {
    __shared__ int cnt[2];
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nf = T.nf, W = pr.W, H = pr.H;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x * blockDim.x >= unsigned(nv)) return;
    uint8_t code = 0;
    if (i < nv) {
    // the vertex's own data, all at once; then its 3x3 depth window (clamped
    // into the image: a repeated edge pixel changes neither the minimum nor
    // the test for an uncovered pixel), read whether or not it is needed
    const bool valid = pr.dvalid[i] != 0;
    const float u = pr.duv[i], v = pr.duv[nv + i];
    const float X = pr.dx[i], Y = pr.dx[nv + i], Z = pr.dx[2 * nv + i];
    const bool cont = pr.vcont[i] != 0;
    // (an invalid vertex's projection may be non-finite: not converted)
    const int px = valid ? int(rintf(u)) : 0, py = valid ? int(rintf(v)) : 0;
    const bool inside = valid && px >= 0 && px < W && py >= 0 && py < H;
    uint32_t zw[9];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int y = min(max(py + dy - 1, 0), H - 1), x = min(max(px + dx - 1, 0), W - 1);
            zw[3 * dy + dx] = pr.zbuf[size_t(y) * W + x];
        }
    if (inside) {
        {
            uint32_t m = 0xffffffffu;
            bool open = false;      // an uncovered pixel in the window: the vertex is on the outline
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const uint32_t z = zw[q];
                if (z != 0u && z < m) m = z;
                open = open || z == 0u;
            }
            bool vis = m == 0xffffffffu ? true : (Z <= (1.0f / __uint_as_float(m)) + 0.05f);
            if (vis) {
                code |= 1;
                if (cont && (open || !pr.outline_only)) {
                    code |= 2;
                    // the sum of the vertex's face normals, in face-list order: the
                    // first kVertFaces face indices loaded together (clamped into the
                    // list), then their normals, then the rare remaining faces
                    constexpr int kVertFaces = 8;
                    const int q0 = T.vf_beg[i], q1 = T.vf_beg[i + 1], qc = max(q1 - 1, 0);
                    int fs[kVertFaces];
#pragma unroll
                    for (int u = 0; u < kVertFaces; ++u) fs[u] = T.vf_face[min(q0 + u, qc)];
                    float fn[kVertFaces][3];
#pragma unroll
                    for (int u = 0; u < kVertFaces; ++u)
#pragma unroll
                        for (int a = 0; a < 3; ++a) fn[u][a] = pr.fcross[a * size_t(nf) + fs[u]];
                    float n[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int u = 0; u < kVertFaces; ++u)
                        if (q0 + u < q1) {
                            n[0] = n[0] + fn[u][0];
                            n[1] = n[1] + fn[u][1];
                            n[2] = n[2] + fn[u][2];
                        }
                    for (int q = q0 + kVertFaces; q < q1; ++q) {
                        int f = T.vf_face[q];
                        n[0] = n[0] + pr.fcross[f];
                        n[1] = n[1] + pr.fcross[nf + f];
                        n[2] = n[2] + pr.fcross[2 * size_t(nf) + f];
                    }
                    float gx, gy;
                    (void)sample_cubic(pr.dt.g(), W, H, u, v, gx, gy);
                    float a = (n[0] * Z - n[2] * X) * pr.fx;
                    float b = (n[1] * Z - n[2] * Y) * pr.fy;
                    float s = a * (-gx) + b * (-gy);
                    size_t pix = size_t(py) * W + px;
                    const bool in_mask = pr.mask[pix] != 0 && pr.dt[pix] >= 1.5f;
                    if (in_mask && s < 0.0f) code = pr.exclude_case2 ? uint8_t(code & ~2) : uint8_t(code | 4);
                    if (code & 2) atomicAdd(cnt + 1, 1);
                }
                atomicAdd(cnt, 1);
            }
        }
    }
    if (pr.w_vel > 0.0f) code |= 8;
    pr.vflags[i] = code;
    int p = T.plan_pos[i];
    pr.pva[p] = X;
    pr.pva[nv + p] = Y;
    pr.pva[2 * nv + p] = Z;
    pr.vcode[p] = code;
    pr.px[p] = pr.xyz[i];
    pr.px[nv + p] = pr.xyz[nv + i];
    pr.px[2 * nv + p] = pr.xyz[2 * nv + i];
    if (pr.rgb) {
        pr.pc[p] = pr.rgb[i];
        pr.pc[nv + p] = pr.rgb[nv + i];
        pr.pc[2 * nv + p] = pr.rgb[2 * nv + i];
    }
    }
    __syncthreads();
    if (threadIdx.x < 2 && cnt[threadIdx.x])
        __hip_atomic_fetch_add(pr.counts.g() + threadIdx.x, cnt[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace cap
