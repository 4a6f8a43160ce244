// Learned warm start: per-node features, a 3-layer per-node network with two
// rounds of mean message passing over the node graph, trained and run with
// BF16 MFMA (v_mfma_f32_16x16x16_bf16) and float32 accumulation and master
// weights.  The paper's own warm start is the previous frame's result
// (Sec. 3.4, displacement warping); learned motion priors are its stated
// future work (Sec. 6).  The plain previous-frame start stays the fallback.
#include <cmath>

#include "device.hpp"

namespace cap {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// ---------------------------------------------------------------- GEMM
// C(i, j) = sum_k A(i, k) B(j, k) [+ bias(j)], A and B bfloat16 with arbitrary
// strides, float32 accumulation, one wave per 16x16 output tile.  Optional
// epilogue: a bfloat16 copy of ReLU(C) into Cb.
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int tn = (g.N + 15) >> 4, tm = (g.M + 15) >> 4;
    if (wave >= tm * tn) return;
    const int ti = wave / tn, tj = wave - ti * tn;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    const int ia = ti * 16 + r, jb = tj * 16 + r;
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        s4v a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + kq + q;
            a[q] = (ia < g.M && k < g.K) ? short(g.A[ia * g.sai + k * g.sak]) : short(0);
            b[q] = (jb < g.N && k < g.K) ? short(g.B[jb * g.sbj + k * g.sbk]) : short(0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int j = tj * 16 + r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + (lane >> 4) * 4 + q;
        if (i < g.M && j < g.N) {
            float v = acc[q];
            if (g.bias) v += g.bias[j];
            g.C[i * g.sci + j * g.scj] = v;
            if (g.relu_copy) g.Cb[i * g.scbi + j] = f2bf(v > 0.0f ? v : 0.0f);
        }
    }
}

// ---------------------------------------------------------------- fused forward
// One workgroup (8 waves) per 16 nodes and layer.  The workgroup first forms
// the layer's 16 x K bf16 input tile in LDS, each element once and with
// coalesced loads: layer 1 standardises the raw features; layers 2 and 3 copy
// ReLU(z_prev) and compute the mean over valid out-edges of ReLU(z_prev) of
// the neighbours (also stored into cat for the backward pass).  Each wave
// then owns output tile t = wave (layer 1 and 2: 8 tiles; layer 3: one) and accumulates over k in steps of
// 16 on MFMA with B = W from global memory.  The rounding points are those
// of the layer definition (bf16 inputs and weights, float32 accumulation in
// ascending k, bias after the sum, the mean of float32 ReLU outputs rounded
// once); all intermediates (Xb, z1, cat1, z2, cat2, y) stay for the backward.
constexpr int kLayerThreads = 512;

// One 16x16 output tile of a layer: the lane's weight fragments (output
// column jb, all of k) are loaded into registers at the start of the kernel,
// before the input tile is formed, so that round of latency overlaps the
// gathers; the MFMA chain then runs over k from LDS.  A fragment is four
// consecutive bf16 of a weight row, one 8-byte load (rows are K elements and
// the weight blocks start on 8-byte boundaries).
template <int K>
__device__ inline void load_wfrag(const uint16_t *__restrict__ W, int jb, int N, s4v (&bw)[K / 16]) {
    const int kq = ((threadIdx.x & 63) >> 4) * 4;
    const uint2 *wrow = reinterpret_cast<const uint2 *>(W + size_t(jb < N ? jb : 0) * K + kq);
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {      // lanes past N load row 0: their output columns are never stored
        const uint2 u = wrow[4 * s];
        bw[s][0] = short(u.x & 0xffffu);
        bw[s][1] = short(u.x >> 16);
        bw[s][2] = short(u.y & 0xffffu);
        bw[s][3] = short(u.y >> 16);
    }
}

// Workgroup barrier that orders LDS accesses only (global loads in flight
// stay in flight across it).
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int K>
__device__ inline f4v tile_mfma(const uint16_t (*As)[K + 8], const s4v (&bw)[K / 16]) {
    const int lane = threadIdx.x & 63, r = lane & 15, kq = (lane >> 4) * 4;
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < K / 16; ++s) {
        s4v a;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = short(As[r][16 * s + kq + q]);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[s], acc, 0, 0, 0);
    }
    return acc;
}

__global__ __launch_bounds__(kLayerThreads) void k_ws_layer1(const float *__restrict__ X, int nn,
                                                             const float *__restrict__ mu, const float *__restrict__ sd,
                                                             const uint16_t *__restrict__ W,
                                                             const float *__restrict__ bias, uint16_t *__restrict__ Xb,
                                                             float *__restrict__ z, uint16_t *__restrict__ cat) {
    static_assert(kLayerThreads / 64 == 8, "one output tile per wave");
    __shared__ uint16_t As[16][32 + 8];
    const int i0 = blockIdx.x * 16;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15;
    s4v bw[2];
    load_wfrag<32>(W, wv * 16 + r, 128, bw);
    for (int idx = threadIdx.x; idx < 16 * 32; idx += blockDim.x) {
        const int r = idx >> 5, k = idx & 31, i = i0 + r;
        uint16_t b = 0;
        if (i < nn) {
            b = f2bf(k < 27 ? (X[size_t(i) * 32 + k] - mu[k]) / sd[k] : 0.0f);
            Xb[size_t(i) * 32 + k] = b;
        }
        As[r][k] = b;
    }
    lds_barrier();
    {
        const int t = wv;
        const f4v acc = tile_mfma<32>(As, bw);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + (lane >> 4) * 4 + q, j = t * 16 + r;
            if (i < nn) {
                const float v = acc[q] + bias[j];
                z[size_t(i) * 128 + j] = v;
                cat[size_t(i) * 256 + j] = f2bf(v > 0.0f ? v : 0.0f);
            }
        }
    }
}

// Layers 2 (NT = 8 output tiles, 128 outputs) and 3 (NT = 1, N = 6 outputs).
// cat: [nn][256] bf16 inputs whose first half is ReLU(z_prev) (written by the
// previous layer); this kernel writes its second half (the neighbour means).
// cat_next (optional): bf16 ReLU copy of this layer's output into the next
// layer's first half.  xdelta (optional): the warm-start update
// x[c][k] = y[k][c] * (0.05 rad, 0.01 m scale) in node-major layout; with
// `upd` as well (N = 6), the block then applies that update to its nodes'
// state (the node update of a PCG solution, from the values in registers).
template <int NT>
__global__ __launch_bounds__(kLayerThreads) void k_ws_layer_mp(uint16_t *__restrict__ cat,
                                                               const float *__restrict__ zp,
                                                               const int *__restrict__ edge_dst, int nn,
                                                               const uint16_t *__restrict__ W,
                                                               const float *__restrict__ bias, int N,
                                                               float *__restrict__ z, uint16_t *__restrict__ cat_next,
                                                               float *__restrict__ xdelta, const ProbDev *__restrict__ upd) {
    static_assert(NT <= kLayerThreads / 64, "at most one output tile per wave");
    __shared__ uint16_t As[16][256 + 8];
    __shared__ int nbs[16][8];
    __shared__ float xs[16][6];     // the block's updates, for `upd`
    const int i0 = blockIdx.x * 16;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15;
    // the neighbour list (every thread loads an entry, the first 128 store
    // them) and the weights, unconditionally (no branches between the loads);
    // the barriers order LDS only
    const int ri = threadIdx.x & 127, ni = i0 + (ri >> 3);
    int nb = edge_dst[(ri & 7) * nn + min(ni, nn - 1)];
    if (ni >= nn) nb = -1;
    s4v bw[16];
    load_wfrag<256>(W, (wv < NT ? wv : 0) * 16 + r, N, bw);
    if (threadIdx.x < 128) nbs[ri >> 3][ri & 7] = nb;
    lds_barrier();
    // the input tile: ReLU(z_prev) copied (2048 values) and the neighbour means
    // (2048 values of 8 loads each), kFill of each per thread, every load of
    // the thread issued before any sum
    constexpr int kFill = 16 * 128 / kLayerThreads;
    int nbr[kFill][8];      // the rows' neighbour lists, all read from LDS before any load
#pragma unroll
    for (int m = 0; m < kFill; ++m)
#pragma unroll
        for (int e = 0; e < 8; ++e) nbr[m][e] = nbs[(threadIdx.x + kLayerThreads * m) >> 7][e];
    uint16_t own[kFill];
    float v[kFill][8];
#pragma unroll
    for (int m = 0; m < kFill; ++m) {
        const int idx = threadIdx.x + kLayerThreads * m, rr = idx >> 7, f = idx & 127, i = i0 + rr;
        own[m] = i < nn ? cat[size_t(i) * 256 + f] : uint16_t(0);
#pragma unroll
        for (int e = 0; e < 8; ++e) {         // safe index when the edge is absent
            const int l = nbr[m][e];
            v[m][e] = i < nn ? zp[size_t(l >= 0 ? l : 0) * 128 + f] : 0.0f;
        }
    }
#pragma unroll
    for (int m = 0; m < kFill; ++m) {
        const int idx = threadIdx.x + kLayerThreads * m, rr = idx >> 7, f = idx & 127, i = i0 + rr;
        float sum = 0.0f;
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (nbr[m][e] >= 0) {
                sum += v[m][e] > 0.0f ? v[m][e] : 0.0f;
                ++cnt;
            }
        const uint16_t b = i < nn ? f2bf(cnt ? sum / float(cnt) : 0.0f) : uint16_t(0);
        if (i < nn) cat[size_t(i) * 256 + 128 + f] = b;
        As[rr][f] = own[m];
        As[rr][128 + f] = b;
    }
    lds_barrier();
    if (wv < NT) {
        const int t = wv;
        const f4v acc = tile_mfma<256>(As, bw);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + (lane >> 4) * 4 + q, j = t * 16 + r;
            if (i < nn && j < N) {
                const float v = acc[q] + bias[j];
                z[size_t(i) * N + j] = v;
                if (cat_next) cat_next[size_t(i) * 256 + j] = f2bf(v > 0.0f ? v : 0.0f);
                if (xdelta) {
                    const float u = v * (j < 3 ? 0.05f : 0.01f);
                    xdelta[size_t(j) * nn + i] = u;
                    if (upd) xs[i - i0][j] = u;
                }
            }
        }
    }
    if (xdelta && upd) {        // (uniform)
        lds_barrier();
        const int k = i0 + int(threadIdx.x);
        if (threadIdx.x < 16 && k < nn) node_update_from(*upd, k, xs[threadIdx.x], xs[threadIdx.x] + 3);
    }
}

template __global__ void k_ws_layer_mp<8>(uint16_t *, const float *, const int *, int, const uint16_t *, const float *,
                                          int, float *, uint16_t *, float *, const ProbDev *);
template __global__ void k_ws_layer_mp<1>(uint16_t *, const float *, const int *, int, const uint16_t *, const float *,
                                          int, float *, uint16_t *, float *, const ProbDev *);

// ---------------------------------------------------------------- message passing (backward)
// Backward through [h; mean(h)] and the ReLU:
// dz[l][f] = (dcat[l][f] + sum over in-edges (k -> l) of dcat[k][width + f] / |N(k)|) * (z[l][f] > 0)
__global__ void k_mean_bwd(const float *__restrict__ dcat, const float *__restrict__ z, int nn,
                           const int *__restrict__ in_beg, const int *__restrict__ in_src,
                           const int *__restrict__ out_cnt, uint16_t *__restrict__ dzb, float *__restrict__ dz,
                           int width) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn * width) return;
    const int l = i / width, f = i - l * width;
    float s = dcat[size_t(l) * 2 * width + f];
    for (int q = in_beg[l]; q < in_beg[l + 1]; ++q) {
        const int k = in_src[q];
        s += dcat[size_t(k) * 2 * width + width + f] / float(out_cnt[k]);
    }
    const float v = z[size_t(l) * width + f] > 0.0f ? s : 0.0f;
    dz[i] = v;
    dzb[i] = f2bf(v);
}

// Column sums (bias gradients): out[j] = sum_i in[i][j].  One block per
// column; strided partial sums, then a fixed-order tree, so the result does
// not depend on timing.
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ in, int rows, int cols,
                                                float *__restrict__ out) {
    __shared__ float part[256];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int i = threadIdx.x; i < rows; i += blockDim.x) s += in[size_t(i) * cols + j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = part[0];
}

// dy = 2 (y - t) / (6 nn), fp32 and bf16; per-item squared error for the loss.
__global__ void k_mse_grad(const float *__restrict__ y, const float *__restrict__ t, int n, float *__restrict__ dy,
                           uint16_t *__restrict__ dyb, float *__restrict__ se) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float d = y[i] - t[i];
    const float g = 2.0f * d / float(n);
    dy[i] = g;
    dyb[i] = f2bf(g);
    se[i] = d * d;
}

// Adam on the float32 master vector, then refresh the bf16 weight copy.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, uint16_t *__restrict__ wb, int n, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float wi = w[i] - lr * mh / (sqrtf(vh) + 1e-8f);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float *__restrict__ in, uint16_t *__restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}


// ---------------------------------------------------------------- features
__device__ inline void log_so3(const float R[9], float w[3]) {
    const float c = fminf(fmaxf(((R[0] + R[4]) + R[8] - 1.0f) * 0.5f, -1.0f), 1.0f);
    const float th = acosf(c);
    const float v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    const float s = th < 1e-4f ? 0.5f + th * th / 12.0f : th / (2.0f * sinf(th));
    for (int a = 0; a < 3; ++a) w[a] = s * v[a];
}

// Raw features of every node of problem blockIdx.y ([nn][32]): axis-angle of
// R_k and t_k (0..5), their change since frame t-2 (6..11, zero without it),
// sign(b) log(1 + |b|) of the right-hand side (12..17), log(1 + diag)
// (18..23), node position minus the mean node position (24..26), zeros.
// A thread's first node has all of its loads issued before the block forms
// the mean position (strided partial sums, then a fixed-order tree), so the
// two overlap; further nodes (more nodes than threads) load afterwards.
struct WsNodeIn {
    float R[9], t[3], R2[9], t2[3], b[6], d[6], g[3];
};

__device__ inline void ws_node_load(const ProbDev &pr, const CAP_GLOBAL float *__restrict__ prev2, int nn, int k,
                                    WsNodeIn &in) {
#pragma unroll
    for (int q = 0; q < 9; ++q) in.R[q] = pr.state[size_t(q) * nn + k];
#pragma unroll
    for (int a = 0; a < 3; ++a) in.t[a] = pr.state[size_t(9 + a) * nn + k];
    if (prev2) {
#pragma unroll
        for (int q = 0; q < 9; ++q) in.R2[q] = prev2[size_t(q) * nn + k];
#pragma unroll
        for (int a = 0; a < 3; ++a) in.t2[a] = prev2[size_t(9 + a) * nn + k];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        in.b[c] = pr.b[size_t(c) * nn + k];
        in.d[c] = pr.diag[size_t(c) * nn + k];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) in.g[a] = pr.gpos[size_t(a) * nn + k];
}

__device__ inline void ws_node_features(const WsNodeIn &in, bool has_prev2, const float mean[3], float *x) {
    float w[3];
    log_so3(in.R, w);
    for (int a = 0; a < 3; ++a) {
        x[a] = w[a];
        x[3 + a] = in.t[a];
    }
    if (has_prev2) {
        float D[9], dw[3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                D[3 * i + j] = (in.R[3 * i] * in.R2[3 * j] + in.R[3 * i + 1] * in.R2[3 * j + 1]) +
                               in.R[3 * i + 2] * in.R2[3 * j + 2];
        log_so3(D, dw);
        for (int a = 0; a < 3; ++a) {
            x[6 + a] = dw[a];
            x[9 + a] = in.t[a] - in.t2[a];
        }
    } else {
        for (int a = 0; a < 6; ++a) x[6 + a] = 0.0f;
    }
    for (int c = 0; c < 6; ++c) {
        x[12 + c] = copysignf(log1pf(fabsf(in.b[c])), in.b[c]);
        x[18 + c] = log1pf(fmaxf(in.d[c], 0.0f));
    }
    for (int a = 0; a < 3; ++a) x[24 + a] = in.g[a] - mean[a];
    for (int a = 27; a < 32; ++a) x[a] = 0.0f;
}

__global__ __launch_bounds__(256) void k_ws_features(const ProbDev *__restrict__ P, float *__restrict__ X) {
    __shared__ float part[3][256];
    __shared__ float mean[3];
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const CAP_GLOBAL float *__restrict__ prev2 = pr.prev2.g();
    const int nn = T.nn;
    const int k0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    WsNodeIn first;
    if (k0 < nn) ws_node_load(pr, prev2, nn, k0, first);
    // mean node position: strided partial sums, then a fixed-order tree over the block
    {
        float s[3] = {0.0f, 0.0f, 0.0f};
        for (int k = threadIdx.x; k < nn; k += blockDim.x)      // node positions (set up per frame)
            for (int a = 0; a < 3; ++a) s[a] += pr.gpos[size_t(a) * nn + k];
        for (int a = 0; a < 3; ++a) part[a][threadIdx.x] = s[a];
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h)
                for (int a = 0; a < 3; ++a) part[a][threadIdx.x] += part[a][threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x < 3) mean[threadIdx.x] = part[threadIdx.x][0] / float(nn);
        __syncthreads();
    }
    const float m[3] = {mean[0], mean[1], mean[2]};
    if (k0 < nn) ws_node_features(first, prev2 != nullptr, m, X + size_t(k0) * 32);
    for (int k = k0 + stride; k < nn; k += stride) {
        WsNodeIn in;
        ws_node_load(pr, prev2, nn, k, in);
        ws_node_features(in, prev2 != nullptr, m, X + size_t(k) * 32);
    }
}


// The learned start's first layer with its features formed in place: one
// 8-wave workgroup per 16 nodes.  The first 256 threads form the mean node
// position exactly as k_ws_features does (the same strided sums and tree), 16
// threads form their nodes' features (into LDS, and into X as k_ws_features
// would), and the layer then proceeds as k_ws_layer1 on those values: the
// same numbers as the two launches, with one launch and no round trip
// through X.
__global__ __launch_bounds__(kLayerThreads) void k_ws_layer1_feat(const ProbDev *__restrict__ P, float *__restrict__ X,
                                                                  const float *__restrict__ mu,
                                                                  const float *__restrict__ sd,
                                                                  const uint16_t *__restrict__ W,
                                                                  const float *__restrict__ bias,
                                                                  uint16_t *__restrict__ Xb, float *__restrict__ z,
                                                                  uint16_t *__restrict__ cat) {
    static_assert(kLayerThreads / 64 == 8 && kLayerThreads >= 256, "one output tile per wave; 256 threads for the mean");
    __shared__ float part[3][256];
    __shared__ float mean[3];
    __shared__ float Xs[16][32];
    __shared__ uint16_t As[16][32 + 8];
    const ProbDev &pr = *P;
    const int nn = pr.T.nn;
    const CAP_GLOBAL float *__restrict__ prev2 = pr.prev2.g();
    const int i0 = blockIdx.x * 16, t = threadIdx.x;
    const int wv = t >> 6, lane = t & 63, r = lane & 15;
    s4v bw[2];
    load_wfrag<32>(W, wv * 16 + r, 128, bw);
    WsNodeIn in;
    const int kn = i0 + t;
    if (t < 16 && kn < nn) ws_node_load(pr, prev2, nn, kn, in);
    {   // mean node position, as in k_ws_features
        float sacc[3] = {0.0f, 0.0f, 0.0f};
        if (t < 256)
            for (int k = t; k < nn; k += 256)
                for (int a = 0; a < 3; ++a) sacc[a] += pr.gpos[size_t(a) * nn + k];
        if (t < 256)
            for (int a = 0; a < 3; ++a) part[a][t] = sacc[a];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h)
                for (int a = 0; a < 3; ++a) part[a][t] += part[a][t + h];
            __syncthreads();
        }
        if (t < 3) mean[t] = part[t][0] / float(nn);
        __syncthreads();
    }
    if (t < 16 && kn < nn) {
        const float m[3] = {mean[0], mean[1], mean[2]};
        ws_node_features(in, prev2 != nullptr, m, Xs[t]);
#pragma unroll
        for (int q = 0; q < 32; ++q) X[size_t(kn) * 32 + q] = Xs[t][q];
    }
    __syncthreads();
    for (int idx = t; idx < 16 * 32; idx += blockDim.x) {      // standardised, as k_ws_layer1
        const int rr = idx >> 5, k = idx & 31, i = i0 + rr;
        uint16_t b = 0;
        if (i < nn) {
            b = f2bf(k < 27 ? (Xs[rr][k] - mu[k]) / sd[k] : 0.0f);
            Xb[size_t(i) * 32 + k] = b;
        }
        As[rr][k] = b;
    }
    lds_barrier();
    const f4v acc = tile_mfma<32>(As, bw);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + (lane >> 4) * 4 + q, j = wv * 16 + r;
        if (i < nn) {
            const float v = acc[q] + bias[j];
            z[size_t(i) * 128 + j] = v;
            cat[size_t(i) * 256 + j] = f2bf(v > 0.0f ? v : 0.0f);
        }
    }
}

// Training target: per node (dw, dt) with R_next = Exp(dw) R_prev and
// t_next = t_prev + dt, divided by (0.05 rad, 0.01 m); layout [nn][6].
__global__ void k_ws_target(const float *__restrict__ prev, const float *__restrict__ next, int nn,
                            float *__restrict__ target) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    float R0[9], R1[9], D[9], dw[3];
    for (int q = 0; q < 9; ++q) { R0[q] = prev[size_t(q) * nn + k]; R1[q] = next[size_t(q) * nn + k]; }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            D[3 * i + j] = (R1[3 * i] * R0[3 * j] + R1[3 * i + 1] * R0[3 * j + 1]) + R1[3 * i + 2] * R0[3 * j + 2];
    log_so3(D, dw);
    for (int a = 0; a < 3; ++a) {
        target[size_t(k) * 6 + a] = dw[a] / 0.05f;
        target[size_t(k) * 6 + 3 + a] = (next[size_t(9 + a) * nn + k] - prev[size_t(9 + a) * nn + k]) / 0.01f;
    }
}

// Feature standardisation from `rows` feature rows ([rows][32]): one workgroup
// per feature, float64 sums in a fixed order; deviation floored at 1e-6.
__global__ __launch_bounds__(256) void k_ws_scaling(const float *__restrict__ X, long long rows, float *mu, float *sd) {
    __shared__ double red[4];
    const int f = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    for (long long i = threadIdx.x; i < rows; i += blockDim.x) {
        const double v = X[i * 32 + f];
        s += v;
        s2 += v * v;
    }
    s = block_sum<256>(s, red);
    s2 = block_sum<256>(s2, red);
    if (threadIdx.x == 0) {
        const double m = s / double(rows);
        const double var = fmax(s2 / double(rows) - m * m, 0.0);
        mu[f] = float(m);
        sd[f] = float(fmax(sqrt(var), 1e-6));
    }
}

}  // namespace cap
