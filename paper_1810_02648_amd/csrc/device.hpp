// Device helpers shared by the kernels (compiled with -ffp-contract=off: every
// float operation below rounds on its own, in the order written).
#pragma once

#include "common.hpp"

namespace cap {

// Cubic-convolution (Keys, a = -0.5) weights for offsets -1..2 and their
// derivatives, in the fixed float32 operation order that the integer
// decisions rely on.
__device__ inline void keys_weights(float f, float w[4], float d[4]) {
    const float h = 0.5f;
    float f2 = f * f;
    float f3 = f2 * f;
    w[0] = ((2.0f * f2 - f3) - f) * h;
    w[1] = ((3.0f * f3 - 5.0f * f2) + 2.0f) * h;
    w[2] = ((4.0f * f2 - 3.0f * f3) + f) * h;
    w[3] = (f3 - f2) * h;
    d[0] = ((4.0f * f - 3.0f * f2) - 1.0f) * h;
    d[1] = (9.0f * f2 - 10.0f * f) * h;
    d[2] = ((8.0f * f - 9.0f * f2) + 1.0f) * h;
    d[3] = (3.0f * f2 - 2.0f * f) * h;
}

// Value and gradient of the cubic interpolant of a [H][W] float image at the
// point (ix + fx, iy + fy) (integer cell, fraction in [0, 1)), clamp-to-edge.
// Rows are accumulated n = 0..3, then m = 0..3.
__device__ inline float sample_cubic_cell(const CAP_GLOBAL float *__restrict__ img, int W, int H, int ix, float fx, int iy,
                                          float fy, float &gu, float &gv) {
    float wx[4], dx[4], wy[4], dy[4];
    keys_weights(fx, wx, dx);
    keys_weights(fy, wy, dy);
    int xs[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) xs[n] = min(max(ix + n - 1, 0), W - 1);
    float val = 0.0f, gx = 0.0f, gy = 0.0f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const CAP_GLOBAL float *row = img + size_t(min(max(iy + m - 1, 0), H - 1)) * W;
        float rx = 0.0f, rv = 0.0f;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            float t = row[xs[n]];
            rx = rx + dx[n] * t;
            rv = rv + wx[n] * t;
        }
        gx = gx + wy[m] * rx;
        gy = gy + dy[m] * rv;
        val = val + wy[m] * rv;
    }
    gu = gx;
    gv = gy;
    return val;
}

// Float32 position: cell = floor(u), fraction = u - floor(u) (the decision recipe).
__device__ inline float sample_cubic(const CAP_GLOBAL float *__restrict__ img, int W, int H, float u, float v, float &gu,
                                     float &gv) {
    const float fu = floorf(u), fv = floorf(v);
    return sample_cubic_cell(img, W, H, int(fu), u - fu, int(fv), v - fv, gu, gv);
}

// Three channels of a [3][H][W] image sharing the stencil.
__device__ inline void sample_cubic3_cell(const CAP_GLOBAL float *__restrict__ img, int W, int H, int ix, float fx, int iy,
                                          float fy, float val[3], float gu[3], float gv[3]) {
    float wx[4], dx[4], wy[4], dy[4];
    keys_weights(fx, wx, dx);
    keys_weights(fy, wy, dy);
    int xs[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) xs[n] = min(max(ix + n - 1, 0), W - 1);
    const size_t plane = size_t(W) * H;
#pragma unroll
    for (int c = 0; c < 3; ++c) { val[c] = 0.0f; gu[c] = 0.0f; gv[c] = 0.0f; }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        size_t ro = size_t(min(max(iy + m - 1, 0), H - 1)) * W;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const CAP_GLOBAL float *row = img + c * plane + ro;
            float rx = 0.0f, rv = 0.0f;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                float t = row[xs[n]];
                rx = rx + dx[n] * t;
                rv = rv + wx[n] * t;
            }
            gu[c] = gu[c] + wy[m] * rx;
            gv[c] = gv[c] + dy[m] * rv;
            val[c] = val[c] + wy[m] * rv;
        }
    }
}

__device__ inline void cross3(const float a[3], const float b[3], float c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Cell and float32 fraction of a float64 image coordinate (clamped far outside).
__device__ inline void cell_of(double u, int &i, float &f) {
    u = fmin(fmax(u, -1.0e6), 1.0e6);
    const double fl = floor(u);
    i = int(fl);
    f = float(u - fl);
    if (f >= 1.0f) f = 0.99999994f;
}

// Start-state geometry of vertex i from its float32 position: projection,
// 1/256-pixel snapping and validity (decision recipe), contour mark cleared.
__device__ inline void store_start_vertex(const ProbDev &pr, int i, float X, float Y, float Z) {
    const int nv = pr.T.nv;
    float u = (pr.fx * X) / Z + pr.cx;
    float vv = (pr.fy * Y) / Z + pr.cy;
    bool valid = Z > 0.0f && fabsf(u) <= 65536.0f && fabsf(vv) <= 65536.0f;
    pr.dx[i] = X;
    pr.dx[nv + i] = Y;
    pr.dx[2 * nv + i] = Z;
    pr.duv[i] = u;
    pr.duv[nv + i] = vv;
    pr.dfix[i] = valid ? int(rintf(u * 256.0f)) : 0;
    pr.dfix[nv + i] = valid ? int(rintf(vv * 256.0f)) : 0;
    pr.dvalid[i] = valid ? 1 : 0;
    pr.vcont[i] = 0;
}

// Node k's update by (dw, dt): R <- Exp(dw) R (Rodrigues, float32), t <- t + dt.
__device__ inline void node_update_from(const ProbDev &pr, int k, const float w[3], const float tau[3]) {
    const int nn = pr.T.nn;
    const float th2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    float A, B;
    if (th2 < 1e-8f) {
        A = 1.0f - th2 / 6.0f;
        B = 0.5f - th2 / 24.0f;
    } else {
        const float th = sqrtf(th2);
        A = sinf(th) / th;
        B = (1.0f - cosf(th)) / th2;
    }
    float K[9] = {0.0f, -w[2], w[1], w[2], 0.0f, -w[0], -w[1], w[0], 0.0f};
    float E[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            float kk = (K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j]) + K[3 * i + 2] * K[6 + j];
            E[3 * i + j] = (i == j ? 1.0f : 0.0f) + A * K[3 * i + j] + B * kk;
        }
    float R[9];
    for (int q = 0; q < 9; ++q) R[q] = pr.state[size_t(q) * nn + k];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            pr.state[size_t(3 * i + j) * nn + k] = (E[3 * i] * R[j] + E[3 * i + 1] * R[3 + j]) + E[3 * i + 2] * R[6 + j];
    for (int a = 0; a < 3; ++a) pr.state[size_t(9 + a) * nn + k] += tau[a];
}

// Sums out[q] = sum over t < n of a[q * stride + t] (q < N, n >= 1) in
// float64 that every lane of every wave forms identically, without LDS or
// barriers: lane l adds a[l], a[l + 64], ... in order (the first four strides'
// loads of all N rows in flight together), then a fixed butterfly across the
// wave (each step adds the same two values in every lane of a pair, so all
// lanes end with the same sums).
template <int N>
__device__ inline void wave_sum_n(const CAP_GLOBAL double *a, int stride, int n, double (&out)[N]) {
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = 0.0;
    for (int t0 = 0; t0 < n; t0 += 64 * U) {
        double x[U][N];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(t0 + lane + 64 * u, n - 1);
#pragma unroll
            for (int q = 0; q < N; ++q) x[u][q] = a[size_t(q) * stride + t];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + lane + 64 * u < n)
#pragma unroll
                for (int q = 0; q < N; ++q) out[q] += x[u][q];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < N; ++q) out[q] += __shfl_xor(out[q], o);
}

// Deterministic block-wide sum of a double: fixed butterfly inside each wave,
// then the wave sums in wave order.  `sh` holds NT/64 doubles.
template <int NT>
__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// The same for N doubles at once (one exchange through LDS); `sh` holds
// NT/64 rows of N doubles.  v[] is replaced by the block sums.
template <int NT, int N>
__device__ inline void block_sum_n(double (&v)[N], double (*sh)[N]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] += __shfl_xor(v[q], o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) sh[wid][q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) r += sh[w][q];
        v[q] = r;
    }
    __syncthreads();
}

}  // namespace cap
