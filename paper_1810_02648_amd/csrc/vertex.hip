// Per-vertex non-rigid stage (Sec. 3.4 energy with the vertex positions as
// the unknowns; Sec. 4 non-rigid solver): template tables, the per-frame
// launch sequence and its kernels.
//
// One thread per vertex block row (Sec. 4: the rows of J^T J are handled per
// vertex, each thread gathering its row's non-zeros).  A row's non-zeros are
// the vertex's own 3x3 block and one block per one-ring neighbour; the
// product J^T |B| J p is applied matrix-free from the per-vertex data block
// H_i = sum |b| G^T G (stored, 6 floats), the temporal weights, and the
// regulariser blocks w_s a_ij I + w_e a_ij u_ij u_ij^T, whose unit edge
// directions u_ij are re-formed from the linearisation point gathered with p.
// No atomics: every vertex writes only its own rows; inner products are
// summed per workgroup and the workgroup sums added by every workgroup of the
// next launch in the same fixed order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"
#include "runtime.hpp"

namespace cap {

int build_topology_template(const int *tri_dev, int nv, int nf, capture_template **out, int device);

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v);
__global__ void k_contour(const ProbDev *P);
__global__ void k_dt_seg(const ProbDev *P);
__global__ void k_prep_raster(const ProbDev *P, int nb_f, int scan);
__global__ void k_prep_cols(const ProbDev *P);
__global__ void k_prep_rows(const ProbDev *P, int nb_rows);
__global__ void k_decide(const ProbDev *P);
__global__ void k_part_labels(const ProbDev *P, const int *parts, int *img);
__global__ void k_part_labels_big(const ProbDev *P, const int *parts, int *img);

constexpr int kVThreads = 128;
constexpr int kRingChunk = 4;       // one-ring neighbours whose gathers are issued together
constexpr int kRowLanes = 8;        // lanes per vertex row in the product
constexpr int kApplyThreads = 1024;
constexpr int kVTerms = 7;          // photo, sil (with b), sil (with |b|), smooth, edge, velocity, acceleration
constexpr int kVLevels = 3;         // distinct Gaussian kernels per solve
constexpr int kVMaxBlur = 15;
// Table 1: non-rigidity weight of material classes 1..7
constexpr double kTable1[7] = {1.0, 2.0, 2.5, 3.0, 50.0, 100.0, 200.0};

// One-ring table of a template, ELL layout [K][nv] (neighbour k of vertex i
// at k * nv + i; rows padded with -1 after the last neighbour).
struct VTemplateDev {
    int nv, K;
    gptr<const int> nbr;
    gptr<const float> ek;     // s_ij / |N_i|: weight of the directed edge i -> j in the energy
    gptr<const float> ea;     // s_ij / |N_i| + s_ij / |N_j|: weight of the edge pair in the normal equations
    gptr<const float> elen;   // |Vhat_i - Vhat_j|
    gptr<const int> parts;    // [nv] body-part label (0: torso), or null
};

// One frame: inputs, decisions and the solver's buffers (all [3][nv] planes).
struct VertexDev {
    VTemplateDev T;
    int nv, nb;                      // vertices, workgroups of the per-vertex kernels
    int nba;                         // workgroups of the product (kRowLanes lanes per vertex)
    int W, H;
    float fx, fy, cx, cy;
    float sw_photo, sw_sil, tau;
    double w_smooth, w_edge, w_vel, w_acc;
    gptr<const float> posed, prev, prev2, rgb, dt;
    gptr<const uint8_t> vflags;
    gptr<float> Vout;                // the caller's positions (start in, solution out)
    gptr<double> V[2], x[2];         // linearisation point and PCG solution of step g in buffer g & 1
    gptr<double> r, u, p[2], Ap;     // PCG vectors (p of iteration j in buffer j & 1)
    gptr<double> dinv;               // Jacobi preconditioner 1 / diag(J^T |B| J)
    gptr<float> Hm;                  // [6][nv] data block H_i (xx, xy, xz, yy, yz, zz)
    gptr<double> ru;                 // [2][nb] per-workgroup r.u of two iterations
    gptr<double> pap;                // [nb] per-workgroup p.Ap
    gptr<double> epart;              // [MAX_GN + 1][kVTerms][nb] per-workgroup energies
    gptr<double> scal;               // [MAX_GN] PCG stopped in step g, then [MAX_GN + 1][kVTerms] energies
    gptr<double> rhs_out, diag_out;  // capture_vertex_linearize outputs (or null)
    gptr<int> ring;                  // [nv] one-ring distance from a snapped vertex (vertex snapping)
    gptr<int> plab[2];               // [H][W] body-part label images (ping-pong of the dilation)
    gptr<int> nsnap;                 // [1] snapped vertices
};

struct BlurW {
    float w[kVMaxBlur];
    int r;
};

// The blur levels of a solve: kernel radii and weights.
struct BlurSet {
    int n;
    int r[kVLevels];
    float w[kVLevels][kVMaxBlur];
};

}  // namespace cap

struct capture_vertex_template {
    cap::VTemplateDev dev;
    capture_template *topo;     // mesh tables for the raster and decision kernels
    void *mem;                  // device one-ring table
    int device;
};

namespace cap {

// ---------------------------------------------------------------- kernels
// Start positions: the decision recipe's float32 geometry, and the first
// linearisation point (read by step 0 as "previous point + previous solution").
// Blocks from nbv on clear the depth buffer instead, 8 x kVThreads pixels each.
constexpr int kZbufPerBlock = 8 * kVThreads;
__global__ __launch_bounds__(kVThreads) void k_vstart(const VertexDev *__restrict__ P, const ProbDev *__restrict__ R,
                                                      int nbv) {
    if (int(blockIdx.x) >= nbv) {
        const size_t hw = size_t(R->W) * R->H, q0 = size_t(blockIdx.x - nbv) * kZbufPerBlock + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kZbufPerBlock / kVThreads; ++u)
            if (q0 + size_t(u) * kVThreads < hw) R->zbuf[q0 + size_t(u) * kVThreads] = 0u;
        return;
    }
    const VertexDev &pr = *P;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < CAPTURE_MAX_GN) pr.scal[threadIdx.x] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x < 3) R->counts[threadIdx.x] = 0;     // visible, contour, large-face queue
    if (i >= nv) return;
    const float X = pr.Vout[i], Y = pr.Vout[nv + i], Z = pr.Vout[2 * size_t(nv) + i];
    store_start_vertex(*R, i, X, Y, Z);
    pr.V[1][i] = X;
    pr.V[1][nv + i] = Y;
    pr.V[1][2 * size_t(nv) + i] = Z;
    for (int a = 0; a < 3; ++a) pr.x[1][a * size_t(nv) + i] = 0.0;
}

// Horizontal passes of every blur level: a row segment of 256 pixels and its
// clamped margins staged in LDS once for the three channels, then each pixel's
// taps (added from -r to r) for each level; out: tmp[level][c][H][W].
constexpr int kBlurMargin = (kVMaxBlur - 1) / 2;
__global__ __launch_bounds__(256) void k_vblur_h(const ProbDev *__restrict__ R, float *__restrict__ tmp, int W, int H,
                                                 BlurSet bs) {
    __shared__ float sh[3][256 + 2 * kBlurMargin];
    const int x0 = blockIdx.x * 256, y = blockIdx.y, t = threadIdx.x;
    const size_t plane = size_t(W) * H;
    const float *img = R->image;
    for (int q = t; q < 256 + 2 * kBlurMargin; q += 256) {
        const int x = min(max(x0 - kBlurMargin + q, 0), W - 1);
        for (int c = 0; c < 3; ++c) sh[c][q] = img[c * plane + size_t(y) * W + x];
    }
    __syncthreads();
    const int x = x0 + t;
    if (x >= W) return;
    for (int l = 0; l < bs.n; ++l) {
        const int r = bs.r[l];
        float w[kVMaxBlur];                  // the level's taps (uniform)
#pragma unroll
        for (int q = 0; q < kVMaxBlur; ++q) w[q] = bs.w[l][q];
        for (int c = 0; c < 3; ++c) {
            // taps unrolled to the largest kernel, every read issued first
            // (clamped into the level's window), then added from -r to r
            const float *row = &sh[c][t + kBlurMargin - r];
            float v[kVMaxBlur];
#pragma unroll
            for (int q = 0; q < kVMaxBlur; ++q) v[q] = row[min(q, 2 * r)];
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < kVMaxBlur; ++q)
                if (q <= 2 * r) acc = acc + w[q] * v[q];
            tmp[(size_t(l) * 3 + c) * plane + size_t(y) * W + x] = acc;
        }
    }
}

// Vertical passes: level blockIdx.z, a tile of 64 columns x 16 rows with its
// clamped margin rows staged in LDS per channel, taps added from -r to r.
constexpr int kBlurTileW = 64, kBlurTileH = 16;
struct BlurOut {
    float *p[kVLevels];
};
__global__ __launch_bounds__(256) void k_vblur_v(const float *__restrict__ tmp, BlurOut out, int W, int H, BlurSet bs) {
    __shared__ float sh[kBlurTileH + 2 * kBlurMargin][kBlurTileW];
    const int l = blockIdx.z, r = bs.r[l];
    float w[kVMaxBlur];                      // the level's taps (uniform)
#pragma unroll
    for (int q = 0; q < kVMaxBlur; ++q) w[q] = bs.w[l][q];
    const int x0 = blockIdx.x * kBlurTileW, y0 = blockIdx.y * kBlurTileH, t = threadIdx.x;
    const int tx = t & (kBlurTileW - 1), ty = t / kBlurTileW;        // 4 row groups of 4 rows
    const size_t plane = size_t(W) * H;
    const int x = min(x0 + tx, W - 1);
    for (int c = 0; c < 3; ++c) {
        const float *src = tmp + (size_t(l) * 3 + c) * plane;
        __syncthreads();
        for (int q = ty; q < kBlurTileH + 2 * r; q += 256 / kBlurTileW) {
            const int y = min(max(y0 - r + q, 0), H - 1);
            sh[q][tx] = src[size_t(y) * W + x];
        }
        __syncthreads();
        if (x0 + tx < W)
            for (int k = 0; k < kBlurTileH / (256 / kBlurTileW); ++k) {
                const int row = ty + k * (256 / kBlurTileW), y = y0 + row;
                if (y >= H) break;
                float v[kVMaxBlur];          // as in the horizontal pass: reads first, then the taps in order
#pragma unroll
                for (int q = 0; q < kVMaxBlur; ++q) v[q] = sh[row + min(q, 2 * r)][tx];
                float acc = 0.0f;
#pragma unroll
                for (int q = 0; q < kVMaxBlur; ++q)
                    if (q <= 2 * r) acc = acc + w[q] * v[q];
                out.p[l][c * plane + size_t(y) * W + x0 + tx] = acc;
            }
    }
}

__device__ inline void load3(const gptr<double> &a, int nv, int i, double v[3]) {
    v[0] = a[i];
    v[1] = a[nv + i];
    v[2] = a[2 * size_t(nv) + i];
}

// Linearisation at step g's point V = V_{g-1} + x_{g-1} (buffers (g-1) & 1):
// residuals, the data block H_i, the gradient J^T B F and diagonal of
// J^T |B| J of the vertex's block row, per-workgroup energies; then the
// first PCG vectors x = 0, r = b = -J^T B F, u = M r and the r.u sums.
// mode 0: full step; 1: energies only, and the point is written to the
// caller's array (float32); 2: full, plus rhs / diag copies to the outputs.
__global__ __launch_bounds__(kVThreads) void k_vlin(const VertexDev *__restrict__ P, const float *__restrict__ img,
                                                    int g, int mode) {
    __shared__ double red[kVThreads / 64][kVTerms + 1];
    const VertexDev &pr = *P;
    const VTemplateDev &T = pr.T;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    const int gp = (g + 1) & 1, gc = g & 1;
    if (mode != 0 && i == 0) pr.nsnap[0] = 0;      // the snapping that may follow counts from here
    double es[kVTerms + 1] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < nv) {
        double V[3], xo[3];
        load3(pr.V[gp], nv, i, V);
        load3(pr.x[gp], nv, i, xo);
        for (int a = 0; a < 3; ++a) V[a] += xo[a];
        const uint8_t code = pr.vflags[i];
        float Hm[6] = {0, 0, 0, 0, 0, 0};
        float gd[3] = {0, 0, 0};
        // data terms: the projection in float64, sampling and Jacobians in float32
        if ((code & 3) && V[2] > 0.0) {
            const double izd = 1.0 / V[2];
            const double ud = double(pr.fx) * V[0] * izd + pr.cx, vd = double(pr.fy) * V[1] * izd + pr.cy;
            int cu, cv;
            float fu, fv;
            cell_of(ud, cu, fu);
            cell_of(vd, cv, fv);
            const float iz = float(izd), X = float(V[0]), Y = float(V[1]);
            const float P0[3] = {pr.fx * iz, 0.0f, -pr.fx * X * iz * iz};
            const float P1[3] = {0.0f, pr.fy * iz, -pr.fy * Y * iz * iz};
            if (code & 1) {
                float val[3], gu[3], gv[3];
                sample_cubic3_cell((const CAP_GLOBAL float *)img, pr.W, pr.H, cu, fu, cv, fv, val, gu, gv);
                float res[3], n2 = 0.0f;
                for (int c = 0; c < 3; ++c) {
                    res[c] = val[c] - pr.rgb[size_t(c) * nv + i];
                    n2 += res[c] * res[c];
                }
                if (!(sqrtf(n2) > pr.tau)) {
                    for (int c = 0; c < 3; ++c) {
                        const float r = pr.sw_photo * res[c];
                        float G[3];
                        for (int a = 0; a < 3; ++a) G[a] = pr.sw_photo * (gu[c] * P0[a] + gv[c] * P1[a]);
                        Hm[0] += G[0] * G[0]; Hm[1] += G[0] * G[1]; Hm[2] += G[0] * G[2];
                        Hm[3] += G[1] * G[1]; Hm[4] += G[1] * G[2]; Hm[5] += G[2] * G[2];
                        for (int a = 0; a < 3; ++a) gd[a] += G[a] * r;
                        es[0] += double(r) * double(r);
                    }
                }
            }
            if (code & 2) {
                float gu, gv;
                const float dval = sample_cubic_cell(pr.dt.g(), pr.W, pr.H, cu, fu, cv, fv, gu, gv);
                const float r = pr.sw_sil * dval;
                const float b = (code & 4) ? -1.0f : 1.0f;
                float G[3];
                for (int a = 0; a < 3; ++a) G[a] = pr.sw_sil * (gu * P0[a] + gv * P1[a]);
                Hm[0] += G[0] * G[0]; Hm[1] += G[0] * G[1]; Hm[2] += G[0] * G[2];
                Hm[3] += G[1] * G[1]; Hm[4] += G[1] * G[2]; Hm[5] += G[2] * G[2];
                for (int a = 0; a < 3; ++a) gd[a] += b * G[a] * r;
                es[1] += double(b) * double(r) * double(r);
                es[2] += double(r) * double(r);
            }
        }
        double gr[3] = {gd[0], gd[1], gd[2]};
        double dg[3] = {Hm[0], Hm[3], Hm[5]};
        // temporal priors (identity Jacobians)
        if (pr.w_vel > 0.0 || pr.w_acc > 0.0) {
            double q1[3], q2[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a) q1[a] = pr.prev[size_t(a) * nv + i];
            if (pr.w_acc > 0.0)
                for (int a = 0; a < 3; ++a) q2[a] = pr.prev2[size_t(a) * nv + i];
            for (int a = 0; a < 3; ++a) {
                if (pr.w_vel > 0.0) {
                    const double d = V[a] - q1[a];
                    gr[a] += pr.w_vel * d;
                    dg[a] += pr.w_vel;
                    es[5] += pr.w_vel * d * d;
                }
                if (pr.w_acc > 0.0) {
                    const double d = (V[a] - 2.0 * q1[a]) + q2[a];
                    gr[a] += pr.w_acc * d;
                    dg[a] += pr.w_acc;
                    es[6] += pr.w_acc * d * d;
                }
            }
        }
        // spatial regularisers over the one-ring
        if (pr.w_smooth > 0.0 || pr.w_edge > 0.0) {
            double S[3];
            for (int a = 0; a < 3; ++a) S[a] = pr.posed[size_t(a) * nv + i];
            // the one-ring in chunks, each chunk's gathers in flight together
            for (int k0 = 0; k0 < T.K; k0 += kRingChunk) {
                int jn[kRingChunk];
                double ek[kRingChunk], ea[kRingChunk], el[kRingChunk], Vj[kRingChunk][3], xj[kRingChunk][3];
                float Sj[kRingChunk][3];
#pragma unroll
                for (int u = 0; u < kRingChunk; ++u) {
                    const int k = min(k0 + u, T.K - 1);
                    const size_t o = size_t(k) * nv + i;
                    jn[u] = k0 + u < T.K ? T.nbr[o] : -1;
                    ek[u] = T.ek[o];
                    ea[u] = T.ea[o];
                    el[u] = T.elen[o];
                }
#pragma unroll
                for (int u = 0; u < kRingChunk; ++u) {
                    const int q = jn[u] < 0 ? i : jn[u];
                    load3(pr.V[gp], nv, q, Vj[u]);
                    load3(pr.x[gp], nv, q, xj[u]);
                    for (int a = 0; a < 3; ++a) Sj[u][a] = pr.posed[size_t(a) * nv + q];
                }
#pragma unroll
                for (int u = 0; u < kRingChunk; ++u) {
                    if (jn[u] < 0) continue;
                    double d[3], sm[3];
                    for (int a = 0; a < 3; ++a) {
                        const double v = Vj[u][a] + xj[u][a];
                        d[a] = V[a] - v;
                        sm[a] = d[a] - (S[a] - double(Sj[u][a]));
                    }
                    if (pr.w_smooth > 0.0) {
                        es[3] += pr.w_smooth * ek[u] * ((sm[0] * sm[0] + sm[1] * sm[1]) + sm[2] * sm[2]);
                        for (int a = 0; a < 3; ++a) {
                            gr[a] += pr.w_smooth * ea[u] * sm[a];
                            dg[a] += pr.w_smooth * ea[u];
                        }
                    }
                    if (pr.w_edge > 0.0) {
                        const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                        const double dl = len - el[u];
                        es[4] += pr.w_edge * ek[u] * dl * dl;
                        if (len > 0.0)
                            for (int a = 0; a < 3; ++a) {
                                const double ua = d[a] / len;
                                gr[a] += pr.w_edge * ea[u] * dl * ua;
                                dg[a] += pr.w_edge * ea[u] * ua * ua;
                            }
                    }
                }
                if (jn[kRingChunk - 1] < 0) break;
            }
        }
        if (mode == 1) {
            for (int a = 0; a < 3; ++a) pr.Vout[size_t(a) * nv + i] = float(V[a]);
        } else {
            for (int a = 0; a < 3; ++a) {
                const size_t o = size_t(a) * nv + i;
                const double di = dg[a] > 0.0 ? 1.0 / dg[a] : 1.0;
                const double b = -gr[a];
                pr.V[gc][o] = V[a];
                pr.x[gc][o] = 0.0;
                pr.r[o] = b;
                pr.u[o] = di * b;
                pr.dinv[o] = di;
                es[kVTerms] += b * (di * b);
                if (mode == 2) {
                    if (pr.rhs_out) pr.rhs_out[o] = b;
                    if (pr.diag_out) pr.diag_out[o] = dg[a];
                }
            }
            for (int q = 0; q < 6; ++q) pr.Hm[size_t(q) * nv + i] = Hm[q];
        }
    }
    block_sum_n<kVThreads, kVTerms + 1>(es, red);
    if (threadIdx.x == 0) {
        for (int t = 0; t < kVTerms; ++t) pr.epart[(size_t(g) * kVTerms + t) * pr.nb + blockIdx.x] = es[t];
        if (mode != 1) pr.ru[blockIdx.x] = es[kVTerms];
    }
}

// PCG (Jacobi, float64 vectors), two launches per iteration j of step g.
// k_vapply: beta from the r.u sums of iterations j and j - 1 (every
// workgroup adds the workgroup sums in the same order), p_j = u + beta p_{j-1}
// for the vertex and, formed again from the stored vectors, for its
// neighbours; then row i of J^T |B| J p_j: H_i p_i + (w_vel + w_acc) p_i +
// sum_j a_ij [w_smooth (p_i - p_j) + w_edge u_ij u_ij^T (p_i - p_j)], and the
// p.Ap sums.  Stops the step's PCG (flag in scal[g]) when r.u == 0.
// product_only: multiply the vector in u (p = u), no stop test (capture_vertex_linearize).
// kRowLanes lanes per vertex row: lane l takes neighbours l, l + kRowLanes, ...
// of the one-ring (their gathers in flight across the lanes), the lanes' sums
// are added by a fixed butterfly, and the row's first lane adds the vertex's
// own block and stores p_j and (J^T |B| J p_j)_i.
__global__ __launch_bounds__(kApplyThreads) void k_vapply(const VertexDev *__restrict__ P, int g, int j,
                                                          int product_only) {
    __shared__ double red[kApplyThreads / 64][1];
    const VertexDev &pr = *P;
    if (pr.scal[g] != 0.0) return;
    const VTemplateDev &T = pr.T;
    const int nv = pr.nv, nb = pr.nb;
    const int gt = blockIdx.x * kApplyThreads + threadIdx.x, i0 = gt / kRowLanes, l = gt % kRowLanes;
    double rz[1] = {1.0}, rzp[1] = {1.0};
    if (!product_only) wave_sum_n<1>(pr.ru.g() + size_t(j & 1) * nb, nb, nb, rz);
    if (rz[0] == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) pr.scal[g] = 1.0;
        return;
    }
    if (j > 0) wave_sum_n<1>(pr.ru.g() + size_t((j + 1) & 1) * nb, nb, nb, rzp);
    const double beta = j > 0 ? rz[0] / rzp[0] : 0.0;
    const gptr<double> pold = pr.p[(j + 1) & 1], pnew = pr.p[j & 1], Vg = pr.V[g & 1];
    auto pval = [&](int n, double q[3]) {
        for (int a = 0; a < 3; ++a) {
            const size_t o = size_t(a) * nv + n;
            q[a] = j > 0 ? pr.u[o] + beta * pold[o] : double(pr.u[o]);
        }
    };
    const int i = min(i0, nv - 1);          // lanes past the last row repeat it and store nothing
    double pi[3], V[3], c[3] = {0.0, 0.0, 0.0};
    pval(i, pi);
    load3(Vg, nv, i, V);
    if (pr.w_smooth > 0.0 || pr.w_edge > 0.0)
        for (int k = l; k < T.K; k += kRowLanes) {
            const int jn = T.nbr[size_t(k) * nv + i];
            if (jn < 0) break;
            const double ea = T.ea[size_t(k) * nv + i];
            double pj[3], Vj[3], dp[3], d[3];
            pval(jn, pj);
            load3(Vg, nv, jn, Vj);
            for (int a = 0; a < 3; ++a) {
                dp[a] = pi[a] - pj[a];
                d[a] = V[a] - Vj[a];
            }
            if (pr.w_smooth > 0.0)
                for (int a = 0; a < 3; ++a) c[a] += pr.w_smooth * ea * dp[a];
            if (pr.w_edge > 0.0) {
                const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                if (len > 0.0) {
                    const double ua[3] = {d[0] / len, d[1] / len, d[2] / len};
                    const double s = pr.w_edge * ea * ((ua[0] * dp[0] + ua[1] * dp[1]) + ua[2] * dp[2]);
                    for (int a = 0; a < 3; ++a) c[a] += s * ua[a];
                }
            }
        }
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] += __shfl_xor(c[a], o);
    double pap[1] = {0.0};
    if (l == 0 && i0 < nv) {
        const double H0 = pr.Hm[i], H1 = pr.Hm[nv + i], H2 = pr.Hm[2 * size_t(nv) + i];
        const double H3 = pr.Hm[3 * size_t(nv) + i], H4 = pr.Hm[4 * size_t(nv) + i], H5 = pr.Hm[5 * size_t(nv) + i];
        const double wt = pr.w_vel + pr.w_acc;
        double out[3];
        out[0] = (((H0 * pi[0] + H1 * pi[1]) + H2 * pi[2]) + wt * pi[0]) + c[0];
        out[1] = (((H1 * pi[0] + H3 * pi[1]) + H4 * pi[2]) + wt * pi[1]) + c[1];
        out[2] = (((H2 * pi[0] + H4 * pi[1]) + H5 * pi[2]) + wt * pi[2]) + c[2];
        for (int a = 0; a < 3; ++a) {
            const size_t o = size_t(a) * nv + i;
            pnew[o] = pi[a];
            pr.Ap[o] = out[a];
        }
        pap[0] = (pi[0] * out[0] + pi[1] * out[1]) + pi[2] * out[2];
    }
    block_sum_n<kApplyThreads, 1>(pap, red);
    if (threadIdx.x == 0) pr.pap[blockIdx.x] = pap[0];
}

// alpha = r.u / p.Ap (stops the step's PCG when p.Ap <= 0, leaving x), then
// x += alpha p, r -= alpha Ap, u = M r and the r.u sums of iteration j + 1.
__global__ __launch_bounds__(kVThreads) void k_vupdate(const VertexDev *__restrict__ P, int g, int j) {
    __shared__ double red[kVThreads / 64][1];
    const VertexDev &pr = *P;
    if (pr.scal[g] != 0.0) return;
    const int nv = pr.nv, nb = pr.nb, i = blockIdx.x * kVThreads + threadIdx.x;
    double pAp[1], rz[1];
    wave_sum_n<1>(pr.pap.g(), pr.nba, pr.nba, pAp);
    wave_sum_n<1>(pr.ru.g() + size_t(j & 1) * nb, nb, nb, rz);
    if (!(pAp[0] > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) pr.scal[g] = 1.0;
        return;
    }
    const double alpha = rz[0] / pAp[0];
    const gptr<double> x = pr.x[g & 1], p = pr.p[j & 1];
    double ru[1] = {0.0};
    if (i < nv)
        for (int a = 0; a < 3; ++a) {
            const size_t o = size_t(a) * nv + i;
            x[o] = x[o] + alpha * p[o];
            const double r = pr.r[o] - alpha * pr.Ap[o];
            const double u = pr.dinv[o] * r;
            pr.r[o] = r;
            pr.u[o] = u;
            ru[0] += r * u;
        }
    block_sum_n<kVThreads, 1>(ru, red);
    if (threadIdx.x == 0) pr.ru[size_t((j + 1) & 1) * nb + blockIdx.x] = ru[0];
}

// Energies of steps 0..G (one workgroup; each wave adds whole rows of
// workgroup partials in a fixed order).
__global__ __launch_bounds__(256) void k_vreport(const VertexDev *__restrict__ P, const int *__restrict__ counts,
                                                  int G) {
    const VertexDev &pr = *P;
    const int nb = pr.nb, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int item = wave; item < (G + 1) * kVTerms; item += 4) {
        double s[1];
        wave_sum_n<1>(pr.epart.g() + size_t(item) * nb, nb, nb, s);
        if (lane == 0) pr.scal[CAPTURE_MAX_GN + item] = s[0];
    }
    if (threadIdx.x == 0) {     // after the energies, so that one read-back takes the whole report
        CAP_GLOBAL double *c = pr.scal.g() + CAPTURE_MAX_GN + (G + 1) * kVTerms;
        c[0] = double(counts[0]);
        c[1] = double(counts[1]);
        c[2] = double(pr.nsnap[0]);
    }
}

// ---------------------------------------------------------------- body-part mask
constexpr int kNoPart = 0x7fffffff;
// One growth step of the part label image over the 3x3 neighbourhood (outside
// the image: no label): torso (0) where any neighbour is torso, else the
// pixel's own label, else the smallest neighbouring label.
__global__ __launch_bounds__(256) void k_part_dilate(const int *__restrict__ src, int *__restrict__ dst, int W, int H) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= W * H) return;
    const int y = q / W, x = q - y * W;
    int v[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int yy = y + dy, xx = x + dx;
            const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
            v[3 * (dy + 1) + dx + 1] = in ? src[size_t(min(max(yy, 0), H - 1)) * W + min(max(xx, 0), W - 1)] : kNoPart;
        }
    int mn = kNoPart;
    bool torso = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        torso = torso || v[k] == 0;
        mn = min(mn, v[k]);
    }
    dst[q] = torso ? 0 : (v[4] != kNoPart ? v[4] : mn);
}

// Contour vertices whose pixel lies in another part's region lose their
// silhouette residual (b_i = 0): flags cleared, contour count reduced.
__global__ __launch_bounds__(kVThreads) void k_part_mask(const VertexDev *__restrict__ P, const ProbDev *__restrict__ R,
                                                         const int *__restrict__ img) {
    const VertexDev &pr = *P;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (i >= nv) return;
    const uint8_t code = R->vflags[i];
    if (!(code & 2)) return;
    const int px = int(rintf(R->duv[i])), py = int(rintf(R->duv[nv + i]));
    const int lab = img[size_t(py) * R->W + px];
    if (lab != kNoPart && lab != pr.T.parts[i]) {
        R->vflags[i] = uint8_t(code & ~6);
        atomicSub(R->counts.ptr + 1, 1);
    }
}

// ---------------------------------------------------------------- vertex snapping
// Contour vertices with b_i = +1 walk on the distance transform from their
// final projection along the negative gradient, u <- u - I_DT(u) g/|g| (at most
// `steps` times, stopping once I_DT <= tol or |g| < 1e-6), if their starting
// distance is at most max_px; the pixel is lifted back at the vertex's depth.
// Out: displacement (0 for the others) and ring 0 / rings + 1.
__global__ __launch_bounds__(kVThreads) void k_vsnap(const VertexDev *__restrict__ P, int G, int steps, float max_px,
                                                     float tol, int rings) {
    const VertexDev &pr = *P;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (i >= nv) return;
    double V[3], xo[3], d[3] = {0.0, 0.0, 0.0};
    load3(pr.V[(G + 1) & 1], nv, i, V);
    load3(pr.x[(G + 1) & 1], nv, i, xo);
    for (int a = 0; a < 3; ++a) V[a] += xo[a];
    const uint8_t code = pr.vflags[i];
    bool snap = false;
    if ((code & 2) && !(code & 4) && V[2] > 0.0) {
        double u = double(pr.fx) * V[0] / V[2] + pr.cx, v = double(pr.fy) * V[1] / V[2] + pr.cy;
        float gu, gv;
        int cu, cv;
        float fu, fv;
        cell_of(u, cu, fu);
        cell_of(v, cv, fv);
        const float d0 = sample_cubic_cell(pr.dt.g(), pr.W, pr.H, cu, fu, cv, fv, gu, gv);
        if (d0 <= max_px) {
            snap = true;
            for (int k = 0; k < steps; ++k) {
                cell_of(u, cu, fu);
                cell_of(v, cv, fv);
                const float dist = sample_cubic_cell(pr.dt.g(), pr.W, pr.H, cu, fu, cv, fv, gu, gv);
                const double g = sqrt(double(gu) * gu + double(gv) * gv);
                if (dist <= tol || g < 1e-6) break;
                u = u - double(dist) * gu / g;
                v = v - double(dist) * gv / g;
            }
            d[0] = (u - pr.cx) * V[2] / pr.fx - V[0];
            d[1] = (v - pr.cy) * V[2] / pr.fy - V[1];
        }
    }
    for (int a = 0; a < 3; ++a) pr.p[0][size_t(a) * nv + i] = d[a];
    pr.ring[i] = snap ? 0 : rings + 1;
    if (snap) atomicAdd(pr.nsnap.ptr, 1);
}

// Ring distance r: a vertex farther than r with a neighbour at r - 1.
__global__ __launch_bounds__(kVThreads) void k_vring(const VertexDev *__restrict__ P, int r) {
    const VertexDev &pr = *P;
    const VTemplateDev &T = pr.T;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (i >= nv || pr.ring[i] <= r) return;
    for (int k = 0; k < T.K; ++k) {
        const int j = T.nbr[size_t(k) * nv + i];
        if (j < 0) break;
        if (pr.ring[j] == r - 1) {
            pr.ring[i] = r;
            return;
        }
    }
}

// One Jacobi sweep of the Laplacian warp: vertices of the band (ring 1..rings)
// take the mean of their neighbours' displacements; the others keep theirs.
__global__ __launch_bounds__(kVThreads) void k_vwarp(const VertexDev *__restrict__ P, int src, int rings) {
    const VertexDev &pr = *P;
    const VTemplateDev &T = pr.T;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (i >= nv) return;
    const gptr<double> a = pr.p[src], b = pr.p[src ^ 1];
    const int rg = pr.ring[i];
    double m[3];
    if (rg >= 1 && rg <= rings) {
        double s[3] = {0.0, 0.0, 0.0};
        int n = 0;
        for (int k = 0; k < T.K; ++k) {
            const int j = T.nbr[size_t(k) * nv + i];
            if (j < 0) break;
            for (int c = 0; c < 3; ++c) s[c] += a[size_t(c) * nv + j];
            ++n;
        }
        for (int c = 0; c < 3; ++c) m[c] = s[c] / n;
    } else {
        for (int c = 0; c < 3; ++c) m[c] = a[size_t(c) * nv + i];
    }
    for (int c = 0; c < 3; ++c) b[size_t(c) * nv + i] = m[c];
}

// The caller's positions: the final point plus the displacement in buffer src.
__global__ __launch_bounds__(kVThreads) void k_vsnap_apply(const VertexDev *__restrict__ P, int G, int src) {
    const VertexDev &pr = *P;
    const int nv = pr.nv, i = blockIdx.x * kVThreads + threadIdx.x;
    if (i >= nv) return;
    double V[3], xo[3];
    load3(pr.V[(G + 1) & 1], nv, i, V);
    load3(pr.x[(G + 1) & 1], nv, i, xo);
    for (int a = 0; a < 3; ++a) pr.Vout[size_t(a) * nv + i] = float((V[a] + xo[a]) + pr.p[src][size_t(a) * nv + i]);
}

namespace {

// Blur weights of kernel size k (odd, 1..15): sigma = 0.3 ((k - 1) / 2 - 1) + 0.8,
// normalised in float64, rounded to float32.
BlurW blur_weights(int k) {
    BlurW b{};
    b.r = (k - 1) / 2;
    const double sigma = 0.3 * ((k - 1) * 0.5 - 1.0) + 0.8;
    double w[kVMaxBlur], s = 0.0;
    for (int d = -b.r; d <= b.r; ++d) {
        w[d + b.r] = std::exp(-double(d) * d / (2.0 * sigma * sigma));
        s += w[d + b.r];
    }
    for (int q = 0; q < 2 * b.r + 1; ++q) b.w[q] = float(w[q] / s);
    return b;
}

struct VRun {
    Run R;                        // the decision kernels' problem (one frame)
    VertexDev vd{};
    VertexDev *dv = nullptr;
    int levels[kVLevels] = {0, 0, 0}, nlev = 0;
    int step_level[CAPTURE_MAX_GN] = {};
    float *blurred[kVLevels] = {nullptr, nullptr, nullptr};
    float *tmp = nullptr;
    bool part_mask = false;
    int part_dilation = 0;
};

int kernel_of(const capture_vertex_params *p, int g) { return p->blur_kernel[g] == 0 ? 3 : p->blur_kernel[g]; }

// Workspace: [ProbDev][VertexDev] then the image, vertex and solver buffers.
size_t carve_vertex(uint8_t *base, const capture_vertex_frame &f, int nlev, ProbDev &pr, VertexDev &vd,
                    float **blurred, float **tmp) {
    const TemplateDev &T = f.tmpl->topo->dev;
    const size_t nv = T.nv, nf = T.nf, hw = size_t(f.camera.width) * f.camera.height;
    const int nb = int(blocks(nv, kVThreads));
    Layout L;
    L.take<ProbDev>(base, 1);
    L.take<VertexDev>(base, 1);
    pr.dt = L.take<float>(base, hw);
    pr.colg = L.take<int>(base, hw);
    const size_t nseg = (size_t(f.camera.height) + 15) / 16 * size_t(f.camera.width);
    pr.seg_first = L.take<int>(base, nseg);
    pr.seg_last = L.take<int>(base, nseg);
    pr.zbuf = L.take<uint32_t>(base, hw);
    pr.contour = L.take<uint8_t>(base, hw);
    pr.dx = L.take<float>(base, 3 * nv);
    pr.duv = L.take<float>(base, 2 * nv);
    pr.dfix = L.take<int>(base, 2 * nv);
    pr.dvalid = L.take<uint8_t>(base, nv);
    pr.vcont = L.take<uint8_t>(base, nv);
    pr.vflags = L.take<uint8_t>(base, nv);
    pr.fcross = L.take<float>(base, 3 * nf);
    pr.bigq = L.take<int>(base, nf);
    pr.px = L.take<float>(base, 3 * nv);
    pr.vcode = L.take<uint8_t>(base, nv);
    pr.pva = L.take<float>(base, 3 * nv);
    pr.counts = L.take<int>(base, 3);
    for (int l = 0; l < nlev; ++l) blurred[l] = L.take<float>(base, 3 * hw);
    *tmp = L.take<float>(base, 3 * hw * size_t(nlev));       // horizontal passes of every level
    for (int q = 0; q < 2; ++q) {
        vd.V[q] = L.take<double>(base, 3 * nv);
        vd.x[q] = L.take<double>(base, 3 * nv);
        vd.p[q] = L.take<double>(base, 3 * nv);
    }
    vd.r = L.take<double>(base, 3 * nv);
    vd.u = L.take<double>(base, 3 * nv);
    vd.Ap = L.take<double>(base, 3 * nv);
    vd.dinv = L.take<double>(base, 3 * nv);
    vd.Hm = L.take<float>(base, 6 * nv);
    vd.ru = L.take<double>(base, 2 * size_t(nb));
    vd.pap = L.take<double>(base, blocks(nv * kRowLanes, kApplyThreads));
    vd.epart = L.take<double>(base, size_t(CAPTURE_MAX_GN + 1) * kVTerms * nb);
    vd.scal = L.take<double>(base, CAPTURE_MAX_GN + size_t(CAPTURE_MAX_GN + 1) * kVTerms + 3);
    vd.ring = L.take<int>(base, nv);
    vd.plab[0] = L.take<int>(base, hw);
    vd.plab[1] = L.take<int>(base, hw);
    vd.nsnap = L.take<int>(base, 1);
    return L.off;
}

int check_vertex_frame(const capture_vertex_frame *f) {
    if (!f || !f->tmpl) return fail(CAPTURE_EINVAL, "vertex frame without template");
    if (!f->posed || !f->rgb || !f->mask || !f->image || !f->V) return fail(CAPTURE_EINVAL, "vertex frame: null array");
    const capture_camera &c = f->camera;
    if (c.width < 1 || c.height < 1 || c.width > kMaxImageSide || c.height > kMaxImageSide)
        return fail(CAPTURE_EUNSUPPORTED, "camera: image sides must be in [1, 4096]");
    if (!std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy) || c.fx == 0.0f ||
        c.fy == 0.0f)
        return fail(CAPTURE_EINVAL, "camera: non-finite or zero intrinsics");
    return CAPTURE_OK;
}

// Distinct Gaussian kernels of the schedule, and each step's level.
int vertex_levels(const capture_vertex_params *p, int *levels, int &nlev, int *step_level) {
    nlev = 0;
    for (int g = 0; g < p->gn_iters; ++g) {
        const int k = kernel_of(p, g);
        if (k < 1 || k > kVMaxBlur || (k & 1) == 0) return fail(CAPTURE_EINVAL, "blur_kernel: odd sizes 1..15 (or 0)");
        int l = 0;
        while (l < nlev && levels[l] != k) ++l;
        if (l == nlev) {
            if (nlev == kVLevels) return fail(CAPTURE_EUNSUPPORTED, "at most 3 distinct blur kernels per solve");
            levels[nlev++] = k;
        }
        step_level[g] = l;
    }
    return CAPTURE_OK;
}

int check_vertex_params(const capture_vertex_params *p, const capture_vertex_frame *f) {
    if (!p) return fail(CAPTURE_EINVAL, "null params");
    if (p->gn_iters < 1 || p->gn_iters > CAPTURE_MAX_GN) return fail(CAPTURE_EINVAL, "gn_iters must be in [1, 32]");
    if (p->pcg_iters < 0) return fail(CAPTURE_EINVAL, "pcg_iters must be >= 0");
    const float w[6] = {p->w_photo, p->w_sil, p->w_smooth, p->w_edge, p->w_vel, p->w_acc};
    for (float x : w)
        if (!std::isfinite(x) || x < 0.0f) return fail(CAPTURE_EINVAL, "weights must be finite and non-negative");
    if (std::isnan(p->tau_color) || p->tau_color < 0.0f) return fail(CAPTURE_EINVAL, "tau_color must be >= 0");
    if (p->flags & ~uint32_t(CAPTURE_FLAG_EXCLUDE_CASE2 | CAPTURE_FLAG_OUTLINE_ONLY | CAPTURE_FLAG_PART_MASK))
        return fail(CAPTURE_EINVAL, "unknown flag bits");
    if ((p->flags & CAPTURE_FLAG_PART_MASK) && !f->tmpl->dev.parts)
        return fail(CAPTURE_EINVAL, "the body-part mask needs a template with part labels");
    if (p->part_dilation < 0 || p->part_dilation > 64) return fail(CAPTURE_EINVAL, "part_dilation must be in [0, 64]");
    if ((p->w_vel > 0.0f || p->w_acc > 0.0f) && !f->prev) return fail(CAPTURE_EINVAL, "temporal terms need prev");
    if (p->w_acc > 0.0f && !f->prev2) return fail(CAPTURE_EINVAL, "the acceleration term needs prev2");
    if (std::isnan(p->snap_max_px) || p->snap_max_px < 0.0f || p->snap_steps < 0 || p->snap_steps > 64 ||
        p->snap_rings < 0 || p->snap_rings > 16 || p->snap_iters < 0 || p->snap_iters > 1024)
        return fail(CAPTURE_EINVAL, "snapping: max_px >= 0, steps 0..64, rings 0..16, iters 0..1024");
    return CAPTURE_OK;
}

int vertex_setup(VRun &P, capture_ctx *ctx, const capture_vertex_frame *f, const capture_vertex_params *prm, void *ws,
                 size_t ws_bytes, void *stream) {
    int rc = check_vertex_frame(f);
    if (rc) return rc;
    if ((rc = check_vertex_params(prm, f))) return rc;
    if (f->tmpl->device != ctx->device) return fail(CAPTURE_EINVAL, "template belongs to another device");
    if ((rc = vertex_levels(prm, P.levels, P.nlev, P.step_level))) return rc;
    ProbDev pr{};
    VertexDev vd{};
    const size_t need = carve_vertex(nullptr, *f, P.nlev, pr, vd, P.blurred, &P.tmp);
    if (!ws || ws_bytes < need) return fail(CAPTURE_ENOMEM, "workspace too small");
    uint8_t *base = static_cast<uint8_t *>(ws);
    carve_vertex(base, *f, P.nlev, pr, vd, P.blurred, &P.tmp);
    const capture_vertex_template &vt = *f->tmpl;
    pr.T = vt.topo->dev;
    pr.xyz = f->posed;
    pr.rgb = nullptr;
    pr.mask = f->mask;
    pr.image = f->image;        // source of the blur levels
    pr.W = f->camera.width;
    pr.H = f->camera.height;
    pr.fx = f->camera.fx; pr.fy = f->camera.fy; pr.cx = f->camera.cx; pr.cy = f->camera.cy;
    pr.exclude_case2 = int(prm->flags & CAPTURE_FLAG_EXCLUDE_CASE2);
    pr.outline_only = int((prm->flags & CAPTURE_FLAG_OUTLINE_ONLY) != 0);
    pr.w_vel = 0.0f;
    pr.target = -INFINITY;
    vd.T = vt.dev;
    vd.nv = vt.dev.nv;
    vd.nb = int(blocks(vd.nv, kVThreads));
    vd.nba = int(blocks(size_t(vd.nv) * kRowLanes, kApplyThreads));
    vd.W = pr.W; vd.H = pr.H;
    vd.fx = pr.fx; vd.fy = pr.fy; vd.cx = pr.cx; vd.cy = pr.cy;
    vd.sw_photo = std::sqrt(prm->w_photo);
    vd.sw_sil = std::sqrt(prm->w_sil);
    vd.tau = prm->tau_color;
    vd.w_smooth = prm->w_smooth;
    vd.w_edge = prm->w_edge;
    vd.w_vel = prm->w_vel;
    vd.w_acc = prm->w_acc;
    vd.posed = f->posed;
    vd.prev = f->prev;
    vd.prev2 = f->prev2;
    vd.rgb = f->rgb;
    vd.dt = pr.dt;
    vd.vflags = pr.vflags;
    vd.Vout = f->V;
    P.part_mask = (prm->flags & CAPTURE_FLAG_PART_MASK) != 0;
    P.part_dilation = prm->part_dilation;
    Run &R = P.R;
    R.ctx = ctx;
    R.prof = &ctx->prof;
    R.n = 1;
    R.probs.resize(1);
    R.probs[0] = pr;
    R.dprobs = reinterpret_cast<ProbDev *>(base);
    R.s = static_cast<hipStream_t>(stream);
    P.vd = vd;
    P.dv = reinterpret_cast<VertexDev *>(base + ((sizeof(ProbDev) + 255) & ~size_t(255)));
    // both descriptors in one upload from the context's pinned staging
    const size_t voff = reinterpret_cast<uint8_t *>(P.dv) - reinterpret_cast<uint8_t *>(R.dprobs);
    uint8_t *stage = static_cast<uint8_t *>(run_staging(R, voff + sizeof(VertexDev)));
    if (!stage) return fail(CAPTURE_ENOMEM, "host staging allocation failed");
    std::memcpy(stage, &R.probs[0], sizeof(ProbDev));
    std::memcpy(stage + voff, &P.vd, sizeof(VertexDev));
    CAP_HIP(hipMemcpyAsync(R.dprobs, stage, voff + sizeof(VertexDev), hipMemcpyHostToDevice, R.s));
    return CAPTURE_OK;
}

// Start geometry, distance transform, blur levels, raster and decisions.
int launch_vertex_decisions(VRun &P) {
    Run &R = P.R;
    hipStream_t s = R.s;
    const ProbDev &pr = R.probs[0];
    const size_t hw = size_t(pr.W) * pr.H;
    const int nv = pr.T.nv;
    // the start geometry (which also zeroes the counters and, in blocks of
    // its own, the depth buffer); contour pixels and column segments; then, as in the
    // deformation-graph path, steps with the same predecessors share a launch
    // (rasterisation + segment scan, large faces + column distances, row pass
    // + contour edges)
    timed(R, K_DEFORM, [&] {
        const int nbv = int(blocks(nv, kVThreads));
        hipLaunchKernelGGL(k_vstart, dim3(nbv + int(blocks(hw, kZbufPerBlock))), dim3(kVThreads), 0, s, P.dv, R.dprobs,
                           nbv);
    });
    const dim3 gpx(blocks(hw, 256));
    timed(R, K_CONTOUR, [&] { hipLaunchKernelGGL(k_contour, gpx, dim3(256), 0, s, R.dprobs); });
    const size_t nsegw = size_t(pr.W) * ((pr.H + 15) / 16);
    const int nb_seg = int(blocks(nsegw, 256)), nb_f = int(blocks(pr.T.nf, 256)), nb_me = int(blocks(pr.T.nmedges, 256));
    timed(R, K_DT_COLS, [&] { hipLaunchKernelGGL(k_dt_seg, dim3(nb_seg), dim3(256), 0, s, R.dprobs); });
    timed(R, K_PREP_RASTER, [&] {
        hipLaunchKernelGGL(k_prep_raster, dim3(nb_f + int(blocks(pr.W, 4))), dim3(256), 0, s, R.dprobs, nb_f, 1);
    });
    timed(R, K_PREP_COLS, [&] {
        hipLaunchKernelGGL(k_prep_cols, dim3(kRasterBigBlocks + nb_seg), dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_DT_ROWS, [&] {
        hipLaunchKernelGGL(k_prep_rows, dim3(pr.H + nb_me), dim3(256), dt_rows_lds(pr.W), s, R.dprobs, pr.H);
    });
    timed(R, K_V_BLUR, [&] {
        BlurSet bs{};
        BlurOut bo{};
        bs.n = P.nlev;
        for (int l = 0; l < P.nlev; ++l) {
            const BlurW bw = blur_weights(P.levels[l]);
            bs.r[l] = bw.r;
            for (int q = 0; q < kVMaxBlur; ++q) bs.w[l][q] = bw.w[q];
            bo.p[l] = P.blurred[l];
        }
        hipLaunchKernelGGL(k_vblur_h, dim3(blocks(pr.W, 256), pr.H), dim3(256), 0, s, R.dprobs, P.tmp, pr.W, pr.H, bs);
        hipLaunchKernelGGL(k_vblur_v, dim3(blocks(pr.W, kBlurTileW), blocks(pr.H, kBlurTileH), P.nlev), dim3(256), 0,
                           s, static_cast<const float *>(P.tmp), bo, pr.W, pr.H, bs);
    });
    timed(R, K_DECIDE, [&] { hipLaunchKernelGGL(k_decide, dim3(blocks(nv, 256)), dim3(256), 0, s, R.dprobs); });
    if (P.part_mask) {
        int *a = P.vd.plab[0].ptr, *b = P.vd.plab[1].ptr;
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks(hw, 256)), dim3(256), 0, s, reinterpret_cast<uint32_t *>(a), hw,
                           uint32_t(kNoPart));
        hipLaunchKernelGGL(k_part_labels, dim3(blocks(pr.T.nf, 256)), dim3(256), 0, s, R.dprobs,
                           static_cast<const int *>(P.vd.T.parts.ptr), a);
        hipLaunchKernelGGL(k_part_labels_big, dim3(kRasterBigBlocks), dim3(256), 0, s, R.dprobs,
                           static_cast<const int *>(P.vd.T.parts.ptr), a);
        for (int k = 0; k < P.part_dilation; ++k) {
            hipLaunchKernelGGL(k_part_dilate, gpx, dim3(256), 0, s, static_cast<const int *>(a), b, pr.W, pr.H);
            std::swap(a, b);
        }
        hipLaunchKernelGGL(k_part_mask, dim3(P.vd.nb), dim3(kVThreads), 0, s, P.dv, R.dprobs,
                           static_cast<const int *>(a));
    }
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

void launch_vlin(VRun &P, int g, int level, int mode) {
    Run &R = P.R;
    timed(R, K_V_LIN, [&] {
        hipLaunchKernelGGL(k_vlin, dim3(P.vd.nb), dim3(kVThreads), 0, R.s, P.dv,
                           static_cast<const float *>(P.blurred[level]), g, mode);
    });
}

// The whole solve: decisions, then per step the linearisation and the PCG
// iterations, then the final energies and their per-step sums.
int launch_vertex_solve(VRun &P, const capture_vertex_params *prm) {
    int rc = launch_vertex_decisions(P);
    if (rc) return rc;
    Run &R = P.R;
    const int G = prm->gn_iters, nb = P.vd.nb;
    for (int g = 0; g < G; ++g) {
        launch_vlin(P, g, P.step_level[g], 0);
        for (int j = 0; j < prm->pcg_iters; ++j) {
            timed(R, K_V_APPLY, [&] {
                hipLaunchKernelGGL(k_vapply, dim3(P.vd.nba), dim3(kApplyThreads), 0, R.s, P.dv, g, j, 0);
            });
            timed(R, K_V_UPDATE, [&] { hipLaunchKernelGGL(k_vupdate, dim3(nb), dim3(kVThreads), 0, R.s, P.dv, g, j); });
        }
    }
    launch_vlin(P, G, P.step_level[G - 1], 1);      // (also zeroes the snapped count)
    if (prm->snap_max_px > 0.0f) {
        const float tol = 0.05f;
        timed(R, K_V_SNAP, [&] {
            hipLaunchKernelGGL(k_vsnap, dim3(nb), dim3(kVThreads), 0, R.s, P.dv, G, prm->snap_steps, prm->snap_max_px,
                               tol, prm->snap_rings);
            for (int r = 1; r <= prm->snap_rings; ++r)
                hipLaunchKernelGGL(k_vring, dim3(nb), dim3(kVThreads), 0, R.s, P.dv, r);
            for (int it = 0; it < prm->snap_iters; ++it)
                hipLaunchKernelGGL(k_vwarp, dim3(nb), dim3(kVThreads), 0, R.s, P.dv, it & 1, prm->snap_rings);
            hipLaunchKernelGGL(k_vsnap_apply, dim3(nb), dim3(kVThreads), 0, R.s, P.dv, G, prm->snap_iters & 1);
        });
    }
    hipLaunchKernelGGL(k_vreport, dim3(1), dim3(256), 0, R.s, P.dv, R.probs[0].counts.ptr, G);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

// One-ring table (ELL) of a mesh with Table 1 weights and rest lengths.
int build_vertex_tables(const std::vector<int> &tri, const std::vector<float> &rest, const std::vector<int> &cls,
                        int nv, int nf, int &K, std::vector<int> &nbr, std::vector<float> &ek,
                        std::vector<float> &ea, std::vector<float> &elen) {
    std::vector<std::vector<int>> ring(nv);
    for (int f = 0; f < nf; ++f)
        for (int e = 0; e < 3; ++e) {
            const int a = tri[size_t(e) * nf + f], b = tri[size_t((e + 1) % 3) * nf + f];
            ring[a].push_back(b);
            ring[b].push_back(a);
        }
    K = 1;
    for (auto &r : ring) {
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        K = std::max<int>(K, int(r.size()));
    }
    if (K > CAPTURE_VERTEX_MAX_RING) return fail(CAPTURE_EUNSUPPORTED, "vertex template: one-ring larger than 32");
    nbr.assign(size_t(K) * nv, -1);
    ek.assign(size_t(K) * nv, 0.0f);
    ea.assign(size_t(K) * nv, 0.0f);
    elen.assign(size_t(K) * nv, 0.0f);
    for (int i = 0; i < nv; ++i) {
        const double di = double(ring[i].size());
        for (size_t k = 0; k < ring[i].size(); ++k) {
            const int j = ring[i][k];
            const double sij = 0.5 * (kTable1[cls[i] - 1] + kTable1[cls[j] - 1]);
            const double dj = double(ring[j].size());
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = double(rest[size_t(a) * nv + i]) - double(rest[size_t(a) * nv + j]);
                d2 += d * d;
            }
            const size_t o = k * nv + i;
            nbr[o] = j;
            ek[o] = float(sij / di);
            ea[o] = float(sij / di + sij / dj);
            elen[o] = float(std::sqrt(d2));
        }
    }
    return CAPTURE_OK;
}

template <class T>
int copy_down_v(std::vector<T> &h, const T *d, size_t n) {
    h.resize(n);
    CAP_HIP(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
    return CAPTURE_OK;
}

}  // namespace
}  // namespace cap

using namespace cap;

extern "C" {

int capture_vertex_template_create(capture_ctx *ctx, const capture_vertex_template_desc *d,
                                   capture_vertex_template **out) {
    if (!ctx || !d || !out) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    const int nv = d->n_vertices, nf = d->n_triangles;
    if (nv < 2 || nf < 1) return fail(CAPTURE_EINVAL, "vertex template: need n_vertices >= 2 and n_triangles >= 1");
    if (nv > (1 << 26)) return fail(CAPTURE_EUNSUPPORTED, "vertex template: too many vertices");
    if (!d->tri || !d->rest || !d->classes) return fail(CAPTURE_EINVAL, "vertex template: null array");
    std::vector<int> tri, cls, parts;
    std::vector<float> rest;
    int rc;
    if ((rc = copy_down_v(tri, d->tri, size_t(3) * nf)) || (rc = copy_down_v(cls, d->classes, size_t(nv))) ||
        (rc = copy_down_v(rest, d->rest, size_t(3) * nv)))
        return rc;
    if (d->parts) {
        if ((rc = copy_down_v(parts, d->parts, size_t(nv)))) return rc;
        for (int q : parts) if (q < 0 || q >= 1 << 20) return fail(CAPTURE_EINVAL, "vertex template: part labels 0..2^20-1");
    }
    for (int v : tri) if (v < 0 || v >= nv) return fail(CAPTURE_EINVAL, "vertex template: triangle index out of range");
    for (int c : cls) if (c < 1 || c > 7) return fail(CAPTURE_EINVAL, "vertex template: material class outside 1..7");
    for (float x : rest) if (!std::isfinite(x)) return fail(CAPTURE_ENONFINITE, "vertex template: non-finite rest position");
    capture_template *topo = nullptr;
    if ((rc = build_topology_template(d->tri, nv, nf, &topo, ctx->device))) return rc;     // manifold check
    int K = 0;
    std::vector<int> nbr;
    std::vector<float> ek, ea, elen;
    if ((rc = build_vertex_tables(tri, rest, cls, nv, nf, K, nbr, ek, ea, elen))) {
        capture_template_destroy(topo);
        return rc;
    }
    const size_t b_n = sizeof(int) * nbr.size(), b_f = sizeof(float) * ek.size(), b_p = sizeof(int) * parts.size();
    void *mem = nullptr;
    if (hipMalloc(&mem, b_n + 3 * b_f + b_p) != hipSuccess) {
        capture_template_destroy(topo);
        return fail(CAPTURE_ENOMEM, "vertex template: device allocation failed");
    }
    uint8_t *m = static_cast<uint8_t *>(mem);
    if (hipMemcpy(m, nbr.data(), b_n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + b_n, ek.data(), b_f, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + b_n + b_f, ea.data(), b_f, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + b_n + 2 * b_f, elen.data(), b_f, hipMemcpyHostToDevice) != hipSuccess ||
        (b_p && hipMemcpy(m + b_n + 3 * b_f, parts.data(), b_p, hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(mem);
        capture_template_destroy(topo);
        return fail(CAPTURE_EHIP, "vertex template: upload failed");
    }
    capture_vertex_template *t = new capture_vertex_template{};
    t->dev.nv = nv;
    t->dev.K = K;
    t->dev.nbr = reinterpret_cast<const int *>(m);
    t->dev.ek = reinterpret_cast<const float *>(m + b_n);
    t->dev.ea = reinterpret_cast<const float *>(m + b_n + b_f);
    t->dev.elen = reinterpret_cast<const float *>(m + b_n + 2 * b_f);
    t->dev.parts = b_p ? reinterpret_cast<const int *>(m + b_n + 3 * b_f) : nullptr;
    t->topo = topo;
    t->mem = mem;
    t->device = ctx->device;
    *out = t;
    return CAPTURE_OK;
}

void capture_vertex_template_destroy(capture_vertex_template *t) {
    if (!t) return;
    (void)hipSetDevice(t->device);
    (void)hipFree(t->mem);
    capture_template_destroy(t->topo);
    delete t;
}

int capture_vertex_workspace_size(capture_ctx *ctx, const capture_vertex_frame *f, const capture_vertex_params *prm,
                                  size_t *bytes) {
    if (!ctx || !bytes) return fail(CAPTURE_EINVAL, "null argument");
    int rc = check_vertex_frame(f);
    if (rc) return rc;
    if ((rc = check_vertex_params(prm, f))) return rc;
    int levels[kVLevels], nlev = 0, step_level[CAPTURE_MAX_GN];
    if ((rc = vertex_levels(prm, levels, nlev, step_level))) return rc;
    ProbDev pr{};
    VertexDev vd{};
    float *bl[kVLevels], *tmp;
    *bytes = carve_vertex(nullptr, *f, nlev, pr, vd, bl, &tmp);
    return CAPTURE_OK;
}

int capture_vertex_solve(capture_ctx *ctx, const capture_vertex_frame *f, const capture_vertex_params *prm,
                         capture_vertex_report *rep, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx || !rep) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    VRun P;
    int rc = vertex_setup(P, ctx, f, prm, ws, ws_bytes, stream);
    if (rc) return rc;
    if (ctx->graphs && !ctx->prof.on) {
        // every kernel argument is a workspace address or a size: the key
        std::string key = "vertex|";
        char buf[256];
        std::snprintf(buf, sizeof buf, "%p|%p|%d %d|%d %d|", (void *)P.R.dprobs, (const void *)f->tmpl,
                      f->camera.width, f->camera.height, prm->gn_iters, prm->pcg_iters);
        key += buf;
        for (int g = 0; g < prm->gn_iters; ++g) key += std::to_string(kernel_of(prm, g)) + ",";
        std::snprintf(buf, sizeof buf, "|%a %d %d %d|%u %d", double(prm->snap_max_px), prm->snap_steps,
                      prm->snap_rings, prm->snap_iters, prm->flags, prm->part_dilation);
        key += buf;
        rc = launch_graph(P.R, key, [&](Run &C) {
            VRun Q = P;
            Q.R = C;
            return launch_vertex_solve(Q, prm);
        });
    } else {
        rc = launch_vertex_solve(P, prm);
    }
    if (rc) return rc;
    const int G = prm->gn_iters;
    // the energies of every step, then the visible, contour and snapped
    // counts, in one read-back into the context's pinned staging (the
    // descriptor upload from it precedes this copy on the stream)
    const size_t nrep = size_t(G + 1) * kVTerms + 3;
    const double *en = static_cast<const double *>(run_staging(P.R, sizeof(double) * nrep));
    if (!en) return fail(CAPTURE_ENOMEM, "host staging allocation failed");
    hipStream_t s = P.R.s;
    CAP_HIP(hipMemcpyAsync(const_cast<double *>(en), P.vd.scal.ptr + CAPTURE_MAX_GN, sizeof(double) * nrep,
                           hipMemcpyDeviceToHost, s));
    CAP_HIP(hipStreamSynchronize(s));
    settle(P.R);
    const int counts[2] = {int(en[nrep - 3]), int(en[nrep - 2])}, nsnap = int(en[nrep - 1]);
    *rep = capture_vertex_report{};
    bool finite = true;
    for (int g = 0; g <= G; ++g) {
        const double *e = en + size_t(g) * kVTerms;
        rep->energy[g] = ((((e[0] + e[1]) + e[3]) + e[4]) + e[5]) + e[6];
        finite = finite && std::isfinite(rep->energy[g]);
    }
    const double *e = en + size_t(G) * kVTerms;
    rep->e_photo = e[0];
    rep->e_sil = e[1];
    rep->e_sil_abs = e[2];
    rep->e_smooth = e[3];
    rep->e_edge = e[4];
    rep->e_vel = e[5];
    rep->e_acc = e[6];
    rep->n_visible = counts[0];
    rep->n_boundary = counts[1];
    rep->gn_done = G;
    rep->n_snapped = nsnap;
    rep->status = finite ? CAPTURE_OK : CAPTURE_ENONFINITE;
    if (!finite) return fail(CAPTURE_ENONFINITE, "non-finite energy in the per-vertex solve");
    return CAPTURE_OK;
}

int capture_vertex_linearize(capture_ctx *ctx, const capture_vertex_frame *f, const capture_vertex_params *prm,
                             double *rhs, double *diag, const double *p, double *Ap, double *energy, uint8_t *vflags,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    VRun P;
    int rc = vertex_setup(P, ctx, f, prm, ws, ws_bytes, stream);
    if (rc) return rc;
    P.vd.rhs_out = rhs;
    P.vd.diag_out = diag;
    Run &R = P.R;
    hipStream_t s = R.s;
    CAP_HIP(hipMemcpyAsync(P.dv, &P.vd, sizeof(VertexDev), hipMemcpyHostToDevice, s));
    if ((rc = launch_vertex_decisions(P))) return rc;
    launch_vlin(P, 0, P.step_level[0], 2);
    const int nv = P.vd.nv;
    if (p && Ap) {
        // the product of the given direction: p is copied into u (iteration 0 multiplies p = u)
        CAP_HIP(hipMemcpyAsync(P.vd.u.ptr, p, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_vapply, dim3(P.vd.nba), dim3(kApplyThreads), 0, s, P.dv, 0, 0, 1);
        CAP_HIP(hipMemcpyAsync(Ap, P.vd.Ap.ptr, sizeof(double) * 3 * nv, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_vreport, dim3(1), dim3(256), 0, s, P.dv, R.probs[0].counts.ptr, 0);
    if (vflags) CAP_HIP(hipMemcpyAsync(vflags, R.probs[0].vflags, nv, hipMemcpyDeviceToDevice, s));
    double en[kVTerms];
    CAP_HIP(hipMemcpyAsync(en, P.vd.scal.ptr + CAPTURE_MAX_GN, sizeof(en), hipMemcpyDeviceToHost, s));
    CAP_HIP(hipGetLastError());
    CAP_HIP(hipStreamSynchronize(s));
    settle(R);
    if (energy)
        for (int q = 0; q < kVTerms; ++q) energy[q] = en[q];
    return CAPTURE_OK;
}

}  // extern "C"
