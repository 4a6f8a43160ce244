// Pose stage kernels (Sec. 3.3 energy, Sec. 4 pose solver): forward
// kinematics, linear-blend skinning of the start pose, Jacobian rows of the
// 2D, 3D and silhouette terms, J^T J on FP64 MFMA tiles and the dense
// Cholesky Gauss-Newton step in one workgroup.
//
// Unknowns: 3 axis-angle values per rotating joint (joint order), the root
// translation t, and the translation t' that maps the root-relative 3D
// detections into the camera frame.  R_j = R_parent(j) Exp(theta_j),
// p_j = p_parent + R_parent (J_j - J_parent), p_root = J_root + t.
// The derivative of a point y carried by joint k's rotation is
// -[y - p_k]x R_parent(k) J_l(theta_k) (left Jacobian of Exp).
//
// Exp and J_l use the series sin(x)/x, (1 - cos x)/x^2, (x - sin x)/x^3 in
// x = |w|^2, each evaluated by nested steps S <- 1 - (x / (k (k + 1))) S with a
// fixed number of terms, so the FP64 rotations do not depend on a libm.
#include "device.hpp"

namespace cap {

constexpr int kExpTerms = 24;

__device__ inline double exp_series(double x, int first) {
    double s = 1.0;
#pragma unroll
    for (int n = kExpTerms; n >= 1; --n) {
        const int k = first + 2 * (n - 1);
        s = 1.0 - (x * (1.0 / double(k * (k + 1)))) * s;    // a reciprocal per term (a constant once unrolled)
    }
    return s;
}

// Local rotation Exp(w) (or J_l(w) with `jac`), row-major.
__device__ inline void exp_or_jl(const double w[3], bool jac, double out[9]) {
    const double x = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    double c1, c2;
    if (!jac) {
        c1 = exp_series(x, 2);
        c2 = 0.5 * exp_series(x, 3);
    } else {
        c1 = 0.5 * exp_series(x, 3);
        c2 = exp_series(x, 4) / 6.0;
    }
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double kk = w[a] * w[b] - (a == b ? x : 0.0);
            out[3 * a + b] = ((a == b ? 1.0 : 0.0) + c1 * K[3 * a + b]) + c2 * kk;
        }
}

__device__ inline void mat3(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = (A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j]) + A[3 * i + 2] * B[6 + j];
}

// Forward kinematics by the whole block: local Exp / J_l per joint in
// parallel, then composition level by level down the tree.  Results go to
// LDS (sR, sp, sA: [nj][9], [nj][3], [nj][9]).
__device__ __forceinline__ void fk_block(const BodyDev &B, const double *pose, double *sR, double *sp, double *sA, double *sL,
                         double *sJ) {
    const int nj = B.nj, t = threadIdx.x, maxdepth = B.maxdepth;
    // this joint's tables in registers up front (one round of loads), so the
    // depth sweep below touches only LDS
    int depth = -1, par = -1;
    double off[3] = {0.0, 0.0, 0.0}, root[3] = {0.0, 0.0, 0.0};
    if (t < nj) {
        depth = B.depth[t];
        par = B.parent[t];
        for (int a = 0; a < 3; ++a) {
            const double rt = B.rest[a][t];
            off[a] = par >= 0 ? rt - B.rest[a][par] : 0.0;
            root[a] = par < 0 ? rt + pose[B.it + a] : 0.0;
        }
    }
    if (t < nj) {
        const int c = B.col[t];
        if (c >= 0) {
            const double w[3] = {pose[c], pose[c + 1], pose[c + 2]};
            exp_or_jl(w, false, sL + 9 * t);
            exp_or_jl(w, true, sJ + 9 * t);
        } else {
            for (int e = 0; e < 9; ++e) {
                sL[9 * t + e] = (e % 4 == 0) ? 1.0 : 0.0;
                sJ[9 * t + e] = 0.0;
            }
        }
    }
    __syncthreads();
    for (int d = 0; d <= maxdepth; ++d) {
        if (depth == d) {
            if (par < 0) {
                for (int e = 0; e < 9; ++e) {
                    sR[9 * t + e] = sL[9 * t + e];
                    sA[9 * t + e] = sJ[9 * t + e];
                }
                for (int a = 0; a < 3; ++a) sp[3 * t + a] = root[a];
            } else {
                mat3(sR + 9 * par, sL + 9 * t, sR + 9 * t);
                mat3(sR + 9 * par, sJ + 9 * t, sA + 9 * t);
                const double *Rp = sR + 9 * par;
                for (int a = 0; a < 3; ++a)
                    sp[3 * t + a] = sp[3 * par + a] + ((Rp[3 * a] * off[0] + Rp[3 * a + 1] * off[1]) + Rp[3 * a + 2] * off[2]);
            }
        }
        __syncthreads();
    }
}

__device__ inline void fk_store(const PoseDev &P, const double *sR, const double *sp, const double *sA) {
    const int nj = P.B.nj;
    for (int e = threadIdx.x; e < 9 * nj; e += blockDim.x) {
        P.jR[e] = sR[e];
        P.jA[e] = sA[e];
    }
    for (int e = threadIdx.x; e < 3 * nj; e += blockDim.x) P.jp[e] = sp[e];
}

// Start of a solve: keep the start pose, clear the status, kinematics at it.
__global__ __launch_bounds__(64) void k_pose_fk(const PoseDev *__restrict__ PP) {
    const PoseDev &P = *PP;
    __shared__ double sR[9 * kMaxJoints], sp[3 * kMaxJoints], sA[9 * kMaxJoints], sL[9 * kMaxJoints],
        sJ[9 * kMaxJoints];
    for (int e = threadIdx.x; e < P.B.nu; e += blockDim.x) P.pose0[e] = P.pose[e];
    if (threadIdx.x == 0) P.status[0] = 0;
    fk_block(P.B, P.pose, sR, sp, sA, sL, sJ);
    fk_store(P, sR, sp, sA);
}

// Linear blend skinning of the start pose, float32 recipe:
// d = v - J_j; q_a = (R_a0 d0 + R_a1 d1) + R_a2 d2; acc_a = acc_a + w (q_a + p_j,a).
// Blocks from nbv on clear the depth buffer instead (2,048 pixels each).
__global__ __launch_bounds__(256) void k_pose_lbs(const PoseDev *__restrict__ PP, const ProbDev *__restrict__ PR,
                                                  int nbv) {
    if (int(blockIdx.x) >= nbv) {
        const size_t hw = size_t(PR->W) * PR->H, q0 = size_t(blockIdx.x - nbv) * 2048 + threadIdx.x;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q0 + size_t(u) * 256 < hw) PR->zbuf[q0 + size_t(u) * 256] = 0u;
        return;
    }
    const PoseDev &P = *PP;
    const BodyDev &B = P.B;
    if (blockIdx.x == 0 && threadIdx.x < 3) PR->counts[threadIdx.x] = 0;     // visible, contour, large-face queue
    __shared__ float sR[9 * kMaxJoints], sp[3 * kMaxJoints], sJ[3 * kMaxJoints];
    for (int e = threadIdx.x; e < 9 * B.nj; e += blockDim.x) sR[e] = float(P.jR[e]);
    for (int e = threadIdx.x; e < 3 * B.nj; e += blockDim.x) {
        sp[e] = float(P.jp[e]);
        sJ[e] = float(B.rest[e % 3][e / 3]);
    }
    __syncthreads();
    const int nv = B.nv;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const float v[3] = {B.xyz[i], B.xyz[nv + i], B.xyz[2 * nv + i]};
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int s = 0; s < 4; ++s) {
        const int j = B.bind_joint[size_t(s) * nv + i];
        const float w = B.bind_w[size_t(s) * nv + i];
        const float d[3] = {v[0] - sJ[3 * j], v[1] - sJ[3 * j + 1], v[2] - sJ[3 * j + 2]};
        for (int a = 0; a < 3; ++a) {
            const float *R = sR + 9 * j + 3 * a;
            const float q = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
            acc[a] = acc[a] + w * (q + sp[3 * j + a]);
        }
    }
    store_start_vertex(*PR, i, acc[0], acc[1], acc[2]);
}

// Contour set B as an ascending list, by one block: entry (vertex << 1) |
// (b_i == -1).  The vertices go in rounds of kListBatch chunks of 1,024, each
// round's flags loaded together; wave ballots count each chunk's entries per
// wave, and after one barrier every thread adds the counts before its own
// (earlier chunks, then earlier waves of its chunk) to place its entries.
constexpr int kListBatch = 8;
__global__ __launch_bounds__(1024) void k_pose_list(const PoseDev *__restrict__ PP) {
    const PoseDev &P = *PP;
    const int nv = P.B.nv;
    __shared__ int wsum[kListBatch][16];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int span = kListBatch * int(blockDim.x);
    for (int c0 = 0; c0 < nv; c0 += span) {
        uint8_t f[kListBatch];
#pragma unroll
        for (int u = 0; u < kListBatch; ++u) {
            const int i = c0 + u * int(blockDim.x) + int(threadIdx.x);
            f[u] = i < nv ? P.vflags[i] : 0;
        }
        int before[kListBatch];
#pragma unroll
        for (int u = 0; u < kListBatch; ++u) {
            const unsigned long long m = __ballot((f[u] & 2) != 0);
            before[u] = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wsum[u][wid] = __popcll(m);
        }
        __syncthreads();          // (also orders base's first store before its reads)
        int run = base;
#pragma unroll
        for (int u = 0; u < kListBatch; ++u) {
            int cw = 0;
            for (int w = 0; w < nw; ++w) {
                if (w == wid) before[u] += run + cw;
                cw += wsum[u][w];
            }
            run += cw;
        }
#pragma unroll
        for (int u = 0; u < kListBatch; ++u)
            if (f[u] & 2) P.blist[before[u]] = ((c0 + u * int(blockDim.x) + int(threadIdx.x)) << 1) | ((f[u] & 4) ? 1 : 0);
        __syncthreads();          // every thread has read base and wsum
        if (threadIdx.x == 0) base = run;
        __syncthreads();
    }
    if (threadIdx.x == 0) P.nb[0] = base;
}

// Cubic convolution (a = -0.5) value and gradient at (u, v), FP64, clamp-to-edge.
__device__ inline double sample_cubic_f64(const CAP_GLOBAL float *__restrict__ img, int W, int H, double u, double v, double &gu,
                                          double &gv) {
    u = fmin(fmax(u, -1.0e6), 1.0e6);
    v = fmin(fmax(v, -1.0e6), 1.0e6);
    const double fu = floor(u), fv = floor(v);
    const int ix = int(fu), iy = int(fv);
    double wx[4], dx[4], wy[4], dy[4];
    const double f[2] = {u - fu, v - fv};
    for (int ax = 0; ax < 2; ++ax) {
        const double t = f[ax], t2 = t * t, t3 = t2 * t;
        double *w = ax ? wy : wx, *d = ax ? dy : dx;
        w[0] = ((2.0 * t2 - t3) - t) * 0.5;
        w[1] = ((3.0 * t3 - 5.0 * t2) + 2.0) * 0.5;
        w[2] = ((4.0 * t2 - 3.0 * t3) + t) * 0.5;
        w[3] = (t3 - t2) * 0.5;
        d[0] = ((4.0 * t - 3.0 * t2) - 1.0) * 0.5;
        d[1] = (9.0 * t2 - 10.0 * t) * 0.5;
        d[2] = ((8.0 * t - 9.0 * t2) + 1.0) * 0.5;
        d[3] = (3.0 * t2 - 2.0 * t) * 0.5;
    }
    double val = 0.0, gx = 0.0, gy = 0.0;
    for (int m = 0; m < 4; ++m) {
        const CAP_GLOBAL float *row = img + size_t(min(max(iy + m - 1, 0), H - 1)) * W;
        double rx = 0.0, rv = 0.0;
        for (int n = 0; n < 4; ++n) {
            const double t = row[min(max(ix + n - 1, 0), W - 1)];
            rx += dx[n] * t;
            rv += wx[n] * t;
        }
        gx += wy[m] * rx;
        gy += dy[m] * rv;
        val += wy[m] * rv;
    }
    gu = gx;
    gv = gy;
    return val;
}

// Row entries of g . dY/dtheta for the rotating joints in `mask`, with
// dsum(k) = sum over carried points of weight * (y - p_k).  Written for every
// unknown column of the row (zeros elsewhere) except t, t' and the F column.
__device__ inline void rotation_entries(const BodyDev &B, CAP_GLOBAL double *row, size_t ld, const double g[3], const double *sp,
                                        const double *sA, const double (*ys)[3], const double *ws,
                                        const uint32_t *masks, int npts) {
    for (int k = 0; k < B.nj; ++k) {
        const int c = B.col[k];
        if (c < 0) continue;
        double d[3] = {0.0, 0.0, 0.0};
        bool any = false;
        for (int s = 0; s < npts; ++s)
            if (masks[s] >> k & 1u) {
                any = true;
                for (int a = 0; a < 3; ++a) d[a] += ws[s] * (ys[s][a] - sp[3 * k + a]);
            }
        if (!any) {
            row[c * ld] = row[(c + 1) * ld] = row[(c + 2) * ld] = 0.0;
            continue;
        }
        const double e[3] = {d[1] * g[2] - d[2] * g[1], d[2] * g[0] - d[0] * g[2], d[0] * g[1] - d[1] * g[0]};
        const double *A = sA + 9 * k;
        for (int cc = 0; cc < 3; ++cc) row[(c + cc) * ld] = (e[0] * A[cc] + e[1] * A[3 + cc]) + e[2] * A[6 + cc];
    }
}

// One Jacobian row per thread: 2 per joint (2D), 3 per joint (3D), 3 per joint
// (temporal stabilisation), one per rotational unknown (joint limits), one per
// contour vertex (silhouette).  Column nu holds b * F.  With energy_only the
// rows are not written.  Per-block energy partials go to epart.
__global__ __launch_bounds__(kPoseRowThreads) void k_pose_rows(const PoseDev *__restrict__ PP, int energy_only) {
    const PoseDev &P = *PP;
    const BodyDev &B = P.B;
    __shared__ double sR[9 * kMaxJoints], sp[3 * kMaxJoints], sA[9 * kMaxJoints];
    __shared__ double red[kPoseRowThreads / 64];
    for (int e = threadIdx.x; e < 9 * B.nj; e += blockDim.x) {
        sR[e] = P.jR[e];
        sA[e] = P.jA[e];
    }
    for (int e = threadIdx.x; e < 3 * B.nj; e += blockDim.x) sp[e] = P.jp[e];
    __syncthreads();
    const int nj = B.nj, nu = B.nu, np_ = B.np;
    const size_t ldr = P.ldr;
    const int nfix = pose_fixed_rows(nj, B.it);
    const int M = nfix + P.nb[0];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double en[kPoseTerms] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (r >= 8 * nj && r < nfix) {
        // joint-limit barrier on rotational unknown q: one entry in the row
        const int q = r - 8 * nj;
        const double th = P.pose[q], lo = P.lim_lo[q], hi = P.lim_hi[q];
        const double jq = th > hi ? P.sanat : (th < lo ? -P.sanat : 0.0);
        const double F = th > hi ? P.sanat * (th - hi) : (th < lo ? P.sanat * (lo - th) : 0.0);
        en[5] = F * F;
        if (!energy_only) {
            CAP_GLOBAL double *row = P.rows.g() + r;
            for (int c = 0; c < np_; ++c) row[c * ldr] = c == q ? jq : (c == nu ? F : 0.0);
        }
    } else if (r < M) {
        CAP_GLOBAL double *row = P.rows.g() + r;      // column-major: entry c at row[c * ldr]
        double g[3], F;
        double ys[4][3], ws[4];
        uint32_t masks[4];
        int npts = 1;
        double tw;                    // weight of the root translation columns
        bool has_tp = false;
        int tpc = 0;
        if (r < 8 * nj) {
            const bool is2d = r < 2 * nj, istemp = r >= 5 * nj;
            const int j = is2d ? r >> 1 : (istemp ? (r - 5 * nj) / 3 : (r - 2 * nj) / 3);
            const int c = is2d ? r & 1 : (istemp ? (r - 5 * nj) % 3 : (r - 2 * nj) % 3);
            const double X = sp[3 * j], Y = sp[3 * j + 1], Z = sp[3 * j + 2];
            if (is2d) {
                const double s = sqrt(P.l2d * P.lam[j]);
                if (c == 0) {
                    const double u = (P.fx * X) / Z + P.cx;
                    F = s * (u - P.p2d[j]);
                    g[0] = s * (P.fx / Z); g[1] = 0.0; g[2] = s * (-(P.fx * X) / (Z * Z));
                } else {
                    const double v = (P.fy * Y) / Z + P.cy;
                    F = s * (v - P.p2d[nj + j]);
                    g[0] = 0.0; g[1] = s * (P.fy / Z); g[2] = s * (-(P.fy * Y) / (Z * Z));
                }
                en[0] = F * F;
            } else if (!istemp) {
                F = P.s3d * ((sp[3 * j + c] - P.p3d[c * nj + j]) - P.pose[B.itp + c]);
                g[0] = g[1] = g[2] = 0.0;
                g[c] = P.s3d;
                has_tp = true;
                tpc = c;
                en[1] = F * F;
            } else {        // temporal stabilisation: sqrt(w_j) (p_j - p_j^{t-1})
                const double st = P.prev_joints ? P.stemp[j] : 0.0;
                F = P.prev_joints ? st * (sp[3 * j + c] - P.prev_joints[c * nj + j]) : 0.0;
                g[0] = g[1] = g[2] = 0.0;
                g[c] = st;
                en[4] = F * F;
            }
            ys[0][0] = X; ys[0][1] = Y; ys[0][2] = Z;
            ws[0] = 1.0;
            masks[0] = B.anc[j] & ~(1u << j);     // a joint does not move with its own rotation
            tw = 1.0;
        } else {
            const int e = P.blist[r - nfix];
            const int i = e >> 1;
            const double bs = (e & 1) ? -1.0 : 1.0;
            const int nv = B.nv;
            const double v[3] = {B.xyz[i], B.xyz[nv + i], B.xyz[2 * nv + i]};
            double V[3] = {0.0, 0.0, 0.0};
            tw = 0.0;
            for (int s = 0; s < 4; ++s) {
                const int j = B.bind_joint[size_t(s) * nv + i];
                ws[s] = B.bind_w[size_t(s) * nv + i];
                masks[s] = B.anc[j];
                const double d[3] = {v[0] - B.rest[0][j], v[1] - B.rest[1][j], v[2] - B.rest[2][j]};
                for (int a = 0; a < 3; ++a) {
                    const double *R = sR + 9 * j + 3 * a;
                    ys[s][a] = ((R[0] * d[0] + R[1] * d[1]) + R[2] * d[2]) + sp[3 * j + a];
                    V[a] += ws[s] * ys[s][a];
                }
                tw += ws[s];
            }
            npts = 4;
            const double X = V[0], Y = V[1], Z = V[2];
            const double u = (P.fx * X) / Z + P.cx, vv = (P.fy * Y) / Z + P.cy;
            double du, dv;
            const double dist = sample_cubic_f64(P.dt.g(), P.W, P.H, u, vv, du, dv);
            const double rr = P.ssil * dist;
            F = bs * rr;
            g[0] = P.ssil * (du * (P.fx / Z));
            g[1] = P.ssil * (dv * (P.fy / Z));
            g[2] = P.ssil * (du * (-(P.fx * X) / (Z * Z)) + dv * (-(P.fy * Y) / (Z * Z)));
            en[2] = bs * rr * rr;
            en[3] = rr * rr;
        }
        if (!energy_only) {
            rotation_entries(B, row, ldr, g, sp, sA, ys, ws, masks, npts);
            for (int a = 0; a < 3; ++a) {
                row[(B.it + a) * ldr] = tw * g[a];
                row[(B.itp + a) * ldr] = 0.0;
            }
            if (has_tp) row[(B.itp + tpc) * ldr] = -P.s3d;
            row[nu * ldr] = F;
            for (int c = nu + 1; c < np_; ++c) row[c * ldr] = 0.0;
        }
    }
    for (int q = 0; q < kPoseTerms; ++q) {
        const double s = block_sum<kPoseRowThreads>(en[q], red);
        if (threadIdx.x == 0) P.epart[size_t(blockIdx.x) * kPoseTerms + q] = s;
    }
}

// Upper-triangle 16x16 tiles of [J | bF]^T [J | bF] on V_MFMA_F64_16X16X4F64,
// one workgroup of 4 waves per tile: wave w takes every 4th group of 32 rows,
// A(i, k) = rows[r + k][I0 + i], B(k, j) = rows[r + k][J0 + j].  Lane l
// supplies element (l % 16, l / 16) of A and (l / 16, l % 16) of B; its
// accumulator register q holds D(4 q + l / 16, l % 16) (one row group per
// register, unlike the 16x16 float32/bf16 shapes whose registers hold
// consecutive rows).  The 4 wave sums are added in wave order, and the tile
// is written into the system [nu][nu + 1] (both triangles; the column of
// b F becomes the right-hand side -J^T B F).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kJtjWaves = 4, kJtjBatch = 8;

__global__ __launch_bounds__(64 * kJtjWaves) void k_pose_jtj(const PoseDev *__restrict__ PP) {
    const PoseDev &P = *PP;
    __shared__ double part[kJtjWaves][256];
    const int np_ = P.B.np, nu = P.B.nu, nt = np_ / kPoseTile;
    int I = 0, rem = blockIdx.x;
    while (rem >= nt - I) { rem -= nt - I; ++I; }
    const int Jt = I + rem;
    const int M = pose_fixed_rows(P.B.nj, P.B.it) + P.nb[0];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const CAP_GLOBAL double *col_a = P.rows.g() + size_t(I * kPoseTile + li) * P.ldr;     // column-major rows
    const CAP_GLOBAL double *col_b = P.rows.g() + size_t(Jt * kPoseTile + li) * P.ldr;
    constexpr int span = 4 * kJtjBatch;
    for (int r0 = wv * span; r0 < M; r0 += kJtjWaves * span) {
        double a[kJtjBatch], bb[kJtjBatch];
#pragma unroll
        for (int u = 0; u < kJtjBatch; ++u) {
            const int r = r0 + 4 * u + lk;
            a[u] = r < M ? col_a[r] : 0.0;
            bb[u] = r < M ? col_b[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kJtjBatch; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[wv][(4 * q + lk) * kPoseTile + li] = acc[q];
    __syncthreads();
    if (wv == 0) {
        for (int q = 0; q < 4; ++q) {
            const int e = (4 * q + lk) * kPoseTile + li;
            double s = part[0][e];
            for (int w = 1; w < kJtjWaves; ++w) s += part[w][e];
            const int gi = I * kPoseTile + 4 * q + lk, gj = Jt * kPoseTile + li;
            if (gi > gj) continue;      // a diagonal tile's lower half is the mirror of its upper half
            if (gi < nu && gj < nu) {
                P.sys[gi * (nu + 1) + gj] = s;
                P.sys[gj * (nu + 1) + gi] = s;
            } else if (gi < nu && gj == nu) {
                P.sys[gi * (nu + 1) + nu] = -s;
            }
        }
    }
}

// One workgroup of kStepThreads.  mode 0: energy of the step, damping,
// elimination of the augmented system [A + mu I | -J^T B F] without pivoting
// (A = L D L^T with the right-hand side carried along: a right-looking update
// of the trailing upper triangle, one barrier per pivot, every pivot tested
// for positivity, which holds exactly for a positive definite system), back
// substitution in one wave with the unknowns in registers (reciprocal pivots
// from the elimination), update, kinematics
// at the new pose.  mode 1: energy only (final).  mode 2: energy only (the
// system is already in place for the caller).
constexpr int kStepThreads = 1024;

__global__ __launch_bounds__(kStepThreads) void k_pose_step(const PoseDev *__restrict__ PP, int gn, int nblk, int mode) {
    const PoseDev &P = *PP;
    const BodyDev &B = P.B;
    const int nu = B.nu, lda = nu + 1;
    const int t = threadIdx.x;
    __shared__ double A[kMaxPoseUnknowns * (kMaxPoseUnknowns + 1)];
    __shared__ double pn[kMaxPoseUnknowns];
    __shared__ double red[kStepThreads / 64];
    __shared__ int bad;
    // energies of the rows kernel's blocks: wave q sums term q, each lane a
    // strided share of the blocks (its loads in flight together), then a
    // fixed butterfly over the lanes
    if (t == 0) bad = 0;
    __syncthreads();
    {
        const int wq = t >> 6, lane = t & 63;
        if (wq < kPoseTerms) {
            double es = 0.0;
            for (int b = lane; b < nblk; b += 64) es += P.epart[size_t(b) * kPoseTerms + wq];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) es += __shfl_xor(es, o);
            if (lane == 0) {
                P.energy[gn * kPoseTerms + wq] = es;
                if (!isfinite(es)) bad = 1;
            }
        }
    }
    __syncthreads();
    if (bad) {
        if (t == 0 && P.status[0] == 0) P.status[0] = CAPTURE_ENONFINITE;
        return;
    }
    if (mode != 0 || P.status[0] != 0) return;
    {   // the system into LDS, eight independent loads in flight per lane
        const int tot = nu * lda;
        for (int e0 = t; e0 < tot; e0 += kStepThreads * 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = e0 + kStepThreads * u < tot ? P.sys[e0 + kStepThreads * u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e0 + kStepThreads * u < tot) A[e0 + kStepThreads * u] = v[u];
        }
    }
    __syncthreads();
    {   // damping mu = 1e-6 max diag
        double m = 0.0;
        for (int i = t; i < nu; i += kStepThreads) m = fmax(m, A[i * lda + i]);
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if ((t & 63) == 0) red[t >> 6] = m;
        __syncthreads();
        double mx = red[0];
        for (int w = 1; w < kStepThreads / 64; ++w) mx = fmax(mx, red[w]);
        if (t < nu) A[t * lda + t] += 1e-6 * mx;
        __syncthreads();
    }
    // elimination: for pivot k, rows i > k of the upper triangle and the
    // right-hand side column: A[i][j] -= (A[k][i] / A[k][k]) A[k][j], j >= i.
    // Pivots go in pairs (k, k + 1) with one barrier per pair: every thread
    // forms the values of row k + 1 after pivot k that it needs itself (the
    // same operations as that row's own update), applies pivot k and then
    // pivot k + 1 to its entries of rows i > k + 1; the owners of row k + 1's
    // columns store that row after the next barrier (the pair still reads its
    // old values; no later pair reads it).  The operations and their order per
    // entry are those of one pivot at a time.  Thread t owns column
    // k + 1 + (t % 128) of every kRowGroups-th row from k + 2 on.
    constexpr int kRowGroups = kStepThreads / 128, kRowsPer = (kMaxPoseUnknowns + kRowGroups - 1) / kRowGroups;
    const int tc = t & 127, tr = t >> 7;
    int row1_at = -1;          // LDS index and value of the thread's pending row k + 1 entry
    double row1 = 0.0;
    for (int k = 0; k < nu; k += 2) {
        if (row1_at >= 0) A[row1_at] = row1;
        row1_at = -1;
        const double akk = A[k * lda + k];
        if (!(akk > 0.0) || !isfinite(akk)) {      // every thread reads the same pivot
            if (t == 0) bad = 1;
            break;
        }
        const double inv = 1.0 / akk;
        const bool two = k + 1 < nu;
        // row k + 1 after pivot k: A1[k+1][c] = A[k+1][c] - (A[k][k+1] / A[k][k]) A[k][c]
        const double f1 = two ? A[k * lda + k + 1] * inv : 0.0;
        double inv1 = 0.0;
        if (two) {
            const double a1 = A[(k + 1) * lda + k + 1] - f1 * A[k * lda + k + 1];
            if (!(a1 > 0.0) || !isfinite(a1)) {
                if (t == 0) bad = 1;
                break;
            }
            inv1 = 1.0 / a1;
        }
        if (t == 0) {                             // reciprocal pivots for the back substitution
            pn[k] = inv;
            if (two) pn[k + 1] = inv1;
        }
        const int j = k + 1 + tc;
        if (j <= nu) {
            const double akj = A[k * lda + j];
            const double a1j = two ? A[(k + 1) * lda + j] - f1 * akj : 0.0;     // A1[k+1][j]
            const int iend = min(j, nu - 1);
            // all of the thread's rows at once: their loads in flight together, then the stores
            double aki[kRowsPer], a1i[kRowsPer], aij[kRowsPer];
#pragma unroll
            for (int u = 0; u < kRowsPer; ++u) {
                const int i = k + 2 + tr + u * kRowGroups;
                aki[u] = i <= iend ? A[k * lda + i] : 0.0;
                a1i[u] = i <= iend ? A[(k + 1) * lda + i] : 0.0;
                aij[u] = i <= iend ? A[i * lda + j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kRowsPer; ++u) {
                const int i = k + 2 + tr + u * kRowGroups;
                if (i <= iend) {
                    const double b = aij[u] - (aki[u] * inv) * akj;                 // pivot k
                    const double a1ki = a1i[u] - f1 * aki[u];                       // A1[k+1][i]
                    A[i * lda + j] = b - (a1ki * inv1) * a1j;                       // pivot k + 1
                }
            }
            if (two && tr == 0) {       // row k + 1 after pivot k, stored after the barrier
                row1_at = (k + 1) * lda + j;
                row1 = a1j;
            }
        }
        __syncthreads();
    }
    if (row1_at >= 0) A[row1_at] = row1;       // (none pending after a bad pivot)
    __syncthreads();
    if (bad) {
        for (int e = t; e < nu; e += kStepThreads) P.pose[e] = P.pose0[e];
        if (t == 0) P.status[0] = CAPTURE_ENOTSPD;
        return;
    }
    // back substitution D L^T delta = z in the first wave: component e lives in
    // lane e % 64 (slot e / 64); after delta_i is known it is taken out of the
    // right-hand sides of the rows above
    double d0s[2] = {0.0, 0.0};
    if (t < 64) {
        double b0 = t < nu ? A[t * lda + nu] : 0.0, b1 = t + 64 < nu ? A[(t + 64) * lda + nu] : 0.0;
        double d0 = 0.0, d1 = 0.0;
        for (int i = nu - 1; i >= 0; --i) {
            const double bi = __shfl(i < 64 ? b0 : b1, i & 63);
            const double di = bi * pn[i];
            if ((i & 63) == t) {
                if (i < 64) d0 = di; else d1 = di;
            }
            if (t < i) b0 -= A[t * lda + i] * di;
            if (t + 64 < i) b1 -= A[(t + 64) * lda + i] * di;
        }
        d0s[0] = d0;
        d0s[1] = d1;
    }
    __syncthreads();      // the reciprocal pivots in pn are no longer needed
    if (t < 64) {
        if (t < nu) {
            pn[t] = P.pose[t] + d0s[0];
            P.pose[t] = pn[t];
        }
        if (t + 64 < nu) {
            pn[t + 64] = P.pose[t + 64] + d0s[1];
            P.pose[t + 64] = pn[t + 64];
        }
    }
    __syncthreads();
    // kinematics at the new pose; its joint tables reuse the system's LDS
    double *sR = A, *sp = sR + 9 * kMaxJoints, *sA = sp + 3 * kMaxJoints, *sL = sA + 9 * kMaxJoints,
           *sJ = sL + 9 * kMaxJoints;
    fk_block(B, pn, sR, sp, sA, sL, sJ);
    fk_store(P, sR, sp, sA);
}

// ---------------------------------------------------------------- skinning, warping, extrapolation
// Skinned mesh at a pose: kinematics per workgroup (in LDS), then the float32
// linear-blend recipe of k_pose_lbs for the workgroup's vertices.
__global__ __launch_bounds__(256) void k_body_skin(BodyDev B, const double *__restrict__ pose, float *__restrict__ out) {
    __shared__ double sR[9 * kMaxJoints], sp[3 * kMaxJoints], sA[9 * kMaxJoints], sL[9 * kMaxJoints],
        sJ[9 * kMaxJoints];
    __shared__ float fR[9 * kMaxJoints], fp[3 * kMaxJoints], fJ[3 * kMaxJoints];
    fk_block(B, pose, sR, sp, sA, sL, sJ);
    for (int e = threadIdx.x; e < 9 * B.nj; e += blockDim.x) fR[e] = float(sR[e]);
    for (int e = threadIdx.x; e < 3 * B.nj; e += blockDim.x) {
        fp[e] = float(sp[e]);
        fJ[e] = float(B.rest[e % 3][e / 3]);
    }
    __syncthreads();
    const int nv = B.nv, i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const float v[3] = {B.xyz[i], B.xyz[nv + i], B.xyz[2 * nv + i]};
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int s = 0; s < 4; ++s) {
        const int j = B.bind_joint[size_t(s) * nv + i];
        const float w = B.bind_w[size_t(s) * nv + i];
        const float d[3] = {v[0] - fJ[3 * j], v[1] - fJ[3 * j + 1], v[2] - fJ[3 * j + 2]};
        for (int a = 0; a < 3; ++a) {
            const float *R = fR + 9 * j + 3 * a;
            const float q = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
            acc[a] = acc[a] + w * (q + fp[3 * j + a]);
        }
    }
    for (int a = 0; a < 3; ++a) out[size_t(a) * nv + i] = acc[a];
}

// Unit quaternion (w, x, y, z) of a rotation matrix (row-major), from the
// largest of the trace and the diagonal entries (Shepperd's method).
__device__ inline void quat_of(const double *R, double *q) {
    const double tr = (R[0] + R[4]) + R[8];
    if (tr > 0.0) {
        const double s = 2.0 * sqrt(tr + 1.0);
        q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        const double s = 2.0 * sqrt(((1.0 + R[0]) - R[4]) - R[8]);
        q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        const double s = 2.0 * sqrt(((1.0 + R[4]) - R[0]) - R[8]);
        q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
    } else {
        const double s = 2.0 * sqrt(((1.0 + R[8]) - R[0]) - R[4]);
        q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
    }
}

// Rotation of a vertex under dual-quaternion skinning: its influences'
// quaternions flipped into the first one's hemisphere, blended, normalised.
__device__ inline void blend_rotation(const BodyDev &B, const double *qj, int i, double M[9]) {
    const int nv = B.nv;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    const int j0 = B.bind_joint[i];
    for (int s = 0; s < 4; ++s) {
        const int j = B.bind_joint[size_t(s) * nv + i];
        const double w = B.bind_w[size_t(s) * nv + i];
        const double dot = ((qj[4 * j] * qj[4 * j0] + qj[4 * j + 1] * qj[4 * j0 + 1]) + qj[4 * j + 2] * qj[4 * j0 + 2]) +
                           qj[4 * j + 3] * qj[4 * j0 + 3];
        const double ws = dot < 0.0 ? -w : w;
        for (int c = 0; c < 4; ++c) q[c] += ws * qj[4 * j + c];
    }
    const double n = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    M[0] = 1.0 - 2.0 * (y * y + z * z); M[1] = 2.0 * (x * y - w * z); M[2] = 2.0 * (x * z + w * y);
    M[3] = 2.0 * (x * y + w * z); M[4] = 1.0 - 2.0 * (x * x + z * z); M[5] = 2.0 * (y * z - w * x);
    M[6] = 2.0 * (x * z - w * y); M[7] = 2.0 * (y * z + w * x); M[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Displacement warping: start = S_cur + M_cur M_prev^T (V_prev - S_prev).
__global__ __launch_bounds__(256) void k_body_warp(BodyDev B, const double *__restrict__ pose_prev,
                                                   const double *__restrict__ pose_cur, const float *__restrict__ Vp,
                                                   const float *__restrict__ Sp, const float *__restrict__ Sc,
                                                   float *__restrict__ out) {
    __shared__ double sR[9 * kMaxJoints], sp[3 * kMaxJoints], sA[9 * kMaxJoints], sL[9 * kMaxJoints],
        sJ[9 * kMaxJoints];
    __shared__ double qp[4 * kMaxJoints], qc[4 * kMaxJoints];
    const int nj = B.nj, t = threadIdx.x;
    fk_block(B, pose_prev, sR, sp, sA, sL, sJ);
    if (t < nj) quat_of(sR + 9 * t, qp + 4 * t);
    __syncthreads();
    fk_block(B, pose_cur, sR, sp, sA, sL, sJ);
    if (t < nj) quat_of(sR + 9 * t, qc + 4 * t);
    __syncthreads();
    const int nv = B.nv, i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double Mp[9], Mc[9], d[3], r[3];
    blend_rotation(B, qp, i, Mp);
    blend_rotation(B, qc, i, Mc);
    for (int a = 0; a < 3; ++a) d[a] = double(Vp[size_t(a) * nv + i]) - double(Sp[size_t(a) * nv + i]);
    for (int a = 0; a < 3; ++a) r[a] = (Mp[a] * d[0] + Mp[3 + a] * d[1]) + Mp[6 + a] * d[2];       // M_prev^T d
    for (int a = 0; a < 3; ++a)
        out[size_t(a) * nv + i] =
            float(double(Sc[size_t(a) * nv + i]) + ((Mc[3 * a] * r[0] + Mc[3 * a + 1] * r[1]) + Mc[3 * a + 2] * r[2]));
}

// Joint positions at a pose, out [3][nj].
__global__ __launch_bounds__(64) void k_body_joints(BodyDev B, const double *__restrict__ pose, double *__restrict__ out) {
    __shared__ double sR[9 * kMaxJoints], sp[3 * kMaxJoints], sA[9 * kMaxJoints], sL[9 * kMaxJoints],
        sJ[9 * kMaxJoints];
    fk_block(B, pose, sR, sp, sA, sL, sJ);
    for (int e = threadIdx.x; e < 3 * B.nj; e += blockDim.x) out[(e % 3) * B.nj + e / 3] = sp[e];
}

// Explicit Euler step of the pose: out = p + (p - p2).
__global__ void k_pose_extrapolate(int nu, const double *__restrict__ p, const double *__restrict__ p2,
                                   double *__restrict__ out) {
    const int e = threadIdx.x;
    if (e < nu) out[e] = p[e] + (p[e] - p2[e]);
}

}  // namespace cap
