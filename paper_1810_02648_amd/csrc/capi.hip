// C ABI entry points: argument checks, workspace layout and the launch
// sequence of the per-frame solve.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "runtime.hpp"

namespace cap {

// kernels defined in the other translation units
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v);
__global__ void k_dt_scan_cols(const ProbDev *P);
__global__ void k_decide(const ProbDev *P);
__global__ void k_prep_image(const ProbDev *P, int nb_init, int nb_px, int gn_iters, float w0, float w1);
__global__ void k_prep_geom(const ProbDev *P, int nb_v);
__global__ void k_prep_raster(const ProbDev *P, int nb_f, int scan);
__global__ void k_prep_cols(const ProbDev *P);
__global__ void k_prep_rows(const ProbDev *P, int nb_rows);
__global__ void k_linearize(const ProbDev *P, const TileDesc *D, int mode);
template <int kSplit, int kMode>
__global__ void k_cg(const ProbDev *P, const TileDesc *D, int j);
__global__ void k_node_init(const ProbDev *P, int check_target);
__global__ void k_node_init_fin(const ProbDev *P, int gn, int energy_only, int check_target, int slot_prev, int gn_iters,
                                int nparts);
__global__ void k_node_gather(const ProbDev *P);
__global__ void k_cg_finish(const ProbDev *P, int n);
__global__ void k_pcg_node(const ProbDev *P, int j, int last);
constexpr int kCgFused = 0, kCgStandard = 1;     // k_cg's arrangements of the PCG iteration
// schedules of at most this many PCG iterations per Gauss-Newton step (on grids
// the chip holds at once) run one launch per iteration
constexpr int kCgFusedMaxIters = 16;
int build_template(const capture_template_desc *d, capture_template **out, int device);

// warm-start kernels (warmstart.hip)
__global__ void k_gemm(Gemm g);
__global__ void k_mean_bwd(const float *dcat, const float *z, int nn, const int *in_beg, const int *in_src,
                           const int *out_cnt, uint16_t *dzb, float *dz, int width);
__global__ void k_colsum(const float *in, int rows, int cols, float *out);
__global__ void k_mse_grad(const float *y, const float *t, int n, float *dy, uint16_t *dyb, float *se);
__global__ void k_adam(float *w, const float *g, float *m, float *v, uint16_t *wb, int n, float lr, float c1, float c2);
__global__ void k_to_bf16(const float *in, uint16_t *out, int n);
__global__ void k_ws_features(const ProbDev *P, float *X);
__global__ void k_ws_layer1_feat(const ProbDev *P, float *X, const float *mu, const float *sd, const uint16_t *W,
                                 const float *bias, uint16_t *Xb, float *z, uint16_t *cat);
__global__ void k_ws_layer1(const float *X, int nn, const float *mu, const float *sd, const uint16_t *W,
                            const float *bias, uint16_t *Xb, float *z, uint16_t *cat);
template <int NT>
__global__ void k_ws_layer_mp(uint16_t *cat, const float *zp, const int *edge_dst, int nn, const uint16_t *W,
                              const float *bias, int N, float *z, uint16_t *cat_next, float *xdelta,
                              const ProbDev *upd);
__global__ void k_ws_target(const float *prev, const float *next, int nn, float *target);
__global__ void k_ws_scaling(const float *X, long long rows, float *mu, float *sd);

namespace {
// The last error message (fixed storage: setting it allocates nothing).
thread_local char g_err[512];
}

void set_error(const std::string &msg) { (void)fail(0, msg.c_str()); }
int fail(int code, const char *msg) {
    std::snprintf(g_err, sizeof g_err, "%s", msg ? msg : "");
    return code;
}
int fail(int code, const std::string &msg) { return fail(code, msg.c_str()); }

// ---------------------------------------------------------------- graph build kernels
__device__ inline float d2f(float ax, float ay, float az, float bx, float by, float bz) {
    float dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

// Farthest-point sampling, one launch per node over the whole chip.  Launch n
// (0 <= n < nn) learns node n: vertex 0 for n = 0, else the argmax of the
// smallest squared distances to the nodes so far, with ties to the lowest
// index.  Every workgroup takes that argmax from the previous launch's
// per-workgroup partials (the order of (value desc, index asc) is total, so
// every workgroup gets the same node, with no atomics and no waiting on other
// workgroups); workgroup 0 stores it.  Then each workgroup lowers the
// distances of its vertices (grid-stride) by the new node's and writes the
// argmax of its vertices as its partial for launch n + 1 (partials alternate
// between two buffers by launch parity).  The distances and the rule are
// those of a one-workgroup loop over all vertices, so the nodes are too.
constexpr int kFpsThreads = 256, kFpsMaxBlocks = 256;

struct ArgMax {
    float v;
    int i;
};
__device__ inline ArgMax argmax_of(ArgMax a, ArgMax b) { return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a; }

__device__ inline ArgMax block_argmax(ArgMax a, ArgMax *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a = argmax_of(a, ArgMax{__shfl_xor(a.v, o), __shfl_xor(a.i, o)});
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    ArgMax r = red[0];
#pragma unroll
    for (int w = 1; w < kFpsThreads / 64; ++w) r = argmax_of(r, red[w]);
    __syncthreads();            // red free for the next use
    return r;
}

__global__ __launch_bounds__(kFpsThreads) void k_fps_step(const float *__restrict__ xyz, int nv, int nn, int n,
                                                          float *__restrict__ mind, float *__restrict__ pv,
                                                          int *__restrict__ pi, int *__restrict__ node_vertex) {
    __shared__ ArgMax red[kFpsThreads / 64];
    const float *X = xyz, *Y = xyz + nv, *Z = xyz + 2 * size_t(nv);
    const int nb = gridDim.x;
    int sel = 0;
    if (n > 0) {
        const int t = threadIdx.x, q = ((n - 1) & 1) * kFpsMaxBlocks;
        const ArgMax a = t < nb ? ArgMax{pv[q + t], pi[q + t]} : ArgMax{-1.0f, 0x7fffffff};
        sel = min(block_argmax(a, red).i, nv - 1);     // (every workgroup has a vertex: the index is one)
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) node_vertex[n] = sel;
    if (n == nn - 1) return;
    const float sx = X[sel], sy = Y[sel], sz = Z[sel];
    ArgMax best{-1.0f, 0x7fffffff};
    for (int v = blockIdx.x * kFpsThreads + threadIdx.x; v < nv; v += nb * kFpsThreads) {
        const float d = d2f(X[v], Y[v], Z[v], sx, sy, sz);
        const float m = n == 0 ? d : (d < mind[v] ? d : mind[v]);
        mind[v] = m;
        if (m > best.v) best = ArgMax{m, v};
    }
    best = block_argmax(best, red);
    if (threadIdx.x == 0) {
        pv[(n & 1) * kFpsMaxBlocks + blockIdx.x] = best.v;
        pi[(n & 1) * kFpsMaxBlocks + blockIdx.x] = best.i;
    }
}

// K nearest among the nodes (skipping `self`), ascending distance, ties -> lower index.
template <int K>
__device__ inline void knn_insert(float d, int k, float *bd, int *bk) {
    if (!(d < bd[K - 1])) return;
    int pos = K - 1;
    while (pos > 0 && d < bd[pos - 1]) {
        bd[pos] = bd[pos - 1];
        bk[pos] = bk[pos - 1];
        --pos;
    }
    bd[pos] = d;
    bk[pos] = k;
}

constexpr int kNodeChunk = 2048;

__global__ __launch_bounds__(256) void k_bind(const float *__restrict__ xyz, int nv, int nn,
                                              const int *__restrict__ node_vertex, int *bind_idx, float *bind_w) {
    __shared__ float gx[kNodeChunk], gy[kNodeChunk], gz[kNodeChunk];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    float px = 0, py = 0, pz = 0;
    if (v < nv) { px = xyz[v]; py = xyz[nv + v]; pz = xyz[2 * size_t(nv) + v]; }
    float bd[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    int bk[4] = {-1, -1, -1, -1};
    for (int c0 = 0; c0 < nn; c0 += kNodeChunk) {
        const int cn = min(kNodeChunk, nn - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += blockDim.x) {
            int gv = node_vertex[c0 + i];
            gx[i] = xyz[gv]; gy[i] = xyz[nv + gv]; gz[i] = xyz[2 * size_t(nv) + gv];
        }
        __syncthreads();
        if (v < nv)
            for (int i = 0; i < cn; ++i) knn_insert<4>(d2f(px, py, pz, gx[i], gy[i], gz[i]), c0 + i, bd, bk);
    }
    if (v >= nv) return;
    const float s2 = bd[3];
    float w[4], sum = 0.0f;
    for (int j = 0; j < 4; ++j) {
        w[j] = s2 > 0.0f ? expf(-bd[j] / (2.0f * s2)) : 1.0f;
        sum += w[j];
    }
    for (int j = 0; j < 4; ++j) {
        bind_idx[size_t(j) * nv + v] = bk[j];
        bind_w[size_t(j) * nv + v] = w[j] / sum;
    }
}

__global__ __launch_bounds__(256) void k_node_edges(const float *__restrict__ xyz, int nv, int nn,
                                                    const int *__restrict__ node_vertex, int *edge_dst) {
    __shared__ float gx[kNodeChunk], gy[kNodeChunk], gz[kNodeChunk];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    float px = 0, py = 0, pz = 0;
    if (k < nn) { int gv = node_vertex[k]; px = xyz[gv]; py = xyz[nv + gv]; pz = xyz[2 * size_t(nv) + gv]; }
    float bd[8];
    int bk[8];
    for (int j = 0; j < 8; ++j) { bd[j] = INFINITY; bk[j] = -1; }
    for (int c0 = 0; c0 < nn; c0 += kNodeChunk) {
        const int cn = min(kNodeChunk, nn - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += blockDim.x) {
            int gv = node_vertex[c0 + i];
            gx[i] = xyz[gv]; gy[i] = xyz[nv + gv]; gz[i] = xyz[2 * size_t(nv) + gv];
        }
        __syncthreads();
        if (k < nn)
            for (int i = 0; i < cn; ++i)
                if (c0 + i != k) knn_insert<8>(d2f(px, py, pz, gx[i], gy[i], gz[i]), c0 + i, bd, bk);
    }
    if (k >= nn) return;
    for (int j = 0; j < 8; ++j) edge_dst[size_t(j) * nn + k] = bk[j];
}

// ---------------------------------------------------------------- workspace layout

void carve(Layout &L, uint8_t *base, const capture_frame &f, ProbDev &pr) {
    const TemplateDev &T = f.tmpl->dev;
    const size_t nv = T.nv, nf = T.nf, nn = T.nn, hw = size_t(f.camera.width) * f.camera.height;
    pr.blurred = L.take<float>(base, 3 * hw);
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
    pr.pc = L.take<float>(base, 3 * nv);
    pr.vcode = L.take<uint8_t>(base, nv);
    pr.Hm = L.take<float>(base, 6 * nv);
    pr.partial = L.take<float>(base, size_t(T.nslots) * 12);
    pr.gpos = L.take<float>(base, size_t(3) * nn);
    pr.dots = L.take<double>(base, size_t(6) * T.ntiles);
    pr.cg = L.take<double>(base, 8);
    pr.nsum = L.take<double>(base, size_t(4) * ((nn + 255) / 256));
    pr.tile_e = L.take<double>(base, size_t(T.ntiles) * kTerms);
    pr.pva = L.take<float>(base, 3 * nv);
    gptr<float> *vecs[6] = {&pr.b, &pr.diag, &pr.dinv, &pr.p, &pr.Ap, &pr.x};
    for (gptr<float> *v : vecs) *v = L.take<float>(base, 6 * nn);
    gptr<double> *dvecs[10] = {&pr.vx[0], &pr.vx[1], &pr.vr[0], &pr.vr[1], &pr.vu[0],
                               &pr.vu[1], &pr.vp[0], &pr.vp[1], &pr.vs[0], &pr.vs[1]};
    for (gptr<double> *v : dvecs) *v = L.take<double>(base, 6 * nn);
    pr.state0 = L.take<float>(base, 12 * nn);
}

struct Plan {
    size_t bytes = 0;
};

// Layout: the descriptors, one block with every problem's scalars and counters
// (read back by a single copy), then each problem's buffers.
int grid_tiles(int n, const capture_frame *frames) {
    long long t = 0;
    for (int i = 0; i < n; ++i) t += frames[i].tmpl->dev.ntiles;
    return int((t + 7) / 8 * 8);
}

Plan plan_workspace(int n, const capture_frame *frames, uint8_t *base, ProbDev *probs) {
    Layout L;
    Plan pl;
    // descriptors, then the tile-kernel work list, one upload
    L.take<uint8_t>(base, sizeof(ProbDev) * n + sizeof(TileDesc) * grid_tiles(n, frames));
    double *scal = L.take<double>(base, size_t(kScalars) * n);
    int *counts = L.take<int>(base, size_t(3) * n);
    for (int i = 0; i < n; ++i) {
        ProbDev pr{};
        carve(L, base, frames[i], pr);
        pr.scal = scal ? scal + size_t(kScalars) * i : nullptr;
        pr.counts = counts ? counts + 3 * i : nullptr;
        if (probs) probs[i] = pr;
    }
    pl.bytes = L.off;
    return pl;
}

bool finite(float x) { return std::isfinite(x); }

int check_frames(int n, const capture_frame *frames) {
    if (n < 1 || !frames) return fail(CAPTURE_EINVAL, "need at least one frame");
    for (int i = 0; i < n; ++i) {
        const capture_frame &f = frames[i];
        if (!f.tmpl) return fail(CAPTURE_EINVAL, "frame without template");
        if (!f.xyz || !f.rgb || !f.mask || !f.image || !f.node_state)
            return fail(CAPTURE_EINVAL, "frame: null array");
        const capture_camera &c = f.camera;
        if (c.width < 1 || c.height < 1 || c.width > kMaxImageSide || c.height > kMaxImageSide)
            return fail(CAPTURE_EUNSUPPORTED, "camera: image sides must be in [1, 4096]");
        if (!finite(c.fx) || !finite(c.fy) || !finite(c.cx) || !finite(c.cy) || c.fx == 0.0f || c.fy == 0.0f)
            return fail(CAPTURE_EINVAL, "camera: non-finite or zero intrinsics");
    }
    return CAPTURE_OK;
}

int check_params(const capture_nonrigid_params *p) {
    if (!p) return fail(CAPTURE_EINVAL, "null params");
    if (p->gn_iters < 1 || p->gn_iters > CAPTURE_MAX_GN) return fail(CAPTURE_EINVAL, "gn_iters must be in [1, 32]");
    if (p->pcg_iters < 0 || p->pcg_iters > 10000) return fail(CAPTURE_EINVAL, "pcg_iters must be in [0, 10000]");
    if (!finite(p->w_sil) || !finite(p->w_photo) || !finite(p->w_arap) || !finite(p->w_vel) || p->w_sil < 0 ||
        p->w_photo < 0 || p->w_arap < 0 || p->w_vel < 0)
        return fail(CAPTURE_EINVAL, "weights must be finite and non-negative");
    if (p->flags & ~uint32_t(CAPTURE_FLAG_EXCLUDE_CASE2 | CAPTURE_FLAG_OUTLINE_ONLY | CAPTURE_FLAG_PCG_STANDARD))
        return fail(CAPTURE_EINVAL, "unknown flag bits");
    if (std::isnan(p->tau_color) || p->tau_color < 0) return fail(CAPTURE_EINVAL, "tau_color must be >= 0 or +inf");
    if (!finite(p->pcg_tol) || p->pcg_tol < 0) return fail(CAPTURE_EINVAL, "pcg_tol must be finite and >= 0");
    return CAPTURE_OK;
}

// What a run should do beyond the per-frame preprocessing.
enum class Stage { Decisions, Linearize, Solve };

const char *kKernelNames[K_COUNT] = {"blur", "contour", "dt_cols", "dt_rows", "deform_start", "raster",
                                     "contour_edges", "decide", "linearize", "node_init", "cg", "cg_node",
                                     "ws_features", "ws_mlp", "pose_lbs", "pose_rows", "pose_jtj",
                                     "pose_step", "prep_image", "prep_geom", "prep_raster",
                                     "prep_cols",
                                     "v_blur", "v_lin", "v_apply", "v_update", "v_snap"};

int setup(Run &R, capture_ctx *ctx, int n, const capture_frame *frames, const capture_nonrigid_params *params,
          void *ws, size_t ws_bytes, void *stream) {
    R.prof = R.fixed_stage ? nullptr : &ctx->prof;
    R.ctx = ctx;
    int rc = check_frames(n, frames);
    if (rc) return rc;
    if (params && (rc = check_params(params))) return rc;
    Plan pl = plan_workspace(n, frames, nullptr, nullptr);
    if (!ws || ws_bytes < pl.bytes) return fail(CAPTURE_ENOMEM, "workspace too small");
    R.n = n;
    R.probs.resize(n);
    uint8_t *base = static_cast<uint8_t *>(ws);
    plan_workspace(n, frames, base, R.probs.data());
    R.dprobs = reinterpret_cast<ProbDev *>(base);
    R.s = static_cast<hipStream_t>(stream);
    const float wsil = params ? params->w_sil : 1.0f, wph = params ? params->w_photo : 0.1f,
                war = params ? params->w_arap : 10.0f;
    const float tau = params ? params->tau_color : INFINITY;     // sigma_c threshold; +inf keeps every residual
    const float wvel = params ? params->w_vel : 0.0f;
    const double tol = params ? double(params->pcg_tol) : 0.0;
    const int excl = params ? int(params->flags & CAPTURE_FLAG_EXCLUDE_CASE2) : 0;
    const int outline = params ? int((params->flags & CAPTURE_FLAG_OUTLINE_ONLY) != 0) : 0;
    for (int i = 0; i < n; ++i) {
        const capture_frame &f = frames[i];
        ProbDev &pr = R.probs[i];
        pr.T = f.tmpl->dev;
        pr.xyz = f.xyz; pr.rgb = f.rgb; pr.mask = f.mask; pr.image = f.image; pr.state = f.node_state;
        pr.W = f.camera.width; pr.H = f.camera.height;
        pr.fx = f.camera.fx; pr.fy = f.camera.fy; pr.cx = f.camera.cx; pr.cy = f.camera.cy;
        pr.sw_sil = std::sqrt(wsil); pr.sw_photo = std::sqrt(wph); pr.sw_arap = std::sqrt(war);
        pr.w_arap = war; pr.tau = tau;
        pr.w_vel = wvel; pr.sw_vel = std::sqrt(wvel); pr.exclude_case2 = excl; pr.outline_only = outline;
        pr.pcg_tol2 = tol * tol;
        pr.target = i == 0 ? R.target : -INFINITY;
        pr.prev2 = i == 0 ? R.prev2 : nullptr;
        const TemplateDev &T = pr.T;
        R.max_nv = std::max(R.max_nv, T.nv);
        R.max_nf = std::max(R.max_nf, T.nf);
        R.max_nn = std::max(R.max_nn, T.nn);
        R.max_me = std::max(R.max_me, T.nmedges);
        R.max_tiles = std::max(R.max_tiles, T.ntiles);
        R.max_hw = std::max(R.max_hw, pr.W * pr.H);
        R.max_w = std::max(R.max_w, pr.W);
        R.max_h = std::max(R.max_h, pr.H);
        // contribution buffers: components at an odd stride (max_contrib | 1)
        R.lds_lin = std::max(R.lds_lin, sizeof(float) * (size_t(T.max_slots) * 16 + size_t(T.max_contrib | 1) * 12));
        R.lds_apply = std::max(R.lds_apply, sizeof(float) * (size_t(T.max_slots) * 20 + size_t(T.max_contrib | 1) * 6));
        R.lds_apply_split =
            std::max(R.lds_apply_split, sizeof(float) * (size_t(T.max_slots) * 20 + size_t(T.max_contrib | 1) * 3));
    }
    // sized once for both the descriptors and the report read-back of `collect`
    R.grid_tiles = grid_tiles(n, frames);
    const size_t desc = sizeof(ProbDev) * n + sizeof(TileDesc) * R.grid_tiles;
    void *stage = run_staging(R, desc + sizeof(double) * kScalars * n + sizeof(int) * 3 * n + 512);
    if (!stage) return fail(R.fixed_stage ? CAPTURE_EUNSUPPORTED : CAPTURE_ENOMEM, "host staging too small or its allocation failed");
    std::memcpy(stage, R.probs.data(), sizeof(ProbDev) * n);
    TileDesc *td = reinterpret_cast<TileDesc *>(static_cast<uint8_t *>(stage) + sizeof(ProbDev) * n);
    int k = 0;
    for (int i = 0; i < n; ++i) {
        const std::vector<int> &tr = frames[i].tmpl->tile_ranges;
        for (int t = 0; t < R.probs[i].T.ntiles; ++t, ++k) {
            const int *r = tr.data() + size_t(6) * t;
            td[k] = TileDesc{i, t, r[0], r[1], r[2], r[3], r[4], r[5]};
        }
    }
    R.total_tiles = k;
    for (; k < R.grid_tiles; ++k) td[k] = TileDesc{-1, 0, 0, 0, 0, 0, 0, 0};
    R.tiles = reinterpret_cast<TileDesc *>(base + sizeof(ProbDev) * n);
    CAP_HIP(hipMemcpyAsync(R.dprobs, stage, desc, hipMemcpyHostToDevice, R.s));
    return CAPTURE_OK;
}


int launch_frame(Run &R, int gn_iters = 0) {
    const int n = R.n;
    hipStream_t s = R.s;
    // Gaussian kernel 3, sigma = 0.3 * ((3 - 1) / 2 - 1) + 0.8 = 0.8, normalised
    const double e1 = std::exp(-1.0 / (2.0 * 0.8 * 0.8));
    const float w0 = float(e1 / (1.0 + 2.0 * e1)), w1 = float(1.0 / (1.0 + 2.0 * e1));
    const size_t nsegw = size_t(R.max_w) * ((R.max_h + 15) / 16);
    const int nb_init = blocks(R.max_hw, 1024), nb_px = blocks(R.max_hw, 256), nb_v = blocks(R.max_nv, 256);
    const int nb_seg = blocks(nsegw, 256), nb_f = blocks(R.max_nf, 256), nb_me = blocks(R.max_me, 256);
    // enough columns in all: the segment scan runs a thread per column in its own launch
    const bool scan_cols = size_t(n) * R.max_w >= kScanColsMin;
    const int nb_scan = scan_cols ? 0 : blocks(R.max_w, 4);
    timed(R, K_PREP_IMAGE, [&] {
        hipLaunchKernelGGL(k_prep_image, dim3(nb_init + 2 * nb_px, n), dim3(256), 0, s, R.dprobs, nb_init, nb_px,
                           gn_iters, w0, w1);
    });
    timed(R, K_PREP_GEOM, [&] {
        hipLaunchKernelGGL(k_prep_geom, dim3(nb_v + nb_seg, n), dim3(256), 0, s, R.dprobs, nb_v);
    });
    timed(R, K_PREP_RASTER, [&] {
        hipLaunchKernelGGL(k_prep_raster, dim3(nb_f + nb_scan, n), dim3(256), 0, s, R.dprobs, nb_f, scan_cols ? 0 : 1);
    });
    if (scan_cols)
        timed(R, K_DT_COLS, [&] {
            hipLaunchKernelGGL(k_dt_scan_cols, dim3(blocks(R.max_w, 64), n), dim3(64), 0, s, R.dprobs);
        });
    timed(R, K_PREP_COLS, [&] {
        hipLaunchKernelGGL(k_prep_cols, dim3(kRasterBigBlocks + nb_seg, n), dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_DT_ROWS, [&] {
        hipLaunchKernelGGL(k_prep_rows, dim3(R.max_h + nb_me, n), dim3(256), dt_rows_lds(R.max_w), s, R.dprobs,
                           R.max_h);
    });
    timed(R, K_DECIDE, [&] {
        hipLaunchKernelGGL(k_decide, dim3(nb_v, n), dim3(256), 0, s, R.dprobs);
    });
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

// One product launch (k_cg, iteration j; j < 0: the product of
// capture_linearize) over all tiles.  Grids that the chip holds at once take
// the one-pass reduction; larger ones the two-pass variant with half the LDS.
void launch_cg(Run &R, int j, bool fused) {
    if (R.grid_tiles > kApplySplitTiles) {
        hipLaunchKernelGGL((k_cg<1, kCgStandard>), dim3(unsigned(R.grid_tiles)), dim3(kTileThreads), R.lds_apply_split,
                           R.s, R.dprobs, R.tiles, j);
    } else if (fused) {
        hipLaunchKernelGGL((k_cg<0, kCgFused>), dim3(unsigned(R.grid_tiles)), dim3(kTileThreads), R.lds_apply, R.s,
                           R.dprobs, R.tiles, j);
    } else {
        hipLaunchKernelGGL((k_cg<0, kCgStandard>), dim3(unsigned(R.grid_tiles)), dim3(kTileThreads), R.lds_apply, R.s,
                           R.dprobs, R.tiles, j);
    }
}

// check_target: see k_node_init (with bit 2, slot_prev and gn_iters of the selection).
void launch_linearize(Run &R, int gn, int energy_only, int check_target = 0, int slot_prev = 0, int gn_iters = 0) {
    timed(R, K_LIN, [&] {
        hipLaunchKernelGGL(k_linearize, dim3(unsigned(R.grid_tiles)), dim3(kTileThreads), R.lds_lin, R.s, R.dprobs, R.tiles,
                           energy_only);
    });
    timed(R, K_NODE_INIT, [&] {
        if (!energy_only)
            hipLaunchKernelGGL(k_node_init, dim3(kInitBlocks, R.n), dim3(kInitThreads), 0, R.s, R.dprobs, check_target);
        hipLaunchKernelGGL(k_node_init_fin, dim3(R.n), dim3(kInitFinThreads), 0, R.s, R.dprobs, gn, energy_only,
                           check_target, slot_prev, gn_iters, kInitBlocks);
    });
}

// Gauss-Newton steps [g0, g1): linearisation (skipped for the first step with
// first_done, when it has already been launched) and the PCG iterations.
void launch_steps(Run &R, const capture_nonrigid_params *prm, int check_target, bool first_done, int g0, int g1) {
    for (int gn = g0; gn < g1; ++gn) {
        if (gn > g0 || !first_done) launch_linearize(R, gn, 0, check_target);
        // one launch per iteration (Chronopoulos-Gear) for short schedules on
        // grids the chip holds at once; otherwise the standard recurrence, a
        // product launch and a node-step launch per iteration
        const int n = prm->pcg_iters;
        const bool fused = R.grid_tiles <= kApplySplitTiles && n <= kCgFusedMaxIters &&
                           !(prm->flags & CAPTURE_FLAG_PCG_STANDARD);
        const dim3 gnode(unsigned(blocks(R.max_nn, 256)), unsigned(R.n));
        for (int j = 0; j < n; ++j) {
            timed(R, K_APPLY, [&] {
                launch_cg(R, j, fused);
            });
            if (!fused)
                timed(R, K_NODE_PCG, [&] {
                    hipLaunchKernelGGL(k_pcg_node, gnode, dim3(256), 0, R.s, R.dprobs, j, j == n - 1 ? 1 : 0);
                });
        }
        if (fused || n == 0)
            timed(R, K_NODE_PCG, [&] {
                hipLaunchKernelGGL(k_cg_finish, gnode, dim3(256), 0, R.s, R.dprobs, n);
            });
    }
}

// The full schedule, then the energy at the final state.
int launch_solve(Run &R, const capture_nonrigid_params *prm, int check_target = 0, bool first_done = false) {
    launch_steps(R, prm, check_target, first_done, 0, prm->gn_iters);
    launch_linearize(R, prm->gn_iters, 1);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

// A solve's launch sequence (preprocessing, decisions, Gauss-Newton/PCG)
// captured once per launch shape into a HIP graph on the context's capture
// stream, then replayed on the caller's stream.  Kernels read everything
// else from the descriptors, which setup uploads before the replay, so one
// graph serves any inputs with the same sizes, workspace and schedule.  The
// sequence holds kernels only (buffers are cleared by kernels, not memsets).
// `key` names everything the sequence bakes into kernel arguments.
std::string shape_key(const Run &R, const capture_nonrigid_params *prm) {
    char key[512];
    std::snprintf(key, sizeof key, "%d|%p|%d %d %d %d %d %d %d %d %d|%zu %zu|%d %d", R.n, (void *)R.dprobs, R.max_nv,
                  R.max_nf, R.max_nn, R.max_hw, R.max_w, R.max_h, R.max_tiles, R.total_tiles, R.max_me, R.lds_lin,
                  R.lds_apply, prm->gn_iters, prm->pcg_iters);
    return key;
}

// Every problem's scalars and counters, copied to pinned host memory in one
// read-back (waits for the stream) into *host.
int read_back(Run &R, const uint8_t **host) {
    const uint8_t *blk = reinterpret_cast<const uint8_t *>(R.probs[0].scal.ptr);
    const size_t off_counts = reinterpret_cast<const uint8_t *>(R.probs[0].counts.ptr) - blk;
    const size_t bytes = off_counts + sizeof(int) * 3 * R.n;
    uint8_t *h = static_cast<uint8_t *>(run_staging(R, bytes));
    if (!h) return fail(CAPTURE_ENOMEM, "host staging too small or its allocation failed");
    CAP_HIP(hipMemcpyAsync(h, blk, bytes, hipMemcpyDeviceToHost, R.s));
    CAP_HIP(hipStreamSynchronize(R.s));
    *host = h;
    return CAPTURE_OK;
}

// The reports from a read-back block.
int reports_from(Run &R, const uint8_t *host, int gn_iters, capture_report *reports,
                 const double **scal_host = nullptr) {
    const uint8_t *blk = reinterpret_cast<const uint8_t *>(R.probs[0].scal.ptr);
    const size_t off_counts = reinterpret_cast<const uint8_t *>(R.probs[0].counts.ptr) - blk;
    const double *scal = reinterpret_cast<const double *>(host);
    if (scal_host) *scal_host = scal;
    const int *counts = reinterpret_cast<const int *>(host + off_counts);
    int status = CAPTURE_OK;
    for (int i = 0; i < R.n; ++i) {
        capture_report &rep = reports[i];
        std::memset(&rep, 0, sizeof(rep));
        const double *sc = scal + size_t(kScalars) * i;
        const int done = std::min(gn_iters, std::max(0, int(sc[3])));
        for (int k = 0; k <= done; ++k) {
            const double *ek = sc + 8 + kTerms * k;
            rep.energy[k] = ek[0] + ek[1] + ek[3] + ek[4];
        }
        const double *e = sc + 8 + kTerms * done;
        rep.e_photo = e[0]; rep.e_sil = e[1]; rep.e_sil_abs = e[2]; rep.e_arap = e[3]; rep.e_vel = e[4];
        rep.n_visible = counts[3 * i];
        rep.n_boundary = counts[3 * i + 1];
        rep.gn_done = done;
        rep.status = std::isfinite(rep.energy[done]) ? CAPTURE_OK : CAPTURE_ENONFINITE;
        if (rep.status) status = rep.status;
    }
    return status;
}

int collect(Run &R, int gn_iters, capture_report *reports, const double **scal_host = nullptr) {
    const uint8_t *host = nullptr;
    const int rc = read_back(R, &host);
    if (rc) return rc;
    settle(R);
    return reports_from(R, host, gn_iters, reports, scal_host);
}


// ---------------------------------------------------------------- warm-start network
constexpr int kOffW1 = 0, kOffB1 = 4096, kOffW2 = 4224, kOffB2 = 36992, kOffW3 = 37120, kOffB3 = 38656;
constexpr int kParams = CAPTURE_WS_PARAMS;
static_assert(kOffB3 + 6 == kParams, "parameter layout");

void gemm(hipStream_t s, const uint16_t *A, long long sai, long long sak, const uint16_t *B, long long sbj,
          long long sbk, float *C, long long sci, long long scj, int M, int N, int K, const float *bias,
          uint16_t *Cb = nullptr, long long scbi = 0) {
    Gemm g{A, sai, sak, B, sbj, sbk, C, sci, scj, M, N, K, bias, Cb, scbi, Cb ? 1 : 0};
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm, dim3((tiles + 3) / 4), dim3(256), 0, s, g);
}

// Forward pass on raw features X (device, [nn][32]) -> net->y [nn][6].
// Network forward: three fused layer kernels (one 8-wave workgroup per 16 nodes); with
// xdelta the last one also writes the scaled update in node-major layout.
// The network's forward pass; with xdelta, the prediction is also written as
// a PCG solution ([6][nn]), and with upd (the problem on the device) applied
// to that problem's node state by the last layer.
void ws_forward(capture_warmstart *net, const TemplateDev &T, const float *X, hipStream_t s, float *xdelta = nullptr,
                const ProbDev *upd = nullptr) {
    const int nn = T.nn;
    const dim3 g(unsigned((nn + 15) / 16));
    if (X)      // (else the first layer has run with its features formed in place: k_ws_layer1_feat)
        hipLaunchKernelGGL(k_ws_layer1, g, dim3(512), 0, s, X, nn, net->mu, net->sd, net->wb + kOffW1, net->w + kOffB1,
                           net->Xb, net->z1, net->c1);
    hipLaunchKernelGGL(k_ws_layer_mp<8>, g, dim3(512), 0, s, net->c1, net->z1, T.edge_dst, nn, net->wb + kOffW2,
                       net->w + kOffB2, 128, net->z2, net->c2, (float *)nullptr, (const ProbDev *)nullptr);
    hipLaunchKernelGGL(k_ws_layer_mp<1>, g, dim3(512), 0, s, net->c2, net->z2, T.edge_dst, nn, net->wb + kOffW3,
                       net->w + kOffB3, 6, net->y, (uint16_t *)nullptr, xdelta, upd);
}

// Backward pass after ws_forward, with targets in net->tgt; gradients into net->g.
void ws_backward(capture_warmstart *net, const TemplateDev &T, hipStream_t s) {
    const int nn = T.nn;
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks(size_t(nn) * 6, 256)), dim3(256), 0, s, net->y, net->tgt, nn * 6,
                       net->dy, net->dyb, net->se);
    gemm(s, net->dyb, 1, 6, net->c2, 1, 256, net->g + kOffW3, 256, 1, 6, 256, nn, nullptr);
    hipLaunchKernelGGL(k_colsum, dim3(6), dim3(256), 0, s, net->dy, nn, 6, net->g + kOffB3);
    gemm(s, net->dyb, 6, 1, net->wb + kOffW3, 1, 256, net->dc, 256, 1, nn, 256, 6, nullptr);
    hipLaunchKernelGGL(k_mean_bwd, dim3(blocks(size_t(nn) * 128, 256)), dim3(256), 0, s, net->dc, net->z2, nn,
                       T.in_beg, T.in_src, T.out_cnt, net->dzb, net->dz, 128);
    gemm(s, net->dzb, 1, 128, net->c1, 1, 256, net->g + kOffW2, 256, 1, 128, 256, nn, nullptr);
    hipLaunchKernelGGL(k_colsum, dim3(128), dim3(256), 0, s, net->dz, nn, 128, net->g + kOffB2);
    gemm(s, net->dzb, 128, 1, net->wb + kOffW2, 1, 256, net->dc, 256, 1, nn, 256, 128, nullptr);
    hipLaunchKernelGGL(k_mean_bwd, dim3(blocks(size_t(nn) * 128, 256)), dim3(256), 0, s, net->dc, net->z1, nn,
                       T.in_beg, T.in_src, T.out_cnt, net->dzb, net->dz, 128);
    gemm(s, net->dzb, 1, 128, net->Xb, 1, 32, net->g + kOffW1, 32, 1, 128, 32, nn, nullptr);
    hipLaunchKernelGGL(k_colsum, dim3(128), dim3(256), 0, s, net->dz, nn, 128, net->g + kOffB1);
}

// ---------------------------------------------------------------- allocation-free solve
// Device scratch of capture_nonrigid_solve_noalloc: one copy of this array on
// every device the library runs on, held until the process ends and shared by
// every such call on that device.  Host code never uses the array's name as a
// device address: its per-device address comes from hipGetSymbolAddress,
// resolved once per device when a context is created on it.
constexpr size_t kNoAllocScratch = size_t(32) << 20;
constexpr size_t kNoAllocStage = size_t(64) << 10;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_dev[kNoAllocDevices] = {};
// Host staging of the allocation-free calls (descriptor upload, report
// read-back): fixed, shared like the device scratch.
alignas(256) uint8_t g_noalloc_stage[kNoAllocStage];
}  // namespace

// The device address of `scratch` on `device` (the current device), looked up
// on the first call for that device.
int resolve_scratch(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device >= kNoAllocDevices) return fail(CAPTURE_EUNSUPPORTED, "device index beyond the scratch table");
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(CAPTURE_EHIP, "hipGetSymbolAddress(scratch) failed");
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return CAPTURE_OK;
}

}  // namespace cap

using namespace cap;

extern "C" {

const char *capture_last_error(void) { return g_err; }

int capture_create(capture_ctx **ctx, int device) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null ctx pointer");
    int count = 0;
    CAP_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CAPTURE_EINVAL, "no such device");
    CAP_HIP(hipSetDevice(device));
    void *scr = nullptr;
    const int rc = device < kNoAllocDevices ? resolve_scratch(device, &scr) : CAPTURE_OK;
    if (rc) return rc;
    *ctx = new capture_ctx();
    (*ctx)->device = device;
    (*ctx)->scratch = scr;
    return CAPTURE_OK;
}

void capture_destroy(capture_ctx *ctx) {
    if (!ctx) return;
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (auto &g : ctx->graph_cache) (void)hipGraphExecDestroy(g.exec);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

int capture_graph_build(capture_ctx *ctx, const float *xyz, int32_t n_vertices, int32_t n_nodes, int32_t *node_vertex,
                        int32_t *bind_idx, float *bind_w, int32_t *edge_dst, void *stream) {
    if (!ctx || !xyz || !node_vertex || !bind_idx || !bind_w || !edge_dst) return fail(CAPTURE_EINVAL, "null argument");
    if (n_nodes < 4 || n_nodes > n_vertices || n_nodes > 65536)
        return fail(CAPTURE_EINVAL, "graph: need 4 <= n_nodes <= n_vertices and n_nodes <= 65536");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // scratch: the vertices' smallest squared distances, then two buffers of
    // per-workgroup partials (value, index) of the farthest-point steps
    float *mind = nullptr;
    const size_t mbytes = (sizeof(float) * size_t(n_vertices) + 255) / 256 * 256;
    if (hipMalloc(&mind, mbytes + 2 * kFpsMaxBlocks * (sizeof(float) + sizeof(int))) != hipSuccess)
        return fail(CAPTURE_ENOMEM, "graph: scratch allocation failed");
    float *pv = reinterpret_cast<float *>(reinterpret_cast<char *>(mind) + mbytes);
    int *pi = reinterpret_cast<int *>(pv + 2 * kFpsMaxBlocks);
    const unsigned nb_fps = std::min(blocks(size_t(n_vertices), kFpsThreads), unsigned(kFpsMaxBlocks));
    for (int n = 0; n < n_nodes; ++n)
        hipLaunchKernelGGL(k_fps_step, dim3(nb_fps), dim3(kFpsThreads), 0, s, xyz, n_vertices, n_nodes, n, mind, pv, pi,
                           node_vertex);
    hipLaunchKernelGGL(k_bind, dim3(blocks(n_vertices, 256)), dim3(256), 0, s, xyz, n_vertices, n_nodes, node_vertex,
                       bind_idx, bind_w);
    hipLaunchKernelGGL(k_node_edges, dim3(blocks(n_nodes, 256)), dim3(256), 0, s, xyz, n_vertices, n_nodes,
                       node_vertex, edge_dst);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mind);
    if (e != hipSuccess) return fail(CAPTURE_EHIP, std::string("graph build: ") + hipGetErrorString(e));
    return CAPTURE_OK;
}

int capture_template_create(capture_ctx *ctx, const capture_template_desc *desc, capture_template **out) {
    if (!ctx || !desc || !out) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    return build_template(desc, out, ctx->device);
}

void capture_template_destroy(capture_template *t) {
    if (!t) return;
    (void)hipFree(t->mem);
    delete t;
}

int capture_template_info_get(const capture_template *t, capture_template_info *out) {
    if (!t || !out) return fail(CAPTURE_EINVAL, "null argument");
    const TemplateDev &D = t->dev;
    *out = capture_template_info{D.nv, D.nf, D.nn, D.ntiles, D.nslots, D.max_slots, D.max_contrib,
                                 t->vertices_per_tile};
    return CAPTURE_OK;
}

int capture_workspace_size(capture_ctx *ctx, int32_t n, const capture_frame *frames, size_t *bytes) {
    if (!ctx || !bytes) return fail(CAPTURE_EINVAL, "null argument");
    int rc = check_frames(n, frames);
    if (rc) return rc;
    *bytes = plan_workspace(n, frames, nullptr, nullptr).bytes;
    return CAPTURE_OK;
}

int capture_batch_solve(capture_ctx *ctx, int32_t n, const capture_frame *frames, const capture_nonrigid_params *params,
                        capture_report *reports, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx || !params || !reports) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    int rc = setup(R, ctx, n, frames, params, workspace, workspace_bytes, stream);
    if (rc) return rc;
    if (ctx->graphs && !ctx->prof.on) {
        rc = launch_graph(R, shape_key(R, params), [&](Run &C) {
            const int r = launch_frame(C, params->gn_iters);
            return r ? r : launch_solve(C, params);
        });
        if (rc) return rc;
    } else {
        if ((rc = launch_frame(R, params->gn_iters))) return rc;      // keeps the start states (frame set-up)
        if ((rc = launch_solve(R, params))) return rc;
    }
    rc = collect(R, params->gn_iters, reports);
    if (rc) {
        for (int i = 0; i < n; ++i)
            if (reports[i].status)
                (void)hipMemcpyAsync(frames[i].node_state, R.probs[i].state0, sizeof(float) * 12 * R.probs[i].T.nn,
                                     hipMemcpyDeviceToDevice, R.s);
        (void)hipStreamSynchronize(R.s);
        return fail(rc, "non-finite energy; node states restored");
    }
    return CAPTURE_OK;
}

int capture_nonrigid_solve(capture_ctx *ctx, const capture_frame *frame, const capture_nonrigid_params *params,
                           capture_report *report, void *workspace, size_t workspace_bytes, void *stream) {
    return capture_batch_solve(ctx, 1, frame, params, report, workspace, workspace_bytes, stream);
}

// The same launch sequence as capture_nonrigid_solve, eagerly launched, with
// the device scratch as workspace and fixed host staging: no device, pinned
// or host allocation on any path that returns CAPTURE_OK.
int capture_nonrigid_solve_noalloc(capture_ctx *ctx, const capture_frame *frame,
                                   const capture_nonrigid_params *params, capture_report *report, void *stream) {
    if (!ctx || !params || !report) return fail(CAPTURE_EINVAL, "null argument");
    int rc = check_frames(1, frame);
    if (rc) return rc;
    if ((rc = check_params(params))) return rc;
    if (!ctx->scratch) return fail(CAPTURE_EUNSUPPORTED, "no device scratch on this device");
    if (plan_workspace(1, frame, nullptr, nullptr).bytes > kNoAllocScratch)
        return fail(CAPTURE_EUNSUPPORTED, "frame needs more than the 32 MiB device scratch of the allocation-free solve");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    R.fixed_stage = g_noalloc_stage;
    R.fixed_stage_bytes = kNoAllocStage;
    if ((rc = setup(R, ctx, 1, frame, params, ctx->scratch, kNoAllocScratch, stream))) return rc;
    if ((rc = launch_frame(R, params->gn_iters))) return rc;
    if ((rc = launch_solve(R, params))) return rc;
    rc = collect(R, params->gn_iters, report);
    if (rc) {
        if (report->status)
            (void)hipMemcpyAsync(frame->node_state, R.probs[0].state0, sizeof(float) * 12 * R.probs[0].T.nn,
                                 hipMemcpyDeviceToDevice, R.s);
        (void)hipStreamSynchronize(R.s);
        return fail(rc, "non-finite energy; node state restored");
    }
    return CAPTURE_OK;
}

int capture_autotune_tiles(capture_ctx *ctx, int32_t n, const capture_template_desc *descs, const capture_frame *frames,
                           const capture_nonrigid_params *params, const int32_t *candidates, int32_t n_candidates,
                           int32_t *best, double *times_ms, void *stream) {
    if (!ctx || !descs || !frames || !params || !candidates || !best) return fail(CAPTURE_EINVAL, "null argument");
    if (n < 1 || n_candidates < 1) return fail(CAPTURE_EINVAL, "need at least one frame and one candidate");
    for (int c = 0; c < n_candidates; ++c)
        if (candidates[c] < 1 || candidates[c] > kMaxTileVerts)
            return fail(CAPTURE_EUNSUPPORTED, "candidate vertices_per_tile must be in [1, 256]");
    int rc = check_frames(n, frames);
    if (rc) return rc;
    if ((rc = check_params(params))) return rc;
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // keep the callers' start states; every trial starts from them
    size_t state_floats = 0;
    for (int i = 0; i < n; ++i) state_floats += size_t(12) * frames[i].tmpl->dev.nn;
    float *saved = nullptr;
    if (hipMalloc(&saved, sizeof(float) * state_floats) != hipSuccess)
        return fail(CAPTURE_ENOMEM, "autotune: device allocation failed");
    auto copy_states = [&](bool save) {
        size_t off = 0;
        for (int i = 0; i < n; ++i) {
            const size_t cnt = size_t(12) * frames[i].tmpl->dev.nn;
            (void)hipMemcpyAsync(save ? saved + off : frames[i].node_state, save ? frames[i].node_state : saved + off,
                                 sizeof(float) * cnt, hipMemcpyDeviceToDevice, s);
            off += cnt;
        }
    };
    copy_states(true);
    std::vector<capture_report> reps(n);
    double best_ms = INFINITY;
    int best_c = -1;
    for (int c = 0; c < n_candidates && rc == CAPTURE_OK; ++c) {
        std::vector<capture_template *> tm(n, nullptr);
        std::vector<capture_frame> fr(frames, frames + n);
        for (int i = 0; i < n && rc == CAPTURE_OK; ++i) {
            capture_template_desc d = descs[i];
            d.vertices_per_tile = candidates[c];
            rc = build_template(&d, &tm[i], ctx->device);
            fr[i].tmpl = tm[i];
        }
        void *ws = nullptr;
        size_t bytes = 0;
        if (rc == CAPTURE_OK) {
            bytes = plan_workspace(n, fr.data(), nullptr, nullptr).bytes;
            if (hipMalloc(&ws, bytes) != hipSuccess) rc = fail(CAPTURE_ENOMEM, "autotune: device allocation failed");
        }
        double t_min = INFINITY;
        for (int rep = 0; rep < 4 && rc == CAPTURE_OK; ++rep) {       // one warm-up, three timed
            copy_states(false);
            if (hipStreamSynchronize(s) != hipSuccess) { rc = fail(CAPTURE_EHIP, "autotune: stream error"); break; }
            const auto t0 = std::chrono::steady_clock::now();
            rc = capture_batch_solve(ctx, n, fr.data(), params, reps.data(), ws, bytes, stream);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rep > 0) t_min = std::min(t_min, ms);
        }
        if (times_ms) times_ms[c] = t_min;
        if (rc == CAPTURE_OK && t_min < best_ms) { best_ms = t_min; best_c = candidates[c]; }
        if (ws) (void)hipFree(ws);
        for (capture_template *t : tm) capture_template_destroy(t);
    }
    copy_states(false);
    (void)hipStreamSynchronize(s);
    (void)hipFree(saved);
    if (rc) return rc;
    *best = best_c;
    return CAPTURE_OK;
}

int capture_frame_decisions(capture_ctx *ctx, const capture_frame *frame, float *dt, float *blurred, uint32_t *zbuf,
                            uint8_t *vflags, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    int rc = setup(R, ctx, 1, frame, nullptr, workspace, workspace_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_frame(R))) return rc;
    const ProbDev &pr = R.probs[0];
    const size_t hw = size_t(pr.W) * pr.H;
    if (dt) CAP_HIP(hipMemcpyAsync(dt, pr.dt, sizeof(float) * hw, hipMemcpyDeviceToDevice, R.s));
    if (blurred) CAP_HIP(hipMemcpyAsync(blurred, pr.blurred, sizeof(float) * 3 * hw, hipMemcpyDeviceToDevice, R.s));
    if (zbuf) CAP_HIP(hipMemcpyAsync(zbuf, pr.zbuf, sizeof(uint32_t) * hw, hipMemcpyDeviceToDevice, R.s));
    if (vflags) CAP_HIP(hipMemcpyAsync(vflags, pr.vflags, pr.T.nv, hipMemcpyDeviceToDevice, R.s));
    CAP_HIP(hipStreamSynchronize(R.s));
    settle(R);
    return CAPTURE_OK;
}

int capture_linearize(capture_ctx *ctx, const capture_frame *frame, const capture_nonrigid_params *params, float *rhs,
                      float *diag, const float *p, float *Ap, double *energy, void *workspace, size_t workspace_bytes,
                      void *stream) {
    if (!ctx || !params) return fail(CAPTURE_EINVAL, "null argument");
    if ((p == nullptr) != (Ap == nullptr)) return fail(CAPTURE_EINVAL, "p and Ap go together");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    int rc = setup(R, ctx, 1, frame, params, workspace, workspace_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_frame(R))) return rc;
    launch_linearize(R, 0, 0);
    const ProbDev &pr = R.probs[0];
    const size_t n6 = size_t(6) * pr.T.nn;
    if (p) {
        const double zero = 0.0;
        CAP_HIP(hipMemcpyAsync(pr.p, p, sizeof(float) * n6, hipMemcpyDeviceToDevice, R.s));
        CAP_HIP(hipMemcpyAsync(pr.scal + 1, &zero, sizeof(double), hipMemcpyHostToDevice, R.s));
        timed(R, K_APPLY, [&] {
            launch_cg(R, -1, false);
        });
        hipLaunchKernelGGL(k_node_gather, dim3(1), dim3(kNodeThreads), 0, R.s, R.dprobs);
        CAP_HIP(hipGetLastError());
        CAP_HIP(hipMemcpyAsync(Ap, pr.Ap, sizeof(float) * n6, hipMemcpyDeviceToDevice, R.s));
    }
    if (rhs) CAP_HIP(hipMemcpyAsync(rhs, pr.b, sizeof(float) * n6, hipMemcpyDeviceToDevice, R.s));
    if (diag) CAP_HIP(hipMemcpyAsync(diag, pr.diag, sizeof(float) * n6, hipMemcpyDeviceToDevice, R.s));
    double sc[kScalars];
    CAP_HIP(hipMemcpyAsync(sc, pr.scal, sizeof(sc), hipMemcpyDeviceToHost, R.s));
    CAP_HIP(hipStreamSynchronize(R.s));
    settle(R);
    if (energy) for (int q = 0; q < kTerms; ++q) energy[q] = sc[8 + q];
    return CAPTURE_OK;
}


int capture_warmstart_create(capture_ctx *ctx, int32_t max_nodes, const float *params, capture_warmstart **out) {
    if (!ctx || !params || !out) return fail(CAPTURE_EINVAL, "null argument");
    if (max_nodes < 1 || max_nodes > 65536) return fail(CAPTURE_EINVAL, "max_nodes must be in [1, 65536]");
    for (int i = 0; i < kParams; ++i)
        if (!std::isfinite(params[i])) return fail(CAPTURE_ENONFINITE, "non-finite initial parameter");
    CAP_HIP(hipSetDevice(ctx->device));
    const size_t nn = size_t(max_nodes);
    Layout L;
    auto plan = [&](uint8_t *base, capture_warmstart *n) {
        L.off = 0;
        n->w = L.take<float>(base, kParams); n->g = L.take<float>(base, kParams);
        n->m = L.take<float>(base, kParams); n->v = L.take<float>(base, kParams);
        n->wb = L.take<uint16_t>(base, kParams);
        n->mu = L.take<float>(base, 32); n->sd = L.take<float>(base, 32);
        n->X = L.take<float>(base, nn * 32); n->Xb = L.take<uint16_t>(base, nn * 32);
        n->z1 = L.take<float>(base, nn * 128); n->c1 = L.take<uint16_t>(base, nn * 256);
        n->z2 = L.take<float>(base, nn * 128); n->c2 = L.take<uint16_t>(base, nn * 256);
        n->y = L.take<float>(base, nn * 6); n->tgt = L.take<float>(base, nn * 6);
        n->dy = L.take<float>(base, nn * 6); n->dyb = L.take<uint16_t>(base, nn * 6);
        n->se = L.take<float>(base, nn * 6); n->dc = L.take<float>(base, nn * 256);
        n->dz = L.take<float>(base, nn * 128); n->dzb = L.take<uint16_t>(base, nn * 128);
    };
    capture_warmstart tmp{};
    plan(nullptr, &tmp);
    void *mem = nullptr;
    if (hipMalloc(&mem, L.off) != hipSuccess) return fail(CAPTURE_ENOMEM, "warm start: device allocation failed");
    capture_warmstart *n = new capture_warmstart{};
    n->device = ctx->device;
    n->max_nodes = max_nodes;
    n->mem = mem;
    plan(static_cast<uint8_t *>(mem), n);
    std::vector<float> zeros(kParams, 0.0f), one(32, 1.0f), zero32(32, 0.0f);
    hipError_t e = hipMemcpy(n->w, params, sizeof(float) * kParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->m, zeros.data(), sizeof(float) * kParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->v, zeros.data(), sizeof(float) * kParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->mu, zero32.data(), sizeof(float) * 32, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->sd, one.data(), sizeof(float) * 32, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks(kParams, 256)), dim3(256), 0, nullptr, n->w, n->wb, kParams);
        e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        (void)hipFree(mem);
        delete n;
        return fail(CAPTURE_EHIP, std::string("warm start: ") + hipGetErrorString(e));
    }
    *out = n;
    return CAPTURE_OK;
}

void capture_warmstart_destroy(capture_warmstart *net) {
    if (!net) return;
    (void)hipFree(net->mem);
    delete net;
}

int capture_warmstart_set_scaling(capture_warmstart *net, const float *mean, const float *stddev) {
    if (!net || !mean || !stddev) return fail(CAPTURE_EINVAL, "null argument");
    for (int i = 0; i < 27; ++i)
        if (!std::isfinite(mean[i]) || !std::isfinite(stddev[i]) || !(stddev[i] > 0.0f))
            return fail(CAPTURE_EINVAL, "scaling: means must be finite and deviations positive");
    CAP_HIP(hipSetDevice(net->device));
    CAP_HIP(hipMemcpy(net->mu, mean, sizeof(float) * 27, hipMemcpyHostToDevice));
    CAP_HIP(hipMemcpy(net->sd, stddev, sizeof(float) * 27, hipMemcpyHostToDevice));
    return CAPTURE_OK;
}

int capture_warmstart_get_params(capture_warmstart *net, float *params, int64_t *adam_steps) {
    if (!net) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(net->device));
    if (params) CAP_HIP(hipMemcpy(params, net->w, sizeof(float) * kParams, hipMemcpyDeviceToHost));
    if (adam_steps) *adam_steps = net->steps;
    return CAPTURE_OK;
}

int capture_warmstart_target(capture_ctx *ctx, int32_t n_nodes, const float *state_prev, const float *state_next,
                             float *target, void *stream) {
    if (!ctx || !state_prev || !state_next || !target) return fail(CAPTURE_EINVAL, "null argument");
    if (n_nodes < 1) return fail(CAPTURE_EINVAL, "n_nodes must be >= 1");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ws_target, dim3(blocks(n_nodes, 256)), dim3(256), 0, s, state_prev, state_next, n_nodes,
                       target);
    CAP_HIP(hipGetLastError());
    CAP_HIP(hipStreamSynchronize(s));
    return CAPTURE_OK;
}

int capture_warmstart_fit_scaling(capture_ctx *ctx, capture_warmstart *net, const float *features, int64_t rows,
                                  void *stream) {
    if (!ctx || !net || !features) return fail(CAPTURE_EINVAL, "null argument");
    if (rows < 1) return fail(CAPTURE_EINVAL, "rows must be >= 1");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ws_scaling, dim3(27), dim3(256), 0, s, features, (long long)rows, net->mu, net->sd);
    CAP_HIP(hipGetLastError());
    CAP_HIP(hipStreamSynchronize(s));
    return CAPTURE_OK;
}

int capture_warmstart_features(capture_ctx *ctx, const capture_frame *frame, const float *state_prev2,
                               const capture_nonrigid_params *params, float *features, void *workspace,
                               size_t workspace_bytes, void *stream) {
    if (!ctx || !params || !features) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    R.prev2 = state_prev2;
    int rc = setup(R, ctx, 1, frame, params, workspace, workspace_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_frame(R))) return rc;
    launch_linearize(R, 0, 0);
    timed(R, K_WS_FEAT, [&] {
        hipLaunchKernelGGL(k_ws_features, dim3(blocks(R.probs[0].T.nn, 256), 1), dim3(256), 0, R.s, R.dprobs,
                           features);
    });
    CAP_HIP(hipGetLastError());
    CAP_HIP(hipStreamSynchronize(R.s));
    settle(R);
    return CAPTURE_OK;
}

int capture_warmstart_forward(capture_ctx *ctx, capture_warmstart *net, const capture_template *tmpl,
                              const float *features, float *y, void *stream) {
    if (!ctx || !net || !tmpl || !features || !y) return fail(CAPTURE_EINVAL, "null argument");
    if (tmpl->dev.nn > net->max_nodes) return fail(CAPTURE_EINVAL, "template has more nodes than the network's max_nodes");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ws_forward(net, tmpl->dev, features, s);
    CAP_HIP(hipGetLastError());
    CAP_HIP(hipMemcpyAsync(y, net->y, sizeof(float) * 6 * tmpl->dev.nn, hipMemcpyDeviceToDevice, s));
    CAP_HIP(hipStreamSynchronize(s));
    return CAPTURE_OK;
}

int capture_warmstart_train_step(capture_ctx *ctx, capture_warmstart *net, const capture_template *tmpl,
                                 const float *features, const float *target, float lr, int update, float *grads,
                                 double *loss, void *stream) {
    if (!ctx || !net || !tmpl || !features || !target) return fail(CAPTURE_EINVAL, "null argument");
    if (tmpl->dev.nn > net->max_nodes) return fail(CAPTURE_EINVAL, "template has more nodes than the network's max_nodes");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(CAPTURE_EINVAL, "lr must be finite and >= 0");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nn = tmpl->dev.nn;
    CAP_HIP(hipMemcpyAsync(net->tgt, target, sizeof(float) * 6 * nn, hipMemcpyDeviceToDevice, s));
    ws_forward(net, tmpl->dev, features, s);
    ws_backward(net, tmpl->dev, s);
    if (grads) CAP_HIP(hipMemcpyAsync(grads, net->g, sizeof(float) * kParams, hipMemcpyDeviceToDevice, s));
    if (update) {
        net->steps += 1;
        const float c1 = float(1.0 - std::pow(0.9, double(net->steps)));
        const float c2 = float(1.0 - std::pow(0.999, double(net->steps)));
        hipLaunchKernelGGL(k_adam, dim3(blocks(kParams, 256)), dim3(256), 0, s, net->w, net->g, net->m, net->v,
                           net->wb, kParams, lr, c1, c2);
    }
    CAP_HIP(hipGetLastError());
    std::vector<float> se(size_t(6) * nn);
    CAP_HIP(hipMemcpyAsync(se.data(), net->se, sizeof(float) * se.size(), hipMemcpyDeviceToHost, s));
    CAP_HIP(hipStreamSynchronize(s));
    if (loss) {
        double acc = 0.0;
        for (float v : se) acc += v;
        *loss = acc / double(se.size());
    }
    return CAPTURE_OK;
}

// Launch sequence of the learned start: preprocessing, linearisation at the
// previous frame's state (features and E(x_{t-1})), the network's prediction
// x' = x (+) delta, Gauss-Newton step 0's full linearisation at x' as the
// energy test, selection (restores x_{t-1} on a rejection; only then does the
// conditional pass linearise the restored start again), then Gauss-Newton.
// With `split`, the sequence ends after Gauss-Newton step 0 and the
// linearisation of step 1 (whose energy test may stop the solve); the caller
// launches the remaining steps only if it did not.
// Step at which a learned-start solve is split (0: not split): the median
// step count of the network's last learned solves (1 before any), if a later
// step remains.
int warm_split_step(const capture_warmstart *net, const capture_nonrigid_params *params, double target) {
    if (params->gn_iters <= 1 || !std::isfinite(target)) return 0;
    int s = 1;
    if (net->n_recent > 0) {
        int v[16];
        std::copy(net->recent_gn, net->recent_gn + net->n_recent, v);
        std::sort(v, v + net->n_recent);
        s = std::max(1, v[net->n_recent / 2]);
    }
    return s < params->gn_iters ? s : 0;
}

int warm_sequence(Run &R, const capture_nonrigid_params *params, capture_warmstart *net, int split) {
    const ProbDev &pr = R.probs[0];
    const int prev_slot = CAPTURE_MAX_GN + 1;     // energy at the given start (x_{t-1})
    int rc = launch_frame(R, params->gn_iters);   // keeps the given state in state0
    if (rc) return rc;
    launch_linearize(R, prev_slot, 0);
    timed(R, K_WS_MLP, [&] {      // features and the prediction, applied to the node state by the last layer
        hipLaunchKernelGGL(k_ws_layer1_feat, dim3(unsigned((pr.T.nn + 15) / 16)), dim3(512), 0, R.s, R.dprobs, net->X,
                           net->mu, net->sd, net->wb + kOffW1, net->w + kOffB1, net->Xb, net->z1, net->c1);
        ws_forward(net, pr.T, nullptr, R.s, pr.x, R.dprobs);
    });
    launch_linearize(R, 0, 0, 1 | 4, prev_slot, params->gn_iters);      // energy test and selection
    timed(R, K_LIN, [&] {
        hipLaunchKernelGGL(k_linearize, dim3(unsigned(R.grid_tiles)), dim3(kTileThreads), R.lds_lin, R.s, R.dprobs,
                           R.tiles, 2);
    });
    timed(R, K_NODE_INIT, [&] {
        hipLaunchKernelGGL(k_node_init, dim3(kInitBlocks, R.n), dim3(kInitThreads), 0, R.s, R.dprobs, 3);
        hipLaunchKernelGGL(k_node_init_fin, dim3(R.n), dim3(kInitFinThreads), 0, R.s, R.dprobs, 0, 0, 3, 0, 0, kInitBlocks);
    });
    if (!split) return launch_solve(R, params, 1, true);
    launch_steps(R, params, 1, true, 0, split);
    launch_linearize(R, split, 0, 1);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

// The rest of a learned-start solve split at step `split`: steps split.. and the final energy.
int warm_rest(Run &R, const capture_nonrigid_params *params, int split) {
    launch_steps(R, params, 1, true, split, params->gn_iters);
    launch_linearize(R, params->gn_iters, 1);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

int capture_nonrigid_solve_warm(capture_ctx *ctx, const capture_frame *frame, const capture_nonrigid_params *params,
                                capture_warmstart *net, const float *state_prev2, double target_energy,
                                capture_report *report, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx || !params || !net || !report || !frame) return fail(CAPTURE_EINVAL, "null argument");
    if (std::isnan(target_energy)) return fail(CAPTURE_EINVAL, "target_energy is NaN");
    if (frame->tmpl && frame->tmpl->dev.nn > net->max_nodes)
        return fail(CAPTURE_EINVAL, "template has more nodes than the network's max_nodes");
    CAP_HIP(hipSetDevice(ctx->device));
    Run R;
    R.target = target_energy;
    R.prev2 = state_prev2;
    int rc = setup(R, ctx, 1, frame, params, workspace, workspace_bytes, stream);
    if (rc) return rc;
    const ProbDev &pr = R.probs[0];
    // A good prediction reaches the target within a step or two: the solve is
    // launched in two parts, the first through the energy test at the start of
    // step `split` (the median step count of recent learned solves), the second
    // only if that test has not stopped it (one read-back of the stop flag in
    // between).  A solve that stops early thus pays neither for the launches of
    // its remaining steps (which would find the stop flag and return) nor, in
    // the common case, for a second round trip.
    const int split = warm_split_step(net, params, target_energy);
    const bool graph = ctx->graphs && !ctx->prof.on;
    char net_key[128];    // the forward pass takes the network, edge table and x as arguments
    std::snprintf(net_key, sizeof net_key, "warm%d|%p|%p|%p|", split, (void *)net,
                  (const void *)pr.T.edge_dst, (void *)pr.x);
    const std::string key = net_key + shape_key(R, params);
    auto first = [&](Run &C) { return warm_sequence(C, params, net, split); };
    rc = graph ? launch_graph(R, key, first) : first(R);
    if (rc) return rc;
    const double *sc = nullptr;
    bool done = false;
    if (split) {      // the read-back of the stop flag brings the whole report along
        const uint8_t *host = nullptr;
        if ((rc = read_back(R, &host))) return rc;
        if (reinterpret_cast<const double *>(host)[2] != 0.0) {      // stopped: nothing more runs
            settle(R);
            rc = reports_from(R, host, params->gn_iters, report, &sc);
            done = true;
        } else {
            auto rest = [&](Run &C) { return warm_rest(C, params, split); };
            rc = graph ? launch_graph(R, "rest|" + key, rest) : rest(R);
            if (rc) return rc;
        }
    }
    if (!done) rc = collect(R, params->gn_iters, report, &sc);
    if (!sc) return rc;
    report->energy_pred = sc[4];
    report->energy_prev = sc[6];
    report->warm_start = sc[5] != 0.0 ? 2 : 1;
    if (std::isfinite(target_energy)) {        // step counts of target-driven solves set the next split
        net->recent_gn[net->recent_pos] = report->gn_done;
        net->recent_pos = (net->recent_pos + 1) % 16;
        net->n_recent = std::min(net->n_recent + 1, 16);
    }
    if (rc) {
        (void)hipMemcpyAsync(frame->node_state, pr.state0, sizeof(float) * 12 * pr.T.nn, hipMemcpyDeviceToDevice, R.s);
        (void)hipStreamSynchronize(R.s);
        return fail(rc, "non-finite energy; node state restored");
    }
    return CAPTURE_OK;
}

int capture_set_graphs(capture_ctx *ctx, int on) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null ctx");
    ctx->graphs = on != 0;
    return CAPTURE_OK;
}

int capture_profile_enable(capture_ctx *ctx, int on) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null ctx");
    ctx->prof.on = on != 0;
    return CAPTURE_OK;
}

int capture_profile_read(capture_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches) {
    if (!ctx || !kernel) return fail(CAPTURE_EINVAL, "null argument");
    for (int k = 0; k < K_COUNT; ++k)
        if (std::strcmp(kernel, kKernelNames[k]) == 0) {
            if (total_ms) *total_ms = ctx->prof.total_ms[k];
            if (launches) *launches = ctx->prof.launches[k];
            ctx->prof.total_ms[k] = 0.0;
            ctx->prof.launches[k] = 0;
            return CAPTURE_OK;
        }
    return fail(CAPTURE_EINVAL, std::string("unknown kernel name: ") + kernel);
}

}  // extern "C"
