// C ABI entry points: argument checks, workspace layout and the launch
// sequence of the per-frame solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.hpp"

namespace cap {

// kernels defined in the other translation units
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v);
__global__ void k_blur(const ProbDev *P, int pass, float w0, float w1);
__global__ void k_contour(const ProbDev *P);
__global__ void k_dt_cols(const ProbDev *P);
__global__ void k_dt_rows(const ProbDev *P);
__global__ void k_deform_start(const ProbDev *P);
__global__ void k_raster(const ProbDev *P);
__global__ void k_contour_edges(const ProbDev *P);
__global__ void k_decide(const ProbDev *P);
__global__ void k_linearize(const ProbDev *P, int mode);
__global__ void k_apply(const ProbDev *P);
__global__ void k_node_init(const ProbDev *P, int gn, int energy_only);
__global__ void k_node_gather(const ProbDev *P);
__global__ void k_node_pcg(const ProbDev *P, int last, int update_only);
int build_template(const capture_template_desc *d, capture_template **out, int device);

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// ---------------------------------------------------------------- graph build kernels
__device__ inline float d2f(float ax, float ay, float az, float bx, float by, float bz) {
    float dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

// Farthest-point sampling in one workgroup; argmax ties -> lowest index.
__global__ __launch_bounds__(1024) void k_fps(const float *__restrict__ xyz, int nv, int nn, float *mind,
                                              int *node_vertex) {
    __shared__ float bv[1024];
    __shared__ int bi[1024];
    __shared__ float sel[3];
    const float *X = xyz, *Y = xyz + nv, *Z = xyz + 2 * size_t(nv);
    if (threadIdx.x == 0) { node_vertex[0] = 0; sel[0] = X[0]; sel[1] = Y[0]; sel[2] = Z[0]; }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x) mind[v] = d2f(X[v], Y[v], Z[v], sel[0], sel[1], sel[2]);
    for (int n = 1; n < nn; ++n) {
        float best = -1.0f;
        int bidx = 0x7fffffff;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            float m = mind[v];
            if (m > best) { best = m; bidx = v; }
        }
        bv[threadIdx.x] = best;
        bi[threadIdx.x] = bidx;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (int(threadIdx.x) < s) {
                float ov = bv[threadIdx.x + s];
                int oi = bi[threadIdx.x + s];
                if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                    bv[threadIdx.x] = ov;
                    bi[threadIdx.x] = oi;
                }
            }
            __syncthreads();
        }
        const int s = bi[0];
        if (threadIdx.x == 0) { node_vertex[n] = s; sel[0] = X[s]; sel[1] = Y[s]; sel[2] = Z[s]; }
        __syncthreads();
        const float sx = sel[0], sy = sel[1], sz = sel[2];
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            float d = d2f(X[v], Y[v], Z[v], sx, sy, sz);
            if (d < mind[v]) mind[v] = d;
        }
        __syncthreads();
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
struct Layout {
    size_t off = 0;
    template <typename T>
    T *take(uint8_t *base, size_t n) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += std::max<size_t>(n, 1) * sizeof(T);
        return p;
    }
};

void carve(Layout &L, uint8_t *base, const capture_frame &f, ProbDev &pr) {
    const TemplateDev &T = f.tmpl->dev;
    const size_t nv = T.nv, nf = T.nf, nn = T.nn, hw = size_t(f.camera.width) * f.camera.height;
    pr.blur_tmp = L.take<float>(base, 3 * hw);
    pr.blurred = L.take<float>(base, 3 * hw);
    pr.dt = L.take<float>(base, hw);
    pr.colg = L.take<int>(base, hw);
    pr.zbuf = L.take<uint32_t>(base, hw);
    pr.contour = L.take<uint8_t>(base, hw);
    pr.dx = L.take<float>(base, 3 * nv);
    pr.duv = L.take<float>(base, 2 * nv);
    pr.dfix = L.take<int>(base, 2 * nv);
    pr.dvalid = L.take<uint8_t>(base, nv);
    pr.vcont = L.take<uint8_t>(base, nv);
    pr.vflags = L.take<uint8_t>(base, nv);
    pr.fcross = L.take<float>(base, 3 * nf);
    pr.px = L.take<float>(base, 3 * nv);
    pr.pc = L.take<float>(base, 3 * nv);
    pr.vcode = L.take<uint8_t>(base, nv);
    pr.Hm = L.take<float>(base, 6 * nv);
    pr.partial = L.take<float>(base, size_t(T.nslots) * 12);
    pr.tile_e = L.take<double>(base, size_t(T.ntiles) * 4);
    float **vecs[8] = {&pr.b, &pr.diag, &pr.dinv, &pr.x, &pr.r, &pr.z, &pr.p, &pr.Ap};
    for (float **v : vecs) *v = L.take<float>(base, 6 * nn);
    pr.scal = L.take<double>(base, kScalars);
    pr.counts = L.take<int>(base, 2);
    pr.state0 = L.take<float>(base, 12 * nn);
}

struct Plan {
    size_t bytes = 0;
};

Plan plan_workspace(int n, const capture_frame *frames, uint8_t *base, std::vector<ProbDev> *probs) {
    Layout L;
    Plan pl;
    L.take<ProbDev>(base, n);
    for (int i = 0; i < n; ++i) {
        ProbDev pr{};
        carve(L, base, frames[i], pr);
        if (probs) (*probs)[i] = pr;
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
    if (!finite(p->w_sil) || !finite(p->w_photo) || !finite(p->w_arap) || p->w_sil < 0 || p->w_photo < 0 || p->w_arap < 0)
        return fail(CAPTURE_EINVAL, "weights must be finite and non-negative");
    if (std::isnan(p->tau_color) || p->tau_color < 0) return fail(CAPTURE_EINVAL, "tau_color must be >= 0 or +inf");
    return CAPTURE_OK;
}

// What a run should do beyond the per-frame preprocessing.
enum class Stage { Decisions, Linearize, Solve };

struct Run {
    Profiler *prof = nullptr;
    int n = 0;
    std::vector<ProbDev> probs;
    ProbDev *dprobs = nullptr;
    int max_nv = 0, max_nf = 0, max_hw = 0, max_w = 0, max_h = 0, max_tiles = 0, max_me = 0;
    size_t lds_lin = 0, lds_apply = 0;
    hipStream_t s = nullptr;
};

const char *kKernelNames[K_COUNT] = {"blur", "contour", "dt_cols", "dt_rows", "deform_start", "raster",
                                     "contour_edges", "decide", "linearize", "node_init", "apply", "node_pcg"};

// Launch `go` bracketed by events when timing is on.
template <typename F>
void timed(Run &R, int kid, F go) {
    Profiler *P = R.prof;
    if (!P || !P->on) { go(); return; }
    while (P->ev.size() < P->used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { go(); return; }
        P->ev.push_back(e);
    }
    const size_t i = P->used;
    P->used += 2;
    (void)hipEventRecord(P->ev[i], R.s);
    go();
    (void)hipEventRecord(P->ev[i + 1], R.s);
    P->pending.push_back({kid, i});
}

// After the stream has been synchronised: fold the event pairs into the totals.
void settle(Run &R) {
    Profiler *P = R.prof;
    if (!P) return;
    for (auto &pe : P->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, P->ev[pe.second], P->ev[pe.second + 1]) == hipSuccess) {
            P->total_ms[pe.first] += ms;
            P->launches[pe.first] += 1;
        }
    }
    P->pending.clear();
    P->used = 0;
}

int setup(Run &R, capture_ctx *ctx, int n, const capture_frame *frames, const capture_nonrigid_params *params,
          void *ws, size_t ws_bytes, void *stream) {
    R.prof = &ctx->prof;
    int rc = check_frames(n, frames);
    if (rc) return rc;
    if (params && (rc = check_params(params))) return rc;
    Plan pl = plan_workspace(n, frames, nullptr, nullptr);
    if (!ws || ws_bytes < pl.bytes) return fail(CAPTURE_ENOMEM, "workspace too small");
    R.n = n;
    R.probs.resize(n);
    uint8_t *base = static_cast<uint8_t *>(ws);
    plan_workspace(n, frames, base, &R.probs);
    R.dprobs = reinterpret_cast<ProbDev *>(base);
    R.s = static_cast<hipStream_t>(stream);
    const float wsil = params ? params->w_sil : 1.0f, wph = params ? params->w_photo : 0.1f,
                war = params ? params->w_arap : 10.0f;
    const float tau = params ? (params->tau_color > 0 ? params->tau_color : INFINITY) : INFINITY;
    for (int i = 0; i < n; ++i) {
        const capture_frame &f = frames[i];
        ProbDev &pr = R.probs[i];
        pr.T = f.tmpl->dev;
        pr.xyz = f.xyz; pr.rgb = f.rgb; pr.mask = f.mask; pr.image = f.image; pr.state = f.node_state;
        pr.W = f.camera.width; pr.H = f.camera.height;
        pr.fx = f.camera.fx; pr.fy = f.camera.fy; pr.cx = f.camera.cx; pr.cy = f.camera.cy;
        pr.sw_sil = std::sqrt(wsil); pr.sw_photo = std::sqrt(wph); pr.sw_arap = std::sqrt(war);
        pr.w_arap = war; pr.tau = tau;
        const TemplateDev &T = pr.T;
        R.max_nv = std::max(R.max_nv, T.nv);
        R.max_nf = std::max(R.max_nf, T.nf);
        R.max_me = std::max(R.max_me, T.nmedges);
        R.max_tiles = std::max(R.max_tiles, T.ntiles);
        R.max_hw = std::max(R.max_hw, pr.W * pr.H);
        R.max_w = std::max(R.max_w, pr.W);
        R.max_h = std::max(R.max_h, pr.H);
        R.lds_lin = std::max(R.lds_lin, sizeof(float) * (size_t(T.max_slots) * 15 + size_t(T.max_contrib) * 12));
        R.lds_apply = std::max(R.lds_apply, sizeof(float) * (size_t(T.max_slots) * 21 + size_t(T.max_contrib) * 6));
    }
    CAP_HIP(hipMemcpyAsync(R.dprobs, R.probs.data(), sizeof(ProbDev) * n, hipMemcpyHostToDevice, R.s));
    return CAPTURE_OK;
}

unsigned blocks(size_t n, unsigned t) { return unsigned((n + t - 1) / t); }

int launch_frame(Run &R) {
    const int n = R.n;
    hipStream_t s = R.s;
    for (int i = 0; i < n; ++i) {
        const ProbDev &pr = R.probs[i];
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks(size_t(pr.W) * pr.H, 256)), dim3(256), 0, s, pr.zbuf,
                           size_t(pr.W) * pr.H, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(pr.counts), size_t(2), 0u);
    }
    // Gaussian kernel 3, sigma = 0.3 * ((3 - 1) / 2 - 1) + 0.8 = 0.8, normalised
    const double e1 = std::exp(-1.0 / (2.0 * 0.8 * 0.8));
    const float w0 = float(e1 / (1.0 + 2.0 * e1)), w1 = float(1.0 / (1.0 + 2.0 * e1));
    const dim3 gpx(blocks(R.max_hw, 256), n), gv(blocks(R.max_nv, 256), n);
    timed(R, K_BLUR, [&] {
    hipLaunchKernelGGL(k_blur, gpx, dim3(256), 0, s, R.dprobs, 0, w0, w1);
    });
    timed(R, K_BLUR, [&] {
    hipLaunchKernelGGL(k_blur, gpx, dim3(256), 0, s, R.dprobs, 1, w0, w1);
    });
    timed(R, K_CONTOUR, [&] {
    hipLaunchKernelGGL(k_contour, gpx, dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_DT_COLS, [&] {
    hipLaunchKernelGGL(k_dt_cols, dim3(blocks(R.max_w, 64), n), dim3(64), 0, s, R.dprobs);
    });
    timed(R, K_DT_ROWS, [&] {
    hipLaunchKernelGGL(k_dt_rows, dim3(R.max_h, n), dim3(256), sizeof(int) * R.max_w, s, R.dprobs);
    });
    timed(R, K_DEFORM, [&] {
    hipLaunchKernelGGL(k_deform_start, gv, dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_RASTER, [&] {
    hipLaunchKernelGGL(k_raster, dim3(blocks(R.max_nf, 256), n), dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_CEDGES, [&] {
    hipLaunchKernelGGL(k_contour_edges, dim3(blocks(R.max_me, 256), n), dim3(256), 0, s, R.dprobs);
    });
    timed(R, K_DECIDE, [&] {
    hipLaunchKernelGGL(k_decide, gv, dim3(256), 0, s, R.dprobs);
    });
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

void launch_linearize(Run &R, int gn, int energy_only) {
    timed(R, K_LIN, [&] {
    hipLaunchKernelGGL(k_linearize, dim3(R.max_tiles, R.n), dim3(kTileThreads), R.lds_lin, R.s, R.dprobs,
                           energy_only);
    });
    timed(R, K_NODE_INIT, [&] {
    hipLaunchKernelGGL(k_node_init, dim3(R.n), dim3(kNodeThreads), 0, R.s, R.dprobs, gn, energy_only);
    });
}

int launch_solve(Run &R, const capture_nonrigid_params *prm) {
    for (int gn = 0; gn < prm->gn_iters; ++gn) {
        launch_linearize(R, gn, 0);
        for (int j = 0; j < prm->pcg_iters; ++j) {
            timed(R, K_APPLY, [&] {
    hipLaunchKernelGGL(k_apply, dim3(R.max_tiles, R.n), dim3(kTileThreads), R.lds_apply, R.s, R.dprobs);
            });
            timed(R, K_NODE_PCG, [&] {
    hipLaunchKernelGGL(k_node_pcg, dim3(R.n), dim3(kNodeThreads), 0, R.s, R.dprobs,
                                   j == prm->pcg_iters - 1 ? 1 : 0, 0);
            });
        }
        if (prm->pcg_iters == 0)
            timed(R, K_NODE_PCG, [&] {
    hipLaunchKernelGGL(k_node_pcg, dim3(R.n), dim3(kNodeThreads), 0, R.s, R.dprobs, 0, 1);
            });
    }
    launch_linearize(R, prm->gn_iters, 1);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

int collect(Run &R, int gn_iters, capture_report *reports) {
    std::vector<double> scal(size_t(kScalars) * R.n);
    std::vector<int> counts(size_t(2) * R.n);
    for (int i = 0; i < R.n; ++i) {
        CAP_HIP(hipMemcpyAsync(scal.data() + size_t(kScalars) * i, R.probs[i].scal, sizeof(double) * kScalars,
                               hipMemcpyDeviceToHost, R.s));
        CAP_HIP(hipMemcpyAsync(counts.data() + 2 * i, R.probs[i].counts, sizeof(int) * 2, hipMemcpyDeviceToHost, R.s));
    }
    CAP_HIP(hipStreamSynchronize(R.s));
    settle(R);
    int status = CAPTURE_OK;
    for (int i = 0; i < R.n; ++i) {
        capture_report &rep = reports[i];
        std::memset(&rep, 0, sizeof(rep));
        const double *sc = scal.data() + size_t(kScalars) * i;
        for (int k = 0; k <= gn_iters; ++k) rep.energy[k] = sc[8 + 4 * k] + sc[8 + 4 * k + 1] + sc[8 + 4 * k + 3];
        const double *e = sc + 8 + 4 * gn_iters;
        rep.e_photo = e[0]; rep.e_sil = e[1]; rep.e_sil_abs = e[2]; rep.e_arap = e[3];
        rep.n_visible = counts[2 * i];
        rep.n_boundary = counts[2 * i + 1];
        rep.gn_done = gn_iters;
        rep.status = std::isfinite(rep.energy[gn_iters]) ? CAPTURE_OK : CAPTURE_ENONFINITE;
        if (rep.status) status = rep.status;
    }
    return status;
}

}  // namespace cap

using namespace cap;

extern "C" {

const char *capture_last_error(void) { return g_err.c_str(); }

int capture_create(capture_ctx **ctx, int device) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null ctx pointer");
    int count = 0;
    CAP_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CAPTURE_EINVAL, "no such device");
    CAP_HIP(hipSetDevice(device));
    *ctx = new capture_ctx();
    (*ctx)->device = device;
    return CAPTURE_OK;
}

void capture_destroy(capture_ctx *ctx) {
    if (!ctx) return;
    for (hipEvent_t e : ctx->prof.ev) (void)hipEventDestroy(e);
    delete ctx;
}

int capture_graph_build(capture_ctx *ctx, const float *xyz, int32_t n_vertices, int32_t n_nodes, int32_t *node_vertex,
                        int32_t *bind_idx, float *bind_w, int32_t *edge_dst, void *stream) {
    if (!ctx || !xyz || !node_vertex || !bind_idx || !bind_w || !edge_dst) return fail(CAPTURE_EINVAL, "null argument");
    if (n_nodes < 4 || n_nodes > n_vertices || n_nodes > 65536)
        return fail(CAPTURE_EINVAL, "graph: need 4 <= n_nodes <= n_vertices and n_nodes <= 65536");
    CAP_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *mind = nullptr;
    if (hipMalloc(&mind, sizeof(float) * size_t(n_vertices)) != hipSuccess)
        return fail(CAPTURE_ENOMEM, "graph: scratch allocation failed");
    hipLaunchKernelGGL(k_fps, dim3(1), dim3(1024), 0, s, xyz, n_vertices, n_nodes, mind, node_vertex);
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
    for (int i = 0; i < n; ++i)
        CAP_HIP(hipMemcpyAsync(R.probs[i].state0, frames[i].node_state, sizeof(float) * 12 * R.probs[i].T.nn,
                               hipMemcpyDeviceToDevice, R.s));
    if ((rc = launch_frame(R))) return rc;
    if ((rc = launch_solve(R, params))) return rc;
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
    hipLaunchKernelGGL(k_apply, dim3(R.max_tiles, 1), dim3(kTileThreads), R.lds_apply, R.s, R.dprobs);
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
    if (energy) for (int q = 0; q < 4; ++q) energy[q] = sc[8 + q];
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
