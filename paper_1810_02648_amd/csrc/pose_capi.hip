// C ABI of the pose stage: body creation, workspace layout and the launch
// sequence of one pose solve (decisions at the start pose, then Gauss-Newton
// steps of rows -> J^T J tiles -> Cholesky step).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.hpp"
#include "runtime.hpp"

namespace cap {

int build_topology_template(const int *tri_dev, int nv, int nf, capture_template **out, int device);

__global__ void k_contour(const ProbDev *P);
__global__ void k_dt_seg(const ProbDev *P);
__global__ void k_prep_raster(const ProbDev *P, int nb_f, int scan);
__global__ void k_prep_cols(const ProbDev *P);
__global__ void k_prep_rows(const ProbDev *P, int nb_rows);
__global__ void k_decide(const ProbDev *P);
__global__ void k_pose_fk(const PoseDev *P);
__global__ void k_pose_lbs(const PoseDev *P, const ProbDev *R, int nbv);
__global__ void k_pose_list(const PoseDev *P);
__global__ void k_pose_rows(const PoseDev *P, int energy_only);
__global__ void k_pose_jtj(const PoseDev *P);
__global__ void k_pose_step(const PoseDev *P, int gn, int nblk, int mode);
__global__ void k_body_skin(BodyDev B, const double *pose, float *out);
__global__ void k_body_warp(BodyDev B, const double *pose_prev, const double *pose_cur, const float *Vp,
                            const float *Sp, const float *Sc, float *out);
__global__ void k_pose_extrapolate(int nu, const double *p, const double *p2, double *out);
__global__ void k_body_joints(BodyDev B, const double *pose, double *out);

namespace {

struct PoseRun {
    Run R;                   // the decision kernels' problem (one frame)
    PoseDev pd{};
    PoseDev *dpose = nullptr;
    int max_rows = 0, row_blocks = 0, ntp = 0;
};

// Workspace: [ProbDev][PoseDev] then the frame buffers, then the pose buffers.
size_t carve_pose(uint8_t *base, const capture_pose_frame &f, ProbDev &pr, PoseDev &pd, int &max_rows) {
    const BodyDev &B = f.body->dev;
    const TemplateDev &T = f.body->topo->dev;
    const size_t nv = T.nv, nf = T.nf, hw = size_t(f.camera.width) * f.camera.height;
    Layout L;
    L.take<ProbDev>(base, 1);
    L.take<PoseDev>(base, 1);
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
    max_rows = pose_fixed_rows(B.nj, B.it) + int(nv);
    pd.jR = L.take<double>(base, size_t(9) * B.nj);
    pd.jp = L.take<double>(base, size_t(3) * B.nj);
    pd.jA = L.take<double>(base, size_t(9) * B.nj);
    pd.pose0 = L.take<double>(base, B.nu);
    pd.blist = L.take<int>(base, nv);
    pd.nb = L.take<int>(base, 1);
    pd.ldr = (max_rows + 63) & ~63;
    pd.rows = L.take<double>(base, size_t(pd.ldr) * B.np);
    pd.epart = L.take<double>(base, size_t(blocks(max_rows, kPoseRowThreads)) * kPoseTerms);
    pd.sys = L.take<double>(base, size_t(B.nu) * (B.nu + 1));
    // the report's items together, so that one read-back takes them
    pd.energy = L.take<double>(base, size_t(CAPTURE_MAX_GN + 1) * kPoseTerms);
    pr.counts = L.take<int>(base, 3);
    pd.status = L.take<int>(base, 1);
    return L.off;
}

int check_pose_frame(const capture_pose_frame *f) {
    if (!f || !f->body) return fail(CAPTURE_EINVAL, "pose frame without body");
    if (!f->mask || !f->p2d || !f->p3d || !f->lambda || !f->pose) return fail(CAPTURE_EINVAL, "pose frame: null array");
    const capture_camera &c = f->camera;
    if (c.width < 1 || c.height < 1 || c.width > kMaxImageSide || c.height > kMaxImageSide)
        return fail(CAPTURE_EUNSUPPORTED, "camera: image sides must be in [1, 4096]");
    if (!std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy) || c.fx == 0.0f ||
        c.fy == 0.0f)
        return fail(CAPTURE_EINVAL, "camera: non-finite or zero intrinsics");
    return CAPTURE_OK;
}

int check_pose_params(const capture_pose_params *p) {
    if (!p) return fail(CAPTURE_EINVAL, "null params");
    if (p->gn_iters < 1 || p->gn_iters > CAPTURE_MAX_GN) return fail(CAPTURE_EINVAL, "gn_iters must be in [1, 32]");
    if (!std::isfinite(p->l2d) || !std::isfinite(p->l3d) || !std::isfinite(p->lsil) || p->l2d < 0 || p->l3d < 0 ||
        p->lsil < 0)
        return fail(CAPTURE_EINVAL, "weights must be finite and non-negative");
    if (p->flags & ~uint32_t(CAPTURE_FLAG_EXCLUDE_CASE2 | CAPTURE_FLAG_OUTLINE_ONLY))
        return fail(CAPTURE_EINVAL, "unknown flag bits");
    for (int j = 0; j < CAPTURE_MAX_JOINTS; ++j)
        if (!std::isfinite(p->l_temporal[j]) || p->l_temporal[j] < 0)
            return fail(CAPTURE_EINVAL, "temporal weights must be finite and non-negative");
    if (!std::isfinite(p->l_anatomic) || p->l_anatomic < 0)
        return fail(CAPTURE_EINVAL, "the joint-limit weight must be finite and non-negative");
    for (int q = 0; q < CAPTURE_MAX_POSE_UNKNOWNS; ++q)
        if (std::isnan(p->theta_min[q]) || std::isnan(p->theta_max[q]) || p->theta_min[q] > p->theta_max[q])
            return fail(CAPTURE_EINVAL, "joint limits: theta_min <= theta_max, no NaN");
    return CAPTURE_OK;
}

int pose_setup(PoseRun &P, capture_ctx *ctx, const capture_pose_frame *f, const capture_pose_params *prm, void *ws,
               size_t ws_bytes, void *stream) {
    int rc = check_pose_frame(f);
    if (rc) return rc;
    if ((rc = check_pose_params(prm))) return rc;
    if (f->body->device != ctx->device) return fail(CAPTURE_EINVAL, "body belongs to another device");
    ProbDev pr{};
    PoseDev pd{};
    int max_rows = 0;
    const size_t need = carve_pose(nullptr, *f, pr, pd, max_rows);
    if (!ws || ws_bytes < need) return fail(CAPTURE_ENOMEM, "workspace too small");
    uint8_t *base = static_cast<uint8_t *>(ws);
    carve_pose(base, *f, pr, pd, max_rows);
    const capture_body &body = *f->body;
    pr.T = body.topo->dev;
    pr.xyz = body.dev.xyz;
    pr.rgb = nullptr;
    pr.mask = f->mask;
    pr.W = f->camera.width;
    pr.H = f->camera.height;
    pr.fx = f->camera.fx; pr.fy = f->camera.fy; pr.cx = f->camera.cx; pr.cy = f->camera.cy;
    pr.exclude_case2 = int(prm->flags & CAPTURE_FLAG_EXCLUDE_CASE2);
    pr.outline_only = int((prm->flags & CAPTURE_FLAG_OUTLINE_ONLY) != 0);
    pr.w_vel = 0.0f;
    pr.target = -INFINITY;
    pd.B = body.dev;
    pd.W = pr.W; pd.H = pr.H;
    pd.fx = f->camera.fx; pd.fy = f->camera.fy; pd.cx = f->camera.cx; pd.cy = f->camera.cy;
    pd.l2d = prm->l2d;
    pd.s3d = std::sqrt(prm->l3d);
    pd.ssil = std::sqrt(prm->lsil);
    pd.p2d = f->p2d; pd.p3d = f->p3d; pd.lam = f->lambda;
    bool temporal = false;
    for (int j = 0; j < body.dev.nj; ++j) {
        pd.stemp[j] = std::sqrt(prm->l_temporal[j]);
        temporal = temporal || prm->l_temporal[j] > 0.0;
    }
    if (temporal && !f->prev_joints) return fail(CAPTURE_EINVAL, "temporal weights without prev_joints");
    pd.prev_joints = temporal ? f->prev_joints : nullptr;
    pd.sanat = std::sqrt(prm->l_anatomic);
    for (int q = 0; q < kMaxPoseUnknowns; ++q) {
        pd.lim_lo[q] = prm->theta_min[q];
        pd.lim_hi[q] = prm->theta_max[q];
    }
    pd.pose = f->pose;
    pd.dt = pr.dt;
    pd.vflags = pr.vflags;
    Run &R = P.R;
    R.ctx = ctx;
    R.prof = &ctx->prof;
    R.n = 1;
    R.probs.resize(1);
    R.probs[0] = pr;
    R.dprobs = reinterpret_cast<ProbDev *>(base);
    R.s = static_cast<hipStream_t>(stream);
    R.max_nv = pr.T.nv; R.max_nf = pr.T.nf; R.max_me = pr.T.nmedges;
    R.max_hw = pr.W * pr.H; R.max_w = pr.W; R.max_h = pr.H;
    P.pd = pd;
    P.dpose = reinterpret_cast<PoseDev *>(base + ((sizeof(ProbDev) + 255) & ~size_t(255)));
    P.max_rows = max_rows;
    P.row_blocks = int(blocks(max_rows, kPoseRowThreads));
    const int nt = pd.B.np / kPoseTile;
    P.ntp = nt * (nt + 1) / 2;
    // both descriptors in one upload from the context's pinned staging
    const size_t poff = reinterpret_cast<uint8_t *>(P.dpose) - reinterpret_cast<uint8_t *>(R.dprobs);
    uint8_t *stage = static_cast<uint8_t *>(run_staging(R, poff + sizeof(PoseDev)));
    if (!stage) return fail(CAPTURE_ENOMEM, "host staging allocation failed");
    std::memcpy(stage, &R.probs[0], sizeof(ProbDev));
    std::memcpy(stage + poff, &P.pd, sizeof(PoseDev));
    CAP_HIP(hipMemcpyAsync(R.dprobs, stage, poff + sizeof(PoseDev), hipMemcpyHostToDevice, R.s));
    return CAPTURE_OK;
}

// Start pose: kinematics, skinning, distance transform, raster and decisions,
// then the contour list.
int launch_pose_decisions(PoseRun &P) {
    Run &R = P.R;
    hipStream_t s = R.s;
    const ProbDev &pr = R.probs[0];
    const size_t hw = size_t(pr.W) * pr.H;
    timed(R, K_POSE_LBS, [&] {           // (the skinning also zeroes the counters and clears the depth buffer)
        const int nbv = int(blocks(pr.T.nv, 256));
        hipLaunchKernelGGL(k_pose_fk, dim3(1), dim3(64), 0, s, P.dpose);
        hipLaunchKernelGGL(k_pose_lbs, dim3(nbv + int(blocks(hw, 2048))), dim3(256), 0, s, P.dpose, R.dprobs, nbv);
    });
    const dim3 gpx(blocks(hw, 256));
    timed(R, K_CONTOUR, [&] { hipLaunchKernelGGL(k_contour, gpx, dim3(256), 0, s, R.dprobs); });
    // steps with the same predecessors share a launch, as in the
    // deformation-graph path: rasterisation + segment scan, large faces +
    // column distances, row pass + contour edges
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
    timed(R, K_DECIDE, [&] {
        hipLaunchKernelGGL(k_decide, dim3(blocks(pr.T.nv, 256)), dim3(256), 0, s, R.dprobs);
        hipLaunchKernelGGL(k_pose_list, dim3(1), dim3(1024), 0, s, P.dpose);
    });
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

// Rows and J^T J tiles at the current pose, then k_pose_step in `mode`.
int launch_pose_step(PoseRun &P, int gn, int mode) {
    Run &R = P.R;
    hipStream_t s = R.s;
    const int energy_only = mode == 1;
    timed(R, K_POSE_ROWS, [&] {
        hipLaunchKernelGGL(k_pose_rows, dim3(P.row_blocks), dim3(kPoseRowThreads), 0, s, P.dpose, energy_only);
    });
    if (!energy_only)
        timed(R, K_POSE_JTJ, [&] {
            hipLaunchKernelGGL(k_pose_jtj, dim3(P.ntp), dim3(256), 0, s, P.dpose);
        });
    timed(R, K_POSE_STEP, [&] {
        hipLaunchKernelGGL(k_pose_step, dim3(1), dim3(1024), 0, s, P.dpose, gn, P.row_blocks, mode);
    });
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

}  // namespace
}  // namespace cap

using namespace cap;

extern "C" {

int capture_body_create(capture_ctx *ctx, const capture_body_desc *d, capture_body **out) {
    if (!ctx || !d || !out) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    const int nv = d->n_vertices, nf = d->n_triangles, nj = d->n_joints;
    if (nj < 1 || nj > kMaxJoints) return fail(CAPTURE_EUNSUPPORTED, "body: n_joints must be in [1, 32]");
    if (nv < 1 || nf < 1) return fail(CAPTURE_EINVAL, "body: need n_vertices >= 1 and n_triangles >= 1");
    if (nv > (1 << 28)) return fail(CAPTURE_EUNSUPPORTED, "body: too many vertices");
    if (!d->tri || !d->xyz || !d->bind_joint || !d->bind_w || !d->parents || !d->rest_joints || !d->has_rotation)
        return fail(CAPTURE_EINVAL, "body: null array");
    BodyDev B{};
    B.nj = nj;
    B.nv = nv;
    int ncol = 0;
    for (int j = 0; j < nj; ++j) {
        const int p = d->parents[j];
        if ((j == 0) != (p < 0) || p >= j || p < -1)
            return fail(CAPTURE_EINVAL, "body: parents must be -1 for joint 0 only and parents[j] < j");
        B.parent[j] = p;
        B.depth[j] = p < 0 ? 0 : B.depth[p] + 1;
        B.anc[j] = (p < 0 ? 0u : B.anc[p]) | (1u << j);
        B.maxdepth = std::max(B.maxdepth, B.depth[j]);
        B.col[j] = d->has_rotation[j] ? ncol : -1;
        if (d->has_rotation[j]) ncol += 3;
        for (int a = 0; a < 3; ++a) {
            const double x = d->rest_joints[size_t(a) * nj + j];
            if (!std::isfinite(x)) return fail(CAPTURE_ENONFINITE, "body: non-finite rest joint");
            B.rest[a][j] = x;
        }
    }
    B.it = ncol;
    B.itp = ncol + 3;
    B.nu = ncol + 6;
    if (B.nu > kMaxPoseUnknowns) return fail(CAPTURE_EUNSUPPORTED, "body: more than 81 unknowns");
    B.np = (B.nu + 1 + kPoseTile - 1) / kPoseTile * kPoseTile;
    // skinning: copy down, check, upload with the rest mesh
    std::vector<int> bj(size_t(4) * nv);
    std::vector<float> bw(size_t(4) * nv), xyz(size_t(3) * nv);
    CAP_HIP(hipMemcpy(bj.data(), d->bind_joint, bj.size() * sizeof(int), hipMemcpyDeviceToHost));
    CAP_HIP(hipMemcpy(bw.data(), d->bind_w, bw.size() * sizeof(float), hipMemcpyDeviceToHost));
    CAP_HIP(hipMemcpy(xyz.data(), d->xyz, xyz.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int v : bj) if (v < 0 || v >= nj) return fail(CAPTURE_EINVAL, "body: bind_joint out of range");
    for (float w : bw) if (!std::isfinite(w)) return fail(CAPTURE_ENONFINITE, "body: non-finite skinning weight");
    for (float x : xyz) if (!std::isfinite(x)) return fail(CAPTURE_ENONFINITE, "body: non-finite vertex");
    capture_template *topo = nullptr;
    int rc = build_topology_template(d->tri, nv, nf, &topo, ctx->device);
    if (rc) return rc;
    const size_t b_xyz = sizeof(float) * xyz.size(), b_bj = sizeof(int) * bj.size(), b_bw = sizeof(float) * bw.size();
    void *mem = nullptr;
    if (hipMalloc(&mem, b_xyz + b_bj + b_bw) != hipSuccess) {
        capture_template_destroy(topo);
        return fail(CAPTURE_ENOMEM, "body: device allocation failed");
    }
    uint8_t *m = static_cast<uint8_t *>(mem);
    if (hipMemcpy(m, xyz.data(), b_xyz, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + b_xyz, bj.data(), b_bj, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m + b_xyz + b_bj, bw.data(), b_bw, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        capture_template_destroy(topo);
        return fail(CAPTURE_EHIP, "body: upload failed");
    }
    B.xyz = reinterpret_cast<const float *>(m);
    B.bind_joint = reinterpret_cast<const int *>(m + b_xyz);
    B.bind_w = reinterpret_cast<const float *>(m + b_xyz + b_bj);
    capture_body *b = new capture_body;
    b->dev = B;
    b->topo = topo;
    b->mem = mem;
    b->device = ctx->device;
    *out = b;
    return CAPTURE_OK;
}

void capture_body_destroy(capture_body *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipFree(b->mem);
    capture_template_destroy(b->topo);
    delete b;
}

int capture_body_unknowns(const capture_body *b, int32_t *n) {
    if (!b || !n) return fail(CAPTURE_EINVAL, "null argument");
    *n = b->dev.nu;
    return CAPTURE_OK;
}

int capture_pose_workspace_size(capture_ctx *ctx, const capture_pose_frame *f, size_t *bytes) {
    if (!ctx || !bytes) return fail(CAPTURE_EINVAL, "null argument");
    int rc = check_pose_frame(f);
    if (rc) return rc;
    ProbDev pr{};
    PoseDev pd{};
    int max_rows = 0;
    *bytes = carve_pose(nullptr, *f, pr, pd, max_rows);
    return CAPTURE_OK;
}

int capture_pose_solve(capture_ctx *ctx, const capture_pose_frame *f, const capture_pose_params *prm,
                       capture_pose_report *rep, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx || !rep) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    PoseRun P;
    int rc = pose_setup(P, ctx, f, prm, ws, ws_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_pose_decisions(P))) return rc;
    const int G = prm->gn_iters;
    for (int g = 0; g < G; ++g)
        if ((rc = launch_pose_step(P, g, 0))) return rc;
    if ((rc = launch_pose_step(P, G, 1))) return rc;
    // energies, counts and status (adjacent in the workspace) in one
    // read-back into the context's pinned staging, after the descriptor
    // upload from it on the stream
    const uint8_t *d0 = reinterpret_cast<const uint8_t *>(P.pd.energy.ptr);
    const size_t off_counts = reinterpret_cast<const uint8_t *>(P.R.probs[0].counts.ptr) - d0;
    const size_t off_status = reinterpret_cast<const uint8_t *>(P.pd.status.ptr) - d0;
    uint8_t *h = static_cast<uint8_t *>(run_staging(P.R, off_status + sizeof(int)));
    if (!h) return fail(CAPTURE_ENOMEM, "host staging allocation failed");
    hipStream_t s = P.R.s;
    CAP_HIP(hipMemcpyAsync(h, d0, off_status + sizeof(int), hipMemcpyDeviceToHost, s));
    CAP_HIP(hipStreamSynchronize(s));
    settle(P.R);
    const double *en = reinterpret_cast<const double *>(h);
    int st = 0, counts[2] = {0, 0};
    std::memcpy(counts, h + off_counts, sizeof(counts));
    std::memcpy(&st, h + off_status, sizeof(int));
    *rep = capture_pose_report{};
    for (int g = 0; g <= G; ++g) {
        const double *e = en + kPoseTerms * g;
        rep->energy[g] = (((e[0] + e[1]) + e[2]) + e[4]) + e[5];
    }
    const double *e = en + kPoseTerms * G;
    rep->e2d = e[0];
    rep->e3d = e[1];
    rep->e_sil = e[2];
    rep->e_sil_abs = e[3];
    rep->e_temporal = e[4];
    rep->e_anatomic = e[5];
    rep->n_visible = counts[0];
    rep->n_boundary = counts[1];
    rep->gn_done = G;
    rep->status = st;
    if (st) return fail(st, st == CAPTURE_ENOTSPD ? "pose system not positive definite; pose restored"
                                                   : "non-finite pose energy; pose restored");
    return CAPTURE_OK;
}

int capture_pose_linearize(capture_ctx *ctx, const capture_pose_frame *f, const capture_pose_params *prm,
                           double *system, double *energy, uint8_t *vflags, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    PoseRun P;
    int rc = pose_setup(P, ctx, f, prm, ws, ws_bytes, stream);
    if (rc) return rc;
    if ((rc = launch_pose_decisions(P))) return rc;
    if ((rc = launch_pose_step(P, 0, 2))) return rc;
    hipStream_t s = P.R.s;
    const int nu = P.pd.B.nu;
    double en[kPoseTerms];
    if (system) CAP_HIP(hipMemcpyAsync(system, P.pd.sys, sizeof(double) * nu * (nu + 1), hipMemcpyDeviceToDevice, s));
    if (vflags) CAP_HIP(hipMemcpyAsync(vflags, P.R.probs[0].vflags, P.pd.B.nv, hipMemcpyDeviceToDevice, s));
    CAP_HIP(hipMemcpyAsync(en, P.pd.energy, sizeof(en), hipMemcpyDeviceToHost, s));
    CAP_HIP(hipStreamSynchronize(s));
    settle(P.R);
    if (energy)
        for (int q = 0; q < kPoseTerms; ++q) energy[q] = en[q];
    return CAPTURE_OK;
}

int capture_body_skin(capture_ctx *ctx, const capture_body *b, const double *pose, float *xyz, void *stream) {
    if (!ctx || !b || !pose || !xyz) return fail(CAPTURE_EINVAL, "null argument");
    if (b->device != ctx->device) return fail(CAPTURE_EINVAL, "body belongs to another device");
    CAP_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_body_skin, dim3(blocks(b->dev.nv, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       b->dev, pose, xyz);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

int capture_body_warp(capture_ctx *ctx, const capture_body *b, const double *pose_prev, const double *pose_cur,
                      const float *V_prev, const float *posed_prev, const float *posed_cur, float *start,
                      void *stream) {
    if (!ctx || !b || !pose_prev || !pose_cur || !V_prev || !posed_prev || !posed_cur || !start)
        return fail(CAPTURE_EINVAL, "null argument");
    if (b->device != ctx->device) return fail(CAPTURE_EINVAL, "body belongs to another device");
    CAP_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_body_warp, dim3(blocks(b->dev.nv, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       b->dev, pose_prev, pose_cur, V_prev, posed_prev, posed_cur, start);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

int capture_body_joints(capture_ctx *ctx, const capture_body *b, const double *pose, double *joints, void *stream) {
    if (!ctx || !b || !pose || !joints) return fail(CAPTURE_EINVAL, "null argument");
    if (b->device != ctx->device) return fail(CAPTURE_EINVAL, "body belongs to another device");
    CAP_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_body_joints, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), b->dev, pose, joints);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

int capture_pose_extrapolate(capture_ctx *ctx, const capture_body *b, const double *pose_prev,
                             const double *pose_prev2, double *pose_out, void *stream) {
    if (!ctx || !b || !pose_prev || !pose_prev2 || !pose_out) return fail(CAPTURE_EINVAL, "null argument");
    CAP_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pose_extrapolate, dim3(1), dim3(128), 0, static_cast<hipStream_t>(stream), b->dev.nu,
                       pose_prev, pose_prev2, pose_out);
    CAP_HIP(hipGetLastError());
    return CAPTURE_OK;
}

}  // extern "C"
