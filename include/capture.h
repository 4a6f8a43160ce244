/*
 * capture.h -- C ABI of the MI355X (gfx950) per-frame Gauss-Newton solvers
 * for monocular human performance capture (LiveCap, Habermann et al.,
 * ACM TOG 2019).
 *
 * Conventions shared by every entry point
 *  - Array arguments are DEVICE pointers unless marked "host".  Multi-channel
 *    arrays are structure-of-arrays: [3][n] means three planes of n values.
 *    Images are row-major [H][W]; pixel (i, j) = (column, row) has its centre
 *    at image coordinates (i, j).
 *  - The caller owns every buffer.  The library never frees caller memory and
 *    keeps no caller pointer past the call, except that a template keeps its
 *    own device copy of the static data it derives (capture_template_create).
 *  - Scratch memory comes from the caller's workspace (capture_workspace_size);
 *    solves allocate nothing.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.  Work
 *    is enqueued on it; solve calls wait for it before returning (the report
 *    is filled on return).
 *  - Errors: negative return codes; capture_last_error() gives a message
 *    (thread-local, valid until the next call on that thread).  Nothing
 *    throws across the ABI.  Arguments are validated before any launch; on an
 *    error return no output has been modified.
 */
#ifndef CAPTURE_H
#define CAPTURE_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define CAPTURE_API __attribute__((visibility("default")))
#else
#define CAPTURE_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CAPTURE_OK = 0,
    CAPTURE_EINVAL = -1,       /* invalid argument (sizes, null pointers, non-manifold mesh) */
    CAPTURE_ENOTSPD = -2,      /* a linear system was not positive definite */
    CAPTURE_ENONFINITE = -3,   /* a non-finite value was found in inputs or results */
    CAPTURE_EHIP = -4,         /* a HIP runtime call failed */
    CAPTURE_ENOMEM = -5,       /* workspace too small, or template allocation failed */
    CAPTURE_EUNSUPPORTED = -6  /* a size beyond a documented limit */
};

#define CAPTURE_BIND_K 4       /* nodes per vertex (embedded deformation binding) */
#define CAPTURE_EDGE_K 8       /* out-edges per node (regulariser graph) */
#define CAPTURE_MAX_GN 32      /* maximum Gauss-Newton steps per solve */

typedef struct capture_ctx capture_ctx;
typedef struct capture_template capture_template;

/* Pinhole camera, world = camera frame (Sec. 3.2: static camera, camera and
 * world space are the same): u = fx*X/Z + cx, v = fy*Y/Z + cy. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} capture_camera;

/* Open a context on HIP device `device`.  *ctx receives an opaque handle. */
CAPTURE_API int capture_create(capture_ctx **ctx, int device);
CAPTURE_API void capture_destroy(capture_ctx *ctx);
CAPTURE_API const char *capture_last_error(void);

/* --------------------------------------------------------------------------
 * Deformation graph (embedded deformation nodes; the paper names this
 * parameterisation as the alternative to per-vertex unknowns, Sec. 6).
 *   xyz          [3][n_vertices]  rest positions (float32)
 *   node_vertex  [n_nodes]        out: farthest-point samples, seeded at vertex
 *                                 0, argmax ties -> lowest vertex index
 *   bind_idx     [4][n_vertices]  out: 4 nearest nodes, ascending distance,
 *                                 ties -> lower node index
 *   bind_w       [4][n_vertices]  out: exp(-d^2 / (2 d4^2)) normalised to sum 1,
 *                                 d4 = distance to the 4th-nearest node
 *   edge_dst     [8][n_nodes]     out: 8 nearest other nodes (ties -> lower
 *                                 index), -1 when fewer exist
 * Squared distances use one float32 recipe ((dx*dx + dy*dy) + dz*dz) so the
 * indices are reproducible bit for bit.  Requires 4 <= n_nodes <= n_vertices
 * and n_nodes <= 65536.  Synchronous (one kernel launch per node for the
 * sampling).  Set-up, not per frame: the call allocates and frees a device
 * scratch of about 4 * n_vertices bytes (plus 4 KiB of per-workgroup partials).
 * ------------------------------------------------------------------------ */
CAPTURE_API int capture_graph_build(capture_ctx *ctx, const float *xyz, int32_t n_vertices, int32_t n_nodes,
                        int32_t *node_vertex, int32_t *bind_idx, float *bind_w, int32_t *edge_dst,
                        void *stream);

/* --------------------------------------------------------------------------
 * Template: static mesh topology plus graph.  Creation reads the arrays once
 * (device pointers), checks them (indices in range, edge-manifold mesh with
 * each edge in one or two faces, binding weights finite) and builds the
 * library's tiled execution plan in its own device memory.  Triangles wind
 * counter-clockwise seen from outside.
 *   nodes_per_tile / vertices_per_tile: 0 = library defaults (autotuned).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_vertices, n_triangles, n_nodes;
    const int32_t *tri;          /* [3][n_triangles] */
    const int32_t *node_vertex;  /* [n_nodes] */
    const int32_t *bind_idx;     /* [4][n_vertices] */
    const float *bind_w;         /* [4][n_vertices] */
    const int32_t *edge_dst;     /* [8][n_nodes], -1 = no edge */
    int32_t vertices_per_tile;   /* 0 = default (256); at most 256 */
} capture_template_desc;

CAPTURE_API int capture_template_create(capture_ctx *ctx, const capture_template_desc *desc,
                            capture_template **out);
CAPTURE_API void capture_template_destroy(capture_template *tmpl);

/* Shape of a template's execution plan (host memory, filled by
 * capture_template_info; no device work).  Tiles are contiguous ranges of the
 * plan's vertex order processed by one workgroup each; a slot is a graph node
 * touched by a tile; contributions are the per-tile (vertex binding or
 * regulariser edge end) terms summed per slot. */
typedef struct {
    int32_t n_vertices, n_triangles, n_nodes;
    int32_t n_tiles, n_slots;       /* tiles, and slots over all tiles */
    int32_t max_slots, max_contrib; /* largest per-tile counts */
    int32_t vertices_per_tile;      /* the cap the plan was built with */
} capture_template_info;

/* Returns CAPTURE_EINVAL for a null argument. */
CAPTURE_API int capture_template_info_get(const capture_template *tmpl, capture_template_info *out);

/* One frame of the non-rigid stage (Sec. 3.4). */
typedef struct {
    const capture_template *tmpl;
    const float *xyz;          /* [3][n_vertices] the frame's input mesh (e.g. the posed
                                  template); graph node k sits at xyz[:, node_vertex[k]] */
    const float *rgb;          /* [3][n_vertices] template vertex colours C, in [0, 1] */
    capture_camera camera;
    const uint8_t *mask;       /* [H][W] foreground silhouette, 0 = background */
    const float *image;        /* [3][H][W] colour frame in [0, 1] */
    float *node_state;         /* [12][n_nodes] in: start, out: solution; per node the
                                  rotation R row-major (9 values) then translation t (3) */
} capture_frame;

/* Weights and schedule.  E = w_photo*sum||sigma_c(I_Gauss(pi(V_i)) - C_i)||^2
 *  + w_sil*sum b_i I_DT(pi(V_i))^2 + w_arap*sum||R_k(g_l - g_k) + g_k + t_k - g_l - t_l||^2
 *  + w_vel*sum_i ||V_i - V_i^a||^2.
 * tau_color: the photometric robust-kernel threshold sigma_c (Sec. 3.4: a
 * vertex's colour residual is set to zero when the norm of its colour
 * difference exceeds tau_color, compared in float32); +inf disables it, 0
 * prunes every residual whose colour difference is not exactly zero.
 * w_vel: the paper's temporal prior E_velocity (Sec. 3.4) over all vertices, with
 * the previous frame's result carried to the current pose: V^a is the input
 * mesh deformed by the start node state (the previous frame's solution);
 * 0 disables it.
 * CAPTURE_FLAG_EXCLUDE_CASE2: contour vertices in the paper's case 2 (inside the
 * image silhouette with the normal opposing z, b_i = -1) get no silhouette
 * residual instead of the literal -I_DT^2, which is unbounded below. */
#define CAPTURE_FLAG_EXCLUDE_CASE2 1u
/* Jacobi-PCG runs in one of two arrangements with the same iterates in exact
 * arithmetic (Sec. 4: a fixed number of PCG iterations per Gauss-Newton step).
 * Schedules of at most 16 iterations on at most 1024 tiles (all frames of the
 * call) take one launch per iteration (Chronopoulos-Gear form); longer
 * schedules and larger grids take the standard recurrence (two launches per
 * iteration), whose rounding stays bounded over hundreds of iterations.
 * CAPTURE_FLAG_PCG_STANDARD always takes the standard recurrence. */
#define CAPTURE_FLAG_PCG_STANDARD 4u
typedef struct {
    float w_sil, w_photo, w_arap, tau_color, w_vel;
    int32_t gn_iters;          /* 1..CAPTURE_MAX_GN */
    int32_t pcg_iters;         /* >= 0 Jacobi-PCG iterations per Gauss-Newton step (the cap when pcg_tol > 0) */
    uint32_t flags;            /* CAPTURE_FLAG_* */
    float pcg_tol;             /* 0: exactly pcg_iters iterations; > 0: a step's PCG also stops once the
                                  residual of the normal equations satisfies ||r|| <= pcg_tol ||b||
                                  (b = -J^T B F; PCG run to convergence) */
} capture_nonrigid_params;

/* Host-side report of one solve. */
typedef struct {
    double energy[CAPTURE_MAX_GN + 1];    /* E at the start of each GN step taken, then the final E
                                             (entries 0..gn_done are valid) */
    double e_photo, e_sil, e_sil_abs, e_arap, e_vel;  /* final per-term energies (e_sil_abs: with |b_i|) */
    double energy_prev, energy_pred;      /* warm start only: E at the given state, E at the predicted start */
    int32_t n_visible, n_boundary;        /* |visible set|, |contour set| */
    int32_t gn_done;                      /* Gauss-Newton steps taken */
    int32_t warm_start;                   /* 0 plain start; 1 predicted start used; 2 predicted start
                                             rejected (higher energy), solve ran from the given state */
    int32_t status;                       /* CAPTURE_OK or a device-detected error */
} capture_report;

/* Workspace bytes for solving the `n` frames together (n = 1 for a single
 * frame).  Frames are host structs; their arrays are not read. */
CAPTURE_API int capture_workspace_size(capture_ctx *ctx, int32_t n, const capture_frame *frames, size_t *bytes);

/* Non-rigid Gauss-Newton solve of one frame (Sec. 3.4 energy, Sec. 4 solver:
 * J^T J delta = -J^T F with J^T J applied matrix-free and solved by
 * Jacobi-preconditioned CG, fixed iteration counts).  The once-per-frame
 * decisions (visible set by depth buffering, contour set B, direction signs
 * b_i) are taken at the start state.  `report` is host memory. */
CAPTURE_API int capture_nonrigid_solve(capture_ctx *ctx, const capture_frame *frame,
                           const capture_nonrigid_params *params, capture_report *report,
                           void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same solve of one frame
 * as capture_nonrigid_solve, with no workspace argument.  Scratch is a 32 MiB
 * device array that the library holds on every device it runs on until the
 * process ends (its address is looked up once per device by capture_create);
 * descriptor upload and report read-back go through a fixed 64 KiB host
 * buffer.  On success the call performs no device, pinned or host allocation
 * and launches eagerly (graphs and kernel timing do not apply).  Every call
 * on a device shares that device's scratch and the one host buffer, and the
 * scratch keeps the last call's contents (the solve initialises everything
 * it reads): calls that overlap, on any stream or thread, race and must be
 * serialised by the caller.  A frame whose workspace (capture_workspace_size)
 * exceeds 32 MiB, e.g. a 1080x1080 image with a 20,000-vertex template fits
 * and a 1200x1200 image does not, or whose descriptors exceed the host
 * buffer, returns CAPTURE_EUNSUPPORTED before any launch.  Errors as for
 * capture_nonrigid_solve. */
CAPTURE_API int capture_nonrigid_solve_noalloc(capture_ctx *ctx, const capture_frame *frame,
                                               const capture_nonrigid_params *params, capture_report *report,
                                               void *stream);

/* The same solve for `n` independent frames of possibly different sizes in one
 * sequence of batched launches.  `frames` and `reports` are host arrays of n;
 * all frames share `params`. */
CAPTURE_API int capture_batch_solve(capture_ctx *ctx, int32_t n, const capture_frame *frames,
                        const capture_nonrigid_params *params, capture_report *reports,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Tile-size autotuner (setup time, not per frame).  For each candidate
 * vertices_per_tile it builds the n templates of `descs` with that tile size,
 * times one batched solve of `frames` (whose tmpl is replaced by the
 * candidate's) three times after a warm-up, and keeps the fastest; *best
 * receives that candidate and times_ms (host, n_candidates, may be NULL) the
 * best time of each.  Every trial starts from the frames' node_state, which is
 * left unchanged.  Allocates and frees its own device memory; synchronous. */
CAPTURE_API int capture_autotune_tiles(capture_ctx *ctx, int32_t n, const capture_template_desc *descs,
                                       const capture_frame *frames, const capture_nonrigid_params *params,
                                       const int32_t *candidates, int32_t n_candidates, int32_t *best,
                                       double *times_ms, void *stream);

/* --------------------------------------------------------------------------
 * Stage entry points: the per-frame preprocessing and one linearisation, with
 * their intermediate results, for callers that need them (and for checking).
 * All outputs are caller-allocated device arrays; any may be NULL.
 * ------------------------------------------------------------------------ */

/* Per-frame preprocessing at the frame's node_state (Sec. 3.2 distance
 * transform, Sec. 3.4 blurred image, visibility, contour set, signs):
 *   dt        [H][W] float   Euclidean distance (px) to the nearest contour pixel
 *   blurred   [3][H][W]      Gaussian blur (kernel 3, sigma 0.8, clamp-to-edge)
 *   zbuf      [H][W] uint32  float bits of the largest inverse depth, 0 = empty
 *   vflags    [n_vertices] uint8: bit0 visible, bit1 contour set B, bit2 b_i = -1 */
CAPTURE_API int capture_frame_decisions(capture_ctx *ctx, const capture_frame *frame, float *dt, float *blurred,
                            uint32_t *zbuf, uint8_t *vflags, void *workspace, size_t workspace_bytes,
                            void *stream);

/* One linearisation at the frame's node_state (decisions taken at the same
 * state), then the matrix-free product:
 *   rhs   [6][n_nodes]  -J^T B F per node (dw_x, dw_y, dw_z, dt_x, dt_y, dt_z)
 *   diag  [6][n_nodes]  diagonal of J^T |B| J
 *   p     [6][n_nodes]  input direction (may be NULL: no product)
 *   Ap    [6][n_nodes]  out: J^T |B| J p
 *   energy (host, 5 doubles): photo, sil (with b_i), sil with |b_i|, arap, velocity */
CAPTURE_API int capture_linearize(capture_ctx *ctx, const capture_frame *frame, const capture_nonrigid_params *params,
                      float *rhs, float *diag, const float *p, float *Ap, double *energy,
                      void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * Learned warm start.  A per-node network (shared weights) with two rounds of
 * mean message passing over the node graph predicts the start update of a
 * frame from the previous frame's node parameters and per-node statistics of
 * the new frame's linearisation at those parameters; the paper's plain start
 * (the previous frame's result, Sec. 3.4) stays the fallback.  Layers:
 *   h1 = ReLU(W1 x + b1) (32 -> 128), m1 = mean over out-neighbours of h1,
 *   h2 = ReLU(W2 [h1; m1] + b2) (256 -> 128), m2 = mean of h2,
 *   y = W3 [h2; m2] + b3 (256 -> 6); update = y * (0.05, 0.05, 0.05 rad, 0.01, 0.01, 0.01 m).
 * Parameter vector (float32, host order): W1 [128][32], b1 [128], W2 [128][256],
 * b2 [128], W3 [6][256], b3 [6]; CAPTURE_WS_PARAMS values.  Matrix products
 * run on BF16 MFMA with float32 accumulation; master weights and Adam state are
 * float32 (Adam: beta 0.9 / 0.999, eps 1e-8).
 * Features per node (32 floats, [n_nodes][32], zero-padded after 27):
 *   axis-angle of R_k, t_k, change of both since frame t-2 (0 without it),
 *   sign(b) log(1 + |b|) of b = -J^T B F (6), log(1 + diag(J^T |B| J)) (6),
 *   node position minus the mean node position (3).
 * ------------------------------------------------------------------------ */
#define CAPTURE_WS_PARAMS 38662
#define CAPTURE_WS_FEATURES 32

typedef struct capture_warmstart capture_warmstart;

/* Network with the given initial parameters (host, CAPTURE_WS_PARAMS floats),
 * activation buffers for up to max_nodes nodes (library-owned device memory). */
CAPTURE_API int capture_warmstart_create(capture_ctx *ctx, int32_t max_nodes, const float *params,
                                         capture_warmstart **out);
CAPTURE_API void capture_warmstart_destroy(capture_warmstart *net);
/* Feature standardisation (host, 27 means and 27 standard deviations > 0). */
CAPTURE_API int capture_warmstart_set_scaling(capture_warmstart *net, const float *mean, const float *stddev);
/* Current float32 parameters (host, CAPTURE_WS_PARAMS) and Adam step count. */
CAPTURE_API int capture_warmstart_get_params(capture_warmstart *net, float *params, int64_t *adam_steps);

/* Fit the feature standardisation to `rows` raw feature rows (device,
 * [rows][32], e.g. all nodes of all training frames): per-feature mean and
 * standard deviation (floored at 1e-6). */
CAPTURE_API int capture_warmstart_fit_scaling(capture_ctx *ctx, capture_warmstart *net, const float *features,
                                              int64_t rows, void *stream);
/* Training target [n_nodes][6] (device): per node (dw, dt) with
 * R_next = Exp(dw) R_prev, t_next = t_prev + dt, divided by (0.05, 0.05, 0.05, 0.01, 0.01, 0.01). */
CAPTURE_API int capture_warmstart_target(capture_ctx *ctx, int32_t n_nodes, const float *state_prev,
                                         const float *state_next, float *target, void *stream);
/* Raw (unstandardised) features [n_nodes][32] at the frame's node_state
 * (device output); state_prev2: [12][n_nodes] node state of frame t-2, or NULL. */
CAPTURE_API int capture_warmstart_features(capture_ctx *ctx, const capture_frame *frame, const float *state_prev2,
                                           const capture_nonrigid_params *params, float *features,
                                           void *workspace, size_t workspace_bytes, void *stream);
/* Network output y [n_nodes][6] (scaled units) for raw features of a template's nodes. */
CAPTURE_API int capture_warmstart_forward(capture_ctx *ctx, capture_warmstart *net, const capture_template *tmpl,
                                          const float *features, float *y, void *stream);
/* One training step on one frame: loss = mean (y - target)^2 over the n_nodes x 6
 * outputs (target in scaled units, [n_nodes][6] device).  grads (device,
 * CAPTURE_WS_PARAMS floats) receives the gradient if not NULL; with `update` the
 * Adam step is applied.  *loss (host) receives the loss before the update. */
CAPTURE_API int capture_warmstart_train_step(capture_ctx *ctx, capture_warmstart *net, const capture_template *tmpl,
                                             const float *features, const float *target, float lr, int update,
                                             float *grads, double *loss, void *stream);
/* Non-rigid solve started by the network: decisions and linearisation at the
 * frame's node_state (the previous frame's result), predicted start x',
 * energies at both; the lower one starts Gauss-Newton, which stops at the
 * start of the first step whose energy is <= target_energy (pass -inf for the
 * full schedule).  report->warm_start tells which start was used.  With a
 * finite target the launches are issued in two parts with one read-back of
 * the stop flag in between; the first part ends at the step count that the
 * network's last 16 target-driven solves needed (median; 1 at first), so the
 * network keeps that history (launch policy only: results do not depend on it). */
CAPTURE_API int capture_nonrigid_solve_warm(capture_ctx *ctx, const capture_frame *frame,
                                            const capture_nonrigid_params *params, capture_warmstart *net,
                                            const float *state_prev2, double target_energy, capture_report *report,
                                            void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * Pose stage (Sec. 3.3 energy, Sec. 4 pose solver).  A skeleton of
 * n_joints joints; each rotating joint carries three axis-angle unknowns
 * (joint order; the root's rotation is the global rotation), followed by the
 * root translation t (3) and the translation t' (3) that maps the
 * root-relative 3D detections into the camera frame: n_unknowns =
 * 3 * (rotating joints) + 6.  Joint rotations compose down the tree,
 * R_j = R_parent Exp(theta_j), p_j = p_parent + R_parent (J_j - J_parent),
 * p_root = J_root + t, and the mesh follows by linear blend skinning (the
 * paper skins with dual quaternions; this library uses LBS) with 4
 * influences per vertex: V_i = sum_s w_s (R_j (v_i - J_j) + p_j).
 * Energy: E = l2d sum_j lambda_j ||pi(p_j) - P2D_j||^2
 *           + l3d sum_j ||p_j - (P3D_j + t')||^2 + lsil sum_{i in B} b_i I_DT(pi(V_i))^2
 *           + E_temporal + E_anatomic (see capture_pose_params),
 * decisions (visible set, contour set B, signs b_i) taken once per solve at
 * the start pose with the same raster and decision rules as the non-rigid
 * stage.  Each Gauss-Newton step solves (J^T J + mu I) delta = -J^T B F with
 * mu = 1e-6 * max diag(J^T J) by a dense FP64 Cholesky factorisation, then
 * theta <- theta + delta (additive axis-angle update).
 * ------------------------------------------------------------------------ */
#define CAPTURE_MAX_JOINTS 32
#define CAPTURE_MAX_POSE_UNKNOWNS 81

typedef struct capture_body capture_body;

typedef struct {
    int32_t n_vertices, n_triangles, n_joints;
    const int32_t *tri;           /* [3][n_triangles] (closed parts may overlap) */
    const float *xyz;             /* [3][n_vertices] rest mesh, skinned to the rest joints */
    const int32_t *bind_joint;    /* [4][n_vertices] joint of each skinning influence */
    const float *bind_w;          /* [4][n_vertices] influence weights (sum 1 per vertex) */
    const int32_t *parents;       /* host [n_joints]: -1 for joint 0 only, otherwise parents[j] < j */
    const double *rest_joints;    /* host [3][n_joints] rest joint positions (metres) */
    const int32_t *has_rotation;  /* host [n_joints]: 1 = the joint carries 3 axis-angle unknowns */
} capture_body_desc;

/* Validates the description (sizes, tree order, indices, edge-manifold mesh,
 * finite weights, n_unknowns <= CAPTURE_MAX_POSE_UNKNOWNS) and keeps a device
 * copy of the mesh tables, skinning and skeleton.  Synchronous. */
CAPTURE_API int capture_body_create(capture_ctx *ctx, const capture_body_desc *desc, capture_body **out);
CAPTURE_API void capture_body_destroy(capture_body *body);
CAPTURE_API int capture_body_unknowns(const capture_body *body, int32_t *n_unknowns);

typedef struct {
    const capture_body *body;
    capture_camera camera;
    const uint8_t *mask;          /* [H][W] foreground silhouette, 0 = background */
    const double *p2d;            /* [2][n_joints] 2D joint detections (pixels) */
    const double *p3d;            /* [3][n_joints] root-relative 3D joint detections (metres) */
    const double *lambda;         /* [n_joints] per-joint 2D confidences, >= 0 */
    double *pose;                 /* [n_unknowns] in: start pose, out: solution */
    const double *prev_joints;    /* [3][n_joints] joint positions of the previous frame (E_temporal), or NULL */
} capture_pose_frame;

/* CAPTURE_FLAG_OUTLINE_ONLY: B keeps only contour vertices on the outline of
 * the rendered model (an uncovered pixel in the 3x3 window around the vertex
 * pixel); contours of parts seen in front of other parts are dropped.  Also
 * CAPTURE_FLAG_EXCLUDE_CASE2 as for the non-rigid stage. */
#define CAPTURE_FLAG_OUTLINE_ONLY 2u
/* Body-part mask of the per-vertex stage's silhouette term (capture_vertex_params). */
#define CAPTURE_FLAG_PART_MASK 8u
/* E_temporal = sum_j l_temporal[j] ||p_j - p_j^{t-1}|| ^2 (Sec. 3.3, temporal
 * stabilisation: l_temporal[j] = lambda_temporal * lambda_j) needs
 * frame->prev_joints when any weight is > 0.  E_anatomic = l_anatomic *
 * sum_q Psi(theta_q) over the rotational unknowns q < 3 * (rotating joints)
 * (Sec. 3.3, joint angle limits: the quadratic barrier outside
 * [theta_min[q], theta_max[q]]; +-inf for an unlimited unknown).  Zero
 * weights leave the terms out. */
typedef struct {
    double l2d, l3d, lsil;        /* term weights, finite and >= 0 */
    int32_t gn_iters;             /* 1..CAPTURE_MAX_GN */
    uint32_t flags;               /* CAPTURE_FLAG_EXCLUDE_CASE2 | CAPTURE_FLAG_OUTLINE_ONLY */
    double l_temporal[CAPTURE_MAX_JOINTS];
    double l_anatomic;
    double theta_min[CAPTURE_MAX_POSE_UNKNOWNS], theta_max[CAPTURE_MAX_POSE_UNKNOWNS];
} capture_pose_params;

typedef struct {
    double energy[CAPTURE_MAX_GN + 1];    /* E at the start of each step, then the final E */
    double e2d, e3d, e_sil, e_sil_abs;    /* final per-term energies (e_sil_abs: with |b_i|) */
    double e_temporal, e_anatomic;
    int32_t n_visible, n_boundary, gn_done;
    int32_t status;                       /* CAPTURE_OK or a device-detected error */
} capture_pose_report;

/* Workspace bytes of one pose frame (a host struct; its arrays are not read). */
CAPTURE_API int capture_pose_workspace_size(capture_ctx *ctx, const capture_pose_frame *frame, size_t *bytes);

/* Gauss-Newton pose solve of one frame.  On a device-detected error (a
 * non-positive Cholesky pivot, a non-finite energy) frame->pose is restored
 * to the start pose and the status is returned. */
CAPTURE_API int capture_pose_solve(capture_ctx *ctx, const capture_pose_frame *frame,
                                   const capture_pose_params *params, capture_pose_report *report,
                                   void *workspace, size_t workspace_bytes, void *stream);

/* Decisions and one linearisation at frame->pose (not modified):
 *   system  [n_unknowns][n_unknowns + 1] (device, may be NULL): J^T J (undamped)
 *           with -J^T B F as the last column
 *   energy  host [6]: 2D, 3D, silhouette (with b_i), silhouette with |b_i|, temporal, joint limits
 *   vflags  [n_vertices] (device, may be NULL): bit0 visible, bit1 in B, bit2 b_i = -1 */
CAPTURE_API int capture_pose_linearize(capture_ctx *ctx, const capture_pose_frame *frame,
                                       const capture_pose_params *params, double *system, double *energy,
                                       uint8_t *vflags, void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * Per-vertex non-rigid stage: the paper's own Stage II parameterisation
 * (Sec. 3.4): the unknowns are the vertex positions V (3 per vertex),
 *   E(V) = w_photo sum_{i visible} ||sigma_c(I_Gauss(pi(V_i)) - C_i)||^2
 *        + w_sil sum_{i in B} b_i I_DT(pi(V_i))^2
 *        + w_smooth sum_i sum_{j in N_i} s_ij/|N_i| ||(V_i - V_j) - (V^S_i - V^S_j)||^2
 *        + w_edge sum_i sum_{j in N_i} s_ij/|N_i| (||V_i - V_j|| - ||Vhat_i - Vhat_j||)^2
 *        + w_vel sum_i ||V_i - V^{t-1}_i||^2 + w_acc sum_i ||V_i - 2 V^{t-1}_i + V^{t-2}_i||^2
 * (Sec. 3.4: dense photometric and silhouette alignment, spatial smoothness,
 * edge length, velocity and acceleration priors).  N_i is the one-ring of
 * vertex i, Vhat the rest pose, V^S the skinned pose result, and
 * s_ij = (s_i + s_j) / 2 with s_i the Table 1 non-rigidity weight of vertex
 * i's material class (Sec. 3.1: class 1..7 -> 1, 2, 2.5, 3, 50, 100, 200).
 * Decisions (visible set, contour set B, signs b_i) are taken once at the
 * start positions with the rules of the embedded-deformation stage.  Each
 * Gauss-Newton step solves J^T |B| J delta = -J^T B F by Jacobi-preconditioned
 * CG (Sec. 4, non-rigid paragraph: rows parallelised per vertex block row,
 * diagonal preconditioner, a fixed number of iterations; the product is
 * applied matrix-free by gathering each vertex's one-ring) and sets
 * V <- V + delta.  The iterate and the CG vectors are float64; residuals,
 * Jacobians and the per-vertex data blocks float32.
 * ------------------------------------------------------------------------ */
#define CAPTURE_VERTEX_MAX_RING 32     /* largest one-ring size a template may have */

typedef struct capture_vertex_template capture_vertex_template;

typedef struct {
    int32_t n_vertices, n_triangles;
    const int32_t *tri;          /* [3][n_triangles] device, counter-clockwise seen from outside; closed
                                    parts may overlap; every edge in one or two faces */
    const float *rest;           /* [3][n_vertices] device: rest pose Vhat (edge rest lengths) */
    const int32_t *classes;      /* [n_vertices] device: material class 1..7 of Table 1 */
    const int32_t *parts;        /* [n_vertices] device: body-part label (0 = torso, < 2^20), or NULL
                                    (needed by CAPTURE_FLAG_PART_MASK) */
} capture_vertex_template_desc;

/* Copies the topology, builds the one-ring table (ELL layout, neighbours in
 * ascending order) with each directed edge's s_ij/|N_i|, the undirected
 * weight s_ij/|N_i| + s_ij/|N_j| and the rest length, and keeps them in
 * library-owned device memory.  CAPTURE_EINVAL for indices or classes out of
 * range or a non-manifold mesh, CAPTURE_EUNSUPPORTED for a one-ring larger
 * than CAPTURE_VERTEX_MAX_RING.  Synchronous. */
CAPTURE_API int capture_vertex_template_create(capture_ctx *ctx, const capture_vertex_template_desc *desc,
                                               capture_vertex_template **out);
CAPTURE_API void capture_vertex_template_destroy(capture_vertex_template *tmpl);

typedef struct {
    const capture_vertex_template *tmpl;
    const float *posed;        /* [3][n_vertices] V^S: the skinned mesh of the pose result */
    const float *prev;         /* [3][n_vertices] V^{t-1}, or NULL (then w_vel and w_acc must be 0) */
    const float *prev2;        /* [3][n_vertices] V^{t-2}, or NULL (then w_acc must be 0) */
    const float *rgb;          /* [3][n_vertices] template vertex colours C, in [0, 1] */
    capture_camera camera;
    const uint8_t *mask;       /* [H][W] foreground silhouette, 0 = background */
    const float *image;        /* [3][H][W] colour frame in [0, 1] */
    float *V;                  /* [3][n_vertices] in: start positions, out: solution */
} capture_vertex_frame;

/* blur_kernel[g]: odd size k in 1..15 of the Gaussian I_Gauss used by
 * Gauss-Newton step g (sigma = 0.3 ((k - 1) / 2 - 1) + 0.8, separable,
 * clamp-to-edge; 0 means 3).  The paper's photometric pyramid (Sec. 3.4: one
 * Gauss-Newton step per level, kernels 15, 9, 3) is {15, 9, 3} with
 * gn_iters = 3; at most 3 distinct sizes per solve.  The final energy uses
 * the last step's image.  flags: CAPTURE_FLAG_EXCLUDE_CASE2,
 * CAPTURE_FLAG_OUTLINE_ONLY as for the other stages. */
typedef struct {
    float w_photo, w_sil, w_smooth, w_edge, w_vel, w_acc, tau_color;
    int32_t gn_iters;          /* 1..CAPTURE_MAX_GN */
    int32_t pcg_iters;         /* >= 0 Jacobi-PCG iterations per Gauss-Newton step */
    uint32_t flags;
    int32_t blur_kernel[CAPTURE_MAX_GN];
    /* Vertex snapping after the solve (Sec. 3.4), off when snap_max_px = 0:
     * contour vertices with b_i = +1 whose distance-transform value at the
     * final projection is at most snap_max_px pixels walk along the negative
     * distance-transform gradient, u <- u - I_DT(u) grad / |grad|, at most
     * snap_steps times (stopping below 0.05 px or where the gradient
     * vanishes), and are lifted back at their depth; vertices within
     * snap_rings one-ring steps of a snapped vertex follow a Laplacian warp:
     * snap_iters Jacobi sweeps of d_i <- mean of the neighbours' d, snapped
     * vertices held at their displacement and vertices farther away at 0.
     * The report's energies are those before snapping. */
    float snap_max_px;
    int32_t snap_steps, snap_rings, snap_iters;
    /* Body-part mask (Sec. 3.4, dense silhouette alignment; flag
     * CAPTURE_FLAG_PART_MASK): the model at the start positions is rendered with
     * per-face part labels (a face takes its first vertex's label; a pixel the
     * label of the face that sets its depth-buffer value, the smallest on
     * ties), grown part_dilation times over 3x3 neighbourhoods with the torso
     * (label 0) taking precedence (a background pixel otherwise takes its
     * smallest neighbouring label), and a contour vertex whose pixel carries
     * another part's label gets b_i = 0 (no silhouette residual). */
    int32_t part_dilation;
} capture_vertex_params;

typedef struct {
    double energy[CAPTURE_MAX_GN + 1];    /* E at the start of each step (with that step's image), then the final E */
    double e_photo, e_sil, e_sil_abs, e_smooth, e_edge, e_vel, e_acc;   /* final per-term energies */
    int32_t n_visible, n_boundary, gn_done;
    int32_t n_snapped;                    /* contour vertices moved by vertex snapping */
    int32_t status;                       /* CAPTURE_OK or CAPTURE_ENONFINITE (a non-finite energy) */
} capture_vertex_report;

/* Workspace bytes of one frame (a host struct; its arrays are not read). */
CAPTURE_API int capture_vertex_workspace_size(capture_ctx *ctx, const capture_vertex_frame *frame,
                                              const capture_vertex_params *params, size_t *bytes);

/* Gauss-Newton solve of one frame.  frame->V is overwritten with the result
 * (also when the report's status is CAPTURE_ENONFINITE, which is returned). */
CAPTURE_API int capture_vertex_solve(capture_ctx *ctx, const capture_vertex_frame *frame,
                                     const capture_vertex_params *params, capture_vertex_report *report,
                                     void *workspace, size_t workspace_bytes, void *stream);

/* Decisions and one linearisation at frame->V (not modified), with the image
 * of step 0, then the matrix-free product:
 *   rhs   [3][n_vertices] -J^T B F        diag [3][n_vertices] diagonal of J^T |B| J
 *   p     [3][n_vertices] input direction (may be NULL)   Ap [3][n_vertices] out: J^T |B| J p
 *   energy (host, 7 doubles): photo, sil, sil with |b_i|, smooth, edge, velocity, acceleration
 *   vflags [n_vertices] (may be NULL): bit0 visible, bit1 in B, bit2 b_i = -1
 * float64 rhs, diag, p and Ap; any output may be NULL. */
CAPTURE_API int capture_vertex_linearize(capture_ctx *ctx, const capture_vertex_frame *frame,
                                         const capture_vertex_params *params, double *rhs, double *diag,
                                         const double *p, double *Ap, double *energy, uint8_t *vflags,
                                         void *workspace, size_t workspace_bytes, void *stream);

/* --------------------------------------------------------------------------
 * Between the stages and between frames.  These calls only enqueue work on
 * `stream` (no host synchronisation, no workspace), so that the stages of
 * consecutive frames can run concurrently on different streams.
 * ------------------------------------------------------------------------ */
/* The skinned mesh V^S of a body at a pose (Sec. 3.1 skinning, with the
 * library's linear blend and the float32 recipe of the pose stage's start
 * positions): pose [n_unknowns] device float64, xyz [3][n_vertices] device out. */
CAPTURE_API int capture_body_skin(capture_ctx *ctx, const capture_body *body, const double *pose, float *xyz,
                                  void *stream);

/* Displacement warping (Sec. 3.4): the previous frame's non-rigid
 * displacement d = V^{t-1} - V^{S,t-1} is taken back to the rest pose by the
 * inverse skinning rotation of the previous pose and carried forward by the
 * current pose's, start = V^{S,t} + M_t M_{t-1}^T d, where M is the rotation
 * of dual-quaternion skinning at the vertex (the unit quaternions of its
 * influencing joints' global rotations, flipped into the first influence's
 * hemisphere, blended by the skinning weights and normalised).  Poses device
 * float64 [n_unknowns]; meshes device [3][n_vertices] float32 (the body's
 * vertex count); start may alias none of the inputs.  Arithmetic in float64. */
CAPTURE_API int capture_body_warp(capture_ctx *ctx, const capture_body *body, const double *pose_prev,
                                  const double *pose_cur, const float *V_prev, const float *posed_prev,
                                  const float *posed_cur, float *start, void *stream);

/* Joint positions p_j at a pose (forward kinematics of the pose stage):
 * pose [n_unknowns] device float64, joints [3][n_joints] device float64 out
 * (e.g. the next frame's capture_pose_frame.prev_joints). */
CAPTURE_API int capture_body_joints(capture_ctx *ctx, const capture_body *body, const double *pose, double *joints,
                                    void *stream);

/* Start pose of the next frame (Sec. 3.3): an explicit Euler step in joint
 * angle space, pose_out = pose_prev + (pose_prev - pose_prev2); device float64
 * [n_unknowns] each. */
CAPTURE_API int capture_pose_extrapolate(capture_ctx *ctx, const capture_body *body, const double *pose_prev,
                                         const double *pose_prev2, double *pose_out, void *stream);

/* Launch mode of capture_batch_solve / capture_nonrigid_solve /
 * capture_nonrigid_solve_warm / capture_vertex_solve.  With `on`, the per-frame launch sequence
 * (preprocessing, decisions, the warm-start prediction and selection, and the
 * full Gauss-Newton/PCG schedule) is captured into a HIP graph the first time
 * a launch shape (frame count, sizes, workspace address, schedule; for the
 * learned start also the network and template) is seen and replayed
 * afterwards (at most 16 graphs per context, least recently used dropped);
 * results are identical to eager launches.  Off by default; while kernel
 * timing is enabled, solves launch eagerly. */
CAPTURE_API int capture_set_graphs(capture_ctx *ctx, int on);

/* --------------------------------------------------------------------------
 * Kernel timing.  While enabled, every launch of the solver kernels is
 * bracketed by HIP events on the call's stream; elapsed times accumulate per
 * kernel until read.  Kernel names: "blur", "contour", "dt_cols", "dt_rows",
 * "deform_start", "raster", "contour_edges", "decide", "linearize",
 * "node_init", "cg", "cg_node", "ws_features", "ws_mlp", "pose_lbs",
 * "pose_rows", "pose_jtj", "pose_step", "prep_image", "prep_geom",
 * "prep_raster", "prep_cols".  "cg" is the matrix-free product J^T |B| J v of
 * a PCG iteration with the vector update before it; "cg_node" the per-node
 * step (for schedules of at most 16 PCG iterations on grids of at most 1024
 * tiles: once per Gauss-Newton step, the last iteration's solution update and
 * the node update; otherwise once per iteration).  The non-rigid stage's per-frame steps run in
 * combined launches: "prep_image" (frame set-up, blur, contour pixels),
 * "prep_geom" (deformed start, column segments), "prep_raster"
 * (rasterisation and, for few image columns, the segment scan; with many
 * columns the scan is its own launch, timed as "dt_cols"), "prep_cols"
 * (large faces, column distances), "dt_rows" (row pass, then contour
 * edges), "decide".  The pose stage launches the steps one by one under the
 * other names.
 * ------------------------------------------------------------------------ */
CAPTURE_API int capture_profile_enable(capture_ctx *ctx, int on);
/* Accumulated time (ms) and launch count of `kernel` since the last read;
 * resets that kernel's counters. */
CAPTURE_API int capture_profile_read(capture_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
