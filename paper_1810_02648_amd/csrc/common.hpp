// Shared host/device declarations of the capture library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/capture.h"

namespace cap {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const char *msg);     // copies msg into a fixed thread-local buffer
int fail(int code, const std::string &msg);

#define CAP_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::cap::fail(CAPTURE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- plan limits
constexpr int kTileThreads = 256;     // threads of a tile workgroup (one vertex each)
constexpr int kMaxTileVerts = 256;    // vertices per tile
constexpr int kMaxTileContrib = 1024; // contributions held in LDS per tile
constexpr int kMaxTileSlots = 200;    // distinct nodes touched by a tile
#ifndef CAP_NODE_THREADS
#define CAP_NODE_THREADS 1024
#endif
constexpr int kNodeThreads = CAP_NODE_THREADS;    // threads of a per-problem node workgroup
constexpr int kInitThreads = 512;     // threads of a post-linearisation node workgroup (k_node_init)
constexpr int kInitBlocks = 8;        // k_node_init workgroups per problem (then k_node_init_fin: one)
constexpr int kInitFinThreads = 256;  // threads of k_node_init_fin
constexpr int kMaxImageSide = 4096;
constexpr int kRasterSmall = 256;         // pixel-box size above which a face is rasterised by a workgroup
constexpr int kRasterBigBlocks = 512;
constexpr int kScanColsMin = 16384;      // image columns (all frames) from which the segment scan runs a thread per column
// Dynamic LDS of the row pass for rows of W pixels: G (int).
inline size_t dt_rows_lds(int W) { return sizeof(int) * size_t(W) + 16; }
#ifndef CAP_APPLY_SPLIT_TILES
#define CAP_APPLY_SPLIT_TILES 1024
#endif
constexpr int kApplySplitTiles = CAP_APPLY_SPLIT_TILES;   // tile grids above this take the two-pass J^T J p reduction
constexpr int kGraphCache = 16;          // captured solve graphs kept per context
constexpr int kTerms = 5;   // energy terms per slot: photo, sil (with b), sil (with |b|), arap, velocity
constexpr int kInitPart = 8 + kTerms * (CAPTURE_MAX_GN + 2);  // energy slot MAX_GN + 1: predicted start
constexpr int kScalars = kInitPart + 2 * kInitBlocks;         // then r.u and b.b per k_node_init workgroup

// A pointer to device global memory.  Indexing it reads and writes through
// the global address space (global_load / global_store): a plain pointer held
// in a struct in memory is generic to the compiler, and generic (flat)
// accesses also count against the scalar-load counter, so every wait for a
// scalar load would wait for them too.  Converts to and from T * for host code.
#define CAP_GLOBAL __attribute__((address_space(1)))
template <class T>
struct gptr {
    T *ptr = nullptr;
    gptr() = default;
    __host__ __device__ gptr(T *q) : ptr(q) {}
    template <class U, class = typename std::enable_if<std::is_convertible<U *, T *>::value>::type>
    __host__ __device__ gptr(const gptr<U> &q) : ptr(q.ptr) {}    // e.g. gptr<float> -> gptr<const float>
    __host__ __device__ operator T *() const { return ptr; }
    __device__ __forceinline__ CAP_GLOBAL T &operator[](size_t i) const { return ((CAP_GLOBAL T *)ptr)[i]; }
    __device__ __forceinline__ CAP_GLOBAL T *g() const { return (CAP_GLOBAL T *)ptr; }
};

// Static per-template data in library-owned device memory (plan order =
// vertices grouped by their nearest node, nodes in breadth-first order of the
// node graph; tiles are contiguous ranges of the plan order).
struct TemplateDev {
    int nv, nf, nn, ntiles, nslots, nmedges, max_slots, max_contrib;
    gptr<const int> tri;            // [3][nf]
    gptr<const int> node_vertex;    // [nn]
    gptr<const int> bind_idx;       // [4][nv] (vertex order)
    gptr<const float> bind_w;       // [4][nv] (vertex order)
    gptr<const int> edge_dst;       // [8][nn]
    gptr<const int> plan_vid;       // [nv] plan position -> vertex
    gptr<const int> plan_pos;       // [nv] vertex -> plan position
    gptr<const float> plan_w;       // [4][nv] binding weights in plan order
    gptr<const uint32_t> plan_slot; // [nv] 4 tile-local slot indices (u8 each)
    gptr<const int> tile_vbeg;      // [ntiles+1]
    gptr<const int> tile_sbeg;      // [ntiles+1] into slot_node / partials
    gptr<const int> slot_node;      // [nslots]
    gptr<const int> tile_obeg;      // [ntiles+1] into owned_*
    gptr<const int> owned_node;     // [nn]
    gptr<const uint8_t> owned_slot; // [nn]
    gptr<const uint8_t> owned_eslot;// [8][nn] slot of each out-edge target, 255 = none
    gptr<const int> list_beg;       // [nslots+1] into list_idx
    gptr<const uint16_t> list_idx;  // tile-local contribution indices, grouped by slot
    gptr<const int> node_pbeg;      // [nn+1] into node_pidx
    gptr<const int> node_pidx;      // global slot indices of each node, tile order (node-major positions)
    gptr<const int> slot_dest;      // [nslots] node-major position of each slot's partial
    gptr<const int> slot_pb;        // [nslots] first partial (node-major position) of the slot's node
    gptr<const int> slot_pe;        // [nslots] end of that range; bit 31 set: the slot's tile owns the node
    gptr<const uint16_t> plan_cpos; // [4][nv] tile-local position of each vertex contribution in slot order
    gptr<const uint32_t> owned_cpos;// [8][nn] positions of an owned edge's two contributions (lo: source, hi: target)
    gptr<const int> vf_beg;         // [nv+1] vertex -> incident faces
    gptr<const int> vf_face;        // [3nf] ascending per vertex
    gptr<const int> medge;          // [4][nmedges]: a, b, f0, f1 (-1 = border)
    gptr<const int> in_beg;         // [nn+1] node graph in-edges (source nodes), ascending
    gptr<const int> in_src;         // [..]
    gptr<const int> out_cnt;        // [nn] number of valid out-edges
};

// One work item of the tile kernels: a tile of one problem with its vertex
// [vb, vb + nvt), slot [sb, sb + ns) and owned-node [ob, ob + nown) ranges.
// Built on the host per solve; prob < 0 marks the padding of the grid.
struct TileDesc {
    int prob, tile, vb, nvt, sb, ns, ob, nown;
};

// One problem (frame) of a batch: template, frame inputs and its workspace.
struct ProbDev {
    TemplateDev T;
    gptr<const float> xyz;
    gptr<const float> rgb;
    gptr<const uint8_t> mask;
    gptr<const float> image;
    gptr<float> state;
    int W, H;
    float fx, fy, cx, cy;
    float sw_sil, sw_photo, sw_arap, w_arap, tau, w_vel, sw_vel;
    double pcg_tol2;             // stop a step's PCG once ||r||^2 <= pcg_tol2 ||b||^2 (0: fixed count)
    int exclude_case2;
    int outline_only;            // contour set B restricted to the rendered model's outline
    // images
    gptr<float> blurred, dt;
    gptr<int> colg;
    gptr<int> seg_first, seg_last;   // [ceil(H/16)][W]
    gptr<uint32_t> zbuf;
    gptr<uint8_t> contour;
    // vertices (vertex order)
    gptr<float> dx;        // [3][nv] deformed position at the start state (float32 recipe)
    gptr<float> duv;       // [2][nv]
    gptr<int> dfix;        // [2][nv] 1/256-pixel fixed point
    gptr<uint8_t> dvalid;  // [nv]
    gptr<uint8_t> vcont;   // [nv]
    gptr<uint8_t> vflags;  // [nv] bit0 visible, bit1 contour set, bit2 b_i = -1
    // faces
    gptr<float> fcross;    // [3][nf]
    // vertices (plan order)
    gptr<float> px;        // [3][nv]
    gptr<float> pc;        // [3][nv]
    gptr<uint8_t> vcode;   // [nv] bit0 visible, bit1 silhouette residual, bit2 b_i = -1, bit3 velocity term
    gptr<float> pva;       // [3][nv] velocity anchor: start positions (float32 recipe)
    gptr<float> Hm;        // [6][nv]
    // tiles / slots
    gptr<float> partial;   // [12][nslots] component-major; positions node-major (node_pbeg ranges)
    gptr<float> gpos;      // [3][nn] node positions (the frame's input mesh at the node vertices)
    gptr<double> tile_e;   // [ntiles][kTerms]
    // nodes
    gptr<float> b, diag, dinv;   // [6][nn] right-hand side, diag(J^T |B| J), Jacobi preconditioner
    gptr<double> vx[2], vr[2], vu[2], vp[2], vs[2];  // [6][nn] PCG vectors (float64), two generations (see k_cg)
    gptr<float> x;         // [6][nn] the warm start's predicted update
    gptr<float> p, Ap;     // [6][nn] product input and output of capture_linearize
    gptr<double> scal;     // [kScalars]: r.u, PCG stopped, stopped, stop step, ..., kTerms energies per GN step
    gptr<double> dots;     // [2][3][ntiles] per-tile r.u, u.Au and r.r sums of two PCG launches
    gptr<double> cg;       // [8]: (gamma, alpha) of two PCG launches, generation of the final x, b.b
    gptr<double> nsum;     // [2][2][node blocks] per-block r.u and r.r of two node steps (standard PCG)
    gptr<int> counts;      // [3] visible, contour set, queued large faces
    gptr<int> bigq;        // [nf] faces left to the large-face pass
    gptr<float> state0;    // [12][nn] copy of the start state (restored on a device-detected error)
    double target;    // stop once the energy at the start of a GN step is <= target (-inf: never)
    gptr<const float> prev2;   // [12][nn] state two frames back (warm-start features), or null
};

// Arguments of the warm-start network's MFMA GEMM: C(i, j) = sum_k A(i, k) B(j, k)
// [+ bias(j)], bf16 operands with arbitrary strides; optional bf16 ReLU copy.
struct Gemm {
    const uint16_t *A;
    long long sai, sak;
    const uint16_t *B;
    long long sbj, sbk;
    float *C;
    long long sci, scj;
    int M, N, K;
    const float *bias;
    uint16_t *Cb;
    long long scbi;
    int relu_copy;
};

// ---------------------------------------------------------------- pose stage
constexpr int kMaxJoints = 32;
constexpr int kMaxPoseUnknowns = 81;     // 3 per rotating joint + root t (3) + t' (3)
constexpr int kPoseTile = 16;            // MFMA f64 16x16x4 tiles of J^T J
constexpr int kPoseMaxCols = 96;         // unknowns + the b*F column, padded to 16
constexpr int kPoseRowThreads = 256;
constexpr int kPoseTerms = 6;            // energy terms: 2D, 3D, silhouette (b), silhouette (|b|), temporal, limits
// Rows of the pose Jacobian before the contour rows: 2D (2 per joint), 3D and
// temporal (3 per joint each), joint limits (one per rotational unknown).
__host__ __device__ inline int pose_fixed_rows(int nj, int it) { return 8 * nj + it; }

// Skeleton and skinning of a body (device copy of the static part).
struct BodyDev {
    int nj, nu, np, it, itp, maxdepth, nv;
    int parent[kMaxJoints], col[kMaxJoints], depth[kMaxJoints];
    uint32_t anc[kMaxJoints];        // bit k set: joint k is j itself or one of its ancestors
    double rest[3][kMaxJoints];      // rest joint positions
    gptr<const float> xyz;                // [3][nv] rest mesh
    gptr<const int> bind_joint;           // [4][nv]
    gptr<const float> bind_w;             // [4][nv]
};

// One pose problem: body, detections, weights and its workspace.
struct PoseDev {
    BodyDev B;
    int W, H;
    double fx, fy, cx, cy;
    double s3d, ssil;                // square roots of the 3D and silhouette weights
    double l2d;
    gptr<const double> p2d, p3d, lam;   // [2][nj], [3][nj], [nj]
    gptr<const double> prev_joints;       // [3][nj] joint positions of the previous frame (temporal term), or null
    double stemp[kMaxJoints];             // square roots of the per-joint temporal weights
    double sanat;                         // square root of the joint-limit weight (0: no term)
    double lim_lo[kMaxPoseUnknowns], lim_hi[kMaxPoseUnknowns];   // limits of the rotational unknowns
    gptr<double> pose;                    // caller's [nu]
    gptr<const float> dt;                 // [H][W]
    gptr<const uint8_t> vflags;           // [nv] decision flags
    gptr<double> jR, jp, jA;            // [nj][9], [nj][3], [nj][9]: global rotations, positions, derivative axes
    gptr<double> pose0;                   // [nu] start pose (restored on a device-detected error)
    gptr<int> blist;                      // [nv] contour set: (vertex << 1) | (b_i == -1), ascending
    gptr<int> nb;                         // [1] |B|
    gptr<double> rows;                    // [np][ldr] Jacobian, column-major (row r, column c at c * ldr + r);
                                     // column nu holds b*F
    int ldr;                         // max_rows rounded up to 64
    gptr<double> epart;                   // [row blocks][kPoseTerms] energy partials
    gptr<double> energy;                  // [MAX_GN + 1][kPoseTerms]
    gptr<double> sys;                     // [nu][nu + 1] system of the current step (J^T J | -J^T B F), undamped
    gptr<int> status;                     // [1]
};

// Optional per-kernel timing with HIP events (capture_profile_*).
enum KernelId {
    K_BLUR, K_CONTOUR, K_DT_COLS, K_DT_ROWS, K_DEFORM, K_RASTER, K_CEDGES, K_DECIDE,
    K_LIN, K_NODE_INIT, K_APPLY, K_NODE_PCG, K_WS_FEAT, K_WS_MLP,
    K_POSE_LBS, K_POSE_ROWS, K_POSE_JTJ, K_POSE_STEP, K_PREP_IMAGE, K_PREP_GEOM, K_PREP_RASTER, K_PREP_COLS,
    K_V_BLUR, K_V_LIN, K_V_APPLY, K_V_UPDATE, K_V_SNAP,
    K_COUNT
};

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> pending;
    double total_ms[K_COUNT] = {};
    long long launches[K_COUNT] = {};
};

}  // namespace cap

struct capture_ctx {
    int device;
    cap::Profiler prof;
    void *pinned = nullptr;      // pinned host staging (descriptors, report read-back)
    size_t pinned_bytes = 0;
    bool graphs = false;         // replay solves from captured HIP graphs
    void *scratch = nullptr;     // this device's address of the allocation-free solve's scratch
    hipStream_t capture_stream = nullptr;
    struct Graph {
        std::string key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graph_cache;   // most recent last, at most kGraphCache entries
};

struct capture_warmstart {
    int device, max_nodes;
    long long steps;
    int recent_gn[16];           // Gauss-Newton steps of the last learned-start solves (ring)
    int n_recent, recent_pos;
    void *mem;
    float *w, *g, *m, *v, *mu, *sd;
    uint16_t *wb;
    float *X, *z1, *z2, *y, *tgt, *dy, *se, *dc, *dz;
    uint16_t *Xb, *c1, *c2, *dyb, *dzb;
};

struct capture_body {
    cap::BodyDev dev;
    capture_template *topo;     // mesh tables for the raster and decision kernels
    void *mem;                  // device copy of xyz and skinning
    int device;
};

struct capture_template {
    cap::TemplateDev dev;
    std::vector<int> tile_ranges;   // host copy: [ntiles][6] vb, nvt, sb, ns, ob, nown
    int vertices_per_tile = 0;
    void *mem;
    size_t bytes;
    int device;
};
