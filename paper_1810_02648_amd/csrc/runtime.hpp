// Host-side launch helpers shared by the entry points (internal).
#pragma once
#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"

namespace cap {

// Bump allocator over a caller workspace (base == nullptr: sizing pass).
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

// Pinned host staging of a context, grown on demand (descriptor uploads and
// report read-backs).  Calls on one context are serialised by the caller.
inline void *staging(capture_ctx *ctx, size_t bytes) {
    if (ctx->pinned_bytes < bytes) {
        if (ctx->pinned) (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        const size_t want = std::max<size_t>(bytes, 64 * 1024);
        if (hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault) != hipSuccess) return nullptr;
        ctx->pinned_bytes = want;
    }
    return ctx->pinned;
}

// Per-problem descriptors on the host: inline storage for one problem (the
// single-frame entry points allocate nothing for it), heap storage for batches.
class ProbList {
  public:
    void resize(int n) {
        n_ = n;
        if (n > 1) heap_.resize(size_t(n));
    }
    ProbDev *data() { return n_ > 1 ? heap_.data() : &one_; }
    const ProbDev *data() const { return n_ > 1 ? heap_.data() : &one_; }
    ProbDev &operator[](size_t i) { return data()[i]; }
    const ProbDev &operator[](size_t i) const { return data()[i]; }
    size_t size() const { return size_t(n_); }

  private:
    int n_ = 0;
    ProbDev one_{};
    std::vector<ProbDev> heap_;
};

struct Run {
    capture_ctx *ctx = nullptr;
    Profiler *prof = nullptr;
    int n = 0;
    ProbList probs;
    ProbDev *dprobs = nullptr;
    int max_nv = 0, max_nf = 0, max_nn = 0, max_hw = 0, max_w = 0, max_h = 0, max_tiles = 0, max_me = 0;
    size_t lds_lin = 0, lds_apply = 0, lds_apply_split = 0;
    TileDesc *tiles = nullptr;   // device [grid_tiles]: tile-kernel work items (die-interleaved grid)
    int total_tiles = 0;         // tiles of all problems
    int grid_tiles = 0;          // total_tiles rounded up to a multiple of 8
    hipStream_t s = nullptr;
    // set before setup; applied to problem 0 (single-frame entry points)
    double target = -INFINITY;
    const float *prev2 = nullptr;
    // allocation-free calls: host staging of fixed size instead of the
    // context's growable pinned buffer, and no kernel timing
    uint8_t *fixed_stage = nullptr;
    size_t fixed_stage_bytes = 0;
};

// Host staging of a run: the fixed buffer when the run has one (nullptr if it
// is too small), else the context's pinned buffer.
inline void *run_staging(Run &R, size_t bytes) {
    if (R.fixed_stage) return bytes <= R.fixed_stage_bytes ? R.fixed_stage : nullptr;
    return staging(R.ctx, bytes);
}

// Launch `go` bracketed by events when timing is on.
template <typename F>
inline void timed(Run &R, int kid, F go) {
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
inline void settle(Run &R) {
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

// Replays the launches of `sequence` (a callable taking a Run whose stream
// it launches on) from a HIP graph cached under `key` in the context,
// capturing it on the context's capture stream the first time.
template <class F>
inline int launch_graph(Run &R, const std::string &key, F &&sequence) {
    capture_ctx *ctx = R.ctx;
    auto &cache = ctx->graph_cache;
    hipGraphExec_t exec = nullptr;
    for (size_t i = 0; i < cache.size(); ++i)
        if (cache[i].key == key) {
            exec = cache[i].exec;
            std::rotate(cache.begin() + i, cache.begin() + i + 1, cache.end());     // most recent last
            break;
        }
    if (!exec) {
        if (!ctx->capture_stream) CAP_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        Run C = R;
        C.s = ctx->capture_stream;
        C.prof = nullptr;
        CAP_HIP(hipStreamBeginCapture(C.s, hipStreamCaptureModeThreadLocal));
        const int rc = sequence(C);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(C.s, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess || !graph) return fail(CAPTURE_EHIP, "graph capture failed");
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(CAPTURE_EHIP, "graph instantiation failed");
        if (cache.size() >= size_t(kGraphCache)) {
            (void)hipGraphExecDestroy(cache.front().exec);
            cache.erase(cache.begin());
        }
        cache.push_back({key, exec});
    }
    CAP_HIP(hipGraphLaunch(exec, R.s));
    return CAPTURE_OK;
}

inline unsigned blocks(size_t n, unsigned t) { return unsigned((n + t - 1) / t); }

}  // namespace cap
