// ctx.h -- the library's context object and host-side helpers shared by
// api.hip (context, mesh upload) and frame.hip (frame orchestration).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hexfc.h"
#include "kern.h"

namespace hexfc {

// Device allocation that only grows.  A replaced allocation is kept until the
// context is destroyed: work already enqueued, and HIP graphs a caller
// captured from earlier frames, may still use it.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    std::vector<void *> retired;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
        for (void *q : retired) (void)hipFree(q);
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, n ? n : 256);
        if (e != hipSuccess) return e;
        if (p) retired.push_back(p);
        p = q;
        bytes = n;
        return hipSuccess;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// The captured batch pipeline and the shapes it was captured for.
struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nv = 0, W = 0, H = 0, tw = 0, th = 0, t_sort = 0;
    const void *ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t bin_cap = 0;
    float *rgba = nullptr;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        nv = 0;
    }
};

}  // namespace hexfc

struct hexfc_ctx {
    int device = 0;
    std::string err;
    // mesh
    int64_t V = 0, C = 0, F = 0;
    hexfc::DevBuf posq, vert0, face, face_px, face_bnd;
    hexfc::DevBuf face_c, face_ord;  // binning order: corner ids, and the canonical face id
    double bbox_lo[3] = {0, 0, 0}, bbox_hi[3] = {0, 0, 0};
    // tuning
    int tw = 8, th = 8, t_sort = 16;
    // workspace (caller-owned)
    uint64_t *ws = nullptr;
    size_t ws_bytes = 0;
    // per-frame scratch, sized for `nv_cap` views
    hexfc::DevBuf bdepth;  // per pixel: depth key of the nearest boundary-surface fragment
    hexfc::DevBuf mlab_c, mlab_z;  // per fragment: shaded colour and depth for multi-layer alpha blending
    hexfc::DevBuf vert_b, vscr, fscr, bslot, views, tile_cnt, tile_fill, tile_off, bins, masks, gpre, count, off, scan_tmp, cls,
        stats, persist, rqueue;
    hexfc::DevBuf count_rm_tmp;
    // learned tail: per-row head, features and pixel ids, fallback lists
    hexfc::DevBuf l_head, l_feat, l_pix, l_fb;
    hexfc::DevBuf frange;  // int4 [views x faces]: both triangles' tile ranges (binning)
    // device address of this GPU's static scratch (allocation-free learned
    // resolve), looked up once per device; nullptr with the reason when the
    // lookup failed
    void *static_scratch = nullptr;
    std::string static_scratch_err;
    int vert_b_views = 0;  // views whose world part is initialised in vert_b
    uint64_t bin_cap = 0;
    int64_t cls_cap = 0;
    uint64_t *h_stats = nullptr;  // pinned
    // host-mapped copy of the device's cross-frame counters (PersistSlot),
    // written by each frame's closing kernel: [0] frames finished, [1 + i] slot i
    volatile uint64_t *h_pub = nullptr;
    uint64_t *d_pub = nullptr;  // its device address
    // the resolve of the longest lists runs on a second stream beside the others
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int res_min_grid[hexfc::NCLASS + 2] = {};  // resident workgroups of each resolve kernel
    // single frames: sizes learned for the current mesh, viewport, tiling and
    // workspace (the first frame of such a combination waits once to learn them)
    bool sized = false;
    int64_t frame_sig[7] = {0, 0, 0, 0, 0, 0, 0};
    int passes_launch = 1;  // screen passes enqueued per frame
    uint64_t mesh_gen = 0;  // bumped by every upload
    hipStream_t last_stream = nullptr;
    hipStream_t cap_stream = nullptr;  // non-blocking stream used to capture the batch graph
    hexfc::BatchGraph bg;
    // state of the last build
    hexfc::Tiling tl{};
    int nv = 1;
    bool lists_valid = false;
    bool have_frame = false;
    bool stats_known = false;  // last_stats holds the class sizes of the current lists
    uint64_t last_frags = 0;
    uint64_t last_stats[hexfc::ST_COUNT] = {};
    std::vector<hexfc::ViewParams> h_views;
    // optional per-launch timing with HIP events on the launch stream
    bool prof = false;
    struct TimedLaunch {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    std::vector<TimedLaunch> pending;
    double acc_ms[hexfc::KID_COUNT_] = {};
    uint64_t acc_n[hexfc::KID_COUNT_] = {};
    ~hexfc_ctx() {
        bg.reset();
        for (auto &t : pending) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (side_stream) (void)hipStreamDestroy(side_stream);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (h_pub) (void)hipHostFree((void *)h_pub);
    }
};

#define FAIL(ctx, code, ...)                  \
    do {                                      \
        char _b[512];                         \
        snprintf(_b, sizeof _b, __VA_ARGS__); \
        (ctx)->err = _b;                      \
        return code;                          \
    } while (0)

#define HIPCHK(ctx, call)                                                                               \
    do {                                                                                                \
        hipError_t _e = (call);                                                                         \
        if (_e != hipSuccess) FAIL(ctx, HEXFC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
    } while (0)

namespace hexfc {

inline hipEvent_t take_event(hexfc_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around the launches of its scope when profiling is on.
struct ScopedTimer {
    hexfc_ctx *ctx;
    hipStream_t s;
    int kid;
    hipEvent_t a = nullptr;
    ScopedTimer(hexfc_ctx *c, hipStream_t st, int k) : ctx(c), s(st), kid(k) {
        if (ctx->prof && (a = take_event(ctx))) (void)hipEventRecord(a, s);
    }
    ~ScopedTimer() {
        if (!a) return;
        hipEvent_t b = take_event(ctx);
        if (!b) {
            ctx->ev_pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        ctx->pending.push_back({kid, a, b});
    }
};

inline hexfc_status set_device(hexfc_ctx *ctx) {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return HEXFC_OK;
}

}  // namespace hexfc
