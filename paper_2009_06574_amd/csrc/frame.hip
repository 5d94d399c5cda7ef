// frame.hip -- frame orchestration on the host: one view (build, resolve,
// render in screen passes, parity export) and batches of views rendered by
// one captured HIP graph, plus the autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <fstream>
#include <sstream>

#include "ctx.h"

using namespace hexfc;

namespace {

hexfc_status check_camera(hexfc_ctx *ctx, const hexfc_camera *cam, Mat3q &M) {
    if (!cam) FAIL(ctx, HEXFC_EINVAL, "null camera");
    if (cam->width < 1 || cam->height < 1 || cam->width > 8192 || cam->height > 8192)
        FAIL(ctx, HEXFC_ERANGE, "viewport %dx%d out of range", cam->width, cam->height);
    const int rows[3] = {0, 1, 3};
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 4; ++j) {
            float v = cam->view_proj[4 * rows[r] + j];
            if (!(std::fabs(v) < 8.0f)) FAIL(ctx, HEXFC_ERANGE, "camera matrix entry out of range");
            M.m[r][j] = (long long)std::nearbyint((double)v * 1048576.0);
        }
    return HEXFC_OK;
}

hexfc_status check_shading(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *sty, const float *rgba) {
    if (!hot || !sty || !rgba) FAIL(ctx, HEXFC_EINVAL, "null hotspot, style or output");
    if (!(hot->radius > 0.f) || !std::isfinite(hot->radius)) FAIL(ctx, HEXFC_EINVAL, "hotspot radius must be > 0");
    if (sty->lens_mode != 0 && sty->lens_mode != 1) FAIL(ctx, HEXFC_EINVAL, "lens_mode must be 0 or 1");
    if (!(sty->desaturate >= 0.f && sty->desaturate <= 1.f)) FAIL(ctx, HEXFC_ERANGE, "desaturate must be in [0, 1]");
    if (!(sty->sil_alpha >= 0.f && sty->sil_alpha <= 1.f)) FAIL(ctx, HEXFC_ERANGE, "sil_alpha must be in [0, 1]");
    if (!(sty->sil_tau >= 0.f) || !std::isfinite(sty->sil_tau)) FAIL(ctx, HEXFC_ERANGE, "sil_tau must be >= 0");
    return HEXFC_OK;
}

void shade_params(ShadeParams &p, const hexfc_hotspot *hot, const hexfc_style *sty) {
    for (int i = 0; i < 3; ++i) p.hc[i] = hot->center[i];
    p.inv_r = 1.0f / hot->radius;
    p.w_base = sty->w_base;
    p.k_focus = sty->k_focus;
    p.halo_w = sty->halo_width;
    p.halo_a = sty->halo_alpha;
    p.darken = sty->darken;
    p.s = sty->accent_s;
    p.bright = sty->accent_brighten;
    p.delta = sty->delta;
    p.lod = sty->lod;
    for (int i = 0; i < 3; ++i) {
        p.lo[i] = sty->tf_rgb_lo[i];
        p.hi[i] = sty->tf_rgb_hi[i];
        p.bg[i] = sty->bg[i];
    }
    p.a_lo = sty->tf_a_lo;
    p.a_hi = sty->tf_a_hi;
    p.lens_mode = sty->lens_mode;
    p.desat = sty->desaturate;
    p.sil_a = sty->sil_alpha;
    p.sil_tau = sty->sil_tau;
}

// View-depth range [w0, w1] of the mesh bbox: clip w (row 3 of the float
// camera matrix) at its 8 corners.  Normalises the learned tail's depth feature.
void depth_range(const hexfc_ctx *ctx, const hexfc_camera *cam, ViewParams &vp) {
    double lo = 1e300, hi = -1e300;
    for (int c = 0; c < 8; ++c) {
        const double x = (c & 1) ? ctx->bbox_hi[0] : ctx->bbox_lo[0];
        const double y = (c & 2) ? ctx->bbox_hi[1] : ctx->bbox_lo[1];
        const double z = (c & 4) ? ctx->bbox_hi[2] : ctx->bbox_lo[2];
        const float *m = cam->view_proj + 12;
        const double w = (double)m[0] * x + (double)m[1] * y + (double)m[2] * z + (double)m[3];
        lo = std::min(lo, w);
        hi = std::max(hi, w);
    }
    if (!(hi > lo)) hi = lo + 1.0;
    vp.w0 = (float)lo;
    vp.w1 = (float)hi;
    for (int i = 0; i < 4; ++i) vp.sp.wrow[i] = cam->view_proj[12 + i];
    vp.sp.zw0 = (float)lo;
    vp.sp.zinv = (float)(1.0 / (hi - lo));
}

Tiling make_tiling(const hexfc_ctx *ctx, int W, int H) {
    Tiling tl;
    tl.W = W;
    tl.H = H;
    tl.TW = ctx->tw;
    tl.TH = ctx->th;
    tl.ntx = (W + tl.TW - 1) / tl.TW;
    tl.nty = (H + tl.TH - 1) / tl.TH;
    tl.ntiles = tl.ntx * tl.nty;
    return tl;
}

// Grows a buffer; a captured batch graph holding the old address is dropped.
hexfc_status grow(hexfc_ctx *ctx, DevBuf &b, size_t bytes) {
    void *old = b.p;
    HIPCHK(ctx, b.ensure(bytes));
    if (b.p != old) ctx->bg.reset();
    return HEXFC_OK;
}

#define TRY(expr)                          \
    do {                                   \
        hexfc_status _s = (expr);          \
        if (_s != HEXFC_OK) return _s;     \
    } while (0)

VertRec *vert_ptr(hexfc_ctx *ctx, int nv) { return nv == 1 ? ctx->vert0.as<VertRec>() : ctx->vert_b.as<VertRec>(); }

hexfc_status ensure_frame_buffers(hexfc_ctx *ctx, int nv, const Tiling &tl) {
    const int64_t TP = (int64_t)tl.TW * tl.TH;
    const int64_t nt = (int64_t)tl.ntiles * nv;
    const int64_t np = nt * TP;
    const int64_t T = 2 * ctx->F;
    if (np >= (int64_t(1) << 31))  // pixel ids are 32-bit (PIX_SKIP reserved)
        FAIL(ctx, HEXFC_ERANGE, "%lld padded pixels in the batch exceed 2^31", (long long)np);
    TRY(grow(ctx, ctx->vscr, sizeof(int4) * ctx->V * nv));
    TRY(grow(ctx, ctx->fscr, sizeof(int4) * 4 * std::max<int64_t>(ctx->F, 1) * nv));
    TRY(grow(ctx, ctx->frange, sizeof(int4) * std::max<int64_t>(ctx->F, 1) * nv));
    TRY(grow(ctx, ctx->bslot, sizeof(uint32_t) * 4 * std::max<int64_t>(ctx->F, 1) * nv));
    if (nv > 1) {
        const void *old = ctx->vert_b.p;
        TRY(grow(ctx, ctx->vert_b, sizeof(VertRec) * ctx->V * nv));
        if (ctx->vert_b.p != old) ctx->vert_b_views = 0;  // a new allocation holds no world data yet
        for (int v = ctx->vert_b_views; v < nv; ++v)  // world part of each view's vertex records
            HIPCHK(ctx, hipMemcpy(ctx->vert_b.as<VertRec>() + (int64_t)v * ctx->V, ctx->vert0.p,
                                  sizeof(VertRec) * ctx->V, hipMemcpyDeviceToDevice));
        ctx->vert_b_views = std::max(ctx->vert_b_views, nv);
    }
    TRY(grow(ctx, ctx->views, sizeof(ViewParams) * nv));
    TRY(grow(ctx, ctx->tile_cnt, sizeof(uint32_t) * 2 * nt));
    TRY(grow(ctx, ctx->tile_fill, sizeof(uint32_t) * nt));
    TRY(grow(ctx, ctx->tile_off, sizeof(uint64_t) * (nt + 1)));
    TRY(grow(ctx, ctx->count, sizeof(uint32_t) * np));
    TRY(grow(ctx, ctx->bdepth, sizeof(uint32_t) * np));
    TRY(grow(ctx, ctx->gpre, sizeof(uint32_t) * nt * RASTER_WG));
    TRY(grow(ctx, ctx->off, sizeof(uint64_t) * (np + 1)));
    TRY(grow(ctx, ctx->scan_tmp, sizeof(uint64_t) * std::max(scan_tmp_elems(np), scan_tmp_elems(nt))));
    if (ctx->cls_cap < np) {
        TRY(grow(ctx, ctx->cls, sizeof(uint32_t) * NCLASS * np));
        ctx->cls_cap = np;
    }
    if (ctx->bin_cap < (uint64_t)(2 * T * nv + 65536)) {
        uint64_t cap = (uint64_t)(2 * T * nv + 65536);
        TRY(grow(ctx, ctx->bins, sizeof(uint32_t) * cap));
        ctx->bin_cap = cap;
    }
    TRY(grow(ctx, ctx->masks, sizeof(uint64_t) * ctx->bin_cap * (TP / 64)));
    return HEXFC_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

uint64_t *pass_tiles(hexfc_ctx *ctx, int k) { return ctx->stats.as<uint64_t>() + ST_PASS + k; }

// The front half of a frame of nv views: transform, binning, coverage count,
// pixel scan; then either the plan of screen passes under the workspace
// budget (single frames, FRONT_PLAN) or one pass over every tile with its
// pixels classified at once (frames that must fit the workspace: the list
// build and batches, FRONT_SINGLE).
enum FrontMode { FRONT_PLAN, FRONT_SINGLE };

void enqueue_classify(hexfc_ctx *ctx, int nv, int k, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_CLASSIFY);
    launch_classify(ctx->tl, nv, k, ctx->count.as<uint32_t>(), ctx->t_sort, ctx->cls.as<uint32_t>(), ctx->cls_cap,
                    ctx->stats.as<uint64_t>(), s);
}

void enqueue_front(hexfc_ctx *ctx, int nv, const Tiling &tl, hipStream_t s, FrontMode mode) {
    const int64_t TP = (int64_t)tl.TW * tl.TH;
    const int64_t nt = (int64_t)tl.ntiles * nv;
    const int64_t np = nt * TP;
    uint64_t *stats = ctx->stats.as<uint64_t>();
    const int4 *fc = ctx->face_c.as<int4>();
    int4 *vscr = ctx->vscr.as<int4>();
    const uint64_t budget = ctx->ws ? ctx->ws_bytes / 8 : 0;
    ctx->tl = tl;
    launch_zero_u64(stats, ST_COUNT, s);
    launch_zero_u32(ctx->tile_cnt.as<uint32_t>(), 2 * nt, s);
    launch_zero_u32(ctx->tile_fill.as<uint32_t>(), nt, s);
    {
        ScopedTimer tm(ctx, s, KID_TRANSFORM);
        launch_transform(ctx->posq.as<int4>(), ctx->V, nv, ctx->views.as<ViewParams>(), tl.W, tl.H,
                         vert_ptr(ctx, nv), vscr, s);
    }
    {
        ScopedTimer tm(ctx, s, KID_BIN_COUNT);
        launch_tri_bin_count(fc, ctx->face_ord.as<uint32_t>(), ctx->F, nv, vscr, ctx->V, tl,
                             ctx->tile_cnt.as<uint32_t>(), ctx->fscr.as<int4>(), ctx->bslot.as<uint32_t>(),
                             ctx->frange.as<int4>(), s);
        launch_scan_u32_u64(ctx->tile_cnt.as<uint32_t>() + nt, nt, ctx->tile_off.as<uint64_t>(),
                            ctx->scan_tmp.as<uint64_t>(), stats + ST_BINS, s);
    }
    {
        ScopedTimer tm(ctx, s, KID_BIN_SCATTER);
        launch_tri_bin_scatter(ctx->frange.as<int4>(), ctx->F, nv, tl, ctx->tile_off.as<uint64_t>(),
                               ctx->tile_cnt.as<uint32_t>(), ctx->tile_fill.as<uint32_t>(), ctx->bins.as<uint32_t>(),
                               ctx->bin_cap, ctx->bslot.as<uint32_t>(), s);
    }
    {
        ScopedTimer tm(ctx, s, KID_COUNT);
        launch_count(tl, nv, ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(), ctx->bin_cap,
                     ctx->fscr.as<int4>(), ctx->F, ctx->count.as<uint32_t>(), ctx->masks.as<uint64_t>(),
                     ctx->gpre.as<uint32_t>(), s);
    }
    {
        ScopedTimer tm(ctx, s, KID_SCAN);
        launch_scan_u32_u64(ctx->count.as<uint32_t>(), np, ctx->off.as<uint64_t>(), ctx->scan_tmp.as<uint64_t>(),
                            stats + ST_FRAGS, s);
    }
    if (mode == FRONT_PLAN) {
        ScopedTimer tm(ctx, s, KID_PLAN);
        launch_plan(tl, ctx->off.as<uint64_t>(), budget, stats, s);
    } else {
        launch_single_pass(nt, stats, s);
    }
    enqueue_classify(ctx, nv, 0, s);  // (the first pass's classes, before any read-back)
}

// Waits for `s` and copies the device statistics of the last frame to the host.
hexfc_status read_stats(hexfc_ctx *ctx, hipStream_t s) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_stats, ctx->stats.p, sizeof(uint64_t) * ST_COUNT, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    memcpy(ctx->last_stats, ctx->h_stats, sizeof(ctx->last_stats));
    ctx->stats_known = true;
    return HEXFC_OK;
}

// View parameters to the device: a single view by value through a kernel
// argument (a graph that captures the frame keeps them), a batch by copy.
hexfc_status set_views(hexfc_ctx *ctx, int nv, hipStream_t s) {
    if (nv == 1) {
        launch_set_view(ctx->h_views[0], ctx->views.as<ViewParams>(), s);
        return HEXFC_OK;
    }
    // (pageable source: the runtime stages it before returning, so the host
    // copy may change right after)
    HIPCHK(ctx, hipMemcpyAsync(ctx->views.p, ctx->h_views.data(), sizeof(ViewParams) * nv, hipMemcpyHostToDevice, s));
    return HEXFC_OK;
}

hexfc_status check_views(hexfc_ctx *ctx, int nv, const hexfc_camera *cams) {
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    if ((int)ctx->h_views.size() < nv) ctx->h_views.resize(nv);
    for (int v = 0; v < nv; ++v) {
        TRY(check_camera(ctx, &cams[v], ctx->h_views[v].M));
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
            FAIL(ctx, HEXFC_EINVAL, "all views of a batch must have the same viewport");
        depth_range(ctx, &cams[v], ctx->h_views[v]);
    }
    return HEXFC_OK;
}

// The front half of a frame with one wait: sizes the per-frame buffers,
// enqueues the front and reads the statistics back (a second time when the
// triangle bins had to grow).
hexfc_status prepare(hexfc_ctx *ctx, int nv, const hexfc_camera *cams, hipStream_t s, FrontMode mode) {
    TRY(set_device(ctx));
    TRY(check_views(ctx, nv, cams));
    const Tiling tl = make_tiling(ctx, cams[0].width, cams[0].height);
    TRY(ensure_frame_buffers(ctx, nv, tl));
    TRY(set_views(ctx, nv, s));
    for (int attempt = 0; attempt < 2; ++attempt) {
        enqueue_front(ctx, nv, tl, s, mode);
        TRY(read_stats(ctx, s));
        const uint64_t need = ctx->last_stats[ST_BINS];
        if (need <= ctx->bin_cap) break;
        const uint64_t cap = need + need / 4 + 65536;
        TRY(grow(ctx, ctx->bins, sizeof(uint32_t) * cap));
        TRY(grow(ctx, ctx->masks, sizeof(uint64_t) * cap * (tl.TW * tl.TH / 64)));
        ctx->bin_cap = cap;
    }
    ctx->nv = nv;
    ctx->have_frame = true;
    ctx->last_frags = ctx->last_stats[ST_FRAGS];
    return HEXFC_OK;
}

ResolveArgs resolve_args(hexfc_ctx *ctx, float *rgba, int pass) {
    ResolveArgs a;
    a.tl = ctx->tl;
    a.mesh.posq = ctx->posq.as<int4>();
    a.mesh.vert = vert_ptr(ctx, ctx->nv);
    a.mesh.face = ctx->face.as<FaceRec>();
    a.mesh.vscr = ctx->vscr.as<int4>();
    a.mesh.face_px = ctx->face_px.as<float4>();
    a.mesh.V = ctx->V;
    a.mesh.F = ctx->F;
    a.views = ctx->views.as<ViewParams>();
    a.count = ctx->count.as<uint32_t>();
    a.off = ctx->off.as<uint64_t>();
    a.rec = ctx->ws;
    a.rec_cap = ctx->ws_bytes / 8;
    a.pass_p0 = 0;
    a.pass_tiles = pass >= 0 ? pass_tiles(ctx, pass) : nullptr;
    a.rgba = rgba;
    a.sorted_out = nullptr;
    a.off_rm = nullptr;
    return a;
}

// The work of one resolve: per length class the list, its size (device or
// host) and the size the host expects (the grid size).
struct ResolveSet {
    ClassWork cls[NCLASS];
    uint32_t est[NCLASS];
};

// Class sizes of pass k when the host knows them (the statistics of these
// lists were read back), else ~0u, and for the short lists (class 0) every
// pixel of the views (the grid covers a bound of that class).
void class_estimates(hexfc_ctx *ctx, int k, uint32_t est[NCLASS]) {
    const bool known = ctx->stats_known && k == 0;
    for (int c = 0; c < NCLASS; ++c) est[c] = known ? (uint32_t)ctx->last_stats[ST_PCLASS + c] : ~0u;
    if (!known) est[0] = (uint32_t)std::min<int64_t>((int64_t)ctx->tl.ntiles * ctx->nv * ctx->tl.TW * ctx->tl.TH, 1 << 30);
}

// The class lists of pass k with their sizes in device memory.
ResolveSet pass_set(hexfc_ctx *ctx, int k) {
    ResolveSet rs;
    for (int c = 0; c < NCLASS; ++c) {
        rs.cls[c].list = ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap;
        rs.cls[c].n_dev = ctx->stats.as<uint64_t>() + ST_PCLASS + k * NCLASS + c;
        rs.cls[c].n_host = 0;
        rs.cls[c].queue = ctx->rqueue.as<uint32_t>() + c * QUEUE_SEGS * QUEUE_STRIDE;
    }
    class_estimates(ctx, k, rs.est);
    return rs;
}

// One resolve: the classes above 256 fragments (4..7) on the side stream,
// forked from `s` and joined back, beside classes 3..0 on `s`; longest
// first on both.  Classes known to be empty are not launched.
hexfc_status enqueue_resolve(hexfc_ctx *ctx, const ResolveSet &rs, const ResolveArgs &a, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_RESOLVE);
    launch_zero_u32(ctx->rqueue.as<uint32_t>(), NCLASS * QUEUE_SEGS * QUEUE_STRIDE, s);  // the classes' work queues
    auto used = [&](int c) { return rs.cls[c].n_dev != nullptr || rs.cls[c].n_host != 0; };
    const bool side = used(4) || used(5) || used(6) || used(7);
    if (side) {
        HIPCHK(ctx, hipEventRecord(ctx->ev_fork, s));
        HIPCHK(ctx, hipStreamWaitEvent(ctx->side_stream, ctx->ev_fork, 0));
        for (int c = NCLASS - 1; c >= 4; --c)
            if (used(c)) {
                ScopedTimer tc(ctx, ctx->side_stream, KID_RESOLVE_C0 + c);
                launch_resolve_class(c, rs.cls[c], rs.est[c], ctx->t_sort, ctx->res_min_grid, a, ctx->side_stream);
            }
    }
    for (int c = 3; c >= 0; --c)
        if (used(c)) {
            ScopedTimer tc(ctx, s, KID_RESOLVE_C0 + c);
            launch_resolve_class(c, rs.cls[c], rs.est[c], ctx->t_sort, ctx->res_min_grid, a, s);
        }
    if (side) {
        HIPCHK(ctx, hipEventRecord(ctx->ev_join, ctx->side_stream));
        HIPCHK(ctx, hipStreamWaitEvent(s, ctx->ev_join, 0));
    }
    return HEXFC_OK;
}

void enqueue_fill(hexfc_ctx *ctx, int nv, int k, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_FILL);
    launch_fill(ctx->tl, nv, pass_tiles(ctx, k), ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(), ctx->bin_cap,
                ctx->fscr.as<int4>(), ctx->F, ctx->off.as<uint64_t>(), ctx->ws, ctx->ws_bytes / 8,
                ctx->masks.as<uint64_t>(), ctx->gpre.as<uint32_t>(), s);
}

// Silhouettes: the boundary depth of pass k's tiles of the current lists, and
// the white overlay once every pass has been resolved.
void boundary_depth(hexfc_ctx *ctx, int nv, int k, hipStream_t s) {
    launch_boundary_depth(ctx->tl, nv, pass_tiles(ctx, k), ctx->views.as<ViewParams>(), ctx->count.as<uint32_t>(),
                          ctx->off.as<uint64_t>(), ctx->ws, ctx->ws_bytes / 8, ctx->face_bnd.as<uint8_t>(),
                          ctx->bdepth.as<uint32_t>(), s);
}
void silhouettes(hexfc_ctx *ctx, int nv, float *rgba, hipStream_t s) {
    launch_silhouette(ctx->tl, nv, ctx->views.as<ViewParams>(), ctx->bdepth.as<uint32_t>(), rgba, s);
}

void finish(hexfc_ctx *ctx, int passes, bool single, hipStream_t s) {
    launch_finish(ctx->stats.as<uint64_t>(), ctx->persist.as<uint64_t>(), ctx->d_pub, ctx->bin_cap, passes,
                  ctx->ws_bytes / 8, single, s);
}

// Grows the triangle bins and the number of screen passes launched per
// frame to the largest needs the device has reported so far (host-mapped
// counters of finished frames; nothing waits for the frames in flight).
hexfc_status grow_from_published(hexfc_ctx *ctx, const Tiling &tl) {
    const uint64_t bins = ctx->h_pub[1 + PS_MAX_BINS], passes = ctx->h_pub[1 + PS_MAX_PASSES];
    if (bins > ctx->bin_cap) {  // (the replaced buffers stay allocated for the frames in flight)
        const uint64_t cap = bins + bins / 4 + 65536;
        TRY(grow(ctx, ctx->bins, sizeof(uint32_t) * cap));
        TRY(grow(ctx, ctx->masks, sizeof(uint64_t) * cap * (tl.TW * tl.TH / 64)));
        ctx->bin_cap = cap;
    }
    if (passes > (uint64_t)ctx->passes_launch) ctx->passes_launch = (int)std::min<uint64_t>(passes, MAX_PASSES);
    return HEXFC_OK;
}

// Disables the per-launch event timing while a stream is being captured.
struct NoTimingInCapture {
    hexfc_ctx *ctx;
    bool saved;
    NoTimingInCapture(hexfc_ctx *c, bool cap) : ctx(c), saved(c->prof) {
        if (cap) ctx->prof = false;
    }
    ~NoTimingInCapture() { ctx->prof = saved; }
};

// Host-known class sizes of the last built lists (the learned and
// approximate resolves size their launches with them): waits for them when
// the lists came from a frame that did not read them back.
hexfc_status need_stats(hexfc_ctx *ctx, hipStream_t s) {
    if (!ctx->stats_known) TRY(read_stats(ctx, s));
    return HEXFC_OK;
}

}  // namespace

extern "C" {

hexfc_status hexfc_build_fragment_lists(hexfc_ctx *ctx, const hexfc_camera *cam, uint32_t *counts_out,
                                        void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    if (!cam) FAIL(ctx, HEXFC_EINVAL, "null camera");
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) FAIL(ctx, HEXFC_ESTATE, "hexfc_build_fragment_lists waits for the stream: not in a capture");
    ctx->last_stream = s;
    ctx->lists_valid = false;
    TRY(prepare(ctx, 1, cam, s, FRONT_SINGLE));
    const Tiling &tl = ctx->tl;
    if (ctx->last_stats[ST_FRAGS] * 8 > ctx->ws_bytes)
        FAIL(ctx, HEXFC_EOVERFLOW, "%llu fragments exceed the workspace (%zu bytes)",
             (unsigned long long)ctx->last_stats[ST_FRAGS], ctx->ws_bytes);
    enqueue_fill(ctx, 1, 0, s);
    if (counts_out) launch_rowmajor_counts(tl, ctx->count.as<uint32_t>(), counts_out, s);
    finish(ctx, 1, true, s);
    HIPCHK(ctx, hipGetLastError());
    ctx->lists_valid = true;
    return HEXFC_OK;
}

hexfc_status hexfc_resolve(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, float *rgba_out,
                           void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->lists_valid) FAIL(ctx, HEXFC_ESTATE, "no fragment lists built");
    TRY(check_shading(ctx, hot, style, rgba_out));
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    NoTimingInCapture nt(ctx, capturing(s));
    ctx->last_stream = s;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(set_views(ctx, 1, s));
    TRY(enqueue_resolve(ctx, pass_set(ctx, 0), resolve_args(ctx, rgba_out, 0), s));
    if (style->sil_alpha > 0.f) {
        boundary_depth(ctx, 1, 0, s);
        silhouettes(ctx, 1, rgba_out, s);
    }
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

hexfc_status hexfc_resolve_approx(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, int method,
                                  int k, float *rgba_out, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->lists_valid || ctx->nv != 1) FAIL(ctx, HEXFC_ESTATE, "no single-view fragment lists built");
    TRY(check_shading(ctx, hot, style, rgba_out));
    if (method != HEXFC_APPROX_MLAB && method != HEXFC_APPROX_MOMENTS) FAIL(ctx, HEXFC_EINVAL, "unknown method %d", method);
    if (method == HEXFC_APPROX_MLAB && (k < 1 || k > 8)) FAIL(ctx, HEXFC_ERANGE, "MLAB layers must be in [1, 8]");
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    TRY(need_stats(ctx, s));
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(set_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, rgba_out, 0);
    if (method == HEXFC_APPROX_MLAB) {  // scratch for the shaded fragments, laid out like the records
        const uint64_t nf = std::min<uint64_t>(ctx->last_stats[ST_FRAGS], ctx->ws_bytes / 8);
        TRY(grow(ctx, ctx->mlab_c, sizeof(float4) * std::max<uint64_t>(nf, 1)));
        TRY(grow(ctx, ctx->mlab_z, sizeof(uint32_t) * std::max<uint64_t>(nf, 1)));
    }
    for (int c = 0; c < NCLASS - 1; ++c)
        launch_resolve_approx(c, ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap,
                              (uint32_t)ctx->last_stats[ST_CLASS + c], method, k, ctx->t_sort, a, ctx->mlab_c.as<float4>(),
                              ctx->mlab_z.as<uint32_t>(), s);
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

hexfc_status hexfc_render_frame(hexfc_ctx *ctx, const hexfc_camera *cam, const hexfc_hotspot *hot,
                                const hexfc_style *style, float *rgba_out, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    Mat3q M;
    TRY(check_camera(ctx, cam, M));  // camera limits first (ERANGE)
    TRY(check_shading(ctx, hot, style, rgba_out));
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const bool cap = capturing(s);
    NoTimingInCapture nt(ctx, cap);
    ctx->last_stream = s;
    ctx->lists_valid = false;
    ctx->stats_known = false;
    if (ctx->h_views.empty()) ctx->h_views.resize(1);
    shade_params(ctx->h_views[0].sp, hot, style);
    const int64_t sig[7] = {cam->width, cam->height, ctx->tw, ctx->th, (int64_t)(uintptr_t)ctx->ws,
                            (int64_t)ctx->ws_bytes, (int64_t)ctx->mesh_gen};
    if (memcmp(sig, ctx->frame_sig, sizeof sig) != 0) {
        // new mesh, viewport, tiling or workspace: forget the sizes learned so far
        memcpy(ctx->frame_sig, sig, sizeof sig);
        ctx->sized = false;
        ctx->passes_launch = 1;
        if (!cap) {
            launch_zero_u64(ctx->persist.as<uint64_t>(), PS_COUNT, s);
            for (int i = 0; i <= PS_COUNT; ++i) ctx->h_pub[i] = 0;
        }
    }
    if (!ctx->sized) {
        // The first frame of a mesh, viewport, tiling and workspace waits once
        // for its statistics: bin and list sizes, screen passes.
        if (cap)
            FAIL(ctx, HEXFC_ESTATE,
                 "render one frame of this mesh, viewport, tiling and workspace before capturing one");
        TRY(prepare(ctx, 1, cam, s, FRONT_PLAN));
        const uint64_t *S = ctx->last_stats;
        if (S[ST_PLAN_ERR])
            FAIL(ctx, HEXFC_EOVERFLOW, "one screen tile's fragments exceed the workspace (or > %d passes)", MAX_PASSES);
        ctx->passes_launch = (int)std::max<uint64_t>(1, S[ST_NPASS]);
        ctx->sized = true;
    } else {
        if (!cap) TRY(grow_from_published(ctx, ctx->tl));
        TRY(check_views(ctx, 1, cam));
        TRY(set_views(ctx, 1, s));
        enqueue_front(ctx, 1, ctx->tl, s, FRONT_PLAN);
        ctx->nv = 1;
        ctx->have_frame = true;
    }
    // the passes, whose tile ranges the device planned: passes beyond the
    // planned number find an empty range and return at once
    const bool sil = style->sil_alpha > 0.f;
    for (int k = 0; k < ctx->passes_launch; ++k) {
        if (k) enqueue_classify(ctx, 1, k, s);
        enqueue_fill(ctx, 1, k, s);
        TRY(enqueue_resolve(ctx, pass_set(ctx, k), resolve_args(ctx, rgba_out, k), s));
        if (sil) boundary_depth(ctx, 1, k, s);
    }
    if (sil) silhouettes(ctx, 1, rgba_out, s);
    finish(ctx, ctx->passes_launch, false, s);
    HIPCHK(ctx, hipGetLastError());
    // one launched pass: the whole frame's lists are in the workspace (or the
    // frame is flagged) and hexfc_resolve / the parity export may follow
    ctx->lists_valid = ctx->passes_launch == 1;
    return HEXFC_OK;
}

hexfc_status hexfc_render_batch(hexfc_ctx *ctx, int n, const hexfc_camera *cams, const hexfc_hotspot *hots,
                                const hexfc_style *styles, float *rgba_out, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (n < 1 || !cams || !hots || !styles || !rgba_out) FAIL(ctx, HEXFC_EINVAL, "bad batch arguments");
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    if ((int)ctx->h_views.size() < n) ctx->h_views.resize(n);
    for (int v = 0; v < n; ++v) {
        TRY(check_camera(ctx, &cams[v], ctx->h_views[v].M));
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
            FAIL(ctx, HEXFC_EINVAL, "all views of a batch must have the same viewport");
        TRY(check_shading(ctx, &hots[v], &styles[v], rgba_out));
        shade_params(ctx->h_views[v].sp, &hots[v], &styles[v]);
        depth_range(ctx, &cams[v], ctx->h_views[v]);
    }
    ctx->lists_valid = false;
    ctx->stats_known = false;
    BatchGraph &g = ctx->bg;
    const bool reuse = g.exec && g.nv == n && g.W == cams[0].width && g.H == cams[0].height && g.tw == ctx->tw &&
                       g.th == ctx->th && g.t_sort == ctx->t_sort && g.ws == ctx->ws && g.ws_bytes == ctx->ws_bytes &&
                       g.bin_cap == ctx->bin_cap && g.rgba == rgba_out;
    if (reuse) {
        TRY(set_views(ctx, n, s));
        HIPCHK(ctx, hipGraphLaunch(g.exec, s));
        return HEXFC_OK;
    }
    g.reset();
    if (capturing(s)) FAIL(ctx, HEXFC_ESTATE, "the first call for a batch shape waits for the stream: not in a capture");
    // sizing pass (synchronous), then capture the whole batch as one graph
    TRY(prepare(ctx, n, cams, s, FRONT_SINGLE));
    const uint64_t *S = ctx->last_stats;
    if (S[ST_FRAGS] * 8 > ctx->ws_bytes)
        FAIL(ctx, HEXFC_EOVERFLOW, "%llu fragments exceed the workspace (%zu bytes)", (unsigned long long)S[ST_FRAGS],
             ctx->ws_bytes);
    {  // headroom for other cameras of the same batch shape
        const uint64_t cap = S[ST_BINS] + S[ST_BINS] / 2 + 65536;
        if (cap > ctx->bin_cap) {
            TRY(grow(ctx, ctx->bins, sizeof(uint32_t) * cap));
            TRY(grow(ctx, ctx->masks, sizeof(uint64_t) * cap * (ctx->tl.TW * ctx->tl.TH / 64)));
            ctx->bin_cap = cap;
        }
    }
    const bool prof = ctx->prof;
    ctx->prof = false;  // no event records inside the captured graph
    hipStream_t cs = ctx->cap_stream;
    HIPCHK(ctx, hipStreamSynchronize(s));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue_front(ctx, n, ctx->tl, cs, FRONT_SINGLE);
        enqueue_fill(ctx, n, 0, cs);
        if (e == hipSuccess && enqueue_resolve(ctx, pass_set(ctx, 0), resolve_args(ctx, rgba_out, 0), cs) != HEXFC_OK)
            e = hipErrorUnknown;
        // silhouettes (the kernels skip the views whose sil_alpha is 0)
        boundary_depth(ctx, n, 0, cs);
        silhouettes(ctx, n, rgba_out, cs);
        finish(ctx, 1, true, cs);
        e = hipStreamEndCapture(cs, &g.graph);
    }
    ctx->prof = prof;
    if (e != hipSuccess) {
        g.reset();
        FAIL(ctx, HEXFC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g.reset();
        FAIL(ctx, HEXFC_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    g.nv = n;
    g.W = cams[0].width;
    g.H = cams[0].height;
    g.tw = ctx->tw;
    g.th = ctx->th;
    g.t_sort = ctx->t_sort;
    g.ws = ctx->ws;
    g.ws_bytes = ctx->ws_bytes;
    g.bin_cap = ctx->bin_cap;
    g.rgba = rgba_out;
    HIPCHK(ctx, hipGraphLaunch(g.exec, s));
    return HEXFC_OK;
}

hexfc_status hexfc_batch_status(hexfc_ctx *ctx, uint64_t *fragments, int *overflow, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->have_frame) FAIL(ctx, HEXFC_ESTATE, "no frame rendered");
    TRY(set_device(ctx));
    TRY(read_stats(ctx, (hipStream_t)stream));
    const uint64_t *S = ctx->last_stats;
    ctx->last_frags = S[ST_FRAGS];
    if (fragments) *fragments = S[ST_FRAGS];
    if (overflow) *overflow = S[ST_FLAGS] ? 1 : 0;
    return HEXFC_OK;
}

hexfc_status hexfc_get_total_fragments(hexfc_ctx *ctx, uint64_t *out) {
    if (!ctx || !out) return HEXFC_EINVAL;
    if (!ctx->have_frame) FAIL(ctx, HEXFC_ESTATE, "no frame built");
    TRY(set_device(ctx));
    TRY(read_stats(ctx, ctx->last_stream));
    *out = ctx->last_stats[ST_FRAGS];
    return HEXFC_OK;
}

hexfc_status hexfc_get_frame_stats(hexfc_ctx *ctx, uint64_t *out, int n) {
    if (!ctx || !out || n < 0) return HEXFC_EINVAL;
    if (!ctx->have_frame) FAIL(ctx, HEXFC_ESTATE, "no frame built");
    TRY(set_device(ctx));
    TRY(read_stats(ctx, ctx->last_stream));
    for (int i = 0; i < n && i < ST_COUNT; ++i) out[i] = ctx->last_stats[i];
    return HEXFC_OK;
}

hexfc_status hexfc_export_sorted_lists(hexfc_ctx *ctx, uint32_t *counts_out, uint64_t *off_out, uint64_t *rec_out,
                                       void *stream) {
    if (!ctx || !counts_out || !off_out || !rec_out) return HEXFC_EINVAL;
    if (!ctx->lists_valid || ctx->nv != 1) FAIL(ctx, HEXFC_ESTATE, "no single-view fragment lists built");
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    ctx->last_stream = s;
    const Tiling &tl = ctx->tl;
    const int64_t n = (int64_t)tl.W * tl.H;
    launch_rowmajor_counts(tl, ctx->count.as<uint32_t>(), counts_out, s);
    HIPCHK(ctx, ctx->count_rm_tmp.ensure(sizeof(uint64_t) * scan_tmp_elems(n)));
    launch_scan_u32_u64(counts_out, n, off_out, ctx->count_rm_tmp.as<uint64_t>(), nullptr, s);
    ResolveArgs a = resolve_args(ctx, nullptr, 0);
    a.sorted_out = rec_out;
    a.off_rm = off_out;
    TRY(enqueue_resolve(ctx, pass_set(ctx, 0), a, s));
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ learned tail
namespace {

// Rows of the learned resolve: pixels of the long-list classes 1..6.
int64_t learned_rows(const hexfc_ctx *ctx) {
    int64_t n = 0;
    for (int c = 1; c < NCLASS - 1; ++c) n += (int64_t)ctx->last_stats[ST_CLASS + c];
    return n;
}

hexfc_status learned_checks(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, int K) {
    if (!ctx->lists_valid || ctx->nv != 1) FAIL(ctx, HEXFC_ESTATE, "no single-view fragment lists built");
    if (!hot || !style) FAIL(ctx, HEXFC_EINVAL, "null hotspot or style");
    if (!(hot->radius > 0.f) || !std::isfinite(hot->radius)) FAIL(ctx, HEXFC_EINVAL, "hotspot radius must be > 0");
    if (style->lens_mode != 0)
        FAIL(ctx, HEXFC_EINVAL, "the learned tail's proxy features are defined for the object-space lens");
    if (K < 1 || K > 64) FAIL(ctx, HEXFC_ERANGE, "K must be in [1, 64]");
    TRY(set_device(ctx));
    TRY(need_stats(ctx, ctx->last_stream));
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    return HEXFC_OK;
}

// Head composites and tail features of every long-list pixel, rows in class order.
// With a.rgba set (the learned resolve), rows whose head hides the tail get
// their final colour here (conf_min, mask: as the resolve's).
void enqueue_tail_features(hexfc_ctx *ctx, const ResolveArgs &a, int K, float *head, float *feat, float *target,
                           uint32_t *pix, bool rowmajor, float conf_min, uint8_t *mask, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_TAIL);
    launch_zero_u32(ctx->rqueue.as<uint32_t>(), NCLASS * QUEUE_SEGS * QUEUE_STRIDE, s);  // the classes' work queues
    int64_t base = 0;
    for (int c = 1; c < NCLASS - 1; ++c) {
        const uint32_t nc = (uint32_t)ctx->last_stats[ST_CLASS + c];
        launch_tail_features(c, ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap, nc,
                             ctx->rqueue.as<uint32_t>() + c * QUEUE_SEGS * QUEUE_STRIDE, K, a, head, feat, target,
                             pix, rowmajor, base, conf_min, mask, s);
        base += nc;
    }
}

// Arguments of the learned resolve, checked before anything is enqueued.
hexfc_status learned_resolve_checks(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                    const float *params, int K, float conf_min, const float *rgba_out) {
    TRY(learned_checks(ctx, hot, style, K));
    if (!params || !rgba_out) FAIL(ctx, HEXFC_EINVAL, "null parameters or output");
    if (!(conf_min >= 0.f && conf_min < 1.f)) FAIL(ctx, HEXFC_ERANGE, "conf_min must be in [0, 1)");
    return HEXFC_OK;
}

// Per-row staging of the learned resolve (rows in class order).
struct LearnedStaging {
    float *head;    // [rows][4]
    float *feat;    // [rows][NFEAT]
    uint32_t *pix;  // [rows]
    uint32_t *fb;   // [rows] fallback entries
};

// The learned resolve on staging of at least `rows` rows: short lists exact,
// long ones head + predicted tail or, below the confidence threshold, the
// exact kernels over the fallback entries.  Allocates nothing.
hexfc_status learned_resolve(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                             const float *params, int K, float conf_min, float *rgba_out, uint8_t *mask_out,
                             int64_t rows, const LearnedStaging &st, hipStream_t s) {
    const Tiling &tl = ctx->tl;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(set_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, rgba_out, 0);
    uint64_t *stats = ctx->stats.as<uint64_t>();
    if (mask_out) launch_fill_u8(mask_out, (int64_t)tl.W * tl.H, 1, s);
    launch_zero_u64(stats + ST_FB, NCLASS, s);
    if (ctx->last_stats[ST_CLASS]) {  // short lists: exact
        ResolveSet rs{};
        rs.cls[0].list = ctx->cls.as<uint32_t>();
        rs.cls[0].queue = ctx->rqueue.as<uint32_t>();
        rs.est[0] = rs.cls[0].n_host = (uint32_t)ctx->last_stats[ST_CLASS];
        TRY(enqueue_resolve(ctx, rs, a, s));
    }
    if (rows) {
        enqueue_tail_features(ctx, a, K, st.head, st.feat, nullptr, st.pix, false, conf_min, mask_out, s);
        // fallback list of class c: the segment of the class's rows
        FallbackBase fbb{};
        int64_t base = 0;
        for (int c = 1; c < NCLASS - 1; ++c) {
            fbb.b[c] = base;
            base += (int64_t)ctx->last_stats[ST_CLASS + c];
        }
        {
            ScopedTimer tm(ctx, s, KID_MLP);
            launch_mlp_apply(params, st.feat, st.head, st.pix, rows, a, ctx->t_sort, K, conf_min, st.fb, fbb, stats,
                             mask_out, s);
        }
        // exact resolve of the fallback pixels, their number per class read
        // on the device (the grids are sized for the class's rows)
        ScopedTimer tm(ctx, s, KID_FALLBACK);
        ResolveSet rs{};
        for (int c = 1; c < NCLASS - 1; ++c) {
            const uint32_t nc = (uint32_t)ctx->last_stats[ST_CLASS + c];
            if (!nc) continue;
            rs.cls[c].list = st.fb + fbb.b[c];
            rs.cls[c].n_dev = stats + ST_FB + c;
            rs.cls[c].queue = ctx->rqueue.as<uint32_t>() + c * QUEUE_SEGS * QUEUE_STRIDE;
            rs.est[c] = nc;
        }
        const bool prof = ctx->prof;
        ctx->prof = false;  // (timed as the fallback)
        const hexfc_status rc = enqueue_resolve(ctx, rs, a, s);
        ctx->prof = prof;
        TRY(rc);
    }
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

}  // namespace

extern "C" {

hexfc_status hexfc_learned_features(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, int K,
                                    float *head_out, float *feat_out, float *target_out, uint32_t *pix_out,
                                    int64_t cap, int64_t *rows_out, void *stream) {
    if (!ctx || !rows_out) return HEXFC_EINVAL;
    if (stream) ctx->last_stream = (hipStream_t)stream;
    TRY(learned_checks(ctx, hot, style, K));
    const int64_t rows = learned_rows(ctx);
    *rows_out = rows;
    if (!head_out && !feat_out && !target_out && !pix_out) return HEXFC_OK;  // size query
    if (!head_out || !feat_out || !pix_out) FAIL(ctx, HEXFC_EINVAL, "null output");
    if (cap < rows) FAIL(ctx, HEXFC_EOVERFLOW, "%lld rows exceed the output capacity %lld", (long long)rows,
                         (long long)cap);
    hipStream_t s = (hipStream_t)stream;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(set_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, nullptr, 0);
    enqueue_tail_features(ctx, a, K, head_out, feat_out, target_out, pix_out, true, 0.f, nullptr, s);
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

hexfc_status hexfc_resolve_learned(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                   const float *params, int K, float conf_min, float *rgba_out, uint8_t *mask_out,
                                   void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (stream) ctx->last_stream = (hipStream_t)stream;
    TRY(learned_resolve_checks(ctx, hot, style, params, K, conf_min, rgba_out));
    const int64_t rows = learned_rows(ctx);
    TRY(grow(ctx, ctx->l_head, sizeof(float4) * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_feat, sizeof(float) * NFEAT * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_pix, sizeof(uint32_t) * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_fb, sizeof(uint32_t) * std::max<int64_t>(rows, 1)));
    const LearnedStaging st{ctx->l_head.as<float>(), ctx->l_feat.as<float>(), ctx->l_pix.as<uint32_t>(),
                            ctx->l_fb.as<uint32_t>()};
    return learned_resolve(ctx, hot, style, params, K, conf_min, rgba_out, mask_out, rows, st, (hipStream_t)stream);
}

hexfc_status hexfc_resolve_learned_noalloc(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                           const float *params, int K, float conf_min, float *rgba_out,
                                           uint8_t *mask_out, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (stream) ctx->last_stream = (hipStream_t)stream;
    TRY(learned_resolve_checks(ctx, hot, style, params, K, conf_min, rgba_out));
    if (!ctx->static_scratch) FAIL(ctx, HEXFC_EDEVICE, "%s", ctx->static_scratch_err.c_str());
    const int64_t rows = learned_rows(ctx);
    if (rows > NOALLOC_MAX_ROWS)
        FAIL(ctx, HEXFC_EOVERFLOW, "%lld long-list pixels exceed the static scratch of %lld rows", (long long)rows,
             (long long)NOALLOC_MAX_ROWS);
    // the static array carved as in the allocating call, for the maximum row
    // count (every offset a multiple of 256 bytes); no entry of it has to
    // start at zero: each row's staging is written before it is read
    uint8_t *base = static_cast<uint8_t *>(ctx->static_scratch);
    const int64_t R = NOALLOC_MAX_ROWS;
    const LearnedStaging st{reinterpret_cast<float *>(base), reinterpret_cast<float *>(base + 16 * R),
                            reinterpret_cast<uint32_t *>(base + (16 + 4 * NFEAT) * R),
                            reinterpret_cast<uint32_t *>(base + (20 + 4 * NFEAT) * R)};
    static_assert((16 + 4 * NFEAT + 8) == LEARNED_ROW_BYTES, "row staging layout");
    // no timing events either (creating one may allocate)
    const bool prof = ctx->prof;
    ctx->prof = false;
    const hexfc_status rc =
        learned_resolve(ctx, hot, style, params, K, conf_min, rgba_out, mask_out, rows, st, (hipStream_t)stream);
    ctx->prof = prof;
    return rc;
}

// ------------------------------------------------------------------ autotuner
// Exhaustive search over the tile shapes and the insertion/bitonic switch; the
// median of three timed runs wins.  Results are cached in a small JSON file
// keyed by device, viewport, mesh size and batch size.  Rendering results do
// not depend on the choice (tested).
static std::string tune_key(const hexfc_ctx *ctx, int n, int W, int H) {
    hipDeviceProp_t p;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&p, ctx->device) == hipSuccess) arch = p.gcnArchName;
    std::ostringstream k;
    k << arch.substr(0, arch.find(':')) << "|" << W << "x" << H << "|V" << ctx->V << "|F" << ctx->F << "|n" << n;
    return k.str();
}

hexfc_status hexfc_autotune(hexfc_ctx *ctx, int n, const hexfc_camera *cams, const hexfc_hotspot *hots,
                            const hexfc_style *styles, float *rgba_out, const char *cache_path, int *choice_out,
                            void *stream) {
    if (!ctx || n < 1 || !cams || !hots || !styles || !rgba_out) return HEXFC_EINVAL;
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const std::string key = tune_key(ctx, n, cams[0].width, cams[0].height);
    std::string cache;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::stringstream ss;
        ss << in.rdbuf();
        cache = ss.str();
        const size_t at = cache.find("\"" + key + "\"");
        if (at != std::string::npos) {
            int tw = 0, th = 0, ts = 0;
            if (sscanf(cache.c_str() + at + key.size() + 2, ": {\"tile_w\": %d, \"tile_h\": %d, \"t_sort\": %d", &tw, &th,
                       &ts) == 3) {
                TRY(hexfc_set_tuning(ctx, tw, th, ts));
                if (choice_out) {
                    choice_out[0] = tw;
                    choice_out[1] = th;
                    choice_out[2] = ts;
                }
                return HEXFC_OK;
            }
        }
    }
    const int tiles[4][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 8}};
    const int sorts[5] = {0, 8, 16, 32, 64};
    double best = 1e30;
    int bw = 8, bh = 8, bs = 16;
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    for (auto &t : tiles)
        for (int ts : sorts) {
            hexfc_status st = hexfc_set_tuning(ctx, t[0], t[1], ts);
            if (st) continue;
            auto run = [&]() -> hexfc_status {
                return n == 1 ? hexfc_render_frame(ctx, cams, hots, styles, rgba_out, stream)
                              : hexfc_render_batch(ctx, n, cams, hots, styles, rgba_out, stream);
            };
            if (run() != HEXFC_OK) continue;  // warm-up (and graph capture)
            float ms[3];
            bool ok = true;
            for (int r = 0; r < 3 && ok; ++r) {
                (void)hipEventRecord(e0, s);
                ok = run() == HEXFC_OK;
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                (void)hipEventElapsedTime(&ms[r], e0, e1);
            }
            if (!ok) continue;
            std::sort(ms, ms + 3);
            if (ms[1] < best) {
                best = ms[1];
                bw = t[0];
                bh = t[1];
                bs = ts;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(hexfc_set_tuning(ctx, bw, bh, bs));
    if (choice_out) {
        choice_out[0] = bw;
        choice_out[1] = bh;
        choice_out[2] = bs;
    }
    if (cache_path) {
        std::ostringstream entry;
        entry << "  \"" << key << "\": {\"tile_w\": " << bw << ", \"tile_h\": " << bh << ", \"t_sort\": " << bs
              << ", \"ms\": " << best << "}";
        std::string body = cache;
        const size_t open = body.find('{'), close = body.rfind('}');
        std::string inner = (open != std::string::npos && close != std::string::npos && close > open)
                                ? body.substr(open + 1, close - open - 1)
                                : std::string();
        while (!inner.empty() && (inner.back() == '\n' || inner.back() == ' ')) inner.pop_back();
        std::ofstream out(cache_path, std::ios::trunc);
        out << "{" << inner << (inner.find('"') != std::string::npos ? ",\n" : "\n") << entry.str() << "\n}\n";
    }
    return HEXFC_OK;
}

}  // extern "C"
