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

// Transform, bin, count, scan, classify (and plan screen passes for one view).
void enqueue_front(hexfc_ctx *ctx, int nv, const Tiling &tl, hipStream_t s, bool plan) {
    const int64_t TP = (int64_t)tl.TW * tl.TH;
    const int64_t nt = (int64_t)tl.ntiles * nv;
    const int64_t np = nt * TP;
    uint64_t *stats = ctx->stats.as<uint64_t>();
    const int4 *fc = ctx->face_c.as<int4>();
    int4 *vscr = ctx->vscr.as<int4>();
    const uint64_t budget = ctx->ws ? ctx->ws_bytes / 8 : 0;
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
                             ctx->tile_cnt.as<uint32_t>(), ctx->fscr.as<int4>(), ctx->bslot.as<uint32_t>(), s);
        launch_scan_u32_u64(ctx->tile_cnt.as<uint32_t>() + nt, nt, ctx->tile_off.as<uint64_t>(),
                            ctx->scan_tmp.as<uint64_t>(), stats + ST_BINS, s);
    }
    {
        ScopedTimer tm(ctx, s, KID_BIN_SCATTER);
        launch_tri_bin_scatter(ctx->fscr.as<int4>(), ctx->F, nv, tl, ctx->tile_off.as<uint64_t>(),
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
    {
        ScopedTimer tm(ctx, s, KID_CLASSIFY);
        launch_classify(tl, 0, nt, ctx->count.as<uint32_t>(), ctx->t_sort, ctx->cls.as<uint32_t>(), ctx->cls_cap,
                        stats, s);
    }
    if (plan) {
        ScopedTimer tm(ctx, s, KID_PLAN);
        launch_plan(tl, ctx->off.as<uint64_t>(), budget, stats, s);
    }
}

hexfc_status read_stats(hexfc_ctx *ctx, hipStream_t s) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_stats, ctx->stats.p, sizeof(uint64_t) * ST_COUNT, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    memcpy(ctx->last_stats, ctx->h_stats, sizeof(ctx->last_stats));
    return HEXFC_OK;
}

hexfc_status upload_views(hexfc_ctx *ctx, int nv, hipStream_t s) {
    // (pageable source: the runtime stages it before returning, so the host
    // copy may change right after)
    HIPCHK(ctx, hipMemcpyAsync(ctx->views.p, ctx->h_views.data(), sizeof(ViewParams) * nv, hipMemcpyHostToDevice, s));
    return HEXFC_OK;
}

// Everything up to the fill for nv views with the given cameras (one sync;
// a second pass only when the triangle bins had to grow).
hexfc_status prepare(hexfc_ctx *ctx, int nv, const hexfc_camera *cams, hipStream_t s, bool plan) {
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    TRY(set_device(ctx));
    if ((int)ctx->h_views.size() < nv) ctx->h_views.resize(nv);
    for (int v = 0; v < nv; ++v) {
        TRY(check_camera(ctx, &cams[v], ctx->h_views[v].M));
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
            FAIL(ctx, HEXFC_EINVAL, "all views of a batch must have the same viewport");
        depth_range(ctx, &cams[v], ctx->h_views[v]);
    }
    const Tiling tl = make_tiling(ctx, cams[0].width, cams[0].height);
    TRY(ensure_frame_buffers(ctx, nv, tl));
    TRY(upload_views(ctx, nv, s));
    for (int attempt = 0; attempt < 2; ++attempt) {
        enqueue_front(ctx, nv, tl, s, plan);
        TRY(read_stats(ctx, s));
        const uint64_t need = ctx->last_stats[ST_BINS];
        if (need <= ctx->bin_cap) break;
        const uint64_t cap = need + need / 4 + 65536;
        TRY(grow(ctx, ctx->bins, sizeof(uint32_t) * cap));
        TRY(grow(ctx, ctx->masks, sizeof(uint64_t) * cap * (tl.TW * tl.TH / 64)));
        ctx->bin_cap = cap;
    }
    ctx->tl = tl;
    ctx->nv = nv;
    ctx->have_frame = true;
    ctx->last_frags = ctx->last_stats[ST_FRAGS];
    return HEXFC_OK;
}

ResolveArgs resolve_args(hexfc_ctx *ctx, float *rgba) {
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
    a.rgba = rgba;
    a.sorted_out = nullptr;
    a.off_rm = nullptr;
    return a;
}

void launch_classes(hexfc_ctx *ctx, const ResolveArgs &a, const uint64_t *cls_counts, const uint64_t *cls_dev,
                    hipStream_t s) {
    for (int c = 0; c < NCLASS - 1; ++c) {
        if (!cls_dev && !cls_counts[c]) continue;
        ScopedTimer tm(ctx, s, KID_RESOLVE0 + c);
        launch_resolve_class(c, ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap,
                             cls_dev ? 0u : (uint32_t)cls_counts[c], cls_dev ? cls_dev + c : nullptr, ctx->t_sort, a,
                             s);
    }
}

// Silhouettes: the boundary depth of the tiles [g0, g1) of the current lists,
// and the white overlay once every pass has been resolved.
void boundary_depth(hexfc_ctx *ctx, int64_t g0, int64_t g1, int64_t pass_p0, hipStream_t s) {
    launch_boundary_depth(ctx->tl, g0, g1, ctx->views.as<ViewParams>(), ctx->count.as<uint32_t>(),
                          ctx->off.as<uint64_t>(), pass_p0, ctx->ws, ctx->ws_bytes / 8, ctx->face_bnd.as<uint8_t>(),
                          ctx->bdepth.as<uint32_t>(), s);
}
void silhouettes(hexfc_ctx *ctx, int nv, float *rgba, hipStream_t s) {
    launch_silhouette(ctx->tl, nv, ctx->views.as<ViewParams>(), ctx->bdepth.as<uint32_t>(), rgba, s);
}

void timed_fill(hexfc_ctx *ctx, int64_t g0, int64_t g1, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_FILL);
    launch_fill(ctx->tl, g0, g1, ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(), ctx->bin_cap,
                ctx->fscr.as<int4>(), ctx->F, ctx->off.as<uint64_t>(), ctx->ws, ctx->ws_bytes / 8,
                ctx->masks.as<uint64_t>(), ctx->gpre.as<uint32_t>(), s);
}

}  // namespace

extern "C" {

hexfc_status hexfc_build_fragment_lists(hexfc_ctx *ctx, const hexfc_camera *cam, uint32_t *counts_out,
                                        void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    hipStream_t s = (hipStream_t)stream;
    ctx->lists_valid = false;
    TRY(prepare(ctx, 1, cam, s, false));
    const Tiling &tl = ctx->tl;
    if (ctx->last_stats[ST_FRAGS] * 8 > ctx->ws_bytes)
        FAIL(ctx, HEXFC_EOVERFLOW, "%llu fragments exceed the workspace (%zu bytes)",
             (unsigned long long)ctx->last_stats[ST_FRAGS], ctx->ws_bytes);
    timed_fill(ctx, 0, tl.ntiles, s);
    if (counts_out) launch_rowmajor_counts(tl, ctx->count.as<uint32_t>(), counts_out, s);
    HIPCHK(ctx, hipGetLastError());
    ctx->lists_valid = true;
    return HEXFC_OK;
}

hexfc_status hexfc_resolve(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, float *rgba_out,
                           void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->lists_valid) FAIL(ctx, HEXFC_ESTATE, "no fragment lists built");
    TRY(check_shading(ctx, hot, style, rgba_out));
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(upload_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, rgba_out);
    launch_classes(ctx, a, ctx->last_stats + ST_CLASS, nullptr, s);
    if (style->sil_alpha > 0.f) {
        boundary_depth(ctx, 0, ctx->tl.ntiles, 0, s);
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
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(upload_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, rgba_out);
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
    hipStream_t s = (hipStream_t)stream;
    ctx->lists_valid = false;
    if (ctx->h_views.empty()) ctx->h_views.resize(1);
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(prepare(ctx, 1, cam, s, true));
    const Tiling &tl = ctx->tl;
    const uint64_t *S = ctx->last_stats;
    if (S[ST_PLAN_ERR])
        FAIL(ctx, HEXFC_EOVERFLOW, "one screen tile's fragments exceed the workspace (or > %d passes)", MAX_PASSES);
    if (S[ST_CLASS + NCLASS - 1]) FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    const int npass = (int)S[ST_NPASS];
    ResolveArgs a = resolve_args(ctx, rgba_out);
    const bool sil = style->sil_alpha > 0.f;
    if (npass <= 1) {
        timed_fill(ctx, 0, tl.ntiles, s);
        launch_classes(ctx, a, S + ST_CLASS, nullptr, s);
        if (sil) {
            boundary_depth(ctx, 0, tl.ntiles, 0, s);
            silhouettes(ctx, 1, rgba_out, s);
        }
        HIPCHK(ctx, hipGetLastError());
        ctx->lists_valid = true;
        return HEXFC_OK;
    }
    // several screen passes: each pass fills and resolves a range of tiles
    uint64_t bounds[MAX_PASSES + 1];
    for (int i = 0; i <= npass; ++i) bounds[i] = S[ST_PASS + i];
    uint64_t *stats = ctx->stats.as<uint64_t>();
    for (int k = 0; k < npass; ++k) {
        const int64_t t0 = (int64_t)bounds[k], t1 = (int64_t)bounds[k + 1];
        launch_zero_u64(stats + ST_CLASS, 2 * NCLASS, s);
        launch_classify(tl, t0, t1, ctx->count.as<uint32_t>(), ctx->t_sort, ctx->cls.as<uint32_t>(), ctx->cls_cap,
                        stats, s);
        TRY(read_stats(ctx, s));
        timed_fill(ctx, t0, t1, s);
        a.pass_p0 = t0 * tl.TW * tl.TH;
        launch_classes(ctx, a, ctx->last_stats + ST_CLASS, nullptr, s);
        if (sil) boundary_depth(ctx, t0, t1, a.pass_p0, s);
        HIPCHK(ctx, hipGetLastError());
    }
    if (sil) silhouettes(ctx, 1, rgba_out, s);
    HIPCHK(ctx, hipGetLastError());
    ctx->last_stats[ST_NPASS] = (uint64_t)npass;
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
    BatchGraph &g = ctx->bg;
    const bool reuse = g.exec && g.nv == n && g.W == cams[0].width && g.H == cams[0].height && g.tw == ctx->tw &&
                       g.th == ctx->th && g.t_sort == ctx->t_sort && g.ws == ctx->ws && g.ws_bytes == ctx->ws_bytes &&
                       g.bin_cap == ctx->bin_cap && g.rgba == rgba_out;
    if (reuse) {
        TRY(upload_views(ctx, n, s));
        HIPCHK(ctx, hipGraphLaunch(g.exec, s));
        return HEXFC_OK;
    }
    g.reset();
    // sizing pass (synchronous), then capture the whole batch as one graph
    TRY(prepare(ctx, n, cams, s, false));
    const uint64_t *S = ctx->last_stats;
    if (S[ST_FRAGS] * 8 > ctx->ws_bytes)
        FAIL(ctx, HEXFC_EOVERFLOW, "%llu fragments exceed the workspace (%zu bytes)", (unsigned long long)S[ST_FRAGS],
             ctx->ws_bytes);
    if (S[ST_CLASS + NCLASS - 1]) FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
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
        enqueue_front(ctx, n, ctx->tl, cs, false);
        launch_fill(ctx->tl, 0, (int64_t)ctx->tl.ntiles * n, ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(),
                    ctx->bin_cap, ctx->fscr.as<int4>(), ctx->F, ctx->off.as<uint64_t>(), ctx->ws, ctx->ws_bytes / 8,
                    ctx->masks.as<uint64_t>(), ctx->gpre.as<uint32_t>(), cs);
        ResolveArgs a = resolve_args(ctx, rgba_out);
        launch_classes(ctx, a, nullptr, ctx->stats.as<uint64_t>() + ST_CLASS, cs);
        // silhouettes (the kernels skip the views whose sil_alpha is 0)
        boundary_depth(ctx, 0, (int64_t)ctx->tl.ntiles * n, 0, cs);
        silhouettes(ctx, n, rgba_out, cs);
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
    if (overflow)
        *overflow = (S[ST_BINS] > ctx->bin_cap || S[ST_FRAGS] * 8 > ctx->ws_bytes || S[ST_CLASS + NCLASS - 1]) ? 1 : 0;
    return HEXFC_OK;
}

hexfc_status hexfc_get_total_fragments(hexfc_ctx *ctx, uint64_t *out) {
    if (!ctx || !out) return HEXFC_EINVAL;
    if (!ctx->have_frame) FAIL(ctx, HEXFC_ESTATE, "no frame built");
    *out = ctx->last_frags;
    return HEXFC_OK;
}

hexfc_status hexfc_get_frame_stats(hexfc_ctx *ctx, uint64_t *out, int n) {
    if (!ctx || !out || n < 0) return HEXFC_EINVAL;
    if (!ctx->have_frame) FAIL(ctx, HEXFC_ESTATE, "no frame built");
    for (int i = 0; i < n && i < ST_COUNT; ++i) out[i] = ctx->last_stats[i];
    return HEXFC_OK;
}

hexfc_status hexfc_export_sorted_lists(hexfc_ctx *ctx, uint32_t *counts_out, uint64_t *off_out, uint64_t *rec_out,
                                       void *stream) {
    if (!ctx || !counts_out || !off_out || !rec_out) return HEXFC_EINVAL;
    if (!ctx->lists_valid || ctx->nv != 1) FAIL(ctx, HEXFC_ESTATE, "no single-view fragment lists built");
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const Tiling &tl = ctx->tl;
    const int64_t n = (int64_t)tl.W * tl.H;
    launch_rowmajor_counts(tl, ctx->count.as<uint32_t>(), counts_out, s);
    HIPCHK(ctx, ctx->count_rm_tmp.ensure(sizeof(uint64_t) * scan_tmp_elems(n)));
    launch_scan_u32_u64(counts_out, n, off_out, ctx->count_rm_tmp.as<uint64_t>(), nullptr, s);
    ResolveArgs a = resolve_args(ctx, nullptr);
    a.sorted_out = rec_out;
    a.off_rm = off_out;
    launch_classes(ctx, a, ctx->last_stats + ST_CLASS, nullptr, s);
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
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    return HEXFC_OK;
}

// Head composites and tail features of every long-list pixel, rows in class order.
void enqueue_tail_features(hexfc_ctx *ctx, const ResolveArgs &a, int K, float *head, float *feat, float *target,
                           uint32_t *pix, bool rowmajor, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_TAIL);
    int64_t base = 0;
    for (int c = 1; c < NCLASS - 1; ++c) {
        const uint32_t nc = (uint32_t)ctx->last_stats[ST_CLASS + c];
        launch_tail_features(c, ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap, nc, K, a, head, feat, target, pix,
                             rowmajor, base, s);
        base += nc;
    }
}

}  // namespace

extern "C" {

hexfc_status hexfc_learned_features(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, int K,
                                    float *head_out, float *feat_out, float *target_out, uint32_t *pix_out,
                                    int64_t cap, int64_t *rows_out, void *stream) {
    if (!ctx || !rows_out) return HEXFC_EINVAL;
    TRY(learned_checks(ctx, hot, style, K));
    const int64_t rows = learned_rows(ctx);
    *rows_out = rows;
    if (!head_out && !feat_out && !target_out && !pix_out) return HEXFC_OK;  // size query
    if (!head_out || !feat_out || !pix_out) FAIL(ctx, HEXFC_EINVAL, "null output");
    if (cap < rows) FAIL(ctx, HEXFC_EOVERFLOW, "%lld rows exceed the output capacity %lld", (long long)rows,
                         (long long)cap);
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(upload_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, nullptr);
    enqueue_tail_features(ctx, a, K, head_out, feat_out, target_out, pix_out, true, s);
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

hexfc_status hexfc_resolve_learned(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                   const float *params, int K, float conf_min, float *rgba_out, uint8_t *mask_out,
                                   void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    TRY(learned_checks(ctx, hot, style, K));
    if (!params || !rgba_out) FAIL(ctx, HEXFC_EINVAL, "null parameters or output");
    if (!(conf_min >= 0.f && conf_min < 1.f)) FAIL(ctx, HEXFC_ERANGE, "conf_min must be in [0, 1)");
    TRY(set_device(ctx));
    hipStream_t s = (hipStream_t)stream;
    const Tiling &tl = ctx->tl;
    const int64_t rows = learned_rows(ctx);
    TRY(grow(ctx, ctx->l_head, sizeof(float4) * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_feat, sizeof(float) * NFEAT * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_pix, sizeof(uint32_t) * std::max<int64_t>(rows, 1)));
    TRY(grow(ctx, ctx->l_fb, sizeof(uint32_t) * std::max<int64_t>(rows, 1)));
    shade_params(ctx->h_views[0].sp, hot, style);
    TRY(upload_views(ctx, 1, s));
    ResolveArgs a = resolve_args(ctx, rgba_out);
    uint64_t *stats = ctx->stats.as<uint64_t>();
    if (mask_out) launch_fill_u8(mask_out, (int64_t)tl.W * tl.H, 1, s);
    launch_zero_u64(stats + ST_FB, NCLASS, s);
    if (ctx->last_stats[ST_CLASS]) {  // short lists: exact
        ScopedTimer tm(ctx, s, KID_RESOLVE0);
        launch_resolve_class(0, ctx->cls.as<uint32_t>(), (uint32_t)ctx->last_stats[ST_CLASS], nullptr, ctx->t_sort, a,
                             s);
    }
    if (rows) {
        float *head = ctx->l_head.as<float>(), *feat = ctx->l_feat.as<float>();
        uint32_t *pix = ctx->l_pix.as<uint32_t>(), *fb = ctx->l_fb.as<uint32_t>();
        enqueue_tail_features(ctx, a, K, head, feat, nullptr, pix, false, s);
        {
            ScopedTimer tm(ctx, s, KID_MLP);
            launch_mlp_apply(params, feat, head, pix, rows, a, ctx->t_sort, K, conf_min, fb, stats, mask_out, s);
        }
        // exact resolve of the fallback pixels: the rows of each class, learned ones skipped
        ScopedTimer tm(ctx, s, KID_FALLBACK);
        int64_t base = 0;
        for (int c = 1; c < NCLASS - 1; ++c) {
            const uint32_t nc = (uint32_t)ctx->last_stats[ST_CLASS + c];
            if (nc) launch_resolve_class(c, fb + base, nc, nullptr, ctx->t_sort, a, s);
            base += nc;
        }
    }
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
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
