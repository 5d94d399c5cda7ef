// api.hip -- host side of libhexfc: context, mesh upload, frame orchestration
// and the C ABI declared in include/hexfc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/hexfc.h"
#include "kern.h"

using namespace hexfc;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, n ? n : 256);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// VTK hexahedron: the 6 faces and, per corner, its three neighbours ordered
// so the unit cube is right-handed at every corner.
const int kFace[6][4] = {{0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};
const int kNb[8][3] = {{1, 3, 4}, {2, 0, 5}, {3, 1, 6}, {0, 2, 7}, {7, 5, 0}, {4, 6, 1}, {5, 7, 2}, {6, 4, 3}};
// local edge table of cell_edge_level
const int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6}, {6, 7}, {7, 4},
                          {0, 4}, {1, 5}, {2, 6}, {3, 7}};

}  // namespace

struct hexfc_ctx {
    int device = 0;
    std::string err;
    // mesh
    int64_t V = 0, C = 0, F = 0;
    DevBuf posq, vert, face, face_c, vscr;
    // tuning
    int tw = 8, th = 8, t_sort = 16;
    // workspace (caller-owned)
    uint64_t *ws = nullptr;
    size_t ws_bytes = 0;
    // per-frame scratch
    DevBuf tile_cnt, tile_fill, tile_off, bins, masks, count, off, scan_tmp, cls, stats;
    DevBuf count_rm_tmp;
    uint64_t bin_cap = 0;
    int64_t cls_cap = 0;
    uint64_t *h_stats = nullptr;  // pinned
    // state of the last build
    Tiling tl{};
    bool lists_valid = false;
    bool have_frame = false;
    uint64_t last_frags = 0;
    uint64_t last_stats[ST_COUNT] = {};
    // optional per-launch timing with HIP events on the launch stream
    bool prof = false;
    struct TimedLaunch {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_pool;
    std::vector<TimedLaunch> pending;
    double acc_ms[KID_COUNT_] = {};
    uint64_t acc_n[KID_COUNT_] = {};
    ~hexfc_ctx() {
        for (auto &t : pending) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace {

hipEvent_t take_event(hexfc_ctx *ctx) {
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

}  // namespace

#define FAIL(ctx, code, ...)                                          \
    do {                                                              \
        char _b[512];                                                 \
        snprintf(_b, sizeof _b, __VA_ARGS__);                         \
        (ctx)->err = _b;                                              \
        return code;                                                  \
    } while (0)

#define HIPCHK(ctx, call)                                                                           \
    do {                                                                                            \
        hipError_t _e = (call);                                                                     \
        if (_e != hipSuccess) FAIL(ctx, HEXFC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(_e)); \
    } while (0)

namespace {

hexfc_status set_device(hexfc_ctx *ctx) {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return HEXFC_OK;
}

// scaled Jacobian of one cell (corners already dequantised): minimum over the
// corners of det[e1,e2,e3] / (|e1||e2||e3|); a zero-length edge gives 0
double cell_scaled_jacobian(const double P[8][3]) {
    double best = 1e300;
    for (int k = 0; k < 8; ++k) {
        double e[3][3], len[3];
        for (int m = 0; m < 3; ++m) {
            for (int a = 0; a < 3; ++a) e[m][a] = P[kNb[k][m]][a] - P[k][a];
            len[m] = std::sqrt(e[m][0] * e[m][0] + e[m][1] * e[m][1] + e[m][2] * e[m][2]);
            if (len[m] == 0.0) return 0.0;
        }
        double cx = e[1][1] * e[2][2] - e[1][2] * e[2][1];
        double cy = e[1][2] * e[2][0] - e[1][0] * e[2][2];
        double cz = e[1][0] * e[2][1] - e[1][1] * e[2][0];
        double det = (e[0][0] * cx + e[0][1] * cy + e[0][2] * cz) / (len[0] * len[1] * len[2]);
        best = std::min(best, det);
    }
    return best;
}

struct EdgeRec {
    uint64_t key;  // (min id << 32) | max id
    float t;
    uint8_t lvl;
};
struct FaceKey {
    uint64_t hi, lo;  // sorted corner ids
    int64_t idx;      // 6*cell + local face
};

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *hexfc_status_string(hexfc_status s) {
    switch (s) {
        case HEXFC_OK: return "ok";
        case HEXFC_EINVAL: return "invalid argument";
        case HEXFC_ERANGE: return "out of range";
        case HEXFC_ENOMEM: return "out of memory";
        case HEXFC_EOVERFLOW: return "overflow";
        case HEXFC_EDEVICE: return "device error";
        case HEXFC_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char *hexfc_last_error(const hexfc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hexfc_status hexfc_create(int device, hexfc_ctx **out) {
    if (!out) return HEXFC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HEXFC_EDEVICE;
    hexfc_ctx *ctx = new (std::nothrow) hexfc_ctx();
    if (!ctx) return HEXFC_ENOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_stats, sizeof(uint64_t) * ST_COUNT, hipHostMallocDefault) != hipSuccess ||
        ctx->stats.ensure(sizeof(uint64_t) * ST_COUNT) != hipSuccess) {
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        delete ctx;
        return HEXFC_EDEVICE;
    }
    *out = ctx;
    return HEXFC_OK;
}

void hexfc_destroy(hexfc_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
    delete ctx;
}

hexfc_status hexfc_set_workspace(hexfc_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx) return HEXFC_EINVAL;
    if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
        FAIL(ctx, HEXFC_EINVAL, "workspace must be 256-byte aligned");
    ctx->ws = dev_ptr ? reinterpret_cast<uint64_t *>(dev_ptr) : nullptr;
    ctx->ws_bytes = dev_ptr ? bytes : 0;
    ctx->lists_valid = false;
    return HEXFC_OK;
}

hexfc_status hexfc_set_tuning(hexfc_ctx *ctx, int tile_w, int tile_h, int t_sort) {
    if (!ctx) return HEXFC_EINVAL;
    bool ok = (tile_w == 8 && tile_h == 8) || (tile_w == 16 && tile_h == 8) || (tile_w == 16 && tile_h == 16) ||
              (tile_w == 32 && tile_h == 8);
    if (!ok) FAIL(ctx, HEXFC_EINVAL, "tile %dx%d not supported (8x8, 16x8, 16x16, 32x8)", tile_w, tile_h);
    if (t_sort < 0 || t_sort > 64) FAIL(ctx, HEXFC_EINVAL, "t_sort must be in [0, 64]");
    ctx->tw = tile_w;
    ctx->th = tile_h;
    ctx->t_sort = t_sort;
    ctx->lists_valid = false;
    return HEXFC_OK;
}

hexfc_status hexfc_upload_mesh(hexfc_ctx *ctx, const float *xyz, int64_t V, const int32_t *hex, int64_t C,
                               const float *cell_scalar, const uint8_t *cell_edge_level) {
    if (!ctx) return HEXFC_EINVAL;
    if (!xyz || V <= 0 || C < 0 || (C > 0 && !hex)) FAIL(ctx, HEXFC_EINVAL, "bad mesh arrays");
    if (V >= (int64_t(1) << 31)) FAIL(ctx, HEXFC_ERANGE, "too many vertices");
    if (C > (int64_t(1) << 28)) FAIL(ctx, HEXFC_ERANGE, "too many cells");
    for (int64_t i = 0; i < 3 * V; ++i)
        if (!(std::fabs(xyz[i]) < 4.0f)) FAIL(ctx, HEXFC_ERANGE, "coordinate %lld out of range", (long long)i);
    for (int64_t i = 0; i < 8 * C; ++i)
        if (hex[i] < 0 || hex[i] >= V) FAIL(ctx, HEXFC_ERANGE, "corner id out of range at %lld", (long long)i);
    if (cell_scalar)
        for (int64_t c = 0; c < C; ++c)
            if (!std::isfinite(cell_scalar[c])) FAIL(ctx, HEXFC_EINVAL, "non-finite cell scalar");

    // quantised positions
    std::vector<int32_t> q(3 * V);
    for (int64_t i = 0; i < 3 * V; ++i) q[i] = (int32_t)std::nearbyint((double)xyz[i] * 65536.0);
    // per-cell importance
    std::vector<double> tc(C);
    double lo = 1e300, hi = -1e300;
    for (int64_t c = 0; c < C; ++c) {
        double raw;
        if (cell_scalar) {
            raw = cell_scalar[c];
        } else {
            double P[8][3];
            for (int k = 0; k < 8; ++k)
                for (int a = 0; a < 3; ++a) P[k][a] = q[3 * (int64_t)hex[8 * c + k] + a] / 65536.0;
            raw = 1.0 - cell_scaled_jacobian(P);
        }
        tc[c] = raw;
        lo = std::min(lo, raw);
        hi = std::max(hi, raw);
    }
    for (int64_t c = 0; c < C; ++c) tc[c] = hi > lo ? (tc[c] - lo) / (hi - lo) : 0.0;
    std::vector<double> tv(V, 0.0);
    for (int64_t c = 0; c < C; ++c)
        for (int k = 0; k < 8; ++k) tv[hex[8 * c + k]] = std::max(tv[hex[8 * c + k]], tc[c]);
    // unique edges: level must agree, importance = max over the sharing cells
    std::vector<EdgeRec> ed((size_t)(12 * C));
    std::vector<double> edt((size_t)(12 * C));
    for (int64_t c = 0; c < C; ++c)
        for (int e = 0; e < 12; ++e) {
            uint32_t a = (uint32_t)hex[8 * c + kEdge[e][0]], b = (uint32_t)hex[8 * c + kEdge[e][1]];
            if (a == b) FAIL(ctx, HEXFC_EINVAL, "cell %lld has a repeated corner", (long long)c);
            EdgeRec &r = ed[12 * c + e];
            r.key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            r.lvl = cell_edge_level ? cell_edge_level[12 * c + e] : 0;
            r.t = 0.f;
            edt[12 * c + e] = tc[c];
        }
    {
        std::vector<int64_t> ord(ed.size());
        for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int64_t)i;
        std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return ed[x].key < ed[y].key; });
        std::vector<EdgeRec> u;
        u.reserve(ed.size() / 3);
        double tmax = 0.0;
        for (size_t i = 0; i < ord.size(); ++i) {
            const EdgeRec &r = ed[ord[i]];
            if (!u.empty() && u.back().key == r.key) {
                if (u.back().lvl != r.lvl) FAIL(ctx, HEXFC_EINVAL, "cells disagree on the level of a shared edge");
                tmax = std::max(tmax, edt[ord[i]]);
            } else {
                if (!u.empty()) u.back().t = (float)tmax;
                u.push_back(r);
                tmax = edt[ord[i]];
            }
        }
        if (!u.empty()) u.back().t = (float)tmax;
        ed.swap(u);
    }
    // unique faces, first-seen order
    std::vector<FaceKey> fr((size_t)(6 * C));
    for (int64_t c = 0; c < C; ++c)
        for (int f = 0; f < 6; ++f) {
            uint32_t k[4];
            for (int i = 0; i < 4; ++i) k[i] = (uint32_t)hex[8 * c + kFace[f][i]];
            std::sort(k, k + 4);
            FaceKey &r = fr[6 * c + f];
            r.hi = ((uint64_t)k[0] << 32) | k[1];
            r.lo = ((uint64_t)k[2] << 32) | k[3];
            r.idx = 6 * c + f;
        }
    std::sort(fr.begin(), fr.end(), [](const FaceKey &x, const FaceKey &y) {
        if (x.hi != y.hi) return x.hi < y.hi;
        if (x.lo != y.lo) return x.lo < y.lo;
        return x.idx < y.idx;
    });
    std::vector<int64_t> first;
    first.reserve(fr.size() / 2 + 1);
    for (size_t i = 0; i < fr.size(); ++i)
        if (i == 0 || fr[i].hi != fr[i - 1].hi || fr[i].lo != fr[i - 1].lo) first.push_back(fr[i].idx);
    std::sort(first.begin(), first.end());
    const int64_t F = (int64_t)first.size();
    if (2 * F >= (int64_t(1) << 31)) FAIL(ctx, HEXFC_ERANGE, "too many faces");
    std::vector<FaceRec> frec(std::max<int64_t>(F, 1));
    for (int64_t f = 0; f < F; ++f) {
        int64_t c = first[f] / 6, lf = first[f] % 6;
        int32_t cv[4];
        for (int i = 0; i < 4; ++i) cv[i] = hex[8 * c + kFace[lf][i]];
        FaceRec &r = frec[f];
        r.c = make_int4(cv[0], cv[1], cv[2], cv[3]);
        float te[4];
        uint32_t lv = 0;
        for (int k = 0; k < 4; ++k) {
            uint32_t a = (uint32_t)cv[k], b = (uint32_t)cv[(k + 1) % 4];
            uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            auto it = std::lower_bound(ed.begin(), ed.end(), key, [](const EdgeRec &e, uint64_t kk) { return e.key < kk; });
            lv |= (uint32_t)it->lvl << (8 * k);
            te[k] = it->t;
        }
        r.te = make_float4(te[0], te[1], te[2], te[3]);
        r.lvl = lv;
        r.pad0 = r.pad1 = r.pad2 = 0;
    }
    // device arrays
    std::vector<int32_t> posq4(4 * V);
    std::vector<VertRec> vrec(V);
    for (int64_t v = 0; v < V; ++v) {
        for (int a = 0; a < 3; ++a) posq4[4 * v + a] = q[3 * v + a];
        posq4[4 * v + 3] = 0;
        vrec[v].world = make_float4((float)(q[3 * v] / 65536.0), (float)(q[3 * v + 1] / 65536.0),
                                    (float)(q[3 * v + 2] / 65536.0), (float)tv[v]);
        vrec[v].scr = make_int4(0, 0, 0, 1);
    }
    hexfc_status st = set_device(ctx);
    if (st) return st;
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, ctx->posq.ensure(sizeof(int32_t) * 4 * V));
    HIPCHK(ctx, ctx->vert.ensure(sizeof(VertRec) * V));
    HIPCHK(ctx, ctx->face.ensure(sizeof(FaceRec) * std::max<int64_t>(F, 1)));
    HIPCHK(ctx, hipMemcpy(ctx->posq.p, posq4.data(), sizeof(int32_t) * 4 * V, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(ctx->vert.p, vrec.data(), sizeof(VertRec) * V, hipMemcpyHostToDevice));
    HIPCHK(ctx, ctx->face_c.ensure(sizeof(int4) * std::max<int64_t>(F, 1)));
    HIPCHK(ctx, ctx->vscr.ensure(sizeof(int4) * V));
    if (F) {
        std::vector<int4> fc(F);
        for (int64_t f = 0; f < F; ++f) fc[f] = frec[f].c;
        HIPCHK(ctx, hipMemcpy(ctx->face.p, frec.data(), sizeof(FaceRec) * F, hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(ctx->face_c.p, fc.data(), sizeof(int4) * F, hipMemcpyHostToDevice));
    }
    ctx->V = V;
    ctx->C = C;
    ctx->F = F;
    ctx->lists_valid = false;
    ctx->have_frame = false;
    return HEXFC_OK;
}

}  // extern "C"

// ================================================================== frame orchestration
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

DevMesh dev_mesh(const hexfc_ctx *ctx) {
    DevMesh m;
    m.posq = ctx->posq.as<int4>();
    m.vert = ctx->vert.as<VertRec>();
    m.face = ctx->face.as<FaceRec>();
    m.face_c = ctx->face_c.as<int4>();
    m.vscr = ctx->vscr.as<int4>();
    m.V = ctx->V;
    m.F = ctx->F;
    return m;
}

hexfc_status read_stats(hexfc_ctx *ctx, hipStream_t s) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_stats, ctx->stats.p, sizeof(uint64_t) * ST_COUNT, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    memcpy(ctx->last_stats, ctx->h_stats, sizeof(ctx->last_stats));
    return HEXFC_OK;
}

// transform, bin, count, scan, classify (whole frame) and plan; one sync
hexfc_status prepare_frame(hexfc_ctx *ctx, const hexfc_camera *cam, hipStream_t s) {
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    Mat3q M;
    hexfc_status st = check_camera(ctx, cam, M);
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    Tiling tl;
    tl.W = cam->width;
    tl.H = cam->height;
    tl.TW = ctx->tw;
    tl.TH = ctx->th;
    tl.ntx = (tl.W + tl.TW - 1) / tl.TW;
    tl.nty = (tl.H + tl.TH - 1) / tl.TH;
    tl.ntiles = tl.ntx * tl.nty;
    const int64_t TP = (int64_t)tl.TW * tl.TH;
    const int64_t np = (int64_t)tl.ntiles * TP;
    const int64_t T = 2 * ctx->F;
    HIPCHK(ctx, ctx->tile_cnt.ensure(sizeof(uint32_t) * tl.ntiles));
    HIPCHK(ctx, ctx->tile_fill.ensure(sizeof(uint32_t) * tl.ntiles));
    HIPCHK(ctx, ctx->tile_off.ensure(sizeof(uint64_t) * (tl.ntiles + 1)));
    HIPCHK(ctx, ctx->count.ensure(sizeof(uint32_t) * np));
    HIPCHK(ctx, ctx->off.ensure(sizeof(uint64_t) * (np + 1)));
    HIPCHK(ctx, ctx->scan_tmp.ensure(sizeof(uint64_t) * std::max(scan_tmp_elems(np), scan_tmp_elems(tl.ntiles))));
    if (ctx->cls_cap < np) {
        HIPCHK(ctx, ctx->cls.ensure(sizeof(uint32_t) * NCLASS * np));
        ctx->cls_cap = np;
    }
    const int nw = (int)(TP / 64);
    if (ctx->bin_cap == 0) {
        uint64_t cap = (uint64_t)(2 * T + 65536);
        HIPCHK(ctx, ctx->bins.ensure(sizeof(uint32_t) * cap));
        ctx->bin_cap = cap;
    }
    HIPCHK(ctx, ctx->masks.ensure(sizeof(uint64_t) * ctx->bin_cap * nw));
    uint64_t *stats = ctx->stats.as<uint64_t>();
    const uint64_t budget = ctx->ws ? ctx->ws_bytes / 8 : 0;
    const int4 *fv = ctx->face_c.as<int4>();
    int4 *vscr = ctx->vscr.as<int4>();
    {
        ScopedTimer tm(ctx, s, KID_TRANSFORM);
        launch_transform(ctx->posq.as<int4>(), ctx->V, M, tl.W, tl.H, ctx->vert.as<VertRec>(), vscr, s);
    }
    launch_zero_u64(stats, ST_COUNT, s);
    launch_zero_u32(ctx->tile_cnt.as<uint32_t>(), tl.ntiles, s);
    {
        ScopedTimer tm(ctx, s, KID_BIN_COUNT);
        launch_tri_bin_count(fv, T, vscr, tl, ctx->tile_cnt.as<uint32_t>(), s);
        launch_scan_u32_u64(ctx->tile_cnt.as<uint32_t>(), tl.ntiles, ctx->tile_off.as<uint64_t>(),
                            ctx->scan_tmp.as<uint64_t>(), stats + ST_BINS, s);
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        launch_zero_u32(ctx->tile_fill.as<uint32_t>(), tl.ntiles, s);
        launch_zero_u64(stats + ST_CLASS, 2 * NCLASS, s);
        {
            ScopedTimer tm(ctx, s, KID_BIN_SCATTER);
            launch_tri_bin_scatter(fv, T, vscr, tl, ctx->tile_off.as<uint64_t>(), ctx->tile_fill.as<uint32_t>(),
                                   ctx->bins.as<uint32_t>(), ctx->bin_cap, s);
        }
        {
            ScopedTimer tm(ctx, s, KID_COUNT);
            launch_count(tl, ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(), ctx->bin_cap, fv, vscr,
                         ctx->count.as<uint32_t>(), ctx->masks.as<uint64_t>(), s);
        }
        {
            ScopedTimer tm(ctx, s, KID_SCAN);
            launch_scan_u32_u64(ctx->count.as<uint32_t>(), np, ctx->off.as<uint64_t>(), ctx->scan_tmp.as<uint64_t>(),
                                stats + ST_FRAGS, s);
        }
        {
            ScopedTimer tm(ctx, s, KID_CLASSIFY);
            launch_classify(tl, 0, tl.ntiles, ctx->count.as<uint32_t>(), ctx->t_sort, ctx->cls.as<uint32_t>(),
                            ctx->cls_cap, stats, s);
        }
        {
            ScopedTimer tm(ctx, s, KID_PLAN);
            launch_plan(tl, ctx->off.as<uint64_t>(), budget, stats, s);
        }
        st = read_stats(ctx, s);
        if (st) return st;
        uint64_t need = ctx->last_stats[ST_BINS];
        if (need <= ctx->bin_cap) break;
        uint64_t cap = need + need / 4 + 65536;
        HIPCHK(ctx, hipStreamSynchronize(s));
        HIPCHK(ctx, ctx->bins.ensure(sizeof(uint32_t) * cap));
        HIPCHK(ctx, ctx->masks.ensure(sizeof(uint64_t) * cap * nw));
        ctx->bin_cap = cap;
    }
    ctx->tl = tl;
    ctx->have_frame = true;
    ctx->last_frags = ctx->last_stats[ST_FRAGS];
    return HEXFC_OK;
}

ResolveArgs resolve_args(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *sty, float *rgba) {
    ResolveArgs a;
    a.tl = ctx->tl;
    a.mesh = dev_mesh(ctx);
    a.count = ctx->count.as<uint32_t>();
    a.off = ctx->off.as<uint64_t>();
    a.rec = ctx->ws;
    a.pass_p0 = 0;
    ShadeParams &p = a.sp;
    if (hot && sty) {
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
    } else {
        memset(&p, 0, sizeof p);
    }
    a.rgba = rgba;
    a.sorted_out = nullptr;
    a.off_rm = nullptr;
    return a;
}

hexfc_status check_shading(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *sty, const float *rgba) {
    if (!hot || !sty || !rgba) FAIL(ctx, HEXFC_EINVAL, "null hotspot, style or output");
    if (!(hot->radius > 0.f) || !std::isfinite(hot->radius)) FAIL(ctx, HEXFC_EINVAL, "hotspot radius must be > 0");
    return HEXFC_OK;
}

void launch_classes(hexfc_ctx *ctx, const ResolveArgs &a, const uint64_t *cls_counts, hipStream_t s) {
    for (int c = 0; c < NCLASS - 1; ++c) {
        if (!cls_counts[c]) continue;
        ScopedTimer tm(ctx, s, KID_RESOLVE0 + c);
        launch_resolve_class(c, ctx->cls.as<uint32_t>() + (int64_t)c * ctx->cls_cap, (uint32_t)cls_counts[c],
                             ctx->t_sort, a, s);
    }
}

void timed_fill(hexfc_ctx *ctx, int t0, int t1, hipStream_t s) {
    ScopedTimer tm(ctx, s, KID_FILL);
    launch_fill(ctx->tl, t0, t1, ctx->tile_off.as<uint64_t>(), ctx->bins.as<uint32_t>(), ctx->bin_cap,
                ctx->face_c.as<int4>(), ctx->vscr.as<int4>(), ctx->off.as<uint64_t>(), ctx->ws,
                ctx->masks.as<uint64_t>(), s);
}

}  // namespace

extern "C" {

hexfc_status hexfc_build_fragment_lists(hexfc_ctx *ctx, const hexfc_camera *cam, uint32_t *counts_out,
                                        void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    hipStream_t s = (hipStream_t)stream;
    ctx->lists_valid = false;
    hexfc_status st = prepare_frame(ctx, cam, s);
    if (st) return st;
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
    hexfc_status st = check_shading(ctx, hot, style, rgba_out);
    if (st) return st;
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    st = set_device(ctx);
    if (st) return st;
    ResolveArgs a = resolve_args(ctx, hot, style, rgba_out);
    launch_classes(ctx, a, ctx->last_stats + ST_CLASS, (hipStream_t)stream);
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

hexfc_status hexfc_render_frame(hexfc_ctx *ctx, const hexfc_camera *cam, const hexfc_hotspot *hot,
                                const hexfc_style *style, float *rgba_out, void *stream) {
    if (!ctx) return HEXFC_EINVAL;
    if (!ctx->ws) FAIL(ctx, HEXFC_ESTATE, "no workspace set");
    if (ctx->V == 0) FAIL(ctx, HEXFC_ESTATE, "no mesh uploaded");
    Mat3q M;
    hexfc_status st = check_camera(ctx, cam, M);  // camera limits first (ERANGE)
    if (st) return st;
    st = check_shading(ctx, hot, style, rgba_out);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    ctx->lists_valid = false;
    st = prepare_frame(ctx, cam, s);
    if (st) return st;
    const Tiling &tl = ctx->tl;
    const uint64_t *S = ctx->last_stats;
    if (S[ST_PLAN_ERR]) FAIL(ctx, HEXFC_EOVERFLOW, "one screen tile's fragments exceed the workspace (or > %d passes)", MAX_PASSES);
    if (S[ST_CLASS + NCLASS - 1]) FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    const int npass = (int)S[ST_NPASS];
    ResolveArgs a = resolve_args(ctx, hot, style, rgba_out);
    if (npass <= 1) {
        timed_fill(ctx, 0, tl.ntiles, s);
        launch_classes(ctx, a, S + ST_CLASS, s);
        HIPCHK(ctx, hipGetLastError());
        ctx->lists_valid = true;
        return HEXFC_OK;
    }
    // several screen passes: each pass fills and resolves a range of tiles
    uint64_t bounds[MAX_PASSES + 1];
    for (int i = 0; i <= npass; ++i) bounds[i] = S[ST_PASS + i];
    uint64_t *stats = ctx->stats.as<uint64_t>();
    for (int k = 0; k < npass; ++k) {
        const int t0 = (int)bounds[k], t1 = (int)bounds[k + 1];
        launch_zero_u64(stats + ST_CLASS, 2 * NCLASS, s);
        launch_classify(tl, t0, t1, ctx->count.as<uint32_t>(), ctx->t_sort, ctx->cls.as<uint32_t>(), ctx->cls_cap,
                        stats, s);
        st = read_stats(ctx, s);
        if (st) return st;
        timed_fill(ctx, t0, t1, s);
        a.pass_p0 = (int64_t)t0 * tl.TW * tl.TH;
        launch_classes(ctx, a, ctx->last_stats + ST_CLASS, s);
        HIPCHK(ctx, hipGetLastError());
    }
    ctx->last_stats[ST_NPASS] = (uint64_t)npass;
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

hexfc_status hexfc_set_profiling(hexfc_ctx *ctx, int enable) {
    if (!ctx) return HEXFC_EINVAL;
    ctx->prof = enable != 0;
    return HEXFC_OK;
}

hexfc_status hexfc_get_kernel_times(hexfc_ctx *ctx, double *ms_out, uint64_t *launches_out, int n) {
    if (!ctx || n < 0) return HEXFC_EINVAL;
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventSynchronize(t.b));
        HIPCHK(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->acc_ms[t.kid] += ms;
        ctx->acc_n[t.kid] += 1;
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->pending.clear();
    for (int i = 0; i < n && i < KID_COUNT_; ++i) {
        if (ms_out) ms_out[i] = ctx->acc_ms[i];
        if (launches_out) launches_out[i] = ctx->acc_n[i];
    }
    for (int i = 0; i < KID_COUNT_; ++i) {
        ctx->acc_ms[i] = 0.0;
        ctx->acc_n[i] = 0;
    }
    return HEXFC_OK;
}

hexfc_status hexfc_export_sorted_lists(hexfc_ctx *ctx, uint32_t *counts_out, uint64_t *off_out, uint64_t *rec_out,
                                       void *stream) {
    if (!ctx || !counts_out || !off_out || !rec_out) return HEXFC_EINVAL;
    if (!ctx->lists_valid) FAIL(ctx, HEXFC_ESTATE, "no fragment lists built");
    if (ctx->last_stats[ST_CLASS + NCLASS - 1])
        FAIL(ctx, HEXFC_EOVERFLOW, "a pixel list exceeds %d fragments", MAX_LIST);
    hexfc_status st = set_device(ctx);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const Tiling &tl = ctx->tl;
    const int64_t n = (int64_t)tl.W * tl.H;
    launch_rowmajor_counts(tl, ctx->count.as<uint32_t>(), counts_out, s);
    HIPCHK(ctx, ctx->count_rm_tmp.ensure(sizeof(uint64_t) * scan_tmp_elems(n)));
    launch_scan_u32_u64(counts_out, n, off_out, ctx->count_rm_tmp.as<uint64_t>(), nullptr, s);
    ResolveArgs a = resolve_args(ctx, nullptr, nullptr, nullptr);
    a.sorted_out = rec_out;
    a.off_rm = off_out;
    launch_classes(ctx, a, ctx->last_stats + ST_CLASS, s);
    HIPCHK(ctx, hipGetLastError());
    return HEXFC_OK;
}

}  // extern "C"
