// api.hip -- host side of libhexfc: context, workspace, tuning, mesh upload
// and per-launch profiling (C ABI of include/hexfc.h; frames: frame.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace hexfc;

// Scratch of hexfc_resolve_learned_noalloc: the per-row staging of the
// learned resolve (head composites, tail features, pixel ids, fallback
// entries) for at most NOALLOC_MAX_ROWS rows.  Each GPU holds one copy from
// the code object's load to the end of the process.  On the host the name is
// only a stand-in: kernels get the device address hipGetSymbolAddress returns.
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];
static_assert(NOALLOC_MAX_ROWS == HEXFC_NOALLOC_MAX_ROWS, "static scratch size as declared");

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices];  // per device, looked up once with that device current

// Device address of the current device's copy of scratch (device = the
// current one); nullptr and the HIP error on failure.
void *scratch_address(int device, hipError_t *err) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    if (!scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        scratch_dev[device] = p;
    }
    return scratch_dev[device];
}

}  // namespace

namespace {

// VTK hexahedron: the 6 faces and, per corner, its three neighbours ordered
// so the unit cube is right-handed at every corner.
const int kFace[6][4] = {{0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};
const int kNb[8][3] = {{1, 3, 4}, {2, 0, 5}, {3, 1, 6}, {0, 2, 7}, {7, 5, 0}, {4, 6, 1}, {5, 7, 2}, {6, 4, 3}};
// local edge table of cell_edge_level
const int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6}, {6, 7}, {7, 4},
                          {0, 4}, {1, 5}, {2, 6}, {3, 7}};

}  // namespace

namespace {


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
    void *pub = nullptr;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_stats, sizeof(uint64_t) * ST_COUNT, hipHostMallocDefault) != hipSuccess ||
        ctx->stats.ensure(sizeof(uint64_t) * ST_COUNT) != hipSuccess ||
        ctx->persist.ensure(sizeof(uint64_t) * PS_COUNT) != hipSuccess ||
        ctx->rqueue.ensure(sizeof(uint32_t) * NCLASS * QUEUE_SEGS * QUEUE_STRIDE) != hipSuccess ||
        hipMemset(ctx->persist.p, 0, sizeof(uint64_t) * PS_COUNT) != hipSuccess ||
        hipHostMalloc(&pub, sizeof(uint64_t) * (PS_COUNT + 1), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->d_pub, pub, 0) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
        ctx->h_stats = nullptr;
        if (pub) (void)hipHostFree(pub);
        delete ctx;
        return HEXFC_EDEVICE;
    }
    memset(pub, 0, sizeof(uint64_t) * (PS_COUNT + 1));
    ctx->h_pub = reinterpret_cast<volatile uint64_t *>(pub);
    resolve_min_grids(device, ctx->res_min_grid);
    hipError_t serr = hipSuccess;
    ctx->static_scratch = scratch_address(device, &serr);
    if (!ctx->static_scratch) {
        ctx->static_scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(serr);
        (void)hipGetLastError();
    }
    if (hipDeviceSynchronize() != hipSuccess) {  // (the counters' zeroing has landed)
        (void)hipHostFree(ctx->h_stats);
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
    ctx->bg.reset();
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
    ctx->bg.reset();
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
    std::vector<int64_t> first, single;  // single: faces of one cell only (the boundary surface)
    first.reserve(fr.size() / 2 + 1);
    for (size_t i = 0; i < fr.size(); ++i)
        if (i == 0 || fr[i].hi != fr[i - 1].hi || fr[i].lo != fr[i - 1].lo) {
            first.push_back(fr[i].idx);
            if (i + 1 == fr.size() || fr[i + 1].hi != fr[i].hi || fr[i + 1].lo != fr[i].lo) single.push_back(fr[i].idx);
        }
    std::sort(first.begin(), first.end());
    std::sort(single.begin(), single.end());
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
    HIPCHK(ctx, ctx->vert0.ensure(sizeof(VertRec) * V));
    HIPCHK(ctx, ctx->face.ensure(sizeof(FaceRec) * std::max<int64_t>(F, 1)));
    HIPCHK(ctx, hipMemcpy(ctx->posq.p, posq4.data(), sizeof(int32_t) * 4 * V, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(ctx->vert0.p, vrec.data(), sizeof(VertRec) * V, hipMemcpyHostToDevice));
    HIPCHK(ctx, ctx->face_c.ensure(sizeof(int4) * std::max<int64_t>(F, 1)));
    HIPCHK(ctx, ctx->face_px.ensure(sizeof(float4) * std::max<int64_t>(F, 1)));
    HIPCHK(ctx, ctx->face_bnd.ensure(std::max<int64_t>(F, 1)));
    if (F) {
        std::vector<uint8_t> bnd(F);
        for (int64_t f = 0, q = 0; f < F; ++f) {  // both lists ascending
            while (q < (int64_t)single.size() && single[q] < first[f]) ++q;
            bnd[f] = q < (int64_t)single.size() && single[q] == first[f];
        }
        HIPCHK(ctx, hipMemcpy(ctx->face_bnd.p, bnd.data(), F, hipMemcpyHostToDevice));
    }
    if (F) {
        std::vector<int4> fc(F);
        std::vector<float4> px(F);  // face centre and mean corner importance (learned-tail proxy)
        for (int64_t f = 0; f < F; ++f) {
            fc[f] = frec[f].c;
            const int cv[4] = {fc[f].x, fc[f].y, fc[f].z, fc[f].w};
            double ctr[3] = {0, 0, 0}, tbar = 0.0;
            for (int k = 0; k < 4; ++k) {
                for (int a = 0; a < 3; ++a) ctr[a] += 0.25 * (q[3 * (int64_t)cv[k] + a] / 65536.0);
                tbar += 0.25 * tv[cv[k]];
            }
            px[f] = make_float4((float)ctr[0], (float)ctr[1], (float)ctr[2], (float)tbar);
        }
        // Binning order: the faces along a Morton curve of their centres, so
        // that the faces of one wave are neighbours on screen as well and
        // meet few distinct tiles (fewer tile atomics).  Records and every
        // other face array keep the canonical (first-seen) face ids.
        std::vector<uint32_t> ord(F);
        {
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int64_t f = 0; f < F; ++f) {
                const double c3[3] = {px[f].x, px[f].y, px[f].z};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], c3[a]);
                    hi[a] = std::max(hi[a], c3[a]);
                }
            }
            auto spread = [](uint64_t x) {  // 21 bits to every third bit
                x &= 0x1fffffull;
                x = (x | (x << 32)) & 0x1f00000000ffffull;
                x = (x | (x << 16)) & 0x1f0000ff0000ffull;
                x = (x | (x << 8)) & 0x100f00f00f00f00full;
                x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
                x = (x | (x << 2)) & 0x1249249249249249ull;
                return x;
            };
            std::vector<uint64_t> code(F);
            for (int64_t f = 0; f < F; ++f) {
                const double c3[3] = {px[f].x, px[f].y, px[f].z};
                uint64_t m = 0;
                for (int a = 0; a < 3; ++a) {
                    const double u = (c3[a] - lo[a]) / std::max(hi[a] - lo[a], 1e-30);
                    m |= spread((uint64_t)std::min(std::max(u * 2097152.0, 0.0), 2097151.0)) << a;
                }
                code[f] = m;
                ord[f] = (uint32_t)f;
            }
            std::sort(ord.begin(), ord.end(),
                      [&](uint32_t x, uint32_t y) { return code[x] != code[y] ? code[x] < code[y] : x < y; });
        }
        std::vector<int4> fco(F);
        for (int64_t i = 0; i < F; ++i) fco[i] = fc[ord[i]];
        HIPCHK(ctx, ctx->face_ord.ensure(sizeof(uint32_t) * F));
        HIPCHK(ctx, hipMemcpy(ctx->face.p, frec.data(), sizeof(FaceRec) * F, hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(ctx->face_c.p, fco.data(), sizeof(int4) * F, hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(ctx->face_ord.p, ord.data(), sizeof(uint32_t) * F, hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(ctx->face_px.p, px.data(), sizeof(float4) * F, hipMemcpyHostToDevice));
    }
    for (int a = 0; a < 3; ++a) {  // bbox of the dequantised positions
        ctx->bbox_lo[a] = 1e300;
        ctx->bbox_hi[a] = -1e300;
    }
    for (int64_t v = 0; v < V; ++v)
        for (int a = 0; a < 3; ++a) {
            const double x = q[3 * v + a] / 65536.0;
            ctx->bbox_lo[a] = std::min(ctx->bbox_lo[a], x);
            ctx->bbox_hi[a] = std::max(ctx->bbox_hi[a], x);
        }
    ctx->V = V;
    ctx->C = C;
    ctx->F = F;
    ctx->mesh_gen += 1;
    ctx->sized = false;
    ctx->lists_valid = false;
    ctx->have_frame = false;
    ctx->vert_b_views = 0;
    ctx->bg.reset();
    return HEXFC_OK;
}

}  // extern "C"

extern "C" {

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

}  // extern "C"
