// kern.h -- internal declarations shared by the library's translation units
// (device data layout, kernel launchers).  Not part of the public ABI.
//
// Every per-frame kernel handles a batch of NV views of the same size: view v
// owns tiles [v*ntiles, (v+1)*ntiles), pixels [v*P_t, (v+1)*P_t) in
// tile-major order (P_t = ntiles * TW * TH), and vertices [v*V, (v+1)*V) of
// the screen arrays.  A single frame is a batch of one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hexfc {

// ---------------------------------------------------------------- constants
constexpr int SUB = 16;                         // sub-pixels per pixel (4 bits)
constexpr int64_t W_NEAR_Q = int64_t(1) << 32;  // w_q below this culls (w < 1/16)
constexpr int64_t GUARD = int64_t(1) << 17;     // |s| >= GUARD culls
constexpr int64_t QNUM = int64_t(1) << 56;      // q = floor(QNUM / w_q)
constexpr uint32_t KMAX = 1u << 24;             // depth field = KMAX - key
constexpr int MAX_PASSES = 64;
constexpr int MAX_LIST = 2048;                  // longest list the learned and approximate resolves take

// length classes: 0 = short (lane per pixel, n <= t_sort), 1..3 = up to 64,
// 128, 256 fragments (wave per pixel, 32-bit keys sorted in registers), 4..6 =
// up to 512, 1024, 2048 (wave per pixel, 64-bit keys in 8, 16, 32 registers
// per lane), 7 = longer (workgroup per pixel: sorted in LDS, or in place in
// the workspace beyond 2048).
constexpr int NCLASS = 8;

// device-side statistics written by the kernels (zeroed at the start of every
// frame; read back by the host only where an entry point says it waits)
enum StatSlot {
    ST_BINS = 0,      // bin entries needed
    ST_FRAGS = 1,     // total fragments
    ST_NPASS = 2,     // passes planned
    ST_PLAN_ERR = 3,  // a single tile exceeds the workspace (or more than MAX_PASSES passes)
    ST_FLAGS = 4,     // FRAME_* flags of the frame (set by the closing kernel)
    ST_CLASS = 8,     // NCLASS class sizes (pixels), all passes
    ST_CLASSF = 16,   // NCLASS class sizes (fragments), all passes
    ST_FB = 24,       // NCLASS pixels sent back to the exact resolve by the learned one
    ST_PASS = 32,     // MAX_PASSES + 1 tile boundaries of the passes
    ST_PCLASS = ST_PASS + MAX_PASSES + 1,  // [MAX_PASSES][NCLASS] class sizes of each pass
    ST_COUNT = ST_PCLASS + MAX_PASSES * NCLASS
};

// flags of a frame (ST_FLAGS): its output is invalid when any is set
enum FrameFlag {
    FRAME_BINS = 1,       // more triangle-bin entries than the bin buffer holds
    FRAME_PASSES = 2,     // more screen passes needed than were launched
    FRAME_PLAN = 4,       // a single screen tile exceeds the workspace, or more than MAX_PASSES passes
    FRAME_WORKSPACE = 8,  // (single-pass frames) more fragments than the workspace holds
};

// device-side counters kept across frames (not zeroed per frame): the
// largest needs seen, so that the host can grow its buffers for later frames
// without waiting on any of them; copied after every frame into host-mapped
// memory by the closing kernel
enum PersistSlot {
    PS_MAX_BINS = 0, PS_MAX_PASSES, PS_FRAMES, PS_FLAGGED, PS_LAST_FLAGS, PS_LAST_FRAGS,
    PS_CLASS = 8,   // NCLASS: per class, the largest size over the passes of the last frame
    PS_COUNT = 16
};

// kernels timed by the optional per-launch HIP-event profiler
enum KernelId {
    KID_TRANSFORM = 0, KID_BIN_COUNT, KID_BIN_SCATTER, KID_COUNT, KID_SCAN, KID_CLASSIFY, KID_PLAN, KID_FILL,
    KID_RESOLVE,   // the resolve (every length class, both streams)
    KID_TAIL,      // learned resolve: head and tail features
    KID_MLP,       // learned resolve: network and compose
    KID_FALLBACK,  // learned resolve: exact fallback
    KID_RESOLVE_C0,  // the resolve kernel of length class c = KID_RESOLVE_C0 + c, on its own stream
    KID_COUNT_ = KID_RESOLVE_C0 + 8
};

struct Mat3q { long long m[3][4]; };  // rows x, y, w of M_q

// One vertex: dequantised world position and importance t_v (set at upload),
// then the view's snapped screen position, inverse depth q and cull flags
// (written by the transform).  32 bytes: one fragment's shading reads whole
// vertices from few cache lines.
struct __align__(32) VertRec {
    float4 world;  // x, y, z, t_v
    int4 scr;      // sx, sy, q, flags (1: behind the near plane, 2: outside the guard band)
};
// One face: corner ids c0..c3, importance t_e and LoD level (4 x u8) of the
// edges k = (c_k, c_{k+1}).  48 bytes.
struct __align__(16) FaceRec {
    int4 c;
    float4 te;
    uint32_t lvl, pad0, pad1, pad2;
};

// Shading constants of one view (hotspot and style, and for the depth cue
// the camera's clip-w row with the mesh's clip-w range).
struct ShadeParams {
    float hc[3], inv_r;
    float w_base, k_focus, halo_w, halo_a, darken, s, bright, delta;
    int lod;
    float lo[3], hi[3], a_lo, a_hi, bg[3];
    int lens_mode;  // 0: object-space sphere, 1: screen-space circle (pixels)
    float desat;    // depth-cue desaturation strength
    float wrow[4], zw0, zinv;
    float sil_a, sil_tau;  // silhouettes: opacity (0: off), relative depth jump
};

// Everything per view that the kernels read from device memory.
struct ViewParams {
    Mat3q M;
    ShadeParams sp;
    float w0, w1;  // view-depth range of the mesh bbox (learned-tail depth feature)
    float pad0, pad1;
};

// A view's parameters, read through the constant address space: the view
// table does not change while a kernel runs, so uniform reads of it become
// scalar loads, and repeated reads need not be repeated (a vector load and a
// wait per use otherwise: the compiler cannot tell that the kernel's stores
// leave the table alone).
typedef const __attribute__((address_space(4))) ViewParams ConstViewParams;
__device__ __forceinline__ const ViewParams &view_params(const ViewParams *views, int64_t v) {
    return *(const ViewParams *)&((ConstViewParams *)views)[v];
}

struct Tiling {
    int W, H, TW, TH, ntx, nty, ntiles;
};

// Mesh arrays resident on the device plus the per-view screen arrays.
struct DevMesh {
    const int4 *posq;      // [V] (X_q, Y_q, Z_q, 0)
    const VertRec *vert;   // [NV*V] world part replicated per view, screen part per view
    const FaceRec *face;   // [F]
    const int4 *vscr;      // [NV*V] screen part alone (dense, for the rasteriser)
    const float4 *face_px; // [F] face centre (xyz) and mean corner importance: learned-tail proxy
    int64_t V, F;
};

// Blocks are dealt round-robin to the 8 XCDs (each with its own L2); remap a
// block index so that every XCD works through one contiguous range.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
    const uint32_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x * q + min(x, r) + i;
}

// Global pixel id -> view and pixel coordinates.
struct PixelRef {
    int64_t view;
    int x, y;
};
__device__ __forceinline__ PixelRef pixel_ref(const Tiling &tl, uint32_t gp) {
    // (tile sides are powers of two; the views' pixels count below 2^32, as their ids do)
    const int sw = __builtin_ctz((unsigned)tl.TW), sh = __builtin_ctz((unsigned)tl.TH), sp = sw + sh;
    const uint32_t pt = (uint32_t)tl.ntiles << sp;
    PixelRef r;
    const uint32_t view = gp / pt;
    const uint32_t p = gp - view * pt;
    const uint32_t tile = p >> sp, l = p & ((1u << sp) - 1u);
    const uint32_t ty = tile / (uint32_t)tl.ntx, tx = tile - ty * (uint32_t)tl.ntx;
    r.view = view;
    r.x = (int)((tx << sw) + (l & (uint32_t)(tl.TW - 1)));
    r.y = (int)((ty << sh) + (l >> sw));
    return r;
}

// Length class of a list of n fragments (see NCLASS).
__device__ __forceinline__ int length_class(uint32_t n, int t_sort) {
    if (n <= (uint32_t)t_sort) return 0;
    if (n <= 64) return 1;
    if (n <= 128) return 2;
    if (n <= 256) return 3;
    if (n <= 512) return 4;
    if (n <= 1024) return 5;
    if (n <= 2048) return 6;
    return 7;
}

// ---------------------------------------------------------------- launchers (geom.hip)
void launch_transform(const int4 *posq, int64_t V, int nv, const ViewParams *views, int W, int H, VertRec *vert,
                      int4 *vscr, hipStream_t s);
// fscr: per (view, face in binning order) the four screen vertices (4 int4),
// written by the binning count pass and read by the scatter, count and fill
// passes; the w of corner 0 holds the canonical face id (-1: culled corner),
// the other w's the transform's culling flags.
// tile_cnt: 2 NT counters (NT = tiles of all views): [0, NT) the entries of
// the faces' first four tiles, whose slots the count pass stores in bslot
// (4 u32 per (view, face)); [NT, 2 NT) the other entries, then the tile
// totals (the scan's input).  The scatter places the first kind from bslot
// and the others after them with atomics on tile_fill.
// face_c / face_ord: the faces' corner ids and canonical ids in binning order.
// Bin entries and fscr are indexed by binning position (entry = 2 position +
// triangle); the fill writes records with canonical triangle ids.
// frange: per (view, binning position) the two triangles' tile ranges
// (x0 | x1 << 16, y0 | y1 << 16 each; x = -1: culled), written by the
// counting pass and read by the scatter pass.
void launch_tri_bin_count(const int4 *face_c, const uint32_t *face_ord, int64_t F, int nv, const int4 *vscr,
                          int64_t V, const Tiling &tl, uint32_t *tile_cnt, int4 *fscr, uint32_t *bslot,
                          int4 *frange, hipStream_t s);
void launch_tri_bin_scatter(const int4 *frange, int64_t F, int nv, const Tiling &tl, const uint64_t *tile_off,
                            const uint32_t *tile_lo, uint32_t *tile_fill, uint32_t *bins, uint64_t bin_cap,
                            const uint32_t *bslot, hipStream_t s);
// Count and fill run 512-lane workgroups per tile.  masks: per bin entry and
// wave, the 64-bit coverage mask; gpre: per tile, RASTER_WG entries (group of
// the workgroup, pixel) with the fragments of the groups before it.  Both are
// written by count and read by fill.
constexpr int RASTER_WG = 512;
void launch_count(const Tiling &tl, int nv, const uint64_t *tile_off, const uint32_t *bins, uint64_t cap,
                  const int4 *fscr, int64_t F, uint32_t *count, uint64_t *masks, uint32_t *gpre, hipStream_t s);
// fill the tiles [pass_tiles[0], pass_tiles[1]) of one pass (device range; the
// grid covers the nv views' tiles, workgroups outside the range return);
// records are relative to off[pass_tiles[0] * TP]; at most rec_cap records
void launch_fill(const Tiling &tl, int nv, const uint64_t *pass_tiles, const uint64_t *tile_off,
                 const uint32_t *bins, uint64_t cap, const int4 *fscr, int64_t F, const uint64_t *off, uint64_t *rec,
                 uint64_t rec_cap, const uint64_t *masks, const uint32_t *gpre, hipStream_t s);
// exclusive scan of n uint32 values into n+1 uint64 values (out[n] = total);
// `stat` (nullable) receives the total.  tmp: scan_tmp_elems(n) uint64s.
size_t scan_tmp_elems(int64_t n);
void launch_scan_u32_u64(const uint32_t *in, int64_t n, uint64_t *out, uint64_t *tmp, uint64_t *stat,
                         hipStream_t s);
void launch_plan(const Tiling &tl, const uint64_t *off, uint64_t budget_recs, uint64_t *stats, hipStream_t s);
// one pass over all ntiles tiles (the pass table of a frame that must fit the workspace)
void launch_single_pass(int64_t ntiles, uint64_t *stats, hipStream_t s);
// pixels of pass k (tiles stats[ST_PASS + k] .. stats[ST_PASS + k + 1]; the grid
// covers the nv views' tiles) into per-class lists (global pixel ids); the
// class sizes go to stats[ST_PCLASS + k NCLASS ...] and are added to the
// frame totals stats[ST_CLASS ...], stats[ST_CLASSF ...]
void launch_classify(const Tiling &tl, int nv, int k, const uint32_t *count, int t_sort, uint32_t *cls_lists,
                     int64_t cls_cap, uint64_t *stats, hipStream_t s);
// closing kernel of a frame: FRAME_* flags into stats[ST_FLAGS], the largest
// needs and frame counters into persist[PS_*], and persist copied to the
// host-mapped `published` (nullable): published[0] = frames finished, then
// persist[0 .. PS_COUNT - 1] at published[1 ..].
void launch_finish(uint64_t *stats, uint64_t *persist, uint64_t *published, uint64_t bin_cap, int passes_launched,
                   uint64_t ws_recs, bool single_pass, hipStream_t s);
// view parameters by value into device memory (a graph capturing the frame keeps them)
void launch_set_view(const ViewParams &vp, ViewParams *dst, hipStream_t s);
void launch_zero_u64(uint64_t *p, int64_t n, hipStream_t s);
void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
void launch_rowmajor_counts(const Tiling &tl, const uint32_t *count_tm, uint32_t *count_rm, hipStream_t s);

// ---------------------------------------------------------------- launchers (resolve.hip)
struct ResolveArgs {
    Tiling tl;
    DevMesh mesh;
    const ViewParams *views;  // [NV]
    const uint32_t *count;    // global tile-major pixels
    const uint64_t *off;
    uint64_t *rec;            // workspace (pass-relative); lists longer than 2048 are sorted in place
    uint64_t rec_cap;         // records the workspace holds
    int64_t pass_p0;          // first global pixel of the pass (when pass_tiles is null)
    const uint64_t *pass_tiles;  // nullable: device [first, end) tiles of the pass; records are
                                 // relative to off[first * TW * TH] (else to off[pass_p0])
    float *rgba;              // [NV][H][W][4], nullable (sort-only)
    uint64_t *sorted_out;     // nullable: sorted records, row-major CSR (single view)
    const uint64_t *off_rm;   // row-major offsets for sorted_out
};
// The pixels of one length class for a resolve launch: a list of global
// pixel ids (entries equal to PIX_SKIP are skipped) and its size, from device
// memory (n_dev) or, when n_dev is null, n_host.
constexpr uint32_t PIX_SKIP = 0xffffffffu;
struct ClassWork {
    const uint32_t *list;
    const uint64_t *n_dev;
    uint32_t n_host;
    uint32_t *queue;  // QUEUE_SEGS * QUEUE_STRIDE u32 of work-queue counters, zero at launch
};
constexpr int QUEUE_STRIDE = 32;  // one counter per 128-byte line
constexpr int QUEUE_SEGS = 64;    // work-queue counters per class (the most any class kernel uses)
// Resolve of class c (see NCLASS).  est: the class size when the host knows
// it (a smaller grid for a short list), else ~0u (a resident grid); the
// kernel takes the true size from device memory either way.
// min_grid: resolve_min_grids(), the workgroups of each class kernel the
// device holds at once (classes 0..7, then class 0 for t_sort <= 32, <= 64).
void resolve_min_grids(int device, int min_grid[NCLASS + 2]);
void launch_resolve_class(int c, const ClassWork &w, uint32_t est, int t_sort, const int min_grid[NCLASS + 2],
                          const ResolveArgs &a, hipStream_t s);

// Learned tail (resolve.hip): for the pixels of long-list class cls, the exact
// composite of the first K sorted fragments (head[4]), 9 tail features and,
// when target != nullptr, the exact composite of the tail (target[4]); row j
// of the outputs is pixel pix_list[j], stored at out_base + j.
constexpr int NFEAT = 9;
// Per-row staging of the learned resolve: head RGBA, NFEAT features, pixel
// id and fallback entry.  The allocation-free variant keeps it in a static
// device array of NOALLOC_MAX_ROWS rows.
constexpr int64_t LEARNED_ROW_BYTES = sizeof(float) * (4 + NFEAT) + 2 * sizeof(uint32_t);
constexpr int64_t NOALLOC_MAX_ROWS = int64_t(1) << 20;  // HEXFC_NOALLOC_MAX_ROWS
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)(NOALLOC_MAX_ROWS * LEARNED_ROW_BYTES);
// pix_out receives the global tile-major pixel id, or with rowmajor the
// image index (view * H + y) * W + x.  With a.rgba set (the learned resolve)
// a pixel whose head is opaque to within 2^-20 and at least conf_min gets
// its final colour here (mask 0) and pix_out PIX_SKIP.  queue: the class's
// QUEUE_SEGS work-queue counters, zero at the launch.
void launch_tail_features(int cls, const uint32_t *pix_list, uint32_t npix, uint32_t *queue, int K,
                          const ResolveArgs &a, float *head, float *feat, float *target, uint32_t *pix_out,
                          bool rowmajor, int64_t out_base, float conf_min, uint8_t *mask, hipStream_t s);

// Silhouettes of the boundary surface: per pixel of the pass's tiles
// (device range pass_tiles[0..1]; the grid covers the nv views' tiles) the
// depth key of its nearest fragment of a boundary face (0: none), for the
// views whose sil_a > 0; then white on the silhouette pixels of all views.
void launch_boundary_depth(const Tiling &tl, int nv, const uint64_t *pass_tiles, const ViewParams *views,
                           const uint32_t *count, const uint64_t *off, const uint64_t *rec, uint64_t rec_cap,
                           const uint8_t *face_bnd, uint32_t *bdepth, hipStream_t s);
void launch_silhouette(const Tiling &tl, int nv, const ViewParams *views, const uint32_t *bdepth, float *rgba,
                       hipStream_t s);

// Approximate order-independent resolves of the pixels of class cls (wave
// per pixel): method 1 multi-layer alpha blending with k nodes (1..8),
// method 2 moment-based transparency (four power moments).
// mc, mz: multi-layer alpha blending scratch (colour and opacity, depth
// field per fragment, laid out like the records); unused by moments.
void launch_resolve_approx(int cls, const uint32_t *pix_list, uint32_t npix, int method, int k, int t_sort,
                           const ResolveArgs &a, float4 *mc, uint32_t *mz, hipStream_t s);

// Learned tail network (learned.hip).  Parameters: FP32 vector of MLP_PARAMS
// floats: mu[9], inv_sigma[9], W1[9][64], b1[64], W2[64][64], b2[64],
// W3[64][5], b3[5]; outputs y[5] = tail RGBA + confidence logit.
constexpr int MLP_PARAMS = 18 + 9 * 64 + 64 + 64 * 64 + 64 + 64 * 5 + 5;
void launch_mlp_forward(const float *params, const float *X, int64_t n, float *Y, hipStream_t s);
void launch_mlp_loss(const float *Y, const float *T, int64_t n, float conf_tol, float *dY, float *loss_sum,
                     hipStream_t s);
void launch_mlp_backward(const float *params, const float *X, const float *dY, int64_t n, float *grad,
                         hipStream_t s);
void launch_adam(float *w, float *m, float *v, const float *g, int count, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s);
// Apply the network to the n rows (rows with pix PIX_SKIP are skipped) and
// compose with their heads.  A row that needs the exact resolve (at most K
// fragments, or confidence below conf_min) is appended to the fallback list
// of its length class c, fb[fb_base.b[c] + i], i counted in stats[ST_FB + c]
// (zero at launch; the list of class c has room for the class's rows); mask
// (nullable) gets 0 where the learned tail was used.
struct FallbackBase {
    int64_t b[NCLASS];
};
void launch_mlp_apply(const float *params, const float *feat, const float *head, const uint32_t *pix, int64_t n,
                      const ResolveArgs &a, int t_sort, int K, float conf_min, uint32_t *fb,
                      const FallbackBase &fb_base, uint64_t *stats, uint8_t *mask, hipStream_t s);
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);

}  // namespace hexfc
