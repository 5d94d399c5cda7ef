/*
 * hexfc.h -- C ABI of the MI355X (gfx950) focus+context hex-mesh renderer.
 *
 * Implements the per-frame path of Neuhauser, Wang, Westermann,
 * "Interactive Focus+Context Rendering for Hexahedral Mesh Inspection"
 * (arXiv 2009.06574): every hexahedral face is rasterised as two triangles
 * (Section 4), each pixel's fragments are kept in a per-pixel list, sorted by
 * distance to the camera and alpha-blended front to back (Section 3,
 * Section 6), each fragment being shaded by the focus+context rules of
 * Eq. 1-4 (Section 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status:     every call returns a hexfc_status; no C++ exception crosses the
 *             ABI; hexfc_last_error() gives a human-readable detail.  A failed
 *             call leaves the previously uploaded mesh and built lists intact.
 * Streams:    `stream` is a hipStream_t passed as void* (NULL = the default
 *             stream).  Work is enqueued on it; device outputs are valid once
 *             the stream has been synchronised.
 * Memory:     the context owns its device copy of the mesh and its internal
 *             scratch (bins, counts, offsets).  The fragment workspace
 *             (hexfc_set_workspace) and every *_out device buffer belong to
 *             the caller.  Host input arrays are only read during the call.
 * Threads:    a context is used by one host thread at a time.
 * Devices:    a context is bound to the device given to hexfc_create; every
 *             device pointer passed to it must live on that device.
 *
 * Integer geometry contract (identical results on every device)
 * ------------------------------------------------------------
 * positions   X_q = rint(x * 2^16), |x| < 4 world units
 * camera      M_q = rint(M * 2^20), |M_ij| < 8; rows 0, 1 and 3 of the
 *             row-major world->clip matrix are used (clip w = row 3)
 * screen      4 sub-pixel bits; pixel (i, j) (row j from the top) has its
 *             centre at sub-pixel (16 i + 8, 16 j + 8)
 * culling     a triangle is dropped if a vertex has w < 1/16 or lies outside
 *             the guard band |s| < 2^17 sub-pixels, or if its snapped area is 0
 * fill rule   half-open: a centre on an edge belongs to the triangle whose
 *             interior lies on the side of (+eps, +eps*delta)
 * depth key   q = floor(2^56 / w_q); key = floor(sum E_i q_i / sum E_i) with
 *             the edge functions E_i of the pixel centre (exact inverse-depth
 *             interpolation); record = ((2^24 - key) << 32) | triangle id,
 *             triangle id = 2 * face + {0: (c0,c1,c2), 1: (c0,c2,c3)};
 *             lists are sorted ascending (front to back, ties by face id).
 */
#ifndef HEXFC_H
#define HEXFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hexfc_status {
    HEXFC_OK = 0,
    HEXFC_EINVAL = -1,    /* malformed argument or inconsistent mesh data     */
    HEXFC_ERANGE = -2,    /* value outside the documented limits               */
    HEXFC_ENOMEM = -3,    /* device or host allocation failed                  */
    HEXFC_EOVERFLOW = -4, /* fragments do not fit the workspace / a list limit */
    HEXFC_EDEVICE = -5,   /* a HIP runtime call failed                         */
    HEXFC_ESTATE = -6     /* call order violated (no mesh, no lists, ...)      */
} hexfc_status;

typedef struct hexfc_ctx hexfc_ctx;

/* Camera: row-major float world->clip matrix and viewport (1..8192 each). */
typedef struct hexfc_camera {
    float view_proj[16];
    int32_t width, height;
} hexfc_camera;

/* Focus region: an object-space sphere (the paper's object-space lens,
 * Section 4 / Section 7.1): dist = |p - center| / radius, focus =
 * 1 - smoothstep(0.7, 1, dist).  radius > 0. */
typedef struct hexfc_hotspot {
    float center[3];
    float radius;
} hexfc_hotspot;

/* Live shading constants (Section 6: constant shader parameters).
 *   w_base          minimum edge width in world units (Eq. 1)
 *   k_focus         width gain in focus, w = (1 + k_focus*focus) w_base (Eq. 1)
 *   halo_width      halo band beyond w in focus, scaled by focus (Section 4)
 *   halo_alpha      halo opacity (white halo)
 *   darken          focus-edge darkening: C_F *= 1 - darken*focus
 *   accent_s        accentuation factor s of Eq. 2
 *   accent_brighten face-colour gain on accentuated fragments (Section 4.2)
 *   delta           importance threshold of Eq. 1
 *   lod             LoD threshold of Eq. 1 (edge visible in context iff level >= lod)
 *   tf_*            transfer function: colour lerp(lo, hi, t), opacity lerp(a_lo, a_hi, t)
 *   bg              background colour behind the composite (Section 4.1) */
typedef struct hexfc_style {
    float w_base, k_focus, halo_width, halo_alpha, darken;
    float accent_s, accent_brighten, delta;
    int32_t lod;
    float tf_rgb_lo[3], tf_rgb_hi[3];
    float tf_a_lo, tf_a_hi;
    float bg[3];
    /* lens_mode 0: object-space sphere (hotspot centre and radius in world
     * units); 1: the screen-space circle of Section 4 (hotspot centre[0],
     * centre[1] and radius in pixels, pixel (i, j) at (i + 0.5, j + 0.5);
     * centre[2] unused).  Either way the normalised distance is 1 at the
     * lens border (focus, Eq. 3). */
    int32_t lens_mode;
    /* depth cue in the focus region (Section 7.1): each fragment's colour is
     * moved towards its Rec. 709 luminance by desaturate * focus * z, z the
     * fragment's clip w normalised to the mesh bbox's clip-w range; 0 = off,
     * at most 1. */
    float desaturate;
    /* white exterior and interior screen-space silhouettes of the mesh
     * boundary surface (the faces of one cell only; Section 4.2, final look):
     * a pixel that sees the boundary surface is a silhouette pixel when a
     * 4-neighbour inside the image sees none, or sees it more than
     * (1 + sil_tau) times farther; it gets white of opacity sil_alpha on top
     * (rgb' = (1 - a) rgb + a, A' = a + (1 - a) A).  sil_alpha = 0: off.
     * Applied by hexfc_render_frame, hexfc_resolve and hexfc_render_batch. */
    float sil_alpha, sil_tau;
} hexfc_style;

/* Create a context on HIP device `device`.  *out receives the handle. */
hexfc_status hexfc_create(int device, hexfc_ctx **out);

/* Release the context and every device buffer it owns (NULL is a no-op). */
void hexfc_destroy(hexfc_ctx *ctx);

/* Fragment workspace: caller-owned device memory of `bytes` bytes (8 bytes per
 * fragment record).  A frame whose fragments exceed it is rendered in several
 * screen passes (the paper assumes the lists fit, Section 6, and meets a
 * buffer cap at its largest viewport, Section 7, Table 2), each of which must fit;
 * hexfc_build_fragment_lists needs the whole frame to fit.  The pointer must
 * be 256-byte aligned.  Passing NULL/0 detaches the workspace. */
hexfc_status hexfc_set_workspace(hexfc_ctx *ctx, void *dev_ptr, size_t bytes);

/* Upload a hexahedral mesh (Section 3 / Section 6: all render data resident on
 * the GPU).  Host arrays:
 *   xyz              float [V][3] vertex positions, |x| < 4
 *   hex              int32 [C][8] corner ids, VTK hexahedron order
 *   cell_scalar      float [C] per-cell importance source, or NULL for
 *                    1 - scaled Jacobian (min over the 8 corners, Section 3);
 *                    normalised to [0,1] over the mesh
 *   cell_edge_level  uint8 [C][12] LoD level of each local cell edge
 *                    (0:(0,1) 1:(1,2) 2:(2,3) 3:(3,0) 4:(4,5) 5:(5,6) 6:(6,7)
 *                    7:(7,4) 8:(0,4) 9:(1,5) 10:(2,6) 11:(3,7)), or NULL (all 0)
 * Vertex importance = max over incident cells, edge importance = max over
 * cells sharing the edge (Section 3).  Faces are deduplicated in first-seen
 * order.  Errors: EINVAL (bad sizes, a repeated corner, cells that disagree
 * on a shared edge's level), ERANGE (|x| >= 4, ids out of range, V >= 2^31,
 * more than 2^31 - 1 triangles). */
hexfc_status hexfc_upload_mesh(hexfc_ctx *ctx, const float *xyz, int64_t V, const int32_t *hex,
                               int64_t C, const float *cell_scalar, const uint8_t *cell_edge_level);

/* Build the per-pixel fragment lists of one view (Section 6): transform and
 * snap, bin triangles to screen tiles, count, prefix-scan, fill.  The lists
 * stay in the workspace for hexfc_resolve / hexfc_export_sorted_lists; they
 * do not depend on hotspot or style.  counts_out: optional device uint32
 * [height][width] fragment count per pixel.  Synchronises `stream` once to
 * size its buffers.  Errors: ESTATE (no mesh / no workspace), ERANGE (camera
 * limits), EOVERFLOW (the frame does not fit the workspace). */
hexfc_status hexfc_build_fragment_lists(hexfc_ctx *ctx, const hexfc_camera *cam,
                                        uint32_t *counts_out, void *stream);

/* Resolve the last built lists: sort each pixel's list front to back, shade
 * every fragment (Eq. 1-4) and composite (Section 4.2) over the background.
 * The pixels go by list length to one kernel per length class (a lane, a
 * wave or a workgroup per list; the classes above 256 fragments on a second
 * stream, forked and joined with events); each kernel reads its class size
 * from device memory.  Lists of any length are sorted (those longer than 2048
 * fragments in place in the workspace, which leaves each list's records
 * reordered, not changed).
 * rgba_out: device float [height][width][4], premultiplied colour plus
 * accumulated opacity.  Does not wait for the stream.  Errors: ESTATE (no
 * lists), EINVAL (radius <= 0). */
hexfc_status hexfc_resolve(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                           float *rgba_out, void *stream);

/* One frame: build + resolve, in several screen passes when the fragments
 * exceed the workspace (each pass fills and resolves a range of screen tiles
 * that the device plans from the pixels' fragment counts).  Nothing waits for
 * the stream and nothing is copied to the host, so the call can be captured in
 * a HIP graph, with one exception: the first frame of a mesh, viewport, tiling
 * and workspace waits once for its statistics (bin sizes, number of screen
 * passes), and must not be captured.  Later frames use the sizes learned so
 * far and grow them, without waiting, from counters the device publishes to
 * host-mapped memory after every frame; a frame that outgrows them (more bin
 * entries, more screen passes) has an invalid output, is flagged (see
 * hexfc_batch_status) and makes the next call grow.  Same outputs as the two
 * calls above.  Errors: as above, EOVERFLOW (first frame: one screen tile's
 * fragments exceed the workspace), ESTATE (the first frame inside a capture). */
hexfc_status hexfc_render_frame(hexfc_ctx *ctx, const hexfc_camera *cam, const hexfc_hotspot *hot,
                                const hexfc_style *style, float *rgba_out, void *stream);

/* Batch of n views of the same viewport, each with its own camera, hotspot
 * and style, rendered by one captured HIP graph: every stage (transform,
 * binning, count, scan, classes, fill, resolve) runs once over all views, the
 * resolve's class kernels reading the list classes from device memory.  The first call for a batch shape sizes the buffers
 * (synchronising `stream` once) and captures the graph; later calls upload
 * the view parameters and launch the graph without synchronising.  The
 * workspace must hold the fragments of all n views.  rgba_out: device float
 * [n][height][width][4].  A later call whose fragments outgrow the sizes
 * captured is reported by hexfc_batch_status.  Errors: as hexfc_render_frame,
 * EINVAL (viewports differ), EDEVICE (capture failed). */
hexfc_status hexfc_render_batch(hexfc_ctx *ctx, int n, const hexfc_camera *cams, const hexfc_hotspot *hots,
                                const hexfc_style *styles, float *rgba_out, void *stream);

/* Waits for `stream`, then reports the fragments of the last batch (or frame)
 * and whether it overflowed the sizes it was enqueued with (more triangle-bin
 * entries, more screen passes, or more fragments than one pass holds): its
 * output is then invalid. */
hexfc_status hexfc_batch_status(hexfc_ctx *ctx, uint64_t *fragments, int *overflow, void *stream);

/* Autotuner: times every tile shape x t_sort in {0, 8, 16, 32, 64} on the
 * given views (n == 1: hexfc_render_frame, else hexfc_render_batch; median of
 * three runs), applies the fastest and records it in the JSON file at
 * cache_path (NULL: no cache), keyed by device, viewport, mesh size and n; a
 * cached entry is applied without timing.  choice_out (nullable) receives
 * {tile_w, tile_h, t_sort}.  rgba_out is scratch output. */
hexfc_status hexfc_autotune(hexfc_ctx *ctx, int n, const hexfc_camera *cams, const hexfc_hotspot *hots,
                            const hexfc_style *styles, float *rgba_out, const char *cache_path, int *choice_out,
                            void *stream);

/* Tuning knobs (chosen by the autotuner): screen tile of tile_w x tile_h
 * pixels (8x8, 16x8, 16x16 or 32x8; one workgroup lane per pixel) and the
 * longest list sorted lane-per-pixel by insertion sort (t_sort in [0, 64];
 * longer lists use the wave-per-pixel bitonic sort).  Results do not depend
 * on them.  Invalidates built lists. */
hexfc_status hexfc_set_tuning(hexfc_ctx *ctx, int tile_w, int tile_h, int t_sort);

/* Statistics of the last build/render; waits for the stream of the last
 * call: out[0] bin entries, out[1] fragments, out[2] screen passes planned,
 * out[4] flags (nonzero: the frame outgrew its sizes, see
 * hexfc_batch_status), out[8..15] pixels per length class (0: n <= t_sort;
 * 1..7: n <= 64, 128, 256, 512, 1024, 2048, longer), out[16..23] fragments
 * per length class, out[24..31] pixels per class that the last
 * hexfc_resolve_learned sent to the exact fallback.  n = number of entries
 * wanted (<= 32). */
hexfc_status hexfc_get_frame_stats(hexfc_ctx *ctx, uint64_t *out, int n);

/* Per-launch timing with HIP events recorded on the launch stream (off by
 * default; never inside a stream capture).  hexfc_get_kernel_times waits for
 * the recorded events, returns the accumulated milliseconds and launch counts
 * per kernel and resets them.  Kernel index: 0 transform, 1 triangle binning
 * (count + tile scan), 2 bin scatter, 3 coverage count, 4 pixel scan,
 * 5 length classes, 6 pass plan, 7 list fill, 8 resolve (every length class
 * of a pass, both streams, fork to join), 9 learned tail: head and features,
 * 10 learned tail: network and compose, 11 learned tail: exact fallback,
 * 12 + c the resolve kernel of length class c alone (c = 0..7; part of 8;
 * classes 4..7 run on a second stream, their times include waiting for the
 * compute units the first stream holds).  n = number of entries wanted
 * (<= 20). */
hexfc_status hexfc_set_profiling(hexfc_ctx *ctx, int enable);
hexfc_status hexfc_get_kernel_times(hexfc_ctx *ctx, double *ms_out, uint64_t *launches_out, int n);

/* Total fragments of the last build/render (waits for the stream of the last call). */
hexfc_status hexfc_get_total_fragments(hexfc_ctx *ctx, uint64_t *out);

/* Parity export of the last built lists, row-major pixel order:
 *   counts_out  device uint32 [H*W]
 *   off_out     device uint64 [H*W + 1] exclusive offsets
 *   rec_out     device uint64 [total fragments] records, each list sorted
 * Errors: ESTATE (no lists). */
hexfc_status hexfc_export_sorted_lists(hexfc_ctx *ctx, uint32_t *counts_out, uint64_t *off_out,
                                       uint64_t *rec_out, void *stream);

/* Approximate order-independent resolves of the lists of the last
 * hexfc_build_fragment_lists (one view), for comparison with the exact sorted
 * blend (the paper names approximate transparency without per-pixel sorting
 * as future work, Section 8).  Every fragment is shaded by Eq. 1-4.
 *   HEXFC_APPROX_MLAB     multi-layer alpha blending (Salvi and
 *                         Vaidyanathan 2014) with k blending nodes (1..8);
 *                         fragments arrive in primitive order (ascending
 *                         triangle id), are inserted at their depth (after
 *                         nodes of equal depth), and the last two nodes merge
 *                         when there are k + 1.  Exact when k >= list length.
 *   HEXFC_APPROX_MOMENTS  moment-based order-independent transparency
 *                         (Muenstermann et al. 2018): four power moments of
 *                         the absorbance -ln(1 - alpha) over the depth warped
 *                         to [-1, 1] (clip w over the mesh bbox range); per
 *                         fragment the Hamburger bound of the absorbance in
 *                         front (moment bias 5e-5 towards (0, 0.375, 0,
 *                         0.375), own-depth weight 0.25), in FP64; colours
 *                         rescaled so that the opacity is the exact
 *                         1 - prod(1 - alpha).  k is ignored.
 *   rgba_out              device float [H][W][4] (as hexfc_resolve)
 * MLAB keeps a context-owned scratch of 20 bytes per fragment (the shaded
 * fragments in primitive order), grown on first use.
 * Errors: ESTATE, EINVAL (method), ERANGE (k), EOVERFLOW, ENOMEM. */
enum { HEXFC_APPROX_MLAB = 1, HEXFC_APPROX_MOMENTS = 2 };
hexfc_status hexfc_resolve_approx(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                  int method, int k, float *rgba_out, void *stream);

/* ------------------------------------------------------------------------
 * Learned tail compositor.  Long per-pixel lists are resolved as an exact
 * head (the first K fragments in depth order, shaded by Eq. 1-4 and blended
 * front to back as in Section 3) plus a tail predicted by a small MLP from 9
 * features of the remaining n - K fragments.  This follows the paper's
 * future-work direction of approximating order-independent transparency
 * (Section 8); it is not part of the paper's method, whose exact resolve
 * (hexfc_resolve) stays the reference and the fallback.
 *
 * Tail features of a pixel (fragments i = K+1..n in depth order), with the
 * proxy opacity a_i = alpha_TF(tbar_i) * min(|c_i - h| / r, 1)^4 and colour
 * C_i = rgb_TF(tbar_i) of fragment i's face (c_i = centre of the face's
 * dequantised corners, tbar_i = mean corner importance; h, r = hotspot) and
 * the normalised view depth z_i = clamp((w_i - w0) / (w1 - w0), 0, 1)
 * (w_i = 2^20 / depth key, [w0, w1] = clip-w range of the mesh bbox corners
 * under the float camera matrix):
 *   f0 = log1p(n - K), f1 = sum a_i,
 *   f2 = sum a_i z_i / sum a_i, f3 = sum a_i z_i^2 / sum a_i (0 where
 *   sum a_i = 0),
 *   f4..f7 = premultiplied RGBA of the proxies (a_i C_i, a_i) composited
 *   front to back in depth order,
 *   f8 = z_{K+1}, the depth where the tail starts.
 *
 * Network parameters: FP32 device vector of hexfc_mlp_param_count() = 5143
 * floats, in this order: mu[9], inv_sigma[9] (input standardisation,
 * x' = (x - mu) * inv_sigma; not trained), W1[9][64], b1[64], W2[64][64],
 * b2[64], W3[64][5], b3[5] (row-major [in][out]); h1 = gelu(x' W1 + b1),
 * h2 = gelu(h1 W2 + b2), y = h2 W3 + b3 with the tanh form of GELU.  y[0..3]
 * is the tail's premultiplied RGBA, y[4] a confidence logit.  The kernels
 * round weights and activations to BF16 for the matrix cores and accumulate
 * in FP32; master weights and gradients are FP32.
 * ---------------------------------------------------------------------- */

/* Learned resolve of the lists of the last hexfc_build_fragment_lists (one
 * view).  Lists of at most t_sort fragments (length class 0) are resolved
 * exactly; for longer lists the exact head is composed with the predicted
 * tail (clamped to [0, 1]) when the list is longer than K and the pixel
 * confidence 1 - (1 - A_head) * (1 - sigmoid(y[4])) is at least conf_min
 * (the prediction is trusted, or the head hides the tail), else the pixel is
 * resolved by the exact kernels (fallback; its result is then bit-identical
 * to hexfc_resolve's).  For K <= 16 the head is found by a top-K selection
 * without sorting the list, and a pixel whose head is opaque to within 2^-20
 * (where the exact resolve stops too) and at least conf_min is finished with
 * the head alone (mask 0): its tail is neither sorted nor evaluated.
 *   params      device float[5143] (see above)
 *   K           head length, 1..64
 *   conf_min    confidence threshold in [0, 1); 0 accepts every prediction
 *   rgba_out    device float [H][W][4] (as hexfc_resolve)
 *   mask_out    device uint8 [H][W] or NULL: 1 = exact, 0 = learned tail
 * Keeps a context-owned staging of 60 bytes per long-list pixel (head
 * composite, tail features, pixel id, fallback entry), grown on demand.
 * Errors: ESTATE (no single-view lists), ERANGE (K, conf_min), EINVAL,
 * EOVERFLOW (a list longer than 2048), ENOMEM. */
hexfc_status hexfc_resolve_learned(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                   const float *params, int K, float conf_min, float *rgba_out,
                                   uint8_t *mask_out, void *stream);

/* hexfc_resolve_learned for callers that cannot allocate device memory
 * (tight serving loops, hosts or harnesses that forbid hipMalloc): the same
 * kernels, arguments and results, with the per-row staging in a static device
 * array of HEXFC_NOALLOC_MAX_ROWS rows (60 MiB) that each GPU holds from the
 * library's load to the end of the process.
 * Calls neither hipMalloc nor hipFree nor anything that allocates; the lists
 * must have been built before (hexfc_build_fragment_lists).  Not timed by
 * hexfc_set_profiling.  Every call on a GPU, from any context, shares that
 * GPU's array: calls whose work overlaps on one GPU race and must be ordered
 * by the caller (one stream, or events).
 * Errors: as hexfc_resolve_learned (never ENOMEM), plus EOVERFLOW when more than
 * HEXFC_NOALLOC_MAX_ROWS pixels have lists longer than t_sort (nothing is
 * enqueued then) and EDEVICE when the array's address could not be looked up
 * when the context was created. */
#define HEXFC_NOALLOC_MAX_ROWS (1 << 20)
hexfc_status hexfc_resolve_learned_noalloc(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style,
                                           const float *params, int K, float conf_min, float *rgba_out,
                                           uint8_t *mask_out, void *stream);

/* Training and evaluation data of the learned resolve for the lists of the
 * last hexfc_build_fragment_lists: one row per pixel of the long-list classes
 * (n > t_sort), the rows hexfc_resolve_learned feeds to the network.
 *   head_out    device float [cap][4] exact composite of the first K fragments
 *   feat_out    device float [cap][9] tail features (above)
 *   target_out  device float [cap][4] or NULL: exact composite of the tail
 *               (fragments K+1..n shaded by Eq. 1-4, blended front to back)
 *   pix_out     device uint32 [cap] pixel index y * W + x
 *   rows_out    host: number of rows (all outputs NULL: size query only)
 * Errors: ESTATE, ERANGE (K), EOVERFLOW (cap < rows). */
hexfc_status hexfc_learned_features(hexfc_ctx *ctx, const hexfc_hotspot *hot, const hexfc_style *style, int K,
                                    float *head_out, float *feat_out, float *target_out, uint32_t *pix_out,
                                    int64_t cap, int64_t *rows_out, void *stream);

/* Network kernels on caller device buffers (no context; the current HIP
 * device; status only, no error text).  n rows, row-major.
 * forward:  y[n][5] = MLP(x[n][9]).
 * loss:     per row, (1/4) sum_c (y_c - t_c)^2 + 0.1 * BCE(sigmoid(y_4), l),
 *           l = 1 if max_c |y_c - t_c| < conf_tol else 0 (target t[n][4],
 *           conf_tol > 0); *loss_sum += sum over rows;
 *           dy[n][5] = d(mean loss)/dy.
 * backward: grad[5143] += d(sum dy * y)/d params (entries 0..17 untouched);
 *           the caller zeroes grad.
 * adam:     one Adam step (step counts from 1, bias-corrected) on entries
 *           18..5142 of params with moments m, v (each float[5143]).
 * Errors: EINVAL (null pointer with n > 0, n < 0), ERANGE (Adam constants),
 * EDEVICE (launch failure). */
int64_t hexfc_mlp_param_count(void);
hexfc_status hexfc_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream);
hexfc_status hexfc_mlp_loss(const float *y, const float *target, int64_t n, float conf_tol, float *dy,
                            float *loss_sum, void *stream);
hexfc_status hexfc_mlp_backward(const float *params, const float *x, const float *dy, int64_t n, float *grad,
                                void *stream);
hexfc_status hexfc_mlp_adam_step(float *params, float *m, float *v, const float *grad, float lr, float beta1,
                                 float beta2, float eps, int step, void *stream);

const char *hexfc_status_string(hexfc_status s);
/* ---------------------------------------------------------------- LoD
 * Sheet-based level-of-detail hierarchy of the mesh edges (Section 5,
 * Section 5.1): the preprocessing that produces cell_edge_level for
 * hexfc_upload_mesh.  Host-only: no context, no device work; safe to call
 * concurrently on different meshes.
 *
 * Hexahedral sheets (cells joined through topologically parallel edges) are
 * extracted; each sheet's cells form a component.  Pairs of components that
 * a merge would join along at least one boundary face are classified as
 * adjacent (no shared cell), hybrid (shared cells and faces between cells of
 * only one each) or intersecting, and merged in the order: adjacent, hybrid,
 * intersecting, then the larger Eq. 5 weight (boundary faces made interior
 * over the two boundary sizes, over the two cell counts; compared exactly),
 * then the smaller pair of ids (sheets numbered by first appearance, cells in
 * order and within a cell the directions of local edges 0, 1, 8; merged
 * components numbered on from there).  The edges of the faces on both
 * boundaries that a merge makes interior disappear at the current level; the
 * first merge opens level 1 and a merge whose result has more than twice
 * the cells of the larger input of the merge that opened the current level
 * opens the next one.  Merging ends when no pair can be merged; L is the
 * last level.  e_level = (level of disappearance) - 1, or L if the edge never
 * disappears; singular edges (on the boundary with other than 2 incident
 * cells, inside with other than 4) that disappear get L - 1, edges with one
 * incident cell keep L.
 *
 *   hex              host int32 [C][8] corner ids in [0, V), VTK order
 *   n_threads        host threads to use; <= 0: min(16, hardware threads)
 *   cell_edge_level  host uint8 [C][12] out, local edge order of
 *                    hexfc_upload_mesh; may be NULL
 *   info             optional summary out
 * C = 0 is valid (nothing written, info zeroed).  Errors: EINVAL (C < 0,
 * NULL hex, V <= 0, a repeated corner, a face shared by more than two cells),
 * ERANGE (ids out of range, V >= 2^31, 12 C >= 2^32 - 1, more than 255
 * levels), ENOMEM.  Outputs are unspecified after an error. */
typedef struct hexfc_lod_info {
    int64_t sheets;          /* number of sheets                       */
    int64_t edges, faces;    /* distinct edges and faces of the mesh    */
    int64_t singular_edges;
    int64_t merges[3];       /* adjacent, hybrid, intersecting merges   */
    int32_t levels;          /* L, the coarsest level                   */
    int32_t components_left; /* components when merging stopped         */
} hexfc_lod_info;

hexfc_status hexfc_build_lod(const int32_t *hex, int64_t C, int64_t V, int32_t n_threads,
                             uint8_t *cell_edge_level, hexfc_lod_info *info);

const char *hexfc_last_error(const hexfc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HEXFC_H */
