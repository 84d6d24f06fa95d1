/*
 * hgs.h -- C ABI of the MI355X (gfx950) forward renderer for hierarchical
 * 3D Gaussian Splatting scenes.
 *
 * The operation (NavGSim, arXiv 2603.15186):
 *   - Sec. III-B: a scene is a tree of anisotropic 3D Gaussians; leaves hold
 *     the fine detail, internal nodes aggregate it; level-of-detail rendering
 *     selects Gaussians from different levels of the tree.
 *   - Eq. (1) and the Supplementary Material: each Gaussian's density is
 *     exp(-1/2 (x - mu)^T Sigma^-1 (x - mu)) with Sigma = R S S^T R^T.
 *   - Sec. III-A: a view is rendered from the camera intrinsics and
 *     extrinsics alone.
 * A render is: a level-of-detail cut through the hierarchy, EWA projection
 * of the cut's Gaussians to 2D conics with spherical-harmonic colour, tile
 * binning with a (tile, depth) radix sort, and front-to-back alpha
 * compositing per 16x16 tile (alpha capped at 0.99, skipped below 1/255,
 * stop before transmittance drops below 1e-4, 3-sigma support).
 *
 * Conventions: world z is up.  Camera frame: x right, y down, z forward.
 * Pixel (i, j) has its centre at (i + 0.5, j + 0.5).  Outputs are planar
 * FP32: rgb[3][H][W], depth[H][W] (sum of w_i z_i, not normalised),
 * alpha[H][W] (1 - final transmittance).
 *
 * Errors: every entry point returns an hgs_status; nothing throws or aborts
 * across the ABI.  hgs_last_error() describes the last failure of a context.
 * A context is not thread-safe: use one per host thread.
 */
#ifndef HGS_H
#define HGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hgs_status;
#define HGS_OK 0
#define HGS_E_INVALID (-1)        /* bad argument (null, NaN, out of range) */
#define HGS_E_STATE (-2)          /* call out of order (e.g. render before load) */
#define HGS_E_OOM (-3)            /* device or host allocation failed */
#define HGS_E_HIP (-4)            /* a HIP runtime call failed */
#define HGS_E_CAPACITY (-5)       /* a work buffer overflowed and regrowth is off */
#define HGS_E_BAD_HIERARCHY (-6)  /* hierarchy arrays are inconsistent */
#define HGS_E_UNSUPPORTED (-7)    /* valid request the library does not support */

/* LOD modes (hgs_set_lod). */
#define HGS_LOD_ALL_LEAVES 0      /* every leaf, no culling */
#define HGS_LOD_THRESHOLD 1       /* projected-size threshold cut */
#define HGS_LOD_LEARNED 2         /* MLP-refined cut, threshold rule as fallback */

/* Options (hgs_set_option). */
#define HGS_OPT_SYNC_CHECK 1      /* 1 (default): hgs_render waits for the GPU and
                                     checks capacities; 0: fully asynchronous,
                                     call hgs_check() after synchronising */
#define HGS_OPT_AUTO_REGROW 2     /* 1 (default): regrow and re-render on overflow */
#define HGS_OPT_COUNT_NALG 3      /* 1: count evaluated (pixel, Gaussian) pairs (not
                                     while HGS_OPT_KEEP_STATE is on) */
#define HGS_OPT_BATCH_DEPTH 4     /* Gaussians staged in LDS per batch: 64, 128 or 256 */
#define HGS_OPT_USE_GRAPH 5       /* 1: capture the render in a hipGraph on first use and
                                     replay it while cameras, LOD, options, scene and
                                     buffers are unchanged (not with stage timing) */
#define HGS_OPT_PERSISTENT 6      /* 1: composite with a persistent tile queue */
#define HGS_OPT_EXACT_TILES 7     /* 1 (default): bin only tiles the ellipse reaches */
#define HGS_OPT_INITIAL_CAPACITY 8 /* >0: restart work buffers at this many entries
                                      (exercises overflow and regrowth); 0: automatic */
#define HGS_OPT_STAGE_TIMING 9    /* 1: time the stages of every render with HIP events
                                     on its stream; setting it clears the sums */
#define HGS_OPT_SORT_DIGIT_BITS 10 /* widest radix digit, 6..11 (default 8); any
                                     value gives the same order */
#define HGS_OPT_PASS_VIEWS 11     /* >0: render at most this many views per pipeline
                                     pass; 0 (default): one pass, split by the
                                     renderer itself when a pass would outgrow
                                     the 2^28-entry index space.  Images do not
                                     depend on the passes. */
#define HGS_OPT_LANES 13          /* 2: split a batch into at least two pipeline passes
                                     that alternate between two work-buffer sets and
                                     two streams, so one pass's compositing overlaps
                                     the next pass's cut, projection and binning
                                     (twice the work-buffer memory); 1 (default): one
                                     set, one stream.  Images do not depend on it. */
#define HGS_OPT_LOD_BLEND 12      /* 1: level-of-detail transition blending (NavGSim
                                     Sec. III-B: transition regions between levels
                                     are smoothly interpolated).  A cut node g with
                                     parent p is drawn with mean, covariance and
                                     SH coefficients p + t (g - p), t = clamp((s_p
                                     - tau) / (s_p - s_g), 0, 1) (1 if s_g >= s_p),
                                     s = 2 max(fx, fy) r / |c - o| a node's
                                     projected bounding-sphere size in pixels; the
                                     first of p's children in the view's cut takes
                                     opacity o_p + t (o_g - o_p), the others t o_g.
                                     Just after p is refined (s_p = tau) exactly
                                     one copy of p is drawn, just before g is
                                     refined (s_g = tau) g itself: the image is
                                     continuous across every refine decision.
                                     Threshold and learned cuts of a hierarchy
                                     only; 0 (default): off. */
#define HGS_OPT_KEEP_STATE 14     /* 1: every render also keeps, per pixel, where its
                                     front-to-back walk stopped and its final
                                     transmittance (8 bytes per pixel of the batch,
                                     context-owned), so that hgs_render_backward
                                     need not replay the forward walk; 0 (default):
                                     not kept, the backward pass replays it.  Images
                                     and gradients do not depend on it. */

#define HGS_OPT_TILE_SHAPE 15       /* binning and compositing tile, (width << 16) | height:
                                       8x8, 16x8, 16x16 (default), 32x8 or 32x16 pixels.
                                       Each pixel's value does not depend on it (the
                                       3-sigma support is per pixel, the order is depth
                                       then cut order).  Kept pixel states and the
                                       backward pass need 16x16. */
#define HGS_OPT_PIXELS_PER_THREAD 16 /* pixels each compositing thread evaluates: 1
                                       (default), 2 or 4 horizontally adjacent pixels,
                                       at least 64 threads per tile.  Images do not
                                       depend on it. */

typedef struct hgs_ctx hgs_ctx;

/* Gaussians, host arrays borrowed for the duration of the call (copied).
 * means[n*3] metres; scales[n*3] metres, > 0; quats[n*4] (w,x,y,z), nonzero,
 * normalised by the renderer; opacity[n] in (0, 1]; sh[n*K*3] with
 * K = (sh_degree+1)^2, index (g*K + k)*3 + channel, k = l*l + l + m
 * (real harmonics with the Condon-Shortley phase); colour is
 * clamp(sum_k sh_k Y_k(d) + 0.5, 0, 1) with d the unit world-space direction
 * from the camera centre to the mean. */
typedef struct {
    int64_t n;
    int32_t sh_degree;            /* 0..3 */
    int32_t reserved;
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacity;
    const float* sh;
} hgs_gaussians;

/* Hierarchy over the same n Gaussians: node k is Gaussian k.  Level-major
 * ids, roots first, children of a node contiguous and one level down:
 * nodes [level_offset[L], level_offset[L+1]) form level L; parent[k] = -1
 * for roots; child_count[k] = 0 for leaves (first_child ignored then).
 * bound[k*4] = (cx, cy, cz, r): a sphere enclosing the 3-sigma spheres of
 * every leaf below k.  Host arrays, borrowed for the call (copied). */
typedef struct {
    int64_t n_nodes;
    const int32_t* parent;
    const int32_t* first_child;
    const int32_t* child_count;
    const float* bound;
    int32_t n_levels;
    int32_t reserved;
    const int64_t* level_offset;  /* n_levels + 1 entries */
} hgs_hierarchy;

/* Pinhole camera.  R maps world to camera coordinates (rows: right, down,
 * forward); position is the camera centre in world coordinates. */
typedef struct {
    int32_t width, height;        /* 1..8192 */
    float fx, fy, cx, cy;         /* pixels */
    float position[3];
    float R[9];                   /* row-major */
    float znear;                  /* metres, > 0 (0.2 by convention) */
    float bg[3];                  /* background colour */
} hgs_camera;

/* Caller-owned device buffers of one view, written on the render stream. */
typedef struct {
    float* rgb;                   /* [3][H][W] */
    float* depth;                 /* [H][W]; may be NULL */
    float* alpha;                 /* [H][W]; may be NULL */
} hgs_output;

/* Counters of the last render (all views), and GPU stage times summed over
 * the renders timed since HGS_OPT_STAGE_TIMING was last set:
 * ms_cut (LOD cut), ms_project (projection), ms_sort (depth sort, pair
 * emission, tile sort, tile ranges), ms_composite (the compositing kernel),
 * ms_total (whole render). */
typedef struct {
    int64_t cut_size;             /* Gaussians selected by the cut */
    int64_t visible;              /* of those, binned to at least one tile */
    int64_t pairs;                /* (tile, Gaussian) pairs sorted */
    int64_t n_alg;                /* evaluated pairs with q <= 9 (if counted) */
    int64_t tiles;                /* tiles composited */
    int64_t regrows;              /* buffer regrowths during the last render */
    int64_t timed_renders;        /* renders summed in the ms_* fields */
    int64_t graph_launches;       /* renders replayed from a captured graph */
    double ms_cut, ms_project, ms_sort, ms_composite, ms_total;
    int64_t passes;               /* pipeline passes of the last render */
    int64_t n_eval;               /* (pixel, list entry) slots the compositor walked,
                                     including q > 9 and stopped pixels (if counted) */
    int64_t timed_backwards;      /* backward passes summed in the ms_bwd_* fields */
    double ms_bwd_composite, ms_bwd_total;   /* compositing part and whole backward pass */
    int64_t visited;              /* (node, view) pairs the cut tested (threshold and learned cuts) */
} hgs_stats;

/* Create a context on HIP device `device`.  *out is set on success. */
hgs_status hgs_create(int32_t device, hgs_ctx** out);

/* Free the context and all device memory it owns.  NULL is ignored. */
void hgs_destroy(hgs_ctx* ctx);

/* Description of the context's last failure ("" if none); owned by the
 * context, valid until its next call.  Safe with ctx == NULL. */
const char* hgs_last_error(const hgs_ctx* ctx);

/* Check a scene on the host only (never touches a device).  Writes a
 * NUL-terminated reason into msg (if msg_len > 0) on failure.
 * Returns HGS_E_INVALID or HGS_E_BAD_HIERARCHY on failure. */
hgs_status hgs_validate_scene(const hgs_gaussians* g, const hgs_hierarchy* h,
                              char* msg, int64_t msg_len);

/* Validate and upload a scene (h == NULL: flat scene).  On failure the
 * previously loaded scene stays in place. */
hgs_status hgs_load_scene(hgs_ctx* ctx, const hgs_gaussians* g, const hgs_hierarchy* h);

/* Set the n >= 1 views of the next renders (copied). */
hgs_status hgs_set_cameras(hgs_ctx* ctx, int32_t n, const hgs_camera* cams);

/* Level-of-detail mode and threshold tau (pixels, > 0): an internal node is
 * refined while its projected size 2 f r / |c - o| (f = max(fx, fy)) exceeds
 * tau, evaluated exactly in FP64 as (2 f r)^2 > tau^2 |c - o|^2.  Flat scenes
 * ignore the mode.  LEARNED needs hgs_load_lod_mlp first (else HGS_E_STATE). */
hgs_status hgs_set_lod(hgs_ctx* ctx, int32_t mode, float tau_px);

/* Set an HGS_OPT_* option. */
hgs_status hgs_set_option(hgs_ctx* ctx, int32_t option, int64_t value);

/* Render every view set by hgs_set_cameras into outs[0..n) on `stream`
 * (a hipStream_t; NULL = default stream).  With HGS_OPT_SYNC_CHECK on, the
 * call returns after the GPU finished and buffers were checked; otherwise
 * it only enqueues. */
hgs_status hgs_render(hgs_ctx* ctx, void* stream, const hgs_output* outs);

/* After an asynchronous render and a stream synchronisation: HGS_OK, or
 * HGS_E_CAPACITY if a work buffer overflowed, or a depth fell outside the
 * range the batch's depth keys were sized for (a camera matrix that is not
 * a rotation can do that): outputs are then invalid, and capacities have
 * been grown, or full-width depth keys chosen, for the next render.  With
 * HGS_OPT_SYNC_CHECK and HGS_OPT_AUTO_REGROW on, hgs_render does this
 * itself and renders again. */
hgs_status hgs_check(hgs_ctx* ctx);

/* Ascending node ids of view `view`'s cut from the last render.  Writes
 * min(count, cap) ids to host_ids and the full count to *count.  When the
 * batch ran in several passes only views of the last pass are available
 * (HGS_E_STATE otherwise); the same holds for hgs_get_projected. */
hgs_status hgs_get_cut(hgs_ctx* ctx, int32_t view, int32_t* host_ids, int64_t cap,
                       int64_t* count);

/* Stage-wise intermediates of view `view` from the last render, in cut
 * order: per Gaussian 12 floats (u, v, conic A, B, C, r, g, b, depth,
 * opacity, tile count, valid).  Conic recomputed from the stored factors. */
hgs_status hgs_get_projected(hgs_ctx* ctx, int32_t view, float* host_out, int64_t cap,
                             int64_t* count);

/* Counters of the last render (synchronises with it). */
hgs_status hgs_get_stats(hgs_ctx* ctx, hgs_stats* out);

/* Launch plan chosen by hgs_autotune. */
typedef struct {
    int32_t batch_depth;          /* HGS_OPT_BATCH_DEPTH */
    int32_t persistent;           /* HGS_OPT_PERSISTENT */
    int32_t sort_digit_bits;      /* HGS_OPT_SORT_DIGIT_BITS */
    int32_t from_cache;           /* 1: read from the plan cache, not timed */
    double ms;                    /* render time of the plan (mean over reps) */
    double ms_default;            /* render time of the default plan */
    int32_t lanes;                /* HGS_OPT_LANES in force (not searched) */
    int32_t reserved;             /* 0 */
    int32_t tile_w, tile_h;       /* HGS_OPT_TILE_SHAPE */
    int32_t pixels_per_thread;    /* HGS_OPT_PIXELS_PER_THREAD */
    int32_t reserved2;            /* 0 */
} hgs_plan;

/* Time the launch choices that do not change the image (tile shape 8x8,
 * 16x8, 16x16, 32x8 or 32x16 with 1, 2 or 4 pixels per compositing thread;
 * compositor batch depth 64/128/256, at most the tile's thread count;
 * persistent or one-workgroup-per-tile compositing for 16x16 tiles; radix
 * digit width 6..11) on the current scene, views, LOD and lanes (kept as
 * set; with kept pixel states, 16x16 tiles only), rendering every view reps
 * >= 1 times per candidate into internal buffers on `stream`, and keep the
 * fastest as the context's options (*out describes it; may be NULL).
 * Coordinate search: compositor choices first, then the digit width.  cache_path (NULL: none) names a text file of earlier plans keyed
 * by scene size, view sizes and LOD; a matching line is applied without
 * timing, a new plan is appended (the key includes the lanes setting).
 * Synchronous; leaves stage timing off. */
hgs_status hgs_autotune(hgs_ctx* ctx, void* stream, const char* cache_path, int32_t reps, hgs_plan* out);

/* Sort n (key, value) pairs on the device by the low `key_bits` bits of the
 * key, stably (LSD radix, digits of up to HGS_OPT_SORT_DIGIT_BITS bits).  keys/vals are device pointers and
 * are sorted in place; the context's scratch memory is used.  For testing
 * the sort on its own. */
hgs_status hgs_sort_pairs(hgs_ctx* ctx, void* stream, uint32_t* keys, uint32_t* vals,
                          int64_t n, int32_t key_bits);

/* Most pairs hgs_sort_pairs_noalloc sorts. */
#define HGS_SORT_NOALLOC_MAX 4194304

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the sort
 * of hgs_sort_pairs -- the same order, stable, by the low key_bits bits,
 * digits of up to HGS_OPT_SORT_DIGIT_BITS bits -- without allocating
 * anything.  keys/vals are n caller-owned device uint32 arrays, sorted in
 * place; 0 <= n <= HGS_SORT_NOALLOC_MAX, else HGS_E_INVALID (nothing is
 * launched).  Its scratch memory (about 36 MB) is one static device array
 * per GPU, shared by every context and call on that GPU and held until the
 * process ends: calls that overlap in time on one GPU race.  Asynchronous
 * on `stream` (no synchronisation, so it may be captured). */
hgs_status hgs_sort_pairs_noalloc(hgs_ctx* ctx, void* stream, uint32_t* keys, uint32_t* vals,
                                  int64_t n, int32_t key_bits);

/* ---------------------------------------------------------------------- */
/* Learned level-of-detail refinement.  The paper's LOD rendering picks     */
/* Gaussians from different tree levels (NavGSim Sec. III-B); the learned  */
/* rule below is the project's: a candidate is a node the threshold rule   */
/* refines whose projected size is at most s_hi pixels; a small network    */
/* (8 features, layers 8-32-32-1, ReLU, BF16 weights, FP32 accumulation)   */
/* decides whether such a node is refined (p >= p_star) or kept.  Outside  */
/* the band the threshold rule applies unchanged (the fallback).           */
/* Features of (node, view), before standardisation: log projected size,  */
/* log camera depth, opacity, child count, variance of the children's DC   */
/* colour, |cos| of the view ray and the node's thinnest axis, level, log  */
/* projected size of the parent.  Parameter layout (1377 values):          */
/* W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3.                      */
/* ---------------------------------------------------------------------- */

/* Per view, a node that the cut never refines (-1: none); used to render a
 * view with one subtree collapsed to its root.  n = number of views. */
hgs_status hgs_set_keep_nodes(hgs_ctx* ctx, int32_t n, const int32_t* nodes);

/* Run the threshold cut of the current views and collect the candidates
 * (refined, projected size <= s_hi) in (level, view, id) order.  Device
 * outputs, cap entries each: entries[2i] = node, entries[2i+1] = view;
 * features[8i..8i+8) raw features; rects[4i..4i+4) = x0, y0, x1, y1 pixel
 * bounds of the node's bounding-sphere projection, clipped to the image.
 * *count = number of candidates; HGS_E_CAPACITY (with *count set) if cap
 * is too small.  Synchronises with `stream`. */
hgs_status hgs_lod_candidates(hgs_ctx* ctx, void* stream, float s_hi_px, uint32_t* entries, float* features,
                              int32_t* rects, int64_t cap, int64_t* count);

/* Install the network used by HGS_LOD_LEARNED (host arrays, copied):
 * bf16_params[1377], feat_mean[8], feat_std[8] (> 0). */
hgs_status hgs_load_lod_mlp(hgs_ctx* ctx, const uint16_t* bf16_params, const float* feat_mean,
                            const float* feat_std, float p_star, float s_hi_px);

/* Logits of n raw feature rows (device features[n*8], device bf16 weights
 * w[1377], host feat_mean/feat_std[8]) into device logits[n]. */
hgs_status hgs_mlp_forward(hgs_ctx* ctx, void* stream, const float* features, int64_t n, const uint16_t* w,
                           const float* feat_mean, const float* feat_std, float* logits);

/* One training step on the batch (device features[n*8], labels[n] in
 * {0,1}): forward with the BF16 weights w, mean binary cross-entropy,
 * backward, and (if lr > 0) an Adam step (beta 0.9/0.999, eps 1e-8, step
 * counts from 1) on the FP32 master weights, after which w = BF16 of the
 * masters.  grad_out[1377] and loss_out[1] (device, optional) receive the
 * gradient and the loss.  Deterministic. */
hgs_status hgs_mlp_train_step(hgs_ctx* ctx, void* stream, const float* features, const float* labels, int64_t n,
                              const float* feat_mean, const float* feat_std, float* master, uint16_t* w,
                              float* adam_m, float* adam_v, int32_t step, float lr, float* grad_out,
                              float* loss_out);

/* The training step's two halves as separate calls (the same kernels, so
 * hgs_mlp_backward followed by hgs_mlp_adam equals hgs_mlp_train_step bit
 * for bit).  hgs_mlp_backward: forward with the BF16 weights w, mean binary
 * cross-entropy and its gradient into grad_out[1377] (device, required),
 * the loss into loss_out[1] (device, optional); weights untouched.
 * hgs_mlp_adam: one Adam step (beta 0.9/0.999, eps 1e-8, step >= 1, lr > 0)
 * of the FP32 master[1377] and moments adam_m, adam_v[1377] with the
 * gradient grad[1377] (all device), then w = BF16 of the masters.  Both
 * deterministic and asynchronous on `stream`. */
hgs_status hgs_mlp_backward(hgs_ctx* ctx, void* stream, const float* features, const float* labels, int64_t n,
                            const float* feat_mean, const float* feat_std, const uint16_t* w, float* grad_out,
                            float* loss_out);
hgs_status hgs_mlp_adam(hgs_ctx* ctx, void* stream, const float* grad, float* master, uint16_t* w, float* adam_m,
                        float* adam_v, int32_t step, float lr);

/* w[1377] = BF16 (nearest, ties to even) of the FP32 master[1377] (device). */
hgs_status hgs_mlp_bf16_from_master(hgs_ctx* ctx, void* stream, const float* master, uint16_t* w);

/* Column mean and standard deviation of device features[n*8] into device
 * mean_std[16] (8 means then 8 deviations, at least 1e-6). */
hgs_status hgs_feature_stats(hgs_ctx* ctx, void* stream, const float* features, int64_t n, float* mean_std);

/* Device-to-device streaming copy of `bytes` (a multiple of 16; both
 * pointers 16-byte aligned, else HGS_E_INVALID), asynchronous on `stream`:
 * the probe of attainable HBM bandwidth (read + write) that the roofline
 * fractions are quoted against beside the 8 TB/s peak. */
hgs_status hgs_stream_copy(hgs_ctx* ctx, void* stream, const void* src, void* dst, int64_t bytes);

/* dst[3][H][W] = 2x2 box average of src[3][2H][2W] (device, planar). */
hgs_status hgs_downsample2x(hgs_ctx* ctx, void* stream, const float* src, int32_t width, int32_t height,
                            float* dst);

/* A w x h planar RGB image compared with the window at (x0, y0) of a
 * ref_w x ref_h planar RGB reference (device pointers). */
typedef struct {
    const float* img;
    const float* ref;
    int32_t w, h, ref_w, ref_h, x0, y0;
} hgs_region;

/* out[i] (device) = mean squared error over the 3 channels of region i.
 * The descriptors are host memory (copied). */
hgs_status hgs_region_mse(hgs_ctx* ctx, void* stream, int32_t n, const hgs_region* regions, float* out);

/* Expand-vs-keep labels of learned-cut candidates (training data of the
 * learned rule; the tree and its level selection are NavGSim Sec. III-B, the
 * rule is the project's).  For candidate i, regions[2i] is its footprint
 * window rendered with the threshold cut (the node refined) and
 * regions[2i + 1] the same window rendered with the node's subtree
 * collapsed to it, both compared with the same crop of a reference image;
 * with MSE_r and MSE_k their mean squared errors (FP32, floored at 1e-10),
 * drop_db[i] = 10 log10(MSE_k / MSE_r), the PSNR the window loses when the
 * node is kept, and labels[i] = 1 when drop_db[i] > label_db, else 0.
 * labels and drop_db (may be NULL) are device float arrays of n entries;
 * the 2n descriptors are host memory (copied).  Asynchronous on `stream`
 * after waiting for its earlier work (the descriptor buffer is reused). */
hgs_status hgs_lod_labels(hgs_ctx* ctx, void* stream, int32_t n, const hgs_region* regions, float label_db,
                          float* labels, float* drop_db);

/* ---------------------------------------------------------------------- */
/* Ground truth of synthetic scenes (evaluation, not the render path): the */
/* exact surfaces the Gaussians approximate, ray cast with supersampling.  */
/* They stand in for the posed photographs a reconstruction is judged      */
/* against (NavGSim Table 2 reports PSNR against real images).             */
/* ---------------------------------------------------------------------- */

/* kind 0: rectangle o + u a + v b, u, v in [0, 1]; kind 1: cylinder side,
 * axis through (o[0], o[1]), z from o[2] to o[2] + h, radius r; kind 2: disk
 * centred at o with radius r, normal +z.  Colour = clamp(col * f(p), 0, 1)
 * with pattern 0: f = 1; 1: 0.85 + 0.15 sign(sin(2 pi x / 0.4)); 2: 0.9 +
 * 0.1 ((floor(x / 0.6) + floor(y / 0.6)) mod 2); 3: 0.55 if (z mod 3) < 0.12
 * else 0.92 + 0.08 sin(2 pi (x + y) / 1.3). */
typedef struct {
    int32_t kind;
    int32_t pattern;
    float o[3], a[3], b[3];
    float col[3];
    float r, h;
} hgs_surface;

/* Copy n surfaces (host) into the context. */
hgs_status hgs_set_surfaces(hgs_ctx* ctx, int32_t n, const hgs_surface* surfaces);

/* Ray cast the surfaces seen by camera view `view` (of hgs_set_cameras)
 * with ss x ss samples per pixel (1..4) into device rgb[3][H][W]; rays that
 * hit nothing take the camera's background. */
hgs_status hgs_render_surfaces(hgs_ctx* ctx, void* stream, int32_t view, int32_t ss, float* rgb);

/* ---------------------------------------------------------------------- */
/* GS-slice collision map (NavGSim Sec. III-C and the Supplementary        */
/* derivation of Gaussian slicing).                                          */

typedef struct {
    double x0, y0;                /* world x, y (metres) of the grid's lower corner */
    double cell;                  /* cell edge (metres), > 0 */
    int32_t nx, ny;               /* cells per row, rows: 1..16384 each */
    int32_t n_planes;             /* 1..256 */
    float rho_min;                /* solid threshold, in (0, 1) */
    const float* heights;         /* host array of n_planes plane heights (metres) */
} hgs_slice_grid;

/* Occupancy of the scene's leaf Gaussians (every Gaussian of a flat scene)
 * on horizontal planes.  A Gaussian cut by the plane z is the 2D Gaussian
 * o exp(-lambda (z - mu_z)^2 / 2) exp(-q / 2), q = (x - mu(z))^T C_xy
 * (x - mu(z)), with C = Sigma^-1, C_xy its xy block, (alpha, beta) solving
 * C_xy (alpha, beta)^T = (c_xz, c_yz)^T, lambda = c_zz - (alpha, beta) .
 * (c_xz, c_yz) and mu(z) = (mu_x, mu_y) - (z - mu_z)(alpha, beta); it is
 * solid where that value is >= rho_min.  Cell (i, j), the closed square
 * [x0 + i cell, x0 + (i+1) cell] x [y0 + j cell, y0 + (j+1) cell], is 1 in
 * plane k of occ when some solid ellipse on plane k meets it, else 0.  occ
 * (device, [n_planes][ny][nx] bytes) and map (device, [ny][nx] bytes: the
 * union over the planes) are caller-owned; either may be NULL, not both.
 * Asynchronous on `stream`.  HGS_E_INVALID on bad sizes, HGS_E_STATE
 * without a scene. */
hgs_status hgs_slice_occupancy(hgs_ctx* ctx, void* stream, const hgs_slice_grid* grid, uint8_t* occ,
                               uint8_t* map);

/* Disc robots against a 2D occupancy map (e.g. the union map of
 * hgs_slice_occupancy), for collision checks of many robots at once:
 * out[q] = 1 when the closed disc of `radius` metres around
 * (xy[2q], xy[2q+1]) meets the closed square [x0 + i cell, x0 + (i+1) cell] x
 * [y0 + j cell, y0 + (j+1) cell] of some occupied cell (map[j * nx + i] != 0),
 * else 0; cells outside the grid are free.  map (device, ny * nx bytes), xy
 * (device, n pairs of doubles) and out (device, n bytes) are caller-owned.
 * Asynchronous on `stream`.  HGS_E_INVALID on bad sizes or radius. */
hgs_status hgs_disc_collision(hgs_ctx* ctx, void* stream, const uint8_t* map, double x0, double y0, double cell,
                              int32_t nx, int32_t ny, int64_t n, const double* xy, double radius, uint8_t* out);

/* Backward pass of the last render (the gradients scene reconstruction
 * optimises with, NavGSim Sec. III-B).  grads[v] holds, for view v, device
 * planar dL/dRGB [3][height][width], dL/dD [height][width] (D = the raw
 * depth output) and dL/dalpha [height][width]; any may be NULL (zero).  The
 * gradients of L with respect to the rendered Gaussians' parameters are
 * ADDED to out's device arrays: means [n][3], scales [n][3], quats [n][4]
 * (w, x, y, z, as given to hgs_load_scene, before normalisation), opacity
 * [n], sh [n][K][3] (K = (degree + 1)^2); n = every node of the scene (only
 * rendered ones receive gradients).  Discrete decisions (q <= 9, alpha >=
 * 1/255, the early stop) carry no gradient, nor does an opacity-weighted
 * alpha capped at 0.99 or a colour channel clamped to [0, 1].  Run on the
 * render's stream after it; the render must have been one pass (no
 * HGS_OPT_PASS_VIEWS split) without HGS_OPT_LOD_BLEND (HGS_E_STATE,
 * HGS_E_UNSUPPORTED).  A render made with HGS_OPT_KEEP_STATE hands over each
 * pixel's stop position and final transmittance; otherwise the backward pass
 * replays the forward walk to find them.  Asynchronous on `stream`; the
 * summation order of the atomic adds is not fixed, so results vary in the
 * last bits. */
typedef struct {
    const float* rgb;
    const float* depth;
    const float* alpha;
} hgs_image_grad;

typedef struct {
    float* means;
    float* scales;
    float* quats;
    float* opacity;
    float* sh;
} hgs_scene_grad;

hgs_status hgs_render_backward(hgs_ctx* ctx, void* stream, const hgs_image_grad* grads, const hgs_scene_grad* out);

/* Shortest-path planning on the navigable areas (NavGSim Sec. III-C: the
 * slice map serves collision checks and path planning; Sec. IV: expert
 * trajectories from a shortest-path planner between random starts and
 * goals).  Grids are row-major [ny][nx]; a cell index is j * nx + i. */

/* Navigable map for a disc robot: nav[j * nx + i] = 1 when the closed disc
 * of `radius` metres around the cell's centre (x0 + (i + 1/2) cell,
 * y0 + (j + 1/2) cell) meets no occupied cell of map (the test of
 * hgs_disc_collision), else 0.  map and nav: device, ny * nx bytes,
 * caller-owned.  Asynchronous on `stream`.  HGS_E_INVALID on bad sizes. */
hgs_status hgs_navigable_map(hgs_ctx* ctx, void* stream, const uint8_t* map, double x0, double y0, double cell,
                             int32_t nx, int32_t ny, double radius, uint8_t* nav);

/* Distance fields to n_goals goal cells over the navigable cells (nav != 0)
 * of an 8-connected grid: orthogonal moves cost 1, diagonal moves sqrt 2
 * and need both side cells navigable.  dist[g * ny * nx + c] (device,
 * caller-owned, n_goals * ny * nx uint64) = a | b << 32 with (a, b) the
 * orthogonal and diagonal moves of a shortest path from cell c to goal g
 * (unique: the cost a + b sqrt 2 determines it), or UINT64_MAX when c is
 * unreachable; a goal outside the grid or on a blocked cell reaches
 * nothing.  goals: host array of n_goals cell indices.  Blocking: returns
 * after the fields are complete; *rounds (may be NULL) receives the number
 * of relaxation rounds.  Grids up to 2^24 cells, 1..16384 per side;
 * n_goals 1..65535.  HGS_E_INVALID on bad sizes. */
hgs_status hgs_distance_fields(hgs_ctx* ctx, void* stream, const uint8_t* nav, int32_t nx, int32_t ny,
                               int32_t n_goals, const int32_t* goals, uint64_t* dist, int64_t* rounds);

/* Trajectories down distance fields: query q starts at cell starts[q] and
 * follows field slots[q]; at each step it moves to the first neighbour, in
 * the order E (+x), W, S (+y), N, SE, SW, NE, NW, that is a legal move and
 * whose pair plus the move's unit equals the current pair, until the goal.
 * lengths[q] = cells on the path, start and goal included (0: start off the
 * grid, slot out of range or start unreachable; -1: dist is not a distance
 * field); the first min(length, cap) cells go to paths[q * cap ...].
 * nav and dist as for hgs_distance_fields; starts, slots, paths, lengths:
 * device, caller-owned.  The library keeps a table of each cell's step per
 * field (n_goals * ny * nx bytes, grown on demand).  Asynchronous on
 * `stream`.  HGS_E_INVALID on bad sizes, HGS_E_OOM if the table cannot
 * grow. */
hgs_status hgs_trace_paths(hgs_ctx* ctx, void* stream, const uint8_t* nav, int32_t nx, int32_t ny,
                           const uint64_t* dist, int32_t n_goals, int64_t n, const int32_t* starts,
                           const int32_t* slots, int32_t cap, int32_t* paths, int32_t* lengths);

#ifdef __cplusplus
}
#endif

#endif /* HGS_H */
