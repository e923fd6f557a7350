/*
 * gs_api.h -- C ABI of libgs, an MI355X (gfx950) differentiable Gaussian-splatting
 * tile rasterizer: the forward and backward hot path of the training step of
 * Trick-GS (arXiv 2501.14534).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer owned by the caller (typically a
 *    PyTorch tensor).  Host structs (gs_gaussians, gs_camera, gs_opts, ...)
 *    are read during the call only.
 *  - The library never allocates, frees or synchronises.  A call validates
 *    its arguments on the host, enqueues kernels on `stream` and returns; no
 *    call reads device memory on the host, so every call may be captured in a
 *    HIP graph.  Scratch memory comes in through `ws` (size from
 *    gs_workspace_size) and is clobbered by the call; the one exception,
 *    gs_mask_loss_noalloc, uses a static device array of the library
 *    instead.  The workspaces of
 *    gs_bin_sort, gs_render_fwd, gs_render_bwd, gs_blend_bwd, gs_project_bwd
 *    and gs_count_hits must be 256-byte aligned (hipMalloc and PyTorch
 *    allocations are); a misaligned one is GS_E_INVALID.
 *  - Layouts are structure-of-arrays with the Gaussian index last: an array
 *    documented [3][n] holds component k of Gaussian i at [k*n + i].
 *  - A "record" is one (view, Gaussian) pair, r = view * n + gaussian.
 *  - V views of one call are batched: their tiles form one key space (global
 *    tile id = view's tile offset + ty * TX + tx, views in call order) and
 *    their pixels are concatenated in call order.
 *  - Return value: GS_OK, or a negative GS_E_* code.  On GS_E_INVALID nothing
 *    was enqueued.  Capacity overflow of the binning is a DEVICE-side status
 *    (see gs_binning); the call that overflows cannot know it.
 */
#ifndef GS_API_H
#define GS_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;
typedef struct ihipStream_t* gs_stream_t; /* a hipStream_t; NULL = the null stream */

enum {
  GS_OK = 0,
  GS_E_INVALID = -1,     /* bad argument: null pointer, size, degree, tile shape ... */
  GS_E_CAPACITY = -2,    /* reported through gs_binning.status, never returned by a call */
  GS_E_HIP = -3,         /* a kernel launch failed; hipGetLastError() is left set */
  GS_E_UNSUPPORTED = -4, /* the current device is not gfx950 */
  GS_E_TOO_LARGE = -5    /* beyond the static scratch of an allocation-free entry point */
};

#define GS_MAX_VIEWS 16       /* views per call */
#define GS_SPLAT_FLOATS 12    /* floats per projected record */
#define GS_GRAD_FLOATS 9      /* floats per record gradient */
#define GS_MAX_BATCH 1024     /* largest per-tile staging batch (the backward stages at most 512 / waves) */

/* Gaussian parameters, raw (before activations).  Sec. 3.1: mean, scale,
 * rotation quaternion, opacity, diffuse colour and SH coefficients; Sec. 3.2.5:
 * the diffuse colour (band 0) is passed separately from SH bands 1..3;
 * Sec. 3.2.1 (Eq. 3): one volume-mask logit per Gaussian, applied to opacity
 * and scales; Sec. 3.2.3 (Eq. 5): one mask logit per SH band 1..3.           */
typedef struct gs_gaussians {
  const float* means;           /* [3][n] world position                                 */
  const float* log_scales;      /* [3][n] log of the three axis scales                   */
  const float* quats;           /* [4][n] rotation (w, x, y, z); normalised internally   */
  const float* opacity_logits;  /* [n]   opacity = sigmoid(logit)                        */
  const float* sh_dc;           /* [3][n] diffuse colour c_dc (RGB)                      */
  const float* sh_rest;         /* [(K-1)][3][n], K = (deg+1)^2, coefficient k >= 1 of
                                   channel c at [((k-1)*3 + c)*n + i]; NULL iff deg == 0 */
  const float* mask_logits;     /* [n] or NULL (no volume mask)                          */
  const float* sh_mask_logits;  /* [3][n] bands 1..3, or NULL (no band masks)            */
  int64_t n;                    /* number of Gaussians, >= 0                             */
  int32_t sh_degree;            /* 0..3                                                  */
  float mask_eps;               /* hard mask M = [sigmoid(m) > mask_eps]                 */
  float sh_mask_eps;            /* hard band mask M^l = [sigmoid(m_l) > sh_mask_eps]     */
} gs_gaussians;

/* Pinhole camera: x_cam = R x_world + t, camera axes x right, y down, z
 * forward; pixel (i, j) has its centre at (i + 0.5, j + 0.5).              */
typedef struct gs_camera {
  float R[9]; /* row-major world -> camera rotation */
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height; /* > 0 */
} gs_camera;

/* Per-call rasterizer options. */
typedef struct gs_opts {
  float near_plane;  /* cull when camera z <= near_plane (e.g. 0.2)                        */
  float tan_clamp;   /* lateral ratio guard of the EWA Jacobian, in half fields of view (1.3) */
  float lowpass;     /* s of Sigma' + sI (Sec. 3.2.4; 0.3), >= 0; see lowpass_progressive  */
  float bg[3];       /* background colour added with the final transmittance              */
  int32_t tile_w;    /* tile width in pixels, power of two                                 */
  int32_t tile_h;    /* tile height in pixels, power of two; tile_w*tile_h in [64, 1024]   */
  int32_t batch_depth;       /* splats staged per batch, 1..GS_MAX_BATCH: per workgroup in the
                                backward (at most 512 / waves), per wave in the forward walks
                                (at most 64); results do not depend on it                   */
  int32_t pixels_per_thread; /* 1, 2 or 4; tile_w*tile_h/ppt a multiple of 64, <= 256      */
  int32_t subtile_cull;      /* 1: each wave walks only the splats whose alpha >= 1/255
                                footprint can reach its pixels (same result, less work); 0: off */
  int32_t bwd_chunk;         /* entries of a tile's list per backward work item: a power of
                                two in [16, 2^20], or 0 for one item per tile.  The forward
                                records each pixel's state at every multiple of bwd_chunk so
                                the backward can walk the chunks of one long list in parallel. */
  int32_t fwd_chunk;         /* entries of a tile's list per forward work item: a power of two
                                in [64, 2^24], or 0 for one item per tile.  Longer lists are
                                walked in chunks in parallel: each chunk starts from the product
                                of the earlier chunks' (1 - alpha) factors, computed by a
                                product pass first; the image equals the single walk's up to
                                rounding.  Needs more workspace (gs_workspace_size). */
  int32_t lowpass_progressive; /* 1: progressive scaling (Sec. 3.2.4): view v uses
                                  s_v = max(lowpass, W_v H_v / (9 pi n)) for the n Gaussians of
                                  the call (computed in double, rounded to float); 0: s = lowpass */
} gs_opts;

/* Projected (view, Gaussian) records, written by gs_project.
 * splats: [V*n][12] floats, 16-byte aligned:
 *   [0] u  [1] v            screen position of the mean (pixels)
 *   [2] A  [3] B  [4] C     conic: inverse of Sigma' + sI, exponent -(A dx^2 + 2B dx dy + C dy^2)/2
 *   [5] o'                  masked opacity
 *   [6] radius              integral, 3 standard deviations of the major axis
 *   [7] depth               camera-space z
 *   [8..10] rgb             view-dependent colour
 *   [11] valid              1 when projected, 0 when culled (then [0..10] are 0)
 * tiles_touched: [V*n] number of tiles the record is binned to (0 = none). */
typedef struct gs_projected {
  float* splats;
  uint32_t* tiles_touched;
} gs_projected;

/* Sorted (tile, depth) lists.  keys/ids/pair_index hold `capacity` entries;
 * after a successful gs_bin_sort the first K = *count are sorted by key, then
 * by id:
 *   key = (global tile << 32) | IEEE bits of the record's depth (keys may be
 *         NULL: the compositing calls do not read them)
 *   id  = record index (view * n + gaussian)
 *   pair_index = position of the pair in emission order, where each record's
 *                pairs are contiguous, records in index order, and a record's
 *                tiles in row-major order of its tile rectangle
 * offsets: [V*n] first emission position of each record's pairs (its
 *          tiles_touched consecutive positions follow).
 * ranges: [total_tiles][2] = [start, end) into keys/ids, [0,0) when empty.
 * order: [total_tiles] or NULL.  When given, gs_bin_sort writes a
 *        permutation of the global tile ids, longest list first (lengths
 *        grouped by powers of two, order within a group unspecified), and
 *        the compositing calls process tiles in that order, so the deepest
 *        tiles of every view start first.  The order affects timing only:
 *        every tile's results are computed independently.  NULL: tile-id order.
 * count, status: device words written by gs_bin_sort.  status = 0 on success,
 * 1 when K > capacity: then no list is written, every range is empty and
 * *count still holds K, so the caller can grow the buffers and run again. */
typedef struct gs_binning {
  uint64_t* keys;
  uint32_t* ids;
  uint32_t* pair_index;
  uint32_t* offsets;
  uint32_t* ranges;
  uint32_t* order;   /* optional */
  uint64_t capacity; /* < 2^32 */
  uint32_t* count;   /* device, 1 word */
  int32_t* status;   /* device, 1 word */
} gs_binning;

/* Gradients, arrays shaped like the parameters.  Any member may be NULL to
 * skip it.  assign = 0: ACCUMULATED (+=) into the arrays (zero them first for
 * a plain gradient); assign = 1: WRITTEN, every Gaussian's entry (zeros where
 * it gets no gradient), so no zeroing is needed.  Either way a member the call
 * does not compute is left as it is: sh_rest and sh_mask_logits at SH degree
 * 0, mask_logits when the Gaussians have no volume-mask logits.  mean2d, if
 * given, is [V][2][n], receives dL/d(u, v) (densification statistics) and is
 * always accumulated; gs_mask_loss always accumulates.                     */
typedef struct gs_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh_dc;
  float* sh_rest;
  float* mask_logits;
  float* sh_mask_logits;
  float* mean2d;
  int32_t assign;
} gs_grads;

/* Number of tiles and pixels of V views under `opts` (host only): the tile
 * grid of the binning rule (each view is cut into ceil(W / tile_w) x
 * ceil(H / tile_h) tiles, views in call order), the sizes a caller needs for
 * the ranges, order, image, T_final and last_contrib arrays.  GS_E_INVALID on
 * a bad camera or option. */
int gs_view_sizes(const gs_camera* cams, int32_t V, const gs_opts* opts, int64_t* total_tiles,
                  int64_t* total_pixels);

/* Bytes of the one workspace buffer that gs_bin_sort, gs_render_fwd and
 * gs_render_bwd (or gs_blend_bwd + gs_project_bwd) share for n Gaussians, V
 * views and a list capacity (host only; 0 on invalid input): the scratch of
 * the depth sort and the tile sort that order each tile's list as Eq. 2's
 * front-to-back composite needs, and the per-chunk pixel states and per-pair
 * gradients of the backward of Eq. 2.  gs_bin_sort
 * uses it as scratch; gs_render_fwd writes the per-chunk pixel states there,
 * and the backward of the same step reads them, so the buffer must not be
 * reused for anything else between the forward and the backward. */
size_t gs_workspace_size(int64_t n, int32_t V, const gs_camera* cams, const gs_opts* opts, uint64_t capacity);

/* Projection of every Gaussian into every view (Sec. 3.1 Eq. 1, Sec. 3.2.4,
 * Eq. 3, Eq. 5, Sec. 3.2.5): activations, hard masks, world->camera, near
 * cull, 3D covariance from scale and rotation, EWA projection with the
 * low-pass s, conic, radius, SH colour (bands 1..deg scaled by their hard
 * masks, clamped at 0) and the number of tiles each record touches.
 * Reads each Gaussian once for all V views.  Writes out->splats and
 * out->tiles_touched ([V*n] records). */
int gs_project(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
               gs_projected* out, gs_stream_t stream);

/* Tile binning and ordering of the records of a gs_project call, which gives
 * every tile the depth-ordered list that the front-to-back composite of Eq. 2
 * walks (Sec. 3.1).  Binning rule: a record touches the tiles of the rectangle
 * [floor((u - r) / tile_w), floor((u + r) / tile_w)] x [same for v and tile_h],
 * clipped to the view, with u - r and u + r single-precision operations; this
 * rectangle holds every pixel centre inside the record's square (the square
 * test of gs_render_fwd), so the lists do not change the image.  Order: by
 * (global tile, depth) with ties in depth broken by record id, so the order is
 * unique.  Implementation: device-wide scans of tiles_touched, a stable LSD
 * radix sort of the visible records by their depth bits, emission of one pair
 * per touched tile in that order, a stable LSD radix sort of the pairs by tile
 * id (together: the order of keys then ids described above), per-tile ranges
 * and, if order is given, the heaviest-first tile schedule.  Returns
 * GS_E_INVALID (nothing enqueued) on null pointers, a misaligned or short
 * workspace, V * n >= 2^32 or capacity >= 2^32; capacity overflow is reported
 * through *status.  Needs ws_bytes >= gs_workspace_size(...). */
int gs_bin_sort(const gs_projected* proj, const gs_camera* cams, int32_t V, int64_t n, const gs_opts* opts,
                gs_binning* out, void* ws, size_t ws_bytes, gs_stream_t stream);

/* Front-to-back compositing of Eq. 2 per pixel over its tile's list:
 * square test |centre - (u,v)| <= radius per axis, alpha = min(0.99, o' exp(-q/2)),
 * skip alpha < 1/255, stop before a Gaussian that would bring the
 * transmittance under 1e-4, output C + T bg.
 * image: [sum_v 3*H_v*W_v] planar per view ([3][H][W]), views concatenated.
 * T_final, last_contrib: [sum_v H_v*W_v]; last_contrib counts the list
 * entries of the pixel's tile up to and including the last composited one.
 * ws (ws_bytes >= gs_workspace_size(...)): receives, for every multiple of
 * opts->bwd_chunk that the walk of a tile passes, each pixel's transmittance
 * there and the colour composited after it; the backward reads them. */
int gs_render_fwd(const gs_projected* proj, const gs_binning* bins, const gs_camera* cams, int32_t V,
                  int64_t n, const gs_opts* opts, float* image, float* T_final, int32_t* last_contrib,
                  void* ws, size_t ws_bytes, gs_stream_t stream);

/* Backward of gs_render_fwd and gs_project for dL/dimage (layout of image):
 * each tile's list is walked back to front from its largest last_contrib, in
 * chunks of opts->bwd_chunk entries that run in parallel, each starting from
 * the state the forward recorded at its end; transmittance is recovered by
 * division within a chunk; per (tile, splat) the 9 partials are
 * summed over the workgroup's pixels in a fixed order and stored once, at the
 * pair's emission position; then, per Gaussian, its pairs are summed in
 * emission order and the chain rule runs to the raw parameters including the
 * straight-through mask gradients (Eq. 3, Eq. 5).  No atomics: the result is
 * bitwise reproducible, and a batched call equals the sum of per-view calls
 * made in view order.  Gradients go to `grads` (added or written, see gs_grads).
 * Needs ws_bytes >= gs_workspace_size(...). */
int gs_render_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                  const gs_projected* proj, const gs_binning* bins, const float* T_final,
                  const int32_t* last_contrib, const float* dL_dimage, gs_grads* grads, void* ws,
                  size_t ws_bytes, gs_stream_t stream);

/* The two halves of gs_render_bwd, for callers that schedule or time them
 * separately.  gs_blend_bwd: the per-tile back-to-front walk only; WRITES
 * the per-pair splat gradients (u, v, A, B, C, o', r, g, b) of the pairs the
 * walk reaches to grad_pair ([capacity][9], indexed by pair_index; 16-byte
 * aligned, else GS_E_INVALID) and marks them in ws; the rows of the pairs
 * behind every pixel's last contributor are left as they are and count as
 * zero (no zeroing needed).
 * gs_project_bwd: per Gaussian, the sum of its pairs' gradients in emission
 * order, then the chain rule to the raw parameters (the second half of
 * gs_render_bwd), added to or written into `grads`.  ws is the workspace of the
 * step's gs_render_fwd (ws_bytes >= gs_workspace_size(...)); grad_pair may
 * point at its start, as it does inside gs_render_bwd.                      */
int gs_blend_bwd(const gs_camera* cams, int32_t V, int64_t n, const gs_opts* opts, const gs_projected* proj,
                 const gs_binning* bins, const float* T_final, const int32_t* last_contrib, const float* dL_dimage,
                 float* grad_pair, const void* ws, size_t ws_bytes, gs_stream_t stream);
int gs_project_bwd(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                   const gs_projected* proj, const gs_binning* bins, const float* grad_pair, gs_grads* grads,
                   void* ws, size_t ws_bytes, gs_stream_t stream);

/* Gradient of the mean squared error over the V views of a rendered image
 * (layout of gs_render_fwd's image), averaged over mean_views views:
 *   L = (1 / mean_views) sum_v mean over 3 H_v W_v of (image - target)^2,
 *   dL/dimage = 2 (image - target) / (3 H_v W_v mean_views).
 * image, target, dL_dimage: device, [sum_v 3 H_v W_v] (dL_dimage WRITTEN; it may
 * alias neither input).  Only the cameras' width and height are read;
 * mean_views >= 1 (V for a plain mean; a per-view call of a V-view batch
 * passes the batch's V).  One elementwise pass, no workspace.               */
int gs_l2_grad(const float* image, const float* target, const gs_camera* cams, int32_t V, int32_t mean_views,
               float* dL_dimage, gs_stream_t stream);

/* Eq. 2 forward and backward for the mean-squared-error loss of gs_l2_grad,
 * in one launch of the compositing walks: the same results, bit for bit, as
 * gs_render_fwd, then gs_l2_grad(image, target, cams, V, mean_views, ...),
 * then gs_render_bwd on the same arguments.  The loss gradient of a pixel
 * needs only that pixel, so the backward of a tile may start once the forward
 * of that tile is done: every tile's forward walk is taken first, in the
 * heaviest-first order, then the backward items, shortest lists first, so that
 * the backward of finished tiles runs while the deepest tiles' forward walks go
 * on; each backward item waits, with a time limit, for its tile's forward (a
 * wait that times out, which the ordering rules out, makes that item's
 * gradients NaN instead of hanging).
 * image, T_final, last_contrib: WRITTEN as by gs_render_fwd.  dL_dimage:
 * device, image layout, or NULL; when given it receives dL/dimage as
 * gs_l2_grad writes it (it may alias neither image nor target).  grads: as
 * gs_render_bwd.  ws_bytes >= gs_workspace_size(...) (the same workspace as
 * the other calls; this call also keeps per-tile flags and its list of
 * backward items in it).  With
 * opts->fwd_chunk != 0 the call runs the three calls above one after the other
 * and then needs dL_dimage (GS_E_INVALID without it).                          */
int gs_render_fwd_bwd_l2(const gs_gaussians* g, const gs_camera* cams, int32_t V, const gs_opts* opts,
                         const gs_projected* proj, const gs_binning* bins, const float* target, int32_t mean_views,
                         float* image, float* T_final, int32_t* last_contrib, float* dL_dimage, gs_grads* grads,
                         void* ws, size_t ws_bytes, gs_stream_t stream);

/* Photometric loss of Eq. 7, its L1 and D-SSIM terms, over the V views of a
 * rendered image (layout of gs_render_fwd's image), and its gradient:
 *   L_v = (1 - lambda) mean|x - y| + lambda (1 - mean SSIM),  L = mean_v L_v
 * SSIM per colour plane with the 11 x 11 Gaussian window of standard
 * deviation 1.5 applied as two 1-D passes (Sec. 3.2.5), zero padding,
 * C1 = 0.01^2, C2 = 0.03^2; d|t|/dt = sign(t) (0 at 0).
 * image, target: device, [sum_v 3 H_v W_v] planar per view, views concatenated.
 * loss: device [V + 1] or NULL: the V per-view losses, then their mean.
 * dL_dimage: device, image layout, or NULL: WRITES dL/dimage of the mean.
 * Only the cameras' width and height are read.  lambda_ssim in [0, 1].
 * ws_bytes >= gs_loss_workspace_size(cams, V).  Deterministic (no atomics). */
size_t gs_loss_workspace_size(const gs_camera* cams, int32_t V);
int gs_loss_l1_dssim(const float* image, const float* target, const gs_camera* cams, int32_t V,
                     float lambda_ssim, float* loss, float* dL_dimage, void* ws, size_t ws_bytes,
                     gs_stream_t stream);

/* Mask terms of Eq. 7: lambda_m L_m + lambda_sh L_sh with
 *   L_m  = mean over the n Gaussians of sigmoid(mask_logit)        (soft volume mask, Eq. 3)
 *   L_sh = mean over the Gaussians of sum_l w_l sigmoid(sh_mask_logit_l), l = 1..sh_degree,
 *          w_l = (2l + 1) / sum_l' (2l' + 1)                       (coefficient-weighted, Sec. 3.2.3)
 * A NULL mask array contributes nothing.  loss: device [1] or NULL (written).
 * grads->mask_logits / sh_mask_logits (if grads and they are non-NULL) are
 * ACCUMULATED (+=).  Only g's mask arrays, n and sh_degree are read.
 * ws_bytes >= gs_mask_loss_workspace_size(n).  Deterministic (no atomics). */
size_t gs_mask_loss_workspace_size(int64_t n);
int gs_mask_loss(const gs_gaussians* g, float lambda_m, float lambda_sh, float* loss, gs_grads* grads, void* ws,
                 size_t ws_bytes, gs_stream_t stream);

/* gs_mask_loss without the workspace argument, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the partial sums live in a static device array of the
 * library (512 KiB per device, held until the process ends) instead of `ws`.
 * Same kernels, same results, bit for bit, as gs_mask_loss.  n at most 2^24
 * Gaussians, else GS_E_TOO_LARGE (nothing enqueued).  The call allocates
 * nothing (no hipMalloc, no library allocation); it reads the array's device
 * address once per device.  Calls that overlap on one device (other streams or
 * threads) share the array and race: serialise them.  Nothing in the array
 * needs clearing between calls. */
int gs_mask_loss_noalloc(const gs_gaussians* g, float lambda_m, float lambda_sh, float* loss, gs_grads* grads,
                         gs_stream_t stream);

/* Ray hits of the significance score (Eq. 4, Sec. 3.2.2): the walk of
 * gs_render_fwd over the same lists and with the same per-pixel decisions,
 * counting instead of blending.  For each Gaussian i, ADDS (+=) to hits[i]
 * the number of pixels of the V views where it is composited (alpha >= 1/255,
 * in front of the point where the transmittance would fall under 1e-4).
 * Call once per batch of views into one caller-zeroed array to sum over a
 * training set.  hits: device [n] uint32.  Writes nothing else; needs no
 * workspace. */
int gs_count_hits(const gs_projected* proj, const gs_binning* bins, const gs_camera* cams, int32_t V, int64_t n,
                  const gs_opts* opts, uint32_t* hits, gs_stream_t stream);

/* Significance score of Eq. 4 from the summed ray hits:
 *   score_i = hits_i * o'_i * min(vol_i / v_q, 1)
 * o'_i = sigmoid(opacity_logit) times the hard volume mask (Eq. 3, when
 * g->mask_logits is given); vol_i = the product of the three scales; v_q the
 * volume at ascending rank ceil(q n) (q = volume_quantile in (0, 1], 0.9 for
 * the normalisation by the largest Gaussians' volume of Sec. 3.2.2; rank
 * computed in double).  Volumes are compared as the float sums of the
 * log-scales.  A Gaussian without hits scores 0.  Only g's log_scales,
 * opacity_logits, mask_logits, mask_eps and n are read.  hits: device [n];
 * score: device [n] (written).  ws_bytes >= gs_significance_workspace_size().
 * Deterministic. */
size_t gs_significance_workspace_size(void);
int gs_significance(const gs_gaussians* g, const uint32_t* hits, float volume_quantile, float* score, void* ws,
                    size_t ws_bytes, gs_stream_t stream);

/* Target blur of progressive training (Sec. 3.2.4; 9 x 9, sigma 2.4 at the
 * start, Sec. 4.2): a ksize x ksize Gaussian, the outer product of two
 * normalised ksize-tap Gaussians of standard deviation sigma, correlated with
 * each [H][W] plane mirrored about its edge pixels (index -1 reads index 1).
 * in, out: device, [sum_v 3 H_v W_v] planar per view, views concatenated (the
 * layout of gs_render_fwd's image); distinct buffers.  Only the cameras' width
 * and height are read.  ksize odd in [1, 31]; sigma > 0.  out is written. */
int gs_blur_views(const float* in, float* out, const gs_camera* cams, int32_t V, int32_t ksize, float sigma,
                  gs_stream_t stream);

/* Target resize of progressive training (Eq. 6): view v is resampled from
 * in_cams[v]'s size W x H to out_cams[v]'s size W' x H' by area averaging:
 * output pixel (x', y') is the mean of the piecewise-constant input over
 * [x' W / W', (x' + 1) W / W') x [y' H / H', (y' + 1) H / H') (exact
 * overlap weights).  in, out: device, views concatenated as above, not
 * overlapping.  Only the cameras' width and height are read. */
int gs_resize_views(const float* in, const gs_camera* in_cams, float* out, const gs_camera* out_cams, int32_t V,
                    gs_stream_t stream);

/* Static description of a return code. */
const char* gs_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GS_API_H */
