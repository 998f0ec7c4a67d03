/*
 * libhigs: MI355X (gfx950) implementation of the forward frame path of
 * HiGS, "A Hierarchical Rendering Architecture for Real-Time 3D Gaussian
 * Splatting" (Pajak, Bisson, Lima; arXiv 2606.00352).
 *
 * The path, in stage order (each stage is a set of HIP kernels):
 *   higs_project  - per-gaussian EWA projection with degree<=3 SH colour
 *                   (sec. 4.2, Projection and SH evaluation).
 *   higs_bin_sort - (macro-tile, depth) pair emission over 64x32-pixel
 *                   macro-tiles (sec. 3.2 / sec. 4.3) and their sort by
 *                   (macro-tile, depth) with ties broken by gaussian id
 *                   (sec. 3.3 / sec. 4.4).
 *   higs_batch    - split of each macro-tile's sorted list into batches of
 *                   at most B_r gaussians, one processing unit each
 *                   (sec. 3.1, Macro-tile hierarchy and work decomposition).
 *   higs_raster   - per-unit rasterisation over the 8x8 render tiles of the
 *                   macro-tile (sec. 3.4, Algorithms 1 and 2) and the
 *                   post-blend merge of the batch partials with Eq. 1.
 *   higs_render   - all of the above in one call.
 *   higs_server_* - a render server: resident scenes, continuous batching of
 *                   frame requests over contexts and streams (serving).
 *   higs_raster_backward - the adjoint of the last frame: gradients of a loss
 *                   on the image (and final transmittance) with respect to
 *                   the gaussian parameters (the backward that the paper's
 *                   Forward-only paragraph outlines).
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers to contiguous row-major float32
 *     unless stated otherwise; the caller owns them and they must stay valid
 *     until the work queued on `stream` has finished.  The library never
 *     frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it and returns without waiting, except
 *     higs_get_counts and higs_debug_copy, which synchronise the stream of
 *     the last call.
 *   - A context owns every intermediate buffer, sized at creation for the
 *     capacities given there; intermediates stay valid until the next call
 *     that rewrites them.  A context is used from one host thread and one
 *     stream at a time.
 *   - Return value: HIGS_OK (0) or a negative HIGS_E_* code; higs_error_string
 *     turns it into text.  Data-dependent capacity overflow (more pairs or
 *     batches than the context holds) cannot be known when the work is
 *     enqueued: it is recorded on the device and the frame stops there —
 *     every later kernel of the frame returns at once, the image and T_out
 *     are filled with NaN, and higs_raster_backward writes NaN gradients.
 *     higs_get_counts reports it (overflow bits, and the number of pairs the
 *     frame asked for; after a pair overflow the batch stage does not run and
 *     the batch count is 0) so the caller can grow the context and render
 *     again.
 *   - Gaussians with a non-finite mean, scale, rotation or opacity, a zero
 *     quaternion, camera-space depth <= near_z, opacity below 1/255, or a
 *     non-positive-definite 2D covariance are culled (not an error).
 */
#ifndef HIGS_H
#define HIGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HIGS_OK 0
#define HIGS_E_INVALID (-1)     /* null pointer, negative size, bad parameter */
#define HIGS_E_NOMEM (-2)       /* device allocation failed */
#define HIGS_E_CAPACITY (-3)    /* a host-known size exceeds the context */
#define HIGS_E_HIP (-4)         /* a HIP runtime call failed */
#define HIGS_E_UNSUPPORTED (-5) /* tile shape or SH degree not implemented */
#define HIGS_E_STATE (-6)       /* stage called before the one it depends on */

/* Overflow bits reported by higs_get_counts. */
#define HIGS_OVF_PAIRS 1u   /* more (macro-tile, gaussian) pairs than max_pairs */
#define HIGS_OVF_BATCHES 2u /* more batches than max_batches */
#define HIGS_ERR_STALL 0x80000000u /* internal: a sort look-back timed out (frame invalid) */

typedef struct higs_ctx higs_ctx;

/* Method parameters (sec. 3.1 and sec. 5.3 of the paper).  Only the paper's
 * tile shape is implemented: tile_px = 8, mt_tiles_x = 8, mt_tiles_y = 4. */
typedef struct {
  int32_t tile_px;    /* render tile edge in pixels: 8 */
  int32_t mt_tiles_x; /* render tiles per macro-tile, horizontally: 8 */
  int32_t mt_tiles_y; /* render tiles per macro-tile, vertically: 4 */
  int32_t batch_cap;  /* B_r, gaussians per processing unit, 1..1024 (1024) */
  int32_t sh_degree;  /* 0..3 (3); sh arrays hold (sh_degree+1)^2 x 3 floats */
  float alpha_max;    /* clamp of alpha (0.99) */
  float t_eps;        /* compositing stops once T < t_eps (1e-4) */
  float near_z;       /* cull at camera-space depth <= near_z (0.2) */
  float dilation;     /* added to the 2D covariance diagonal (0.3) */
  int32_t sort_mode;  /* HIGS_SORT_ONESWEEP (default) or HIGS_SORT_SEGMENTED */
  int32_t raster_precision; /* HIGS_RASTER_FP32 (default) or HIGS_RASTER_FP16 */
  int32_t sh_format;  /* HIGS_SH_FLOAT32 (default) or HIGS_SH_PACKED32 */
  int32_t max_views;  /* views one frame of higs_render_views may hold, 1..HIGS_MAX_VIEWS (1) */
  int32_t use_graphs; /* 1: replay frames from HIP graphs (see below); 0 (default): launch each kernel */
  int32_t raster_chain; /* batches of one macro-tile that a raster workgroup takes in order,
                           1..64 (64): within them it leaves out a render tile once the product
                           of the earlier batches' transmittances is below t_eps at all 64 of
                           its pixels, where the merge of Eq. 1 stops reading; 1: every
                           (macro-tile, batch) unit is rasterised in full */
  int32_t fuse_merge;   /* 1 (default): a raster work item takes all batches of one
                           macro-tile and folds their partials into its pixels itself, by
                           Eq. 1 in the merge's order and arithmetic (the same image and T,
                           bit for bit, in either raster_precision); no partials are stored,
                           no merge kernel runs, and raster_chain is not used.  0: the
                           partials and the merge kernel, which higs_raster_backward reads
                           (with 1 it first rasterises the frame again with partials) */
} higs_params;

#define HIGS_MAX_VIEWS 64

/* Reduced-precision mode (sec. 3.5 "Numerical representation" and sec. 4.5
 * "Numerical format"): HIGS_RASTER_FP16 rasterises in packed half precision
 * (prescaled Cholesky factors, coordinates relative to the macro-tile centre,
 * two pixels per lane, 8-byte partials) and checks the transmittance cut-off
 * once per 64 gaussians instead of per gaussian.  Projection, pairs, sort
 * order and batches are the float32 mode's, bit for bit; the image is not held
 * to the float32 tolerance (the paper judges this mode by PSNR against the
 * float32 renderer).  higs_raster_backward is not available in this mode. */
#define HIGS_RASTER_FP32 0
#define HIGS_RASTER_FP16 1
/* SH input of higs_project: HIGS_SH_FLOAT32 = float [n, (deg+1)^2, 3];
 * HIGS_SH_PACKED32 = the 32-byte representation of sec. 4.2 written by
 * higs_sh_compress (degree 3 only). */
#define HIGS_SH_FLOAT32 0
#define HIGS_SH_PACKED32 1

/* How pairs are binned and depth-ordered; both give the same (macro-tile,
 * depth, id) order.  SEGMENTED: binning straight into per-macro-tile segments
 * and an independent sort of each (sec. 3.2-3.3, 4.3-4.4); ONESWEEP: a global
 * LSD radix sort of composite (macro-tile, depth) keys. */
#define HIGS_SORT_SEGMENTED 0
#define HIGS_SORT_ONESWEEP 1

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  Pixel (i, j)
 * has its centre at (i + 0.5, j + 0.5).  HOST memory. */
typedef struct {
  int32_t width, height;   /* image size in pixels, >= 1 */
  float fx, fy, cx, cy;    /* focal lengths and principal point, pixels */
  float world_to_cam[12];  /* row-major [R | t]: x_cam = R x_world + t */
  float background[3];     /* added as T * background to the composite */
} higs_camera;

/* Sizes of the last frame; filled by higs_get_counts. */
typedef struct {
  int64_t n_gaussians; /* gaussians submitted to higs_project */
  int64_t n_visible;   /* gaussians with at least one macro-tile pair */
  int64_t n_pairs;     /* (macro-tile, gaussian) pairs emitted */
  int64_t n_batches;   /* (macro-tile, batch) processing units */
  uint32_t overflow;   /* HIGS_OVF_* bits */
  int32_t sort_passes; /* radix passes that moved data (a pass whose digit is
                          the same for every key is skipped) */
  int64_t n_evaluations; /* pixel-gaussian evaluations of the rasteriser
                            (64 per gaussian per render tile visited), or -1
                            unless HIGS_DEBUG_COUNT_EVALS is set */
  int32_t sort_pair_bytes; /* bytes per pair that each radix pass reads and
                              writes: 8 when key and gaussian id share one
                              64-bit word, 12 when the id travels in an array
                              of its own; 0 in segmented mode */
  int32_t graphs;       /* HIP graphs the context holds (params->use_graphs) */
} higs_counts;

/* Writes the paper's defaults into *p. */
void higs_default_params(higs_params* p);

/* Creates a context on HIP device `device` with every intermediate sized for
 * at most max_gaussians gaussians, max_pairs pairs, max_batches processing
 * units and max_width x max_height images.  *out receives the handle.
 * Returns HIGS_E_UNSUPPORTED for a tile shape other than 8x8 / 8x4 or
 * sh_degree > 3, HIGS_E_INVALID for non-positive capacities or a batch_cap
 * outside 1..1024, HIGS_E_NOMEM if the device memory is not there. */
int higs_ctx_create(int device, const higs_params* params, int64_t max_gaussians,
                    int64_t max_pairs, int64_t max_batches, int32_t max_width,
                    int32_t max_height, higs_ctx** out);

/* Releases the context and its device memory (synchronises its stream). */
int higs_ctx_destroy(higs_ctx* ctx);

/* Device memory (bytes) a context created with these capacities allocates
 * (host-only arithmetic, no device call; negative HIGS_E_INVALID for
 * non-positive sizes).  The adjoint buffers of higs_raster_backward come on
 * top (max_batches * 16 KiB + max_gaussians * 64 B). */
int64_t higs_ctx_footprint(const higs_params* params, int64_t max_gaussians, int64_t max_pairs,
                           int64_t max_batches, int32_t max_width, int32_t max_height);

/* Stage 1: projects n gaussians for `cam` (sec. 4.2).  Inputs (device):
 *   means [n,3], scales [n,3] (linear), quats [n,4] as (w,x,y,z), any norm,
 *   opacities [n] (in [0,1]), sh [n, (sh_degree+1)^2, 3].
 * The camera is copied; later stages of the frame use it.  n may be 0.
 * HIGS_E_CAPACITY if n > max_gaussians or the image exceeds max size. */
int higs_project(higs_ctx* ctx, int64_t n, const float* means, const float* scales,
                 const float* quats, const float* opacities, const float* sh,
                 const higs_camera* cam, void* stream);

/* Stage 2: emits every (macro-tile, gaussian) pair whose opacity-level
 * ellipse {q <= 2 ln(255 o)} meets the macro-tile's rectangle (sec. 3.2) in
 * gaussian-id order, and sorts them by (macro-tile, float32 depth bits,
 * gaussian id) (sec. 3.3).  Needs higs_project of the same frame. */
int higs_bin_sort(higs_ctx* ctx, void* stream);

/* Stage 3: per macro-tile, ceil(n / batch_cap) batches in (macro-tile,
 * batch) order (sec. 3.1).  Needs higs_bin_sort of the same frame. */
int higs_batch(higs_ctx* ctx, void* stream);

/* Stage 4: rasterises every processing unit from (C, T) = (0, 1) with
 * front-to-back blending, alpha = min(alpha_max, o exp(-q/2)), skipping
 * alpha < 1/255 and stopping once T < t_eps, then merges the partials of each
 * render tile in batch order with Eq. 1 (C = C0 + T0 C1 + T0 T1 C2 + ...,
 * stopping once the product of T drops below t_eps).  Outputs (device):
 *   image [height, width, 3] = C + T * background;
 *   T_out [height, width] final transmittance, or NULL.
 * Needs higs_batch of the same frame. */
int higs_raster(higs_ctx* ctx, float* image, float* T_out, void* stream);

/* All four stages for one frame. */
int higs_render(higs_ctx* ctx, int64_t n, const float* means, const float* scales,
                const float* quats, const float* opacities, const float* sh,
                const higs_camera* cam, float* image, float* T_out, void* stream);

/* Several views in one frame: every stage runs once, in one launch per kernel,
 * for n_views cameras of one image size, each with its own scene arrays and
 * image (serving many requests per launch).  View v's gaussians and
 * macro-tiles get ranges of their own in the frame (the pair keys carry the
 * view in their macro-tile field), so the emission, the sort, the batch split
 * and the rasteriser treat the views as one larger frame; each image is the
 * one higs_render gives for that view alone, bit for bit.  The context must be
 * created with params->max_views >= n_views; max_gaussians bounds each view's
 * n; max_pairs and max_batches bound the frame's totals (all views).  Every
 * view's camera must have the size of views[0].camera (else HIGS_E_INVALID).
 * Not with the segmented sort mode, and not followed by higs_raster_backward.
 * The views array (host) is read before the call returns. */
typedef struct {
  int64_t n;                /* gaussians of this view's scene */
  const float *means, *scales, *quats, *opacities, *sh;  /* device, as higs_project */
  higs_camera camera;       /* host */
  float* image;             /* device [H, W, 3] */
  float* T_out;             /* device [H, W] or NULL */
} higs_view;
int higs_render_views(higs_ctx* ctx, int32_t n_views, const higs_view* views, void* stream);

/* Graph replay (params->use_graphs = 1): higs_render and higs_render_views
 * record a frame of each new shape (view count, the frame's largest scene
 * rounded up to 1,024 gaussians, image size) into a HIP graph on first use and
 * replay it afterwards, one launch per frame.  The graph's kernels read the
 * views (scene arrays, camera, image) from a device table that the graph's
 * first node copies from a pinned host buffer of that graph; before writing
 * the buffer the call waits for the graph's previous replay to complete, so
 * frames of one shape on one context do not overlap on the host.  The image
 * is the one the per-kernel launch gives, bit for bit.  Frames on the legacy
 * default stream (stream = NULL), with timers (higs_set_timing) or debug
 * flags, and in the segmented sort mode launch kernel by kernel.  A context
 * keeps at most 32 graphs (least recently used are destroyed).  Only
 * higs_render and higs_render_views replay; the staged calls (higs_project
 * ...) always launch kernel by kernel. */

/* Adjoint of the last frame rendered on ctx (the paper is forward-only; its
 * Forward-only paragraph outlines this backward: the post-blend merge of
 * Eq. 1 becomes a prefix scan of transmittance over the batches, the point
 * where transmittance saturates is recovered per (pixel, batch), and the
 * blend is reversed by dividing by (1 - alpha) in float32).
 *   dL_dimage  [H, W, 3] float32: gradient of the loss with respect to the
 *              image higs_raster wrote (H, W of that frame's camera).
 *   dL_dT      [H, W] float32 or NULL (zero): gradient with respect to the
 *              final transmittance T_out.
 *   dmeans [n, 3], dscales [n, 3], dquats [n, 4], dopacities [n],
 *   dsh [n, (sh_degree + 1)^2, 3]: outputs, written in full (zero for
 *              culled and off-screen gaussians); gradients with respect to
 *              the arrays given to higs_project, in their layouts (scales
 *              linear, opacities after the sigmoid, quaternions as given,
 *              unnormalised).
 * The scene arrays passed to the frame's higs_project must still hold the
 * same values: the adjoint re-reads them.  The discrete structure (culls,
 * pairs, depth order, batches, which gaussians composite at a pixel, the
 * alpha clamp at alpha_max) is held fixed, as its derivative is zero almost
 * everywhere.  Per-gaussian sums are accumulated with float atomics, so
 * results vary in the last bits from run to run.  Needs a completed
 * higs_raster on ctx since its last higs_project (else HIGS_E_STATE); the
 * first call allocates the adjoint's buffers (max_batches * 16 KiB +
 * max_gaussians * 64 B; HIGS_E_NOMEM if that fails).  Every gradient is NaN
 * when the frame overflowed its capacities (higs_get_counts). */
int higs_raster_backward(higs_ctx* ctx, const float* dL_dimage, const float* dL_dT,
                         float* dmeans, float* dscales, float* dquats, float* dopacities,
                         float* dsh, void* stream);

/* Packed SH (sec. 4.2, the 32-byte SH representation): the colour
 * coefficients of every gaussian go to YCoCg (luma, two chroma differences),
 * are scaled per basis and component by a high percentile (99.9%) of their
 * magnitude over the gaussians with opacity >= 1/255, pass through a
 * square-root gamma and are quantised to 6 bits of luma and 4 of chroma (the
 * DC basis to 12 and 10 bits), 32 bytes per gaussian after a 256-byte header
 * of 48 float32 scales.  higs_sh_packed_bytes(n) is the size of that buffer.
 * higs_sh_compress writes it from sh [n, 16, 3] and opacities [n] (device)
 * into `packed` (device, 16-byte aligned, higs_sh_packed_bytes(n) bytes,
 * caller-owned); it runs on the current device, allocates a 196 KiB work area
 * and synchronises the stream before returning.  A context created with
 * sh_format = HIGS_SH_PACKED32 then takes `packed` as the sh argument of
 * higs_project. */
int64_t higs_sh_packed_bytes(int64_t n);
int higs_sh_compress(int64_t n, const float* sh, const float* opacities, void* packed,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops and harnesses that forbid hipMalloc): one frame of
 * the whole path, as higs_render with the default parameters, with every
 * intermediate in a static device array of the library (80 MiB, held on each
 * device the library runs on until the process ends) instead of a context.
 * Allocates nothing: no hipMalloc, no hipFree.  Limits: n <= 131072
 * gaussians, images up to 1024 x 1024, at most 524288 (macro-tile, gaussian)
 * pairs per frame (more: the frame stops and the image and T_out are NaN, as
 * for a context's capacity overflow); larger n or images return
 * HIGS_E_CAPACITY before any work is queued.  Arguments as for higs_render,
 * on the current HIP device.  Every call on a device shares that device's
 * array, which keeps the last call's intermediates: calls that overlap on one
 * device (other streams, other host threads) race, so a caller serialises
 * them (one stream, or an event between calls). */
int higs_render_noalloc(int64_t n, const float* means, const float* scales, const float* quats,
                        const float* opacities, const float* sh, const higs_camera* cam,
                        float* image, float* T_out, void* stream);

/* ---- Serving ---------------------------------------------------------------
 * A render server keeps several scenes resident on the device and renders a
 * stream of requests (scene, camera, resolution class) with continuous
 * batching.  Its frame contexts live in one device arena of hbm_budget bytes,
 * allocated by higs_server_create: a request is admitted as soon as a context
 * of its resolution class is idle, or a new one's range fits the arena (idle
 * contexts of other classes are released to make room, least recently used
 * first); no device memory is allocated or freed while serving.  An admitted
 * frame also takes the next queued requests of the same class and image size,
 * up to the class's views per frame, and renders them in one launch per
 * kernel (higs_render_views).  Every context renders on a HIP stream of its
 * own, so admitted frames overlap on the device; with use_graphs the frames
 * are replayed from HIP graphs.  The server is driven from one host thread:
 * higs_server_submit queues, higs_server_poll retires finished frames and
 * admits queued ones; neither blocks.  A request's image is the same rendered
 * alone (higs_render with the class's batch_cap) or in the mix.  The paper
 * renders single frames; this is the serving loop around its frame path. */
typedef struct higs_server higs_server;

#define HIGS_MAX_CLASSES 4
typedef struct {
  int32_t n_classes;                     /* resolution classes, 1..HIGS_MAX_CLASSES */
  int32_t width[HIGS_MAX_CLASSES];       /* largest image of each class */
  int32_t height[HIGS_MAX_CLASSES];
  int64_t max_pairs[HIGS_MAX_CLASSES];   /* pair capacity per view of the class */
  int64_t max_gaussians;                 /* the largest scene */
  int64_t hbm_budget;                    /* bytes of the context arena (allocated at once) */
  int32_t max_in_flight;                 /* frames rendering at once (1 with one view per
                                            frame: the plain one-frame-at-a-time renderer) */
  int32_t views_per_frame[HIGS_MAX_CLASSES]; /* requests one frame may hold (0 or 1: one);
                                            higs_server_tune or _set_class may change it */
  int32_t use_graphs;                    /* 1: frames replayed from HIP graphs */
} higs_server_config;

typedef struct {
  int64_t request_id;
  float gpu_ms;       /* device time of the request's frame, events on its stream */
  uint32_t overflow;  /* HIGS_OVF_* bits of the frame (its images are then NaN) */
  int32_t cls;
  int32_t views;      /* requests the frame rendered */
} higs_completion;

typedef struct {
  int32_t queued, in_flight, contexts;
  int64_t bytes;      /* arena bytes held by frame contexts */
  int64_t completed, evictions;
  int64_t frames;     /* frames launched (each renders 1..views_per_frame requests) */
  int32_t views_per_frame[HIGS_MAX_CLASSES];
  int32_t batch_cap[HIGS_MAX_CLASSES];
} higs_server_stats;

/* params: NULL for the defaults.  HIGS_E_NOMEM if the arena cannot be
 * allocated.
 * higs_server_add_scene: the scene arrays are device pointers owned by the
 * caller that must stay valid and unchanged while the server renders them;
 * stream: the stream on which the arrays were written (an event recorded on it
 * now orders every frame of the scene after that work; NULL is the legacy
 * default stream).
 * higs_server_submit: image is device [H, W, 3] of the camera's size (at most
 * the class size, else HIGS_E_CAPACITY), written when the request completes;
 * stream: the caller's stream whose work so far must precede the frame (an
 * event is recorded on it now; NULL is the legacy default stream).  The image
 * is final once higs_server_poll has returned the request.
 * higs_server_poll returns the number of completions written to done
 * (<= max_done; completions of a frame that do not fit wait for the next
 * call), or a negative error; an error met after completions were retired is
 * returned by the next call that has none to report. */
int higs_server_create(int device, const higs_params* params, const higs_server_config* cfg,
                       higs_server** out);
int higs_server_destroy(higs_server* server);
int higs_server_add_scene(higs_server* server, int32_t scene_id, int64_t n, const float* means,
                          const float* scales, const float* quats, const float* opacities,
                          const float* sh, void* stream);
int higs_server_submit(higs_server* server, int64_t request_id, int32_t scene_id, int32_t cls,
                       const higs_camera* cam, float* image, void* stream);
int higs_server_poll(higs_server* server, higs_completion* done, int32_t max_done);
int higs_server_get_stats(higs_server* server, higs_server_stats* out);

/* Autotuner: for class cls, renders `frames` frames of scene_id at the
 * cameras given (cycled; each of the class size) for every candidate of
 * views per frame in {1, 2, 4, 8, 16} (those whose context fits the arena)
 * and, with allow_batch_cap, B_r in {1024, 512, 256} (other values change the
 * batch boundaries, so images are then no longer those of B_r = 1024 bit for
 * bit); each trial keeps up to max_in_flight frames in flight on as many
 * contexts as the class's share of the arena (1 / n_classes) holds.  The
 * setting with the fewest views per frame (then the largest B_r) within 3% of
 * the fastest trial (requests per second) becomes the class's.  The server
 * must be idle (HIGS_E_STATE otherwise); its idle contexts are released.
 * HIGS_E_CAPACITY if no candidate's context fits the share.  Synchronises the
 * device. */
#define HIGS_TUNE_MAX_TRIALS 16
typedef struct {
  int32_t views_per_frame, batch_cap;   /* chosen */
  int32_t n_trials;
  int32_t trial_views[HIGS_TUNE_MAX_TRIALS];
  int32_t trial_batch_cap[HIGS_TUNE_MAX_TRIALS];
  float trial_fps[HIGS_TUNE_MAX_TRIALS];   /* requests per second */
} higs_tune_report;
int higs_server_tune(higs_server* server, int32_t cls, int32_t scene_id, int32_t n_cams,
                     const higs_camera* cams, int32_t frames, int32_t allow_batch_cap,
                     higs_tune_report* out);
/* Sets a class's views per frame and B_r for contexts created from now on. */
int higs_server_set_class(higs_server* server, int32_t cls, int32_t views_per_frame,
                          int32_t batch_cap);

/* Synchronises the stream of the last call and reports the frame's sizes. */
int higs_get_counts(higs_ctx* ctx, higs_counts* out);

/* Intermediate buffers that higs_debug_copy can read back (tests). */
#define HIGS_DBG_PROJ 1     /* float32 [8][n]: mx, my, a, b, c, tau, key bits, count bits
                               (rows of culled gaussians: key = 0, count = 0, rest undefined;
                               mx .. tau are stored for every gaussian that passes the
                               culling only under HIGS_DEBUG_PROJ_FIELDS, otherwise only
                               for those whose macro-tile list the emission re-derives) */
#define HIGS_DBG_RECORDS 2  /* float32 [n][12]: mx, my, l0, l1, l2, o, r, g, b, tau, 0, 0
                               (defined for gaussians with count > 0) */
#define HIGS_DBG_PAIRS 3    /* uint64 keys [n_pairs] then uint32 ids [n_pairs], emission order
                               (needs HIGS_DEBUG_KEEP_PAIRS); key = macro-tile << 32 | depth bits */
#define HIGS_DBG_SORTED 4   /* same layout, sorted */
#define HIGS_DBG_MT_OFFSETS 5 /* uint32 [n_macro_tiles + 1]: first sorted pair of each macro-tile */
#define HIGS_DBG_BATCHES 6  /* uint32 [n_batches][3]: macro-tile, start, length */
#define HIGS_DBG_ACTIVE 7   /* uint32 [n_batches]: bit t = render tile t written by the unit
                               (ACTIVE and PARTIALS: frames with fuse_merge = 0, else
                               HIGS_E_STATE) */
#define HIGS_DBG_PARTIALS 8 /* float32 [n_batches][32][64][4]: R, G, B, T per pixel, valid
                               where the active bit is set; pixel p of tile t sits at
                               (t % 8 * 8 + p % 8, t / 8 * 8 + p / 8) in the macro-tile */

/* Debug options (bit flags): HIGS_DEBUG_KEEP_PAIRS keeps a copy of the emitted pairs
 * before the sort (allocates max_pairs * 12 bytes on first use) so that
 * HIGS_DBG_PAIRS can read them back. */
#define HIGS_DEBUG_KEEP_PAIRS 1
/* HIGS_DEBUG_COUNT_EVALS makes the rasteriser count its evaluations
 * (reported in higs_counts.n_evaluations; adds one atomic per tile). */
#define HIGS_DEBUG_COUNT_EVALS 2
/* HIGS_DEBUG_PROJ_FIELDS makes the projection store the six binning fields of
 * every gaussian that passes the culling (24 bytes each), for HIGS_DBG_PROJ.
 * Without it they are stored only where the emission needs them: gaussians
 * whose macro-tile list does not fit the compact span word. */
#define HIGS_DEBUG_PROJ_FIELDS 4
/* HIGS_DEBUG_TWO_WORD_PAIRS keeps each pair's key and gaussian id in separate
 * arrays even when they fit one 64-bit word (the layout frames with a wide key
 * and many gaussians use), so that tests can run that sort path on any scene. */
#define HIGS_DEBUG_TWO_WORD_PAIRS 8
int higs_set_debug(higs_ctx* ctx, int flags);

/* Copies `bytes` bytes of buffer `which` (HIGS_DBG_*) into HOST memory
 * `host_dst`, after synchronising.  HIGS_E_INVALID if `bytes` exceeds the
 * buffer's current content. */
int higs_debug_copy(higs_ctx* ctx, int which, void* host_dst, size_t bytes);

/* Per-kernel device times, measured with HIP events recorded on the frame's
 * stream around each kernel group.  higs_set_timing(ctx, n) keeps the events
 * of the last n frames (1..1024; 0 turns timing off, the default) without
 * any host synchronisation; higs_get_timers synchronises and writes the mean
 * over those frames, ms[HIGS_TIMER_*] in milliseconds. */
#define HIGS_TIMER_PROJECT 0 /* projection + SH + per-gaussian pair counts */
#define HIGS_TIMER_SCAN 1    /* pair counts and their scan (segmented: per-macro-tile
                                counts and segment offsets) */
#define HIGS_TIMER_FILL 2    /* pair emission */
#define HIGS_TIMER_SORT 3    /* all radix-sort kernels */
#define HIGS_TIMER_BATCH 4   /* macro-tile offsets + batch table */
#define HIGS_TIMER_RASTER 5  /* per-unit rasteriser */
#define HIGS_TIMER_MERGE 6   /* post-blend merge */
#define HIGS_NUM_TIMERS 7
int higs_set_timing(higs_ctx* ctx, int n_frames);
int higs_get_timers(higs_ctx* ctx, float ms[HIGS_NUM_TIMERS]);

/* Static text for a return code. */
const char* higs_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* HIGS_H */
