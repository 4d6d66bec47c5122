/*
 * libslic: SLIC superpixels on one AMD Instinct MI355X (gfx950).
 *
 * The method is the one gSLICr (Ren, Prisacariu and Reid, arXiv 1509.04232)
 * runs on a GPU: convert the image to CIELAB, place centres on a grid of
 * step S, perturb them to the lowest-gradient pixel nearby, then alternate
 * (associate every pixel with the nearest of the nine centres around its
 * grid cell under Eq. 1's distance; move each centre to the mean of its
 * pixels), and finally enforce connectivity.
 *
 * Conventions shared by every entry point
 *  - Pointers named d_* are device pointers on the current HIP device; the
 *    caller owns every device buffer (input, outputs, workspace).  A context
 *    (slic_ctx) owns only its host-side record.
 *  - `hip_stream` is a hipStream_t (NULL: the null stream).  All device work
 *    is enqueued on it and nothing synchronises the host, except where an
 *    entry point says so.
 *  - Arguments are validated on the host before anything is enqueued; on
 *    SLIC_EINVAL nothing was enqueued and a context is unchanged.  A failed
 *    HIP call returns SLIC_EHIP and poisons the context: later calls on it
 *    return SLIC_ESTATE.  No C++ exception crosses this interface.
 *  - A context is not thread-safe; distinct contexts are independent but
 *    must not share a workspace while both are in use.
 *  - Arithmetic: FP32 in a fixed operation order without contraction, exact
 *    integer centre sums; results are bit-identical to the CPU reference and
 *    independent of launch shapes and run-to-run scheduling.
 */
#ifndef SLIC_H
#define SLIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slic_ctx slic_ctx;

enum {
    SLIC_OK = 0,
    SLIC_EINVAL = 1, /* invalid argument or workspace too small */
    SLIC_ENOMEM = 2, /* host allocation failed */
    SLIC_EHIP = 3,   /* a HIP runtime call failed (no device, launch error, ...) */
    SLIC_ESTATE = 4  /* call not valid in the context's state, or context poisoned */
};

enum {
    SLIC_PERTURB_SEEDS = 1,   /* move each seed to the lowest-gradient pixel of its 3x3 window
                                 (Section 2's seed perturbation) */
    /* colour planes other than CIELAB (the listing's colour-space setting):
     * XYZ scaled by 100 (D65 white -> 100, 100, 100), or the R, G, B bytes
     * as floats; at most one of the two */
    SLIC_COLOR_XYZ = 2,
    SLIC_COLOR_RGB = 4,
    /* the distance of the SLIC paper the method builds on instead of Eq. 1:
     * D^2 = d_lab^2 + (m/S)^2 d_xy^2 (same candidates; its energy term is D) */
    SLIC_DISTANCE_SQUARED = 8
};

/* The problem statement of Section 2: an image of N = width*height pixels,
 * the grid interval S (or the desired superpixel count K, S = sqrt(N/K)),
 * and the compactness m of Eq. 1. */
typedef struct {
    int32_t width, height; /* >= 1 each, width*height < 2^31 */
    int32_t pitch;         /* bytes between input rows, >= width*channels */
    int32_t channels;      /* 3: R,G,B bytes; 4: R,G,B,x (the paper's 4-byte pixels) */
    int32_t S;             /* grid step >= 1, or 0 to derive it from K */
    int32_t K;             /* desired superpixel count, used only when S == 0:
                              S = max(1, floor(sqrt(N/K) + 0.5)) */
    float m;               /* compactness, finite and >= 0, with (m/S) times the
                              image diagonal at most 1e15 (distances stay finite) */
    int32_t flags;         /* SLIC_PERTURB_SEEDS, SLIC_COLOR_XYZ or SLIC_COLOR_RGB,
                              SLIC_DISTANCE_SQUARED, or 0 (a batch shares one distance) */
    int32_t min_segment;   /* connectivity: components smaller than this many pixels
                              are merged; 0: merge when 4*size < S*S */
} slic_params;

/* Device workspace needed by slic_init / slic_segment for these parameters,
 * in bytes (pure host computation).  0 if the parameters are invalid. */
size_t slic_workspace_bytes(const slic_params* p);

/* Grid of Sections 2-3: the integer step S and the ns_c x ns_r map of
 * centres, ns_c = ceil(width/S), ns_r = ceil(height/S); cluster k of cell
 * (cx, cy) is k = cy*ns_c + cx.  Pure host; any output pointer may be NULL. */
int slic_grid(const slic_params* p, int32_t* S, int32_t* ns_c, int32_t* ns_r);

/* Section 4's listing up to the first association: converts d_rgb
 * (height rows of `pitch` bytes) to CIELAB, seeds the centres (Section 3,
 * cluster centre initialisation) and associates every pixel once.  On
 * success *out receives a new context bound to the workspace, the stream and
 * the current device.  d_rgb may be reused once this work has completed on
 * the stream.  d_ws must be 256-byte aligned, ws_bytes >=
 * slic_workspace_bytes(p). */
int slic_init(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb, void* hip_stream,
              void* d_ws, size_t ws_bytes);

/* Video warm start (the paper's use case is a live camera stream): like
 * slic_init, but the centres are d_centres (device float[K][5], (L, a, b,
 * x, y), finite; typically the previous frame's slic_get_centres with the
 * same parameters) instead of seeds, so a few rounds reach the energy that
 * seeding needs many for.  d_centres may be reused once the call's work has
 * completed on the stream. */
int slic_init_from_centres(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb,
                           const float* d_centres, void* hip_stream, void* d_ws, size_t ws_bytes);

/* A frame started from a given first association (a label map computed
 * elsewhere, e.g. a predicted one): like slic_init, but d_labels0 (device
 * int32[height][width], row-major, cluster k = row * ns_c + column of
 * slic_grid's grid) takes the place of the association with the seeds, so
 * the first update of slic_iterate moves each centre to the mean of the
 * pixels given to it; a centre given no pixel keeps its seed (Section 3,
 * cluster centre initialisation).  Entries outside [0, K) take no part in
 * that update and stand for the pixel's own grid cell in the context's
 * labels.  d_labels0 may be reused once the call's work has completed on
 * the stream.  Same workspace and errors as slic_init. */
int slic_init_from_labels(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb,
                          const int32_t* d_labels0, void* hip_stream, void* d_ws, size_t ws_bytes);

/* n_iters >= 0 rounds of (update every centre to the mean of its pixels;
 * associate every pixel), the loop body of Section 4's listing.
 * slic_iterate(c, a) followed by slic_iterate(c, b) equals
 * slic_iterate(c, a + b).  SLIC_ESTATE after slic_enforce_connectivity. */
int slic_iterate(slic_ctx* ctx, int32_t n_iters);

/* Section 2's stopping rule: rounds of (update, associate) until the L1
 * distance between the centres before and after an update, summed over all
 * centres and their five components (L, a, b, x, y) with each |difference|
 * rounded to a multiple of 2^-18, is below threshold * K (threshold: the
 * mean shift per centre, >= 0), at most max_iters rounds.  The round that
 * meets the rule still associates.  The decision is taken on the device
 * (later launches exit at once), so nothing synchronises the host;
 * *d_iters_done (device int32, may be NULL) receives the rounds run.
 * Afterwards the context is final: slic_iterate returns SLIC_ESTATE, the
 * energy, copies and connectivity remain available. */
int slic_iterate_converge(slic_ctx* ctx, int32_t max_iters, float threshold,
                          int32_t* d_iters_done);

/* Connectivity clean-up (Section 2, last step): relabels the context's
 * label map in place into 4-connected segments, merging every segment below
 * the size threshold (slic_params.min_segment) into the segment left of
 * (or, at a row start, above) its first pixel; segments are numbered 0..
 * in raster order of their first pixel.  *d_n_segments (device int32, may
 * be NULL) receives their count.  Afterwards slic_iterate and slic_energy
 * return SLIC_ESTATE; the centres stay those of the last association. */
int slic_enforce_connectivity(slic_ctx* ctx, int32_t* d_n_segments);

/* The paper's own clean-up (Section 3's connectivity step), a cheaper
 * alternative to slic_enforce_connectivity that does not guarantee
 * connected segments: `passes` (>= 0; the paper uses 2) one-thread-per-pixel
 * passes in which a pixel none of whose 4-neighbours inside the image shares
 * its label takes the label that occurs most often among them (ties: the
 * first in the order up, left, right, down); each pass reads the map the
 * previous one wrote.  Relabels the context's label map in place; labels stay
 * cluster indices.  Afterwards slic_iterate and slic_energy return
 * SLIC_ESTATE. */
int slic_filter_stray(slic_ctx* ctx, int32_t passes);

/* Copies of the context's state (device to device, on the context's
 * stream).  Labels: int32[height*width], row-major.  Centres: float[K][5]
 * = (L, a, b, x, y) as used by the last association; counts: int32[K]
 * pixels per centre at the last update (0 before any update), may be NULL.
 * Lab: three planar float[height*width] arrays. */
int slic_get_labels(const slic_ctx* ctx, int32_t* d_labels);
int slic_get_centres(const slic_ctx* ctx, float* d_centres, int32_t* d_counts);
int slic_get_lab(const slic_ctx* ctx, float* d_L, float* d_a, float* d_b);

/* Energy: the mean over pixels of Eq. 1's D_s between each pixel and the
 * centre it is associated with (double, written to *d_out).  Deterministic.
 * SLIC_ESTATE after slic_enforce_connectivity. */
int slic_energy(const slic_ctx* ctx, double* d_out);

/* The whole of Section 4's listing in one call: init, n_iters rounds,
 * optionally the energy (d_energy != NULL, taken before connectivity),
 * optionally connectivity (enforce != 0).  Outputs: d_labels int32[H*W]
 * (required), d_centres float[K][5] (may be NULL), d_n_segments int32 (may
 * be NULL; written only when enforce != 0). */
int slic_segment(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters, int32_t enforce,
                 int32_t* d_labels, float* d_centres, double* d_energy, int32_t* d_n_segments,
                 void* hip_stream, void* d_ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * slic_segment without a workspace argument.  The workspace is a
 * 256-byte-aligned array of SLIC_NOALLOC_MAX_WORKSPACE bytes that the library
 * holds on each device it runs on until the process ends; the call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Arguments, outputs and results are those of slic_segment, bit for bit.
 * SLIC_EINVAL when slic_workspace_bytes(p) exceeds SLIC_NOALLOC_MAX_WORKSPACE
 * (72 MiB: a 1920x1080 frame at any S >= 7).  Every call on one device shares
 * that device's array and leaves its contents behind (each call initialises
 * what it reads): calls that overlap on one device, on different streams or
 * from different threads, race and give wrong results; serialise them. */
#define SLIC_NOALLOC_MAX_WORKSPACE (72u << 20)
int slic_segment_noalloc(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters,
                         int32_t enforce, int32_t* d_labels, float* d_centres, double* d_energy,
                         int32_t* d_n_segments, void* hip_stream);

void slic_destroy(slic_ctx* ctx);
const char* slic_strerror(int code);

/* Launch variants of the association kernel (Section 3's per-pixel step)
 * and their autotuner.  Every variant computes bit-identical results; they
 * differ in the pixels each thread owns (vec horizontally adjacent pixels in
 * each of `rows` rows) and hence the workgroup's tile.  Variant ids run from
 * 1 to slic_assign_variants().  The choice is kept per (width, height, S) in
 * a process-wide table that contexts read when they are created.
 *  - slic_assign_variant_info: the shape of a variant (outputs may be NULL).
 *  - slic_set_assign_variant: record a variant (0: back to the built-in
 *    choice); SLIC_EINVAL if the variant cannot run that shape.
 *  - slic_get_assign_variant: the variant a new context would use.
 *  - slic_autotune: times `reps` runs of slic_init + n_iters iterations for
 *    every variant that supports p (after one warm-up run each), on the given
 *    image, stream and workspace, records the fastest in the table and returns
 *    it with its time per iteration in milliseconds.  Synchronises the host. */
int32_t slic_assign_variants(void);
int slic_assign_variant_info(int32_t variant, int32_t* vec, int32_t* rows, int32_t* tile_w,
                             int32_t* tile_h);
int slic_set_assign_variant(int32_t width, int32_t height, int32_t S, int32_t variant);
int slic_get_assign_variant(int32_t width, int32_t height, int32_t S, int32_t* variant);
int slic_autotune(const slic_params* p, const uint8_t* d_rgb, int32_t n_iters, int32_t reps,
                  void* hip_stream, void* d_ws, size_t ws_bytes, int32_t* best_variant,
                  float* best_ms_per_iter);

/* Batches: many images of uneven sizes and grid steps segmented together.
 * Every launch of the pipeline covers all images: one conversion+seeding
 * launch, 1 + n_iters association launches (workgroups walk a table of
 * (image, tile) pairs), then, with `enforce`, the five connectivity
 * launches (per image instead when an image exceeds 4,194,304 pixels).  The
 * results equal n_images separate slic_segment calls bit for bit.
 *  - slic_batch_workspace_bytes: device workspace for the batch (every
 *    image's own workspace plus the tile tables); 0 if any params invalid.
 *  - slic_batch_create: validates every image, lays out the workspace,
 *    waits for the device to finish its pending work (hipDeviceSynchronize,
 *    so no kernel still running on any stream can touch the workspace),
 *    uploads the tables (synchronous host-to-device copies) and, if
 *    use_graph, captures the whole pipeline into a HIP graph.  `variant` is
 *    an association variant every image supports, or 0 for the largest such
 *    tile.  d_rgb[i], d_labels[i] (int32[H_i*W_i]) and d_n_segments
 *    (int32[n_images], may be NULL, written only with enforce) are the
 *    caller's device buffers and must stay valid while the batch exists.
 *  - slic_batch_run: enqueues the pipeline on hip_stream (one graph launch
 *    with use_graph).  May be called repeatedly (the images are re-read).
 *  - slic_batch_autotune: times `reps` runs per variant that every image
 *    supports, keeps the fastest (re-capturing the graph) and returns it with
 *    its time per run in milliseconds.  Synchronises the host.
 *  - slic_segment_batch: create (no graph), run, destroy in one call. */
typedef struct slic_batch slic_batch;
size_t slic_batch_workspace_bytes(const slic_params* per_image, int32_t n_images);
int slic_batch_create(slic_batch** out, const slic_params* per_image, int32_t n_images,
                      const uint8_t* const* d_rgb, int32_t* const* d_labels, int32_t n_iters,
                      int32_t enforce, int32_t* d_n_segments, int32_t variant, int32_t use_graph,
                      void* d_ws, size_t ws_bytes);
int slic_batch_run(slic_batch* b, void* hip_stream);
int slic_batch_autotune(slic_batch* b, void* hip_stream, int32_t reps, int32_t* best_variant,
                        float* best_ms);
void slic_batch_destroy(slic_batch* b);
int slic_segment_batch(const slic_params* per_image, const uint8_t* const* d_rgb, int32_t n_images,
                       int32_t n_iters, int32_t enforce, int32_t* const* d_labels,
                       int32_t* d_n_segments, void* hip_stream, void* d_ws, size_t ws_bytes);

/* Learned warm start (an extension beyond the paper, whose Section 4 loop
 * starts every frame from grid seeds).  A small convolutional net predicts,
 * per pixel, which of the nine grid cells around the pixel's own cell holds
 * the centre the pixel is associated with after plain SLIC; the decoded
 * label map replaces the first association, so fewer (update, associate)
 * rounds reach the same energy.
 *
 * The net: input (L/100, a/128, b/128) of the CIELAB image; 3x3 convolution
 * 3 -> 32, ReLU, 3x3 convolution 32 -> 32, ReLU, 3x3 convolution 32 -> 9,
 * plus a learned bias per grid phase P[(y mod S) * S + (x mod S)][9] added to
 * the nine logits.  Zero padding at the borders of the region it runs on.
 * Inputs, weights and activations are rounded to bfloat16 (nearest even),
 * accumulation is FP32 (matrix cores); biases and P stay FP32.
 * Parameters: one device float vector of slic_net_param_count(S) values,
 *   W1[9][32][3], b1[32], W2[9][32][32], b2[32], W3[9][9][32], b3[9],
 *   P[S*S][9],
 * with W[tap][out][in], tap = (dy + 1) * 3 + (dx + 1) weighting the input at
 * (x + dx, y + dy).  Class c of the logits names the cell (cy + c / 3 - 1,
 * cx + c % 3 - 1) around the pixel's cell (cx, cy) = (x / S, y / S),
 * clamped into the grid.
 *
 * Training works on batches of crops: crop i is the crop_w x crop_h region
 * of an image whose top-left pixel is (ox, oy); pixels beyond the image's
 * right or bottom edge are zero inputs and carry no target.  Grid phases are
 * those of the full image. */
typedef struct {
    const float* d_L;         /* planar CIELAB of the image, float[img_h * img_w] each */
    const float* d_a;
    const float* d_b;
    const int32_t* d_labels;  /* the image's converged labels (slic_net_targets only), else NULL */
    int32_t img_w, img_h;     /* image size */
    int32_t ox, oy;           /* crop origin, 0 <= ox < img_w, 0 <= oy < img_h */
} slic_net_crop;

/* Number of parameters for grid step S (1 <= S <= 32; 0 otherwise). */
int32_t slic_net_param_count(int32_t S);

/* Device workspace of the net calls below for n_crops (1..32) crops of
 * crop_w x crop_h pixels at grid step S (about 330 bytes per pixel); 0 if the
 * shape is invalid. */
size_t slic_net_workspace_bytes(int32_t n_crops, int32_t crop_w, int32_t crop_h, int32_t S);

/* Forward pass: writes d_logits float[n_crops][crop_h][crop_w][9]. */
int slic_net_forward(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                     int32_t S, const float* d_params, float* d_logits, void* hip_stream,
                     void* d_ws, size_t ws_bytes);

/* Mean softmax cross-entropy over the pixels whose target (int32[n_crops]
 * [crop_h][crop_w], class 0..8, or -1: no target) is a class, and its
 * gradient with respect to every parameter (d_grad: float[param_count],
 * overwritten; the rounded weights' gradients are passed straight through).
 * *d_loss (device double, may be NULL) receives the loss.  Deterministic:
 * partial sums per workgroup are added in a fixed order. */
int slic_net_loss_grad(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                       int32_t S, const float* d_params, const int32_t* d_target, float* d_grad,
                       double* d_loss, void* hip_stream, void* d_ws, size_t ws_bytes);

/* Training targets from each crop's d_labels (grid-indexed cluster labels):
 * the class (dy + 1) * 3 + (dx + 1) of the label's cell (cx + dx, cy + dy)
 * relative to the pixel's cell, -1 if it is not one of the nine or the
 * pixel lies outside the image.  d_target: int32[n_crops][crop_h][crop_w]. */
int slic_net_targets(const slic_net_crop* crops, int32_t n_crops, int32_t crop_w, int32_t crop_h,
                     int32_t S, int32_t* d_target, void* hip_stream);

/* One Adam step (Kingma and Ba) on count parameters: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step))
 * + eps); step >= 1 counts from 1.  d_m and d_v start at zero. */
int slic_net_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t count,
                  int32_t step, float lr, float beta1, float beta2, float eps, void* hip_stream);

/* A prepared net for inference: the bf16 weight copies in the layouts the
 * kernels read, followed by the FP32 parameters and the decode's minimum
 * confidence.  slic_net_prepared_bytes is the size of that device buffer
 * (the same for every S; it must be 256-byte aligned); slic_net_prepare
 * fills it from d_params (slic_net_param_count(S) floats, enqueued on the
 * stream).  min_confidence (finite, >= 0): only pixels whose best class
 * has softmax probability >= min_confidence vote in the first centre update
 * of a warm start (0: every pixel; above 1: none, so the first update
 * keeps the seeds); every pixel still carries its decoded label.  Prepare
 * once per parameter set, then run any number of frames with the same step
 * S: the library records the S each buffer was prepared for (per device and
 * address), and the warm-start calls reject a buffer prepared for another S,
 * or not filled by slic_net_prepare on that device, with SLIC_EINVAL.
 * SLIC_EINVAL for S outside 1..32, a negative, NaN or infinite
 * min_confidence, or a missing or misaligned buffer. */
size_t slic_net_prepared_bytes(void);
int slic_net_prepare(int32_t S, const float* d_params, float min_confidence, void* d_net,
                     void* hip_stream);

/* Warm-started segmentation.  slic_warm_init converts d_rgb, seeds the
 * centres exactly as slic_init does, runs the prepared net d_net (prepared
 * for the step S of p, 1 <= S <= 32) on the whole image in one fused kernel
 * and takes its decoded label map as the first association (in place of
 * slic_init's association with the seeds).  The context then behaves as one
 * from slic_init: slic_iterate(ctx, n) runs n rounds of (update,
 * associate), the first update using the net's labels of the pixels that
 * vote (the prepared net's minimum confidence); a cluster that no voting
 * pixel chose keeps its seed.  Workspace: slic_warm_workspace_bytes(p)
 * (equal to slic_workspace_bytes(p); 0 if S is beyond the net's range).
 * slic_warm_segment runs init, n_iters rounds, the energy (d_energy may be
 * NULL) and, with enforce, connectivity, like slic_segment.
 * Gate: the warm result is meant to replace plain SLIC only where its energy
 * is at most 1.01 times plain SLIC's; that comparison is the caller's (it
 * needs the plain energy). */
size_t slic_warm_workspace_bytes(const slic_params* p);
int slic_warm_init(slic_ctx** out, const slic_params* p, const uint8_t* d_rgb, const void* d_net,
                   void* hip_stream, void* d_ws, size_t ws_bytes);
int slic_warm_segment(const slic_params* p, const uint8_t* d_rgb, const void* d_net,
                      int32_t n_iters, int32_t enforce, int32_t* d_labels, float* d_centres,
                      double* d_energy, int32_t* d_n_segments, void* hip_stream, void* d_ws,
                      size_t ws_bytes);

/* Kernel timing for measurement.  slic_timing_enable(1) forgets earlier
 * records and starts recording: every kernel launch of the library is then
 * bracketed by HIP events on the stream it is launched on.
 * slic_timing_enable(0) stops recording and keeps the records.
 * slic_timing_read synchronises on the recorded events and returns the
 * summed duration in milliseconds and the launch count of the kernels whose
 * name starts with `kernel_prefix` (NULL: all).  Not for concurrent use from
 * several host threads. */
int slic_timing_enable(int32_t on);
int slic_timing_read(const char* kernel_prefix, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SLIC_H */
