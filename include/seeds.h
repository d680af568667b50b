/*
 * seeds.h - C ABI of libseeds: SEEDS superpixel refinement on AMD Instinct
 * MI355X (gfx950).
 *
 * SEEDS (Van den Bergh, Boix, Roig, Van Gool, "SEEDS: Superpixels Extracted
 * via Energy-Driven Sampling") starts from a regular grid of superpixels
 * (Sec. 5.1) and refines it by hill climbing (Sec. 5): blocks of pixels,
 * from the largest block size down to 2x2, and then single pixels move to a
 * neighbouring superpixel when the energy E = H + gamma G grows (Sec. 4).
 * H is the colour-histogram term (eqs. eqColorSum, eqColorMain,
 * eqColorHistogram), evaluated for a move with the histogram intersection of
 * Prop. 1 (Sec. 5.3.1); G is the 3x3 boundary term (eqs. boundaryterm,
 * eqBoundaryMain), evaluated for pixel moves with Prop. 2 (Sec. 5.3.2).
 * Accepted moves update two histograms (Sec. 5.3.3).
 *
 * Schedule. Every sweep of a level visits the nine unit classes
 * c = 3 (uy mod 3) + (ux mod 3) in order; in one phase every boundary unit of
 * class c picks its best 4-neighbour label from the state at the start of the
 * phase (ties: smaller label) and moves if the gain is strictly positive.
 * Units of one class are at least three apart, so the moves of a phase never
 * touch each other's neighbourhoods. A unit may leave label k only if k stays
 * connected around it (4-connectivity, Sec. 3). The result is deterministic:
 * labels, histograms and sizes do not depend on launch shapes or timing.
 *
 * All arithmetic is integer. Counts are pixel counts; the energy changes used
 * are exact in count form (H' = sum_k sum_j h_k(j)^2,
 * G' = sum_i sum_k b_i(k)^2):
 *   pixel p of bin j, k -> n: g = (h_n(j) - h_k(j) + 1) + gamma (W_n + |K_p| - W_k)
 *     where W_x = sum over the pixels i of p's 3x3 of the count of label x in
 *     i's 3x3 patch (patches clipped to the image) and |K_p| the number of
 *     in-image pixels of p's 3x3;
 *   block l with m pixels, k -> n, rule INTERSECT (Prop. 1):
 *     move iff int(c_n, c_l) > int(c_{k\l}, c_l), normalised intersections
 *     compared exactly by cross-multiplication;
 *   block rule EXACT: g = sum_j h_l(j) (h_n(j) - h_k(j) + h_l(j)) (half the
 *     change of H'); under EXACT a block move k -> n is dropped when n is the
 *     source of another accepted block move of the same phase.
 *
 * Errors. Every call returns a seeds_status; seeds_last_error() returns a
 * thread-local description of the last failure on the calling thread.
 * SEEDS_E_INVAL is returned before any device work. After SEEDS_E_DEVICE the
 * context is poisoned: every call except seeds_destroy returns SEEDS_E_STATE.
 *
 * Threading. A context is not thread-safe; distinct contexts may be used
 * concurrently from different threads and streams.
 *
 * Streams. hip_stream is a hipStream_t (NULL = the null stream). Device work
 * is enqueued on it; calls return before it completes unless stated.
 */
#ifndef SEEDS_H
#define SEEDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct seeds_ctx seeds_ctx;

typedef enum {
    SEEDS_OK = 0,
    SEEDS_E_INVAL = -1,  /* bad argument; nothing was enqueued                 */
    SEEDS_E_NOMEM = -2,  /* device or host allocation failed                    */
    SEEDS_E_DEVICE = -3, /* a HIP call or kernel failed; the context is poisoned */
    SEEDS_E_STATE = -4   /* the context is poisoned or in the wrong state       */
} seeds_status;

typedef enum {
    SEEDS_BLOCK_INTERSECT = 0, /* Prop. 1: normalised histogram intersection   */
    SEEDS_BLOCK_EXACT = 1      /* exact change of the colour term, drop rule   */
} seeds_block_rule;

typedef struct {
    int32_t levels;           /* L in [1,8]: block sides 2^(L-1) .. 2, then pixels   */
    int32_t bins_per_channel; /* B in [1,6]: B^3 colour bins (Sec. 4.1; paper: 5)    */
    int32_t iters_per_level;  /* I >= 0: sweeps per level                            */
    int32_t gamma;            /* weight of the boundary term in [0,65536]; 0 = off   */
    int32_t block_rule;       /* seeds_block_rule                                    */
} seeds_params;

/* Parameters used by the paper's experiments where it states them (5 bins per
 * channel, gamma = 1, 3x3 patches, Sec. 6.2), with L = 4 and I = 4.           */
seeds_status seeds_default_params(seeds_params *p);

/* Superpixel grid of Sec. 5.1 without touching the device: gx columns and gy
 * rows, gx = round(sqrt(K W / H)), gy = round(K / gx) (halves round up).
 * SEEDS_E_INVAL when a superpixel would be narrower or shorter than one
 * top block of side 2^(levels-1), or when an argument is out of range.        */
seeds_status seeds_grid(int32_t H, int32_t W, int32_t num_superpixels, int32_t levels,
                        int32_t *gx, int32_t *gy);

/* Create a context for one H x W image and initialise it (Sec. 5.1):
 * quantise the image into B^3 bins, lay the gx x gy grid over the top
 * blocks, build every superpixel's colour histogram and size.
 *   rgb             device pointer to H rows of W interleaved R,G,B bytes;
 *                   row r starts at rgb + r * row_pitch_bytes (>= 3 W). Read in
 *                   stream order; the caller keeps it alive until then.
 *   num_superpixels requested K; the grid gives K_eff = gx * gy.
 * Limits: H, W >= 1, H * W < 2^23, 2^(levels-1) <= min(H, W).
 * The context owns all device memory it allocates (freed by seeds_destroy).   */
seeds_status seeds_init(seeds_ctx **out, const uint8_t *rgb, int32_t H, int32_t W,
                        int64_t row_pitch_bytes, int32_t num_superpixels,
                        const seeds_params *p, void *hip_stream);

/* Re-initialise an existing single-image context from a new image of the same
 * size and parameters (no allocation): quantise, grid, histograms, schedule
 * reset. A batch context takes seeds_batch_reinit.                            */
seeds_status seeds_reinit(seeds_ctx *ctx, const uint8_t *rgb, int64_t row_pitch_bytes,
                          void *hip_stream);

/* Run the refinement schedule (Sec. 5.2): on a freshly initialised context,
 * every block level from side 2^(L-1) down to 2 and then the pixel level, I
 * sweeps each; on a context that has finished it, I more pixel-level sweeps.  */
seeds_status seeds_refine(seeds_ctx *ctx, void *hip_stream);

/* Run at most max_phases phases of the schedule (max_phases < 0: all); the
 * state may stop at a block level, which is a valid partition (Sec. 5.4).
 * *phases_done (may be NULL) receives the number of phases enqueued.          */
seeds_status seeds_refine_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *phases_done,
                                 void *hip_stream);

/* Write the H x W int32 labels (row-major, values in [0, K_eff)) to out.
 * out_is_host = 0: out is a device pointer, the copy is enqueued on the stream.
 * out_is_host = 1: out is host memory; the call waits for the stream.         */
seeds_status seeds_labels(const seeds_ctx *ctx, int32_t *out, int32_t out_is_host,
                          void *hip_stream);

/* K_eff = gx * gy of the context (or -1 for NULL). */
int32_t seeds_num_superpixels(const seeds_ctx *ctx);

/* Test hook: colour histograms (K_eff x B^3 int32, row-major) and sizes
 * (K_eff int32) as pixel counts. Either pointer may be NULL. Same out_is_host
 * convention as seeds_labels.                                                 */
seeds_status seeds_histograms(const seeds_ctx *ctx, int32_t *hist, int32_t *size,
                              int32_t out_is_host, void *hip_stream);

/* Test hook: current level of the context (0 = pixel level) or -1 for NULL.   */
int32_t seeds_level(const seeds_ctx *ctx);

/* Test hook: the energies of the current state in count form (Sec. 4), as
 * exact 64-bit integers written to host memory:
 *   *h_energy = H' = sum_k sum_j h_k(j)^2 over the colour histograms;
 *   *g_energy = G' = sum_i sum_k b_i(k)^2, b_i(k) the number of pixels of
 *               label k in the 3x3 patch around pixel i (clipped at the image
 *               border), on the pixel labels seeds_labels would return.
 * Hill climbing with the exact block rule never lowers H' at block levels,
 * nor H' + gamma G' at pixel level. SEEDS_E_INVAL for NULL outputs; the call
 * waits for the stream (no allocation: it uses the context's own memory).   */
seeds_status seeds_energy(const seeds_ctx *ctx, int64_t *h_energy, int64_t *g_energy,
                          void *hip_stream);

/* Test hook: the boundary units of every image of the context (Sec. 5.2: a
 * block, or at pixel level a pixel, whose 4-neighbourhood in the image holds
 * another label; only these units are proposed for a move, and only their
 * colour bins are read to decide). Counted on the unit grid of `level`:
 * level = -1 is each image's current level; level in [0, seeds_level(ctx)]
 * is min(level, L - 1) of each image, with the labels its units inherit from
 * the current grid (as after the level transitions that precede the next
 * phase at that level). For class cls in [0,8] (units with
 * 3 (uy mod 3) + (ux mod 3) = cls) or every class (cls = -1), units[i] and
 * pixels[i] (host arrays of seeds_batch_count entries; either may be NULL)
 * receive image i's boundary units and the image pixels they cover. Waits
 * for the stream; no allocation.                                            */
seeds_status seeds_boundary_units(const seeds_ctx *ctx, int32_t level, int32_t cls,
                                  int64_t *units, int64_t *pixels, void *hip_stream);

/* ---- Snapshots -----------------------------------------------------------
 * The refinement can be stopped after any phase and resumed later (Sec. 5.4:
 * the partition is valid at every step). A snapshot holds the whole state of
 * a context between calls: every image's colour bins, its labels on the unit
 * grid of its current level, its colour histograms and sizes, and the
 * schedule cursor (level, sweep, class). Restored into a context created for
 * images of the same sizes, K, levels and parameters (seeds_init or
 * seeds_batch_init, any pixels), the context continues exactly as the
 * original would have: labels, histograms and sizes bit for bit.
 * seeds_snapshot_size gives the bytes the current state needs (it depends on
 * the level). seeds_snapshot writes them to host memory `host` of `bytes`
 * bytes (SEEDS_E_INVAL if too small) and waits for the stream; seeds_restore
 * reads them back (SEEDS_E_INVAL, before any device work, for a buffer that
 * is not a snapshot of a matching context) and waits for the stream. A
 * snapshot is native-endian and tied to this library version.             */
seeds_status seeds_snapshot_size(const seeds_ctx *ctx, int64_t *bytes);
seeds_status seeds_snapshot(const seeds_ctx *ctx, void *host, int64_t bytes, void *hip_stream);
seeds_status seeds_restore(seeds_ctx *ctx, const void *host, int64_t bytes, void *hip_stream);

typedef enum {
    SEEDS_LAUNCH_GRAPH = 0,      /* default: one kernel per phase, the launches of a
                                    whole refine call captured once into a HIP
                                    graph and replayed (partial runs launch
                                    directly)                                     */
    SEEDS_LAUNCH_STEPS = 1,      /* the same kernels, launched one by one         */
    SEEDS_LAUNCH_PERSISTENT = 2  /* one cooperative launch per refine call with
                                    grid-wide barriers between phases             */
} seeds_launch_mode;

/* Choose how later refine calls are launched. Results are identical in all
 * modes; the mode only changes the launch structure. SEEDS_LAUNCH_PERSISTENT
 * is for single-image contexts (SEEDS_E_INVAL on a batch).                   */
seeds_status seeds_set_launch_mode(seeds_ctx *ctx, int32_t mode);

/* ---- Tuning ---------------------------------------------------------------
 * How the launches map work to workgroups. The choice never changes a
 * result: labels, histograms and sizes are the same for every setting.
 *   pixel_compaction  1: pixel phases first test every pixel of the class
 *                     cheaply and pack the movable ones into dense wavefronts
 *                     for the full decision; 0: every thread decides its own
 *                     pixel (more arithmetic, one dependent round of loads
 *                     less).
 *   xcd_remap         1: workgroups are numbered so that each of the eight
 *                     XCDs works a contiguous band of the image (fewer L2
 *                     misses); 0: hardware order.
 *   items_per_group   1, 2 or 4: work items (a 64 x 4 tile of class pixels,
 *                     or one round of class blocks) each workgroup of a
 *                     phase launch takes; more items mean fewer, longer
 *                     workgroups.
 *   init_rows         8, 16 or 32: rows of the 64-column tiles of the
 *                     initialisation kernel (2, 4 or 8 pixels per thread).
 *   warm_rows         8, 16 or 32: the same for the warm-start kernel.
 *   block_ppl         1 or 4: pixels of a block each lane holds in the block
 *                     phases of block sides 2, 4 and 8 (1: 4, 16 and 64
 *                     lanes per block; 4: 1, 4 and 16 lanes, so a wavefront
 *                     decides four times as many blocks at once). Larger
 *                     blocks always take 64 lanes. In a batch with
 *                     block_ppl 4 and items_per_group > 1, the block phases'
 *                     per-workgroup delta tables are four times larger.
 * Default: pixel_compaction 0, xcd_remap 1, items_per_group 1, init_rows 16,
 * warm_rows 16, block_ppl 1.                                                */
typedef struct {
    int32_t pixel_compaction;
    int32_t xcd_remap;
    int32_t items_per_group;
    int32_t init_rows;
    int32_t warm_rows;
    int32_t block_ppl;
} seeds_tuning;

seeds_status seeds_get_tuning(const seeds_ctx *ctx, seeds_tuning *out);
seeds_status seeds_set_tuning(seeds_ctx *ctx, const seeds_tuning *t);

/* Autotuner. First the phase mapping: every combination of pixel_compaction,
 * xcd_remap and items_per_group (12 variants, block_ppl 1) is timed on whole
 * refinements of the context's own images (reps runs after one warm-up that
 * captures the graph; median). Then block_ppl 4 with each items_per_group and
 * the compaction and remap of the fastest so far (3 variants); the fastest of
 * the 15 is kept. Then init_rows (3 variants), timed on initialisations, and
 * warm_rows (3 variants), timed on warm starts of the same images after one
 * refinement. The context is re-initialised at the end, so it returns freshly
 * initialised (as after seeds_reinit); the call waits for the stream.
 * *chosen and ms_per_variant[SEEDS_TUNE_VARIANTS] (either may be NULL)
 * receive the choice and the medians: entry v < 12 is the mapping with
 * items_per_group = 1, 2, 4 for v / 4 = 0, 1, 2 and, within,
 * v % 4 = 2 (1 - xcd_remap) + (1 - pixel_compaction); entry 12 + i block_ppl
 * 4 with items_per_group 1, 2, 4 for i = 0, 1, 2; entry 15 + r the
 * initialisation and entry 18 + r the warm start with 8, 16, 32 rows for
 * r = 0, 1, 2. Not for SEEDS_LAUNCH_PERSISTENT; reps in [1,50].              */
#define SEEDS_TUNE_VARIANTS 21
seeds_status seeds_autotune(seeds_ctx *ctx, int32_t reps, seeds_tuning *chosen,
                            float *ms_per_variant, void *hip_stream);

/* Wait for the stream and report device-side failures of earlier refine
 * calls (a grid barrier that timed out, an overflowing move log) as
 * SEEDS_E_DEVICE. seeds_labels and seeds_histograms with host outputs do the
 * same check.                                                                */
seeds_status seeds_sync(seeds_ctx *ctx, void *hip_stream);

/* ---- Streams ------------------------------------------------------------
 * Warm start for the next frame of a video stream (the paper names video as
 * an input the framework adapts to, Sec. 7, and its refinement can stop and
 * resume at any time, Sec. 5.4). The context keeps the previous frame's pixel
 * labels; the call bins the new frame (Sec. 4.1), recounts every
 * superpixel's colour histogram and size from those labels (eq.
 * eqColorHistogram) and marks the schedule finished, so that the next
 * seeds_refine runs I pixel-level sweeps on the new frame.
 *   rgb, row_pitch_bytes  as for seeds_init (same H and W as the context);
 *                         read in stream order.
 * SEEDS_E_STATE unless the labels are at pixel level (refine the first frame
 * to the end first). No allocation.                                          */
seeds_status seeds_warm_start(seeds_ctx *ctx, const uint8_t *rgb, int64_t row_pitch_bytes,
                              void *hip_stream);

/* ---- Batches ------------------------------------------------------------
 * A batch context refines several independent images together: each image
 * gets exactly the labels, histograms and sizes that a single-image context
 * would give it (the method treats every image on its own, Sec. 5), and one
 * launch per phase serves all of them. Images may differ in size, K and
 * levels; bins, sweeps, gamma and the block rule are shared. The schedules
 * are aligned at their end: with Lmax the most levels of any image, the
 * batch walks the levels Lmax-1 .. 0 and an image of L levels takes part from
 * level L-1 down. seeds_refine, seeds_refine_phases, seeds_set_launch_mode
 * (graph and steps modes) and seeds_sync work on batches as on single images;
 * seeds_level reports the batch's level (an image with fewer levels is at
 * min(that, levels - 1)). The single-image calls seeds_labels,
 * seeds_histograms and seeds_num_superpixels refer to image 0.              */
#define SEEDS_MAX_BATCH 4096

typedef struct {
    const uint8_t *rgb;      /* device pointer, as for seeds_init                    */
    int32_t height, width;   /* H, W                                                 */
    int64_t row_pitch_bytes; /* >= 3 W                                               */
    int32_t num_superpixels; /* requested K                                          */
    int32_t levels;          /* L of this image, in [1,8]                            */
} seeds_image;

/* Create a batch context for count (1 .. SEEDS_MAX_BATCH) images and
 * initialise every image (Sec. 5.1). p supplies bins, sweeps, gamma and the
 * block rule (p->levels is ignored: each image has its own). Each image must
 * satisfy the limits of seeds_init, and the state of the whole batch must
 * stay below 2^31 cells: per image K_eff (hs + 1) rounded up to a multiple of
 * 64, where hs is B^3 rounded up to a multiple of 8. An image that fails a
 * check names its index in the error text. The call waits for the stream
 * once (the batch tables are uploaded).                                      */
seeds_status seeds_batch_init(seeds_ctx **out, const seeds_image *images, int32_t count,
                              const seeds_params *p, void *hip_stream);

/* Re-initialise every image of the context from new pixels of the same sizes:
 * rgb[i] and row_pitch_bytes[i] (host arrays of seeds_batch_count entries).
 * When a pointer or pitch differs from the previous call the call waits for
 * the stream before uploading the new table; with unchanged pointers it
 * enqueues only.                                                             */
seeds_status seeds_batch_reinit(seeds_ctx *ctx, const uint8_t *const *rgb,
                                const int64_t *row_pitch_bytes, void *hip_stream);

/* seeds_warm_start for every image of a batch context: rgb[i] and
 * row_pitch_bytes[i] as for seeds_batch_reinit (waits for the stream when a
 * pointer or pitch changed).                                                 */
seeds_status seeds_batch_warm_start(seeds_ctx *ctx, const uint8_t *const *rgb,
                                    const int64_t *row_pitch_bytes, void *hip_stream);

/* Number of images of the context (1 for seeds_init contexts; -1 for NULL). */
int32_t seeds_batch_count(const seeds_ctx *ctx);

/* seeds_labels, seeds_histograms, seeds_num_superpixels and seeds_energy for
 * image `image` of the context (SEEDS_E_INVAL, or -1, when the index is out of
 * range).                                                                    */
seeds_status seeds_batch_labels(const seeds_ctx *ctx, int32_t image, int32_t *out,
                                int32_t out_is_host, void *hip_stream);
seeds_status seeds_batch_histograms(const seeds_ctx *ctx, int32_t image, int32_t *hist,
                                    int32_t *size, int32_t out_is_host, void *hip_stream);
int32_t seeds_batch_num_superpixels(const seeds_ctx *ctx, int32_t image);

/* seeds_batch_labels to device memory for every image of the context at
 * once: outs is a host array of seeds_batch_count(ctx) device pointers,
 * outs[i] receiving image i's H_i x W_i int32 labels (row-major), written in
 * stream order without waiting. Images whose labels are 16-bit pixel labels
 * are converted together, up to 64 per launch; any other image takes its own
 * copy. SEEDS_E_INVAL (before any device work) for a NULL ctx, outs or
 * outs[i]; SEEDS_E_DEVICE if a launch fails (the context is then
 * poisoned, as for seeds_batch_labels).                                      */
seeds_status seeds_batch_labels_all(const seeds_ctx *ctx, int32_t *const *outs,
                                    void *hip_stream);
seeds_status seeds_batch_energy(const seeds_ctx *ctx, int32_t image, int64_t *h_energy,
                                int64_t *g_energy, void *hip_stream);

/* ---- Serving -------------------------------------------------------------
 * A request loop with continuous batching. Requests (images on the device)
 * are submitted at any time; each seeds_server_step enqueues one tick on the
 * server's stream: the images admitted in this tick are initialised, every
 * image in flight advances by one phase of its own schedule (levels L-1 .. 0,
 * I sweeps of nine classes; an image joins at its top level while others are
 * in the middle of theirs), and the labels of images whose schedule ended are
 * written to their outputs. Requests are admitted in arrival order while the
 * device memory budget (pixels, histograms, move logs) and max_inflight
 * allow; an image's memory returns to the pool two ticks after its last
 * phase. Every result equals that of a single-image context with the same
 * parameters, bit for bit. Only the Prop. 1 block rule is served.          */
typedef struct seeds_server seeds_server;

typedef struct {
    int32_t bins_per_channel; /* B in [1,6]                                        */
    int32_t iters_per_level;  /* I >= 1                                            */
    int32_t gamma;            /* boundary-term weight, [0,65536]                  */
    int32_t max_levels;       /* largest L of any request, [1,8]                  */
    int64_t hbm_budget_bytes; /* device memory of the server, [64 MiB, 128 GiB]:
                                 60% pixels (7 B per pixel), 8% histograms, 32%
                                 move logs                                         */
    int32_t max_inflight;     /* most images refined together, [1,65536]          */
    int32_t pixel_compaction; /* launch mapping as in seeds_tuning (0 or 1)       */
    int32_t xcd_remap;        /* (0 or 1); results do not depend on either        */
    int32_t items_per_group;  /* 1, 2 or 4, as in seeds_tuning                     */
} seeds_server_params;

typedef struct {
    int64_t submitted, admitted, completed, ticks;
    int64_t queued, inflight, peak_inflight;
    int64_t bytes_in_use, peak_bytes_in_use, budget_bytes; /* pixels + histograms */
} seeds_server_stats;

/* B = 5, I = 4, gamma = 1, max_levels = 4, 4 GiB, 512 images, no pixel
 * compaction, hardware workgroup order and two work items per workgroup (the
 * mapping measured fastest for mixed request traffic).                      */
seeds_status seeds_server_default_params(seeds_server_params *p);

/* Create a server whose ticks run on hip_stream; allocates the budget once.  */
seeds_status seeds_server_create(seeds_server **out, const seeds_server_params *p,
                                 void *hip_stream);

/* Queue one request: an H x W image as for seeds_init (device pointer, kept
 * alive until its labels are reported), num_superpixels and levels
 * (<= max_levels), and where its H x W int32 labels go (out_is_host = 1:
 * host memory, which should be pinned so the copy stays asynchronous).
 * SEEDS_E_INVAL for bad arguments or an image that cannot fit the budget.
 * *request_id (may be NULL) identifies it in seeds_server_poll.             */
seeds_status seeds_server_submit(seeds_server *s, const uint8_t *rgb, int32_t H, int32_t W,
                                 int64_t row_pitch_bytes, int32_t num_superpixels,
                                 int32_t levels, int32_t *labels_out, int32_t out_is_host,
                                 int64_t *request_id);

/* Enqueue one tick (admission, initialisation, level transitions, one phase
 * of every image in flight, label outputs). The host may run up to 8 ticks
 * ahead of the device; the call waits when it is that far ahead.
 * *pending (may be NULL) receives the requests not yet finished on the host
 * side (queued, in flight, or waiting for their memory to return).          */
seeds_status seeds_server_step(seeds_server *s, int32_t *pending);

/* Report requests whose labels have been written (device work complete):
 * up to max_ids ids into done_ids, their number in *n_done. Each request is
 * reported once.                                                             */
seeds_status seeds_server_poll(seeds_server *s, int64_t *done_ids, int32_t max_ids,
                               int32_t *n_done);

/* Counters of the server (host-side bookkeeping).                            */
seeds_status seeds_server_get_stats(const seeds_server *s, seeds_server_stats *out);

/* Wait for the stream, then release the server and every request. NULL is
 * accepted.                                                                  */
seeds_status seeds_server_destroy(seeds_server *s);

/* ---- Quality metrics -----------------------------------------------------
 * UE, CUE, ASA and BR of Sec. 6.1 for a segmentation s against a ground
 * truth g, as exact integer numerators:
 *   UE  = ue / pixels,  ue  = sum_i sum_{k: s_k meets g_i} |s_k - g_i|  (eq. ue)
 *   ASA = asa / pixels, asa = sum_k max_i |s_k & g_i|
 *   CUE = cue / pixels, cue = sum_k |s_k - g_max(s_k)| (= pixels - asa)
 *   BR  = br_hits / br_total: ground-truth boundary pixels with a boundary
 *         pixel of s at Euclidean distance < eps, over all ground-truth
 *         boundary pixels. A pixel is a boundary pixel of a segmentation when
 *         one of its in-image 4-neighbours carries another segment.        */
typedef struct {
    int64_t pixels;
    int64_t ue;
    int64_t asa;
    int64_t cue;
    int64_t br_hits;
    int64_t br_total;
} seeds_quality;

/* labels, truth: device pointers to H x W int32, row-major, with values in
 * [0, num_labels) and [0, num_truth). eps in [1, 64] (the paper uses 2).
 * num_labels * num_truth <= 2^28 (the overlap table). The call allocates the
 * table in stream order, waits for the stream and writes *out (host).
 * Out-of-range values are detected on the device: the call then returns
 * SEEDS_E_INVAL after the device work (every other SEEDS_E_INVAL comes
 * before it).                                                              */
seeds_status seeds_quality_metrics(const int32_t *labels, const int32_t *truth, int32_t H,
                                   int32_t W, int32_t num_labels, int32_t num_truth, int32_t eps,
                                   seeds_quality *out, void *hip_stream);

/* ---- Allocation-free refinement -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc. One call does
 * what seeds_init, seeds_refine (the whole schedule), seeds_labels to device
 * memory and seeds_destroy do together, with the same kernels and the same
 * result, but every buffer beyond rgb and labels_out lives in a fixed device
 * array of SEEDS_NOALLOC_MAX_BYTES that the library holds on each device it
 * runs on until the process ends. The call allocates nothing (no hipMalloc,
 * no graph, no stream) and only enqueues kernels on hip_stream; it returns
 * before they complete.
 *   rgb, H, W, row_pitch_bytes, num_superpixels, p  as for seeds_init;
 *   labels_out  device pointer to H x W int32 (row-major, values in
 *               [0, K_eff)), written in stream order.
 * SEEDS_E_INVAL (before any device work) for the arguments seeds_init
 * refuses, NULL pointers, and images whose state does not fit the array
 * (a 1920 x 1080 image with 4 levels and B = 5 needs about 25 MB; the two
 * histogram copies take about 1 KB per superpixel at B = 5; the text names
 * the bytes needed). The first call on a device resolves the array's
 * address there (make it outside stream capture). Every call on a device
 * shares its one array: calls whose work overlaps on one device (other
 * threads, other streams without ordering) race and give wrong labels.
 * Device-side failures are not reported by the call.                        */
#define SEEDS_NOALLOC_MAX_BYTES (64u << 20)

seeds_status seeds_segment_noalloc(const uint8_t *rgb, int32_t H, int32_t W,
                                   int64_t row_pitch_bytes, int32_t num_superpixels,
                                   const seeds_params *p, int32_t *labels_out, void *hip_stream);

/* ---- Measurement ----------------------------------------------------------
 * LDS-atomic throughput of the current device, the secondary roof of the
 * refinement kernels: 4096 workgroups of 256 lanes each add 1024 times to
 * their own LDS word (no bank or address conflicts), timed with events on
 * hip_stream (best of three after a warm-up). *ginst_per_s receives 64-lane
 * wavefront atomic instructions per second, in units of 1e9. Allocates a
 * little device memory and waits for the stream.                          */
seeds_status seeds_lds_atomic_rate(double *ginst_per_s, void *hip_stream);

/* Latency floor of a phase launch on the current device: chains of `launches`
 * launches (a HIP graph on a private stream, best of three replays after a
 * warm-up) with the shape of one phase launch, `groups` workgroups of 256
 * lanes, doing us[0] nothing, us[1] one round of coalesced loads (fourteen
 * 2-byte loads per lane, 7 KB per workgroup, like a pixel tile's window),
 * us[2] that round, then five dependent loads per lane from a 512 KB table
 * (the histogram cells of a decision) and a few global atomics per workgroup.
 * us[0..2] receive microseconds per launch. groups in [1,65536], launches in
 * [1,4096]. Allocates device memory for the call, waits for hip_stream first
 * and for its own stream at the end.                                        */
seeds_status seeds_launch_floor(int32_t groups, int32_t launches, double *us, void *hip_stream);

/* Traffic probes: three kernels of exactly known memory traffic, for scaling
 * a profiler's byte counters (rocprofv3 FETCH_SIZE, WRITE_SIZE) to the access
 * kinds of the refinement kernels, which mostly read scattered 4-byte words
 * and add to them atomically. A buffer of `lines` 128-byte lines (a power of
 * two in [2^10, 2^22]), every int32 word 0x01010101, is touched line by line,
 * each line exactly once per kernel, in this stream order:
 *   k_probe_stream   reads the whole buffer with coalesced 16-byte loads;
 *   k_probe_scatter  reads one 4-byte word per line, the lines in a permuted
 *                    order (the 64 lanes of a wavefront hit 64 distinct lines);
 *   k_probe_atomic   adds 1 to one 4-byte word per line, same order.
 * us[0..2] receive each kernel's event-timed duration in microseconds (one
 * launch each, after an untimed one-workgroup launch of each kernel; under a
 * profiler these are dispatches 4, 5 and 6 of the call, its own durations
 * are the ones to read). Allocates the buffer for the call, waits for hip_stream,
 * and checks what each kernel summed (SEEDS_E_DEVICE on a mismatch);
 * SEEDS_E_INVAL for a NULL us or an invalid `lines`.                        */
seeds_status seeds_traffic_probe(int64_t lines, double *us, void *hip_stream);

/* Release the context and its device memory (after synchronising the stream
 * it last used). NULL is accepted.                                            */
seeds_status seeds_destroy(seeds_ctx *ctx);

/* ---- Fault injection (tests of the error paths) ---------------------------
 * Make the library's own code fail on purpose, on the host, without touching
 * the device: after `after` more operations of `kind`, the next one reports a
 * failure instead of running (after < 0 disarms; the setting is global to
 * the process and used once). SEEDS_FAULT_ALLOC: the device allocation of
 * seeds_init / seeds_batch_init / seeds_server_create fails as if out of
 * memory (SEEDS_E_NOMEM, nothing is leaked). SEEDS_FAULT_LAUNCH: a kernel
 * launch of a context (initialisation, a phase, a level transition, a warm
 * start) or of a server tick fails; the call returns SEEDS_E_DEVICE and the
 * context or server is poisoned, as after a real launch failure.            */
#define SEEDS_FAULT_ALLOC 0
#define SEEDS_FAULT_LAUNCH 1

seeds_status seeds_debug_inject_fault(int32_t kind, int32_t after);

/* Thread-local text of the last error on this thread ("" if none). */
const char *seeds_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEEDS_H */
