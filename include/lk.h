/*
 * lk.h -- C ABI of liblkmi, pyramidal Lucas-Kanade feature tracking on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation.  The paper tracks every keypoint of a frame into the next
 * frame (temporal tracking) and from the left into the right camera (the
 * cross-camera gate of Sec. V-A) with pyramidal LK optical flow (Sec. III,
 * Sec. IV).  Its front-end contract passes keypoints as a stacked N x 2 array
 * of pixel coordinates (Eq. 1, P in R^{N x 2}); LK needs keypoints only, no
 * descriptors (Sec. III-A).  The paper does not define LK itself; this
 * library computes the classical pyramidal form (Bouguet), step by step:
 *
 *   1. Gaussian pyramid: level l = every second sample of level l-1 blurred
 *      by the binomial [1 4 6 4 1]/16 kernel in x and y, reflect-101 borders;
 *      level sizes (n+1)/2.  Level 0 is the 8-bit frame itself.
 *   2. Scharr gradients ([3 10 3] x [-1 0 1] / 32) on each level grid,
 *      reflect-101 borders.
 *   3. Per keypoint p, per level l from coarse to fine: template T and its
 *      gradients (Gx, Gy) sampled bilinearly on the win x win grid around
 *      c = p / 2^l (taps clamped to the level); G = sum [Gx^2 GxGy; GxGy Gy^2];
 *      the point is lost (LK_LOST_EIG) if lambda_min(G) / (win^2 255^2) is
 *      below min_eig.  Then up to max_iters Gauss-Newton steps:
 *      q = c + g + d; lost (LK_LOST_OOB) if q leaves [-h, W_l-1+h] x
 *      [-h, H_l-1+h] (h = (win-1)/2); b = sum (T - J(q + x)) (Gx, Gy);
 *      eta = G^-1 b; d += eta; stop when |eta| < eps.  Next level starts
 *      from g = 2 (g + d).
 *   4. End point q = p + g + d; lost (LK_LOST_OOB) unless q lies in the
 *      image; residual = mean |T - J(q + x)| over the level-0 window.
 *   5. Forward-backward check (fb_thresh > 0): the same pass from the next
 *      frame back to the previous one, started at q with zero initial flow;
 *      LK_LOST_FB if that pass is lost or ends farther than fb_thresh from p.
 *
 * Coordinates: pixel centres at integers, (0, 0) the centre of the top-left
 * pixel, x to the right, y down; level l coordinates are level-0 ones times
 * 2^-l.  Keypoints are float32 (x, y) pairs, N x 2, interleaved.
 *
 * Conventions of every entry point:
 *   - Ownership: the library owns context, pyramid and server objects; the
 *     caller owns every array passed in (d_* = device memory, h_* = host).
 *   - Asynchrony: lk_build_pyramid* and lk_track* only enqueue work on the
 *     given stream (a hipStream_t; NULL is the null stream) and return;
 *     outputs are valid once that stream has reached the enqueued work.
 *   - Errors: every entry point returns an lk_result.  Arguments are checked
 *     on the host before anything is enqueued; on error nothing is enqueued
 *     or written and lk_last_error() returns a message (per thread).  No C++
 *     exception crosses this interface.  A device fault is reported as
 *     LK_ERR_DEVICE by the call that observes it.
 *   - Per-point status is data, not an error: lost points still get an end
 *     point and residual, which carry no meaning.
 *   - Objects are not thread safe unless stated; distinct objects may be
 *     used from distinct threads.
 */
#ifndef LKMI_LK_H
#define LKMI_LK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LK_SUCCESS = 0,
    LK_ERR_INVALID_ARG = 1,      /* bad argument; nothing was enqueued */
    LK_ERR_OUT_OF_MEMORY = 2,    /* device or pinned allocation failed, or budget exceeded */
    LK_ERR_DEVICE = 3,           /* HIP runtime or kernel error */
    LK_ERR_BUSY = 4,             /* server: no slot or budget right now; retry later */
    LK_ERR_NOT_READY = 5,        /* server: result not complete yet */
    LK_ERR_NOT_FOUND = 6,        /* server: unknown stream or ticket */
    LK_ERR_NOT_IMPLEMENTED = 7
} lk_result;

/* Storage of pyramid levels >= 1 (level 0 is always the 8-bit frame). */
enum {
    LK_STORAGE_F32 = 0,  /* float levels; gradients computed on the fly from the levels */
    LK_STORAGE_F16 = 1   /* binary16 levels (round to nearest even) and binary16 gradients
                            (Gx, Gy) of every level, built from the stored levels: stored
                            as interleaved planes for levels >= 1; those of level 0 (exact
                            on the 8-bit frame, then rounded) are formed where they are
                            used, with the same bits; tracker arithmetic stays float32 */
};

/* Per-point status codes written to d_status (uint8). */
enum { LK_OK = 0, LK_LOST_EIG = 1, LK_LOST_OOB = 2, LK_LOST_FB = 3 };

#define LK_MAX_LEVELS 8
#define LK_MAX_WIN 31          /* largest window side the tracker kernels are built for */

typedef struct lk_context lk_context;
typedef struct lk_pyramid lk_pyramid;
typedef struct lk_server lk_server;
typedef void *lk_stream;              /* hipStream_t */

/* Tracker parameters.  Valid ranges: win odd in [3, LK_MAX_WIN]; levels in
 * [1, pyramid levels]; max_iters in [1, 1000]; eps > 0; min_eig >= 0;
 * fb_thresh >= 0 (0 disables the forward-backward check); use_guess 0 or 1.
 * Defaults (lk_params_default): 21, 3, 30, 0.01, 1e-6, 0, 0. */
typedef struct {
    int32_t win;          /* window side in pixels (odd) */
    int32_t levels;       /* pyramid levels used, counted from level 0 */
    int32_t max_iters;    /* Gauss-Newton iterations per level */
    int32_t use_guess;    /* 1: d_guess holds initial end-point guesses */
    float eps;            /* stop when |eta| < eps (level pixels) */
    float min_eig;        /* LK_LOST_EIG threshold on lambda_min / (win^2 * 255^2) */
    float fb_thresh;      /* forward-backward threshold in level-0 pixels, 0 = off */
    int32_t reserved;     /* must be 0 */
} lk_params;

lk_params lk_params_default(void);

/* Checks params against the ranges above for pyramids of pyr_levels levels
 * (1..LK_MAX_LEVELS): LK_SUCCESS, or LK_ERR_INVALID_ARG with the reason in
 * lk_last_error().  Every entry point that takes lk_params applies the same
 * check before it enqueues anything; this one needs no device. */
lk_result lk_params_check(const lk_params *params, int32_t pyr_levels);

/* Human-readable message of the last failed call on this thread ("" if none). */
const char *lk_last_error(void);

/* ---- context ------------------------------------------------------------
 * A context binds the library to one device and accounts the device memory
 * it allocates against hbm_budget_bytes (0 = no limit).  The device becomes
 * current on the calling thread. */
lk_result lk_context_create(int32_t device, uint64_t hbm_budget_bytes, lk_context **out);
void lk_context_destroy(lk_context *ctx);           /* waits for the device; NULL is a no-op */
/* Device bytes currently held by objects of this context. */
uint64_t lk_context_bytes_in_use(const lk_context *ctx);

/* ---- pyramids (steps 1-2) -------------------------------------------------
 * lk_pyramid_create allocates the levels >= 1 of a w x h frame (and, for
 * LK_STORAGE_F16, their gradient planes) in one device allocation.  Level 0 is
 * not copied: lk_build_pyramid records d_img (8-bit, row pitch in bytes,
 * pitch >= w) and reads it during the build and during every later
 * lk_track* that uses the pyramid, so the caller keeps that buffer valid and
 * unchanged until such work has completed.  The coarsest level must be at
 * least 4 x 4 pixels (else LK_ERR_INVALID_ARG).  lk_pyramid_destroy frees the
 * memory; the caller first makes sure no enqueued work still uses it. */
lk_result lk_pyramid_create(lk_context *ctx, int32_t w, int32_t h, int32_t levels, int32_t storage,
                            lk_pyramid **out);
lk_result lk_pyramid_destroy(lk_pyramid *pyr);
lk_result lk_pyramid_info(const lk_pyramid *pyr, int32_t *w, int32_t *h, int32_t *levels,
                          int32_t *storage);
lk_result lk_build_pyramid(lk_context *ctx, lk_pyramid *pyr, const uint8_t *d_img, int32_t pitch,
                           lk_stream stream);
/* Builds n pyramids in one launch per level (the frames may differ in size,
 * level count and storage).  h_pyrs, h_imgs, h_pitches are host arrays of n. */
lk_result lk_build_pyramids(lk_context *ctx, lk_pyramid *const *h_pyrs, const uint8_t *const *h_imgs,
                            const int32_t *h_pitches, int32_t n, lk_stream stream);
/* Copies level l (0 <= l < levels; level 0 is the 8-bit frame of the last
 * build, which must still exist) into d_dst as float32, row-major, width W_l
 * (diagnostics and tests).  For LK_STORAGE_F16 pyramids, d_grad (nullable)
 * receives the level's float32 (Gx, Gy) pairs, 2 W_l floats per row. */
lk_result lk_pyramid_read_level(lk_context *ctx, const lk_pyramid *pyr, int32_t level, float *d_dst,
                                float *d_grad, lk_stream stream);

/* ---- tracking (steps 3-5) -------------------------------------------------
 * Tracks n points (d_pts: float32 N x 2) from pyramid prev into pyramid next
 * (same size, same storage, at least params->levels levels).  d_guess
 * (float32 N x 2) is read only when params->use_guess is 1.  Outputs:
 * d_out_pts (float32 N x 2), d_status (uint8 N), d_residual (float32 N, gray
 * levels), and, if d_iters is not NULL, per-point iteration counts (int32
 * N x 2 x params->levels: forward levels 0..L-1, then backward levels).
 * Points outside the frame or not finite are LK_LOST_OOB.  n == 0 is valid
 * and enqueues nothing. */
lk_result lk_track(lk_context *ctx, const lk_pyramid *prev, const lk_pyramid *next, const float *d_pts,
                   const float *d_guess, int32_t n, const lk_params *params, float *d_out_pts,
                   uint8_t *d_status, float *d_residual, int32_t *d_iters, lk_stream stream);

/* Many independent pairs in one launch.  Item i tracks points
 * [pt_offset, pt_offset + n) of the concatenated arrays from prev into next;
 * items may differ in frame size and point count but share params.  Every
 * result is bit-identical to the lk_track call of the same item. */
typedef struct {
    const lk_pyramid *prev;
    const lk_pyramid *next;
    int64_t pt_offset;
    int32_t n;
    int32_t reserved;     /* must be 0 */
} lk_pair;

lk_result lk_track_batched(lk_context *ctx, const lk_pair *h_pairs, int32_t n_pairs, const float *d_pts,
                           const float *d_guess, const lk_params *params, float *d_out_pts,
                           uint8_t *d_status, float *d_residual, int32_t *d_iters, lk_stream stream);

/* lk_track_batched for callers that cannot allocate memory during the call
 * (serving loops and harnesses that forbid hipMalloc): same arguments, same
 * kernels, same results bit for bit, but the call allocates nothing.  The
 * batch table (one entry per pair) goes into a fixed device array of the
 * library, LK_NOALLOC_MAX_PAIRS entries (160 KiB), one per GPU, held from the
 * first lk_context_create on that GPU until the process ends, and is copied
 * there from a pinned host table the context allocated at creation.
 * n_pairs > LK_NOALLOC_MAX_PAIRS: LK_ERR_INVALID_ARG, nothing enqueued.
 * Every call on one GPU shares that array and keeps the last call's table:
 * calls on one GPU that can overlap on the device (different streams without
 * ordering between them, or several contexts or threads) race; order them on
 * one stream.  The host waits until the same context's previous table upload
 * has ended before it rewrites the pinned table. */
#define LK_NOALLOC_MAX_PAIRS 4096
lk_result lk_track_batched_noalloc(lk_context *ctx, const lk_pair *h_pairs, int32_t n_pairs, const float *d_pts,
                                   const float *d_guess, const lk_params *params, float *d_out_pts,
                                   uint8_t *d_status, float *d_residual, int32_t *d_iters, lk_stream stream);

/* ---- prepared batched steps (hipGraph, persistent launch, autotuner) ------
 * A prepared step rebuilds the pyramids of n_builds frames (one launch per
 * level for all of them) and then tracks every pair of n_pairs in one
 * tracker launch -- the steady state of many camera streams, where each
 * stream's previous pyramid stays resident and only its new frame is built.
 * All pointers and shapes are fixed at creation; the job tables live in
 * device memory, so lk_batch_run enqueues no copies.  Results are
 * bit-identical to lk_build_pyramid + lk_track of each pair.
 *
 * Execution shapes (lk_exec_config) change speed, never results:
 *   persistent = 0: one wavefront per keypoint, hardware dispatch;
 *   persistent = 1: a grid of blocks_per_cu workgroups per compute unit,
 *     each wavefront taking keypoints from per-XCD work counters (and
 *     stealing from other XCDs when its own range is done);
 *   use_graph = 1: the whole step is recorded into a HIP graph at creation
 *     (and after lk_batch_tune) and replayed by lk_batch_run.
 *   waves_per_group (hardware dispatch): wavefronts per workgroup;
 *   chunk (persistent grid): keypoints per work fetch.
 * lk_batch_tune times every candidate shape on this batch (after about 20 ms
 * of untimed steps that bring the device to its steady clock; reps launches
 * each, HIP events), keeps the fastest and returns it.  Creation and tuning
 * synchronize the device; lk_batch_run does not. */
typedef struct {
    int32_t n_builds;
    lk_pyramid *const *build_pyrs;     /* host array of n_builds pyramids to rebuild */
    const uint8_t *const *build_imgs;  /* host array of their 8-bit frames (device pointers) */
    const int32_t *build_pitches;      /* host array of row pitches in bytes */
    int32_t n_pairs;
    const lk_pair *pairs;              /* host array of n_pairs pairs */
    const float *d_pts;
    const float *d_guess;
    lk_params params;
    float *d_out_pts;
    uint8_t *d_status;
    float *d_residual;
    int32_t *d_iters;                  /* nullable */
} lk_batch_desc;

typedef struct {
    int32_t persistent;                /* 0: hardware dispatch; 1: persistent grid */
    int32_t blocks_per_cu;             /* persistent grid: workgroups per compute unit, 1..64 */
    int32_t use_graph;                 /* 1: the step is recorded into a HIP graph and replayed */
    int32_t chunk;                     /* persistent grid: keypoints a wavefront takes per fetch,
                                          1..1024 (0: 16) */
    int32_t waves_per_group;           /* hardware dispatch: wavefronts per workgroup, 0 (the
                                          layout's default) or, for win 21 only, 1, 2 or 4 */
    int32_t reserved;                  /* must be 0 */
} lk_exec_config;

typedef struct lk_batch lk_batch;

lk_result lk_batch_create(lk_context *ctx, const lk_batch_desc *desc, const lk_exec_config *cfg /* NULL: defaults */,
                          lk_batch **out);
lk_result lk_batch_run(lk_batch *b, lk_stream stream);
lk_result lk_batch_tune(lk_batch *b, lk_stream stream, int32_t reps, lk_exec_config *best, float *best_ms);
lk_result lk_batch_config(const lk_batch *b, lk_exec_config *cfg);
lk_result lk_batch_destroy(lk_batch *b);   /* waits for the batch's work */

/* Table of tuned execution shapes.  lk_batch_create with cfg == NULL takes
 * the shape of the table row that matches the device's architecture (the
 * gfx name before any ':'), the batch's win, levels and storage, and the
 * buckets of its mean frame size and mean keypoint count per pair; with no
 * matching row (or no pairs) it takes {0, 0, 1, 0, 0, 0}.  The table is read
 * from the file named by the environment variable LKMI_EXEC_TABLE, else from
 * lk_exec_table.txt in the directory of the library, when a lookup first
 * sees that path (a missing file is an empty table; rows whose shape is not
 * valid for their window are skipped).  Format: one row per line,
 * "arch win levels storage res_bucket kp_bucket persistent blocks_per_cu
 * use_graph chunk waves_per_group [ms_per_step]", '#' starts a comment.
 *
 * lk_exec_buckets: res_bucket of a mean level-0 pixel count per pair (0:
 * below 400,000, 1: below 700,000, 2: below 1,500,000, 3: below 3,000,000,
 * 4: above) and kp_bucket of a mean keypoint count per pair (0: below 256,
 * 1: below 512, 2: below 1024, 3: below 2048, 4: above).  Host only.
 * lk_exec_table_lookup: the shape lk_batch_create(cfg = NULL) would take for
 * desc, *found = 1 if a table row matched. */
lk_result lk_exec_buckets(int64_t mean_pixels, int32_t mean_points, int32_t *res_bucket, int32_t *kp_bucket);
lk_result lk_exec_table_lookup(lk_context *ctx, const lk_batch_desc *desc, lk_exec_config *out, int32_t *found);

/* ---- corner detection (Shi-Tomasi "good features to track") -------------
 * The paper's GFTT+LK front-end seeds and tops up its tracks with this
 * detector before LK runs (Sec. IV; the keypoint-count study of Sec. V-E).
 * The paper does not define it; the classical definition is computed, and
 * the result is exact (the corners and their order are those of the
 * definition, bit for bit):
 *   1. integer Scharr gradients ([3 10 3] x [-1 0 1], unscaled) of the 8-bit
 *      frame, reflect-101 borders;
 *   2. per pixel a = sum gx^2, b = sum gx gy, c = sum gy^2 over the
 *      (2 radius + 1)^2 block around it, reflect-101 borders (integers);
 *   3. response R = lambda_min = ((a + c) - sqrt((a - c)^2 + 4 b^2)) / 2 in
 *      binary64, one rounding per operation, in the order t = a - c, t * t,
 *      (4 b) b, their sum, its square root, (a + c) minus it, times 0.5;
 *   4. candidates: pixels at least `border` from every edge with R > 0,
 *      R > quality * max(0, max R over the frame), and R not below any of its
 *      (up to 8) in-frame neighbours;
 *   5. candidates in order of R descending, ties by raster index (y w + x)
 *      ascending, are accepted while no accepted corner and no occupied point
 *      lies at squared distance < min_dist^2 (occupied points at binary64
 *      distance from the integer pixel), until max_corners are accepted.
 * A detector owns a device workspace for up to max_frames frames and
 * max_pixels pixels per call (32.125 bytes per pixel plus 2080 per frame);
 * calls on one detector share it, so they must be ordered on one stream (or
 * by the caller).  lk_detect_corners only enqueues work (one small table copy
 * and five launches). */
#define LK_GFTT_MAX_CORNERS 4096

typedef struct {
    int32_t radius;          /* block half-size, 0..3 */
    int32_t min_dist;        /* pixels, >= 0 */
    int32_t max_corners;     /* 0..LK_GFTT_MAX_CORNERS per frame */
    int32_t border;          /* pixels excluded at every edge, >= 0 */
    double quality;          /* >= 0, finite */
} lk_gftt_params;

typedef struct {
    const uint8_t *img;      /* device, h rows of pitch bytes; w, h in [3, 32768] */
    int32_t w, h, pitch;
    int32_t n_occupied;      /* points that block their neighbourhood, >= 0 */
    const float *occupied;   /* device, n_occupied x 2 (x, y); NULL iff n_occupied == 0 */
    float *out_xy;           /* device, max_corners x 2: accepted corners in order */
    int32_t *count;          /* device, one int32: number of corners written */
    double *response;        /* device, nullable: h x w map of R (row pitch w) */
} lk_gftt_frame;

typedef struct lk_detector lk_detector;

lk_result lk_detector_create(lk_context *ctx, int32_t max_frames, int64_t max_pixels, lk_detector **out);
lk_result lk_detect_corners(lk_detector *det, const lk_gftt_frame *h_frames, int32_t n_frames,
                            const lk_gftt_params *params, lk_stream stream);
lk_result lk_detector_destroy(lk_detector *det);   /* waits for the device */

/* ---- track pools (the track lifecycle after LK) ---------------------------
 * A pool keeps, for each of n_streams camera streams, up to `cap` live tracks
 * on the device: position, 64-bit identity and, in stereo mode, the position
 * in the right camera.  One lifecycle step per frame, for any subset of the
 * streams.  Associated features keep their identity and unmatched new
 * detections start new tracks (Sec. III-C, feature matching); in stereo mode
 * only features that pass the cross-camera optical-flow check enter the
 * temporal pool, in mono mode the pool is carried over by temporal tracking
 * alone (Sec. V, the Botanic Garden discussion).  One step of stream s:
 *   1. temporal pass: its live tracks are tracked from `prev` to `next`
 *      (lk_track with the temporal parameters); with prev NULL (a first
 *      frame) there is no pass and every live track ends;
 *   2. carry-over: tracks with status LK_OK move to their end points and keep
 *      their identities, in pool order; the others end;
 *   3. top-up: corners of `next`'s level 0 (lk_detect_corners with the
 *      detection parameters and the survivors as occupied points) are
 *      appended in rank order until there are detect->max_corners candidates
 *      (none when the survivors already reach it);
 *   4. gate, when `right` is given: every candidate is tracked from `next` to
 *      `right` with the stereo parameters (forward-backward check as set) and
 *      only those with status LK_OK stay, with their right-camera positions;
 *   5. commit: admitted new candidates take the stream's next identities in
 *      order; identities start at 0 and are never reused.
 * The result is the composition of lk_track and lk_detect_corners on the same
 * inputs.  Nothing returns to the host: counts, identities and statistics are
 * read from the state arrays when the caller wants them.
 *
 * State (caller-owned device arrays, see lk_pool_state): the live tracks of
 * stream s are entries [s cap, s cap + count[s]).  count and next_id must be
 * zero before the first step (or use lk_pool_reset).  Scratch: the
 * intermediate results of a step live in pool-owned device memory, or in
 * caller arrays when lk_pool_create gets an lk_pool_scratch (then they can be
 * read after the step).  Steps on one pool must be ordered on one stream. */
typedef struct lk_pool lk_pool;

typedef struct {
    float *pts;              /* n_streams x cap x 2 (x, y) */
    int64_t *ids;            /* n_streams x cap */
    float *right;            /* n_streams x cap x 2: right-camera positions; nullable if no step is gated */
    int32_t *count;          /* n_streams: live tracks */
    int64_t *next_id;        /* n_streams: next unused identity */
    int32_t *stats;          /* n_streams x 4, nullable: of the stream's last step, the previous count,
                                the carried tracks, the new candidates, the admitted tracks */
} lk_pool_state;

typedef struct {             /* every array n_streams x cap (x 2 for positions), device */
    float *t_pts;            /* temporal pass over the previous pool: end points */
    uint8_t *t_status;       /*   and status */
    float *c_pts;            /* candidates: survivors, then new corners */
    int64_t *c_ids;          /*   identities (-1: new) */
    int32_t *c_count;        /* n_streams: candidates */
    float *s_pts;            /* gate pass over the candidates: right-camera end points */
    uint8_t *s_status;       /*   and status */
} lk_pool_scratch;

typedef struct {
    int32_t stream;               /* pool stream index, 0..n_streams-1, distinct within a call */
    int32_t reserved;             /* must be 0 */
    const lk_pyramid *prev;       /* left pyramid of frame t-1, or NULL */
    const lk_pyramid *next;       /* left pyramid of frame t; its level 0 is the detection frame */
    const lk_pyramid *right;      /* right pyramid of frame t, or NULL (no gate) */
} lk_pool_frame;

/* n_streams >= 1, cap in [1, LK_GFTT_MAX_CORNERS], n_streams x cap <= 2^26;
 * max_pixels: level-0 pixels of all frames of one step, at most (the
 * detector's workspace).  scratch: nullable. */
lk_result lk_pool_create(lk_context *ctx, int32_t n_streams, int32_t cap, int64_t max_pixels,
                         const lk_pool_state *state, const lk_pool_scratch *scratch, lk_pool **out);
/* temporal: needed when some frame has prev, stereo: when some frame has
 * right (use_guess must be 0 in both); detect->max_corners <= cap is the
 * top-up target.  Only enqueues work. */
lk_result lk_pool_step(lk_pool *pool, const lk_pool_frame *h_frames, int32_t n_frames, const lk_params *temporal,
                       const lk_params *stereo, const lk_gftt_params *detect, lk_stream stream);
/* Every stream empty, identities from 0 (enqueued). */
lk_result lk_pool_reset(lk_pool *pool, lk_stream stream);
lk_result lk_pool_destroy(lk_pool *pool);   /* waits for the device */

/* ---- epipolar check (geometric verification after LK) ---------------------
 * The paper verifies temporal correspondences geometrically: points are
 * moved to the normalized image plane with the intrinsics, an essential
 * matrix is estimated robustly and correspondences more than 1 px from their
 * epipolar line are rejected (Sec. III-C).  Computed here as
 * hypothesis-and-score over many sets (e.g. one per camera stream) at once:
 *   1. hypothesis k of a set is 8 correspondences, indices given by the
 *      caller (the random draws are inputs);
 *   2. its model is the linear eight-point estimate: E with x_q^T E x_p = 0
 *      for the 8 samples, x = K^-1 (u, v, 1), the null vector of the 8 x 9
 *      system (binary64, elimination with complete pivoting); samples that
 *      repeat an index or leave [0, n), or a system of numerical rank < 8
 *      (a pivot below 1e-10 times the largest entry), give no model;
 *   3. in pixels F = K^-T E K^-1; the error of correspondence i is the
 *      distance of q_i to the epipolar line l = F (p_i, 1); it is an inlier
 *      when that distance is at most threshold_px (binary64, decided as
 *      (q.l)^2 <= t^2 (l1^2 + l2^2) with l1^2 + l2^2 > 0);
 *   4. the best hypothesis has the most inliers (ties: the lowest index);
 *      its inlier mask and model are written.
 * Results are exact up to the rounding of the binary64 solve: a
 * correspondence can flip only when its distance is within about 1e-9 px
 * of the threshold. */
typedef struct {
    const float *p;          /* device, n x 2: positions in the earlier frame (pixels) */
    const float *q;          /* device, n x 2: positions in the later frame */
    int32_t n;               /* correspondences, >= 0 */
    int32_t h;               /* hypotheses, >= 0 */
    const int32_t *samples;  /* device, h x 8 indices into [0, n) */
    float fx, fy, cx, cy;    /* intrinsics: focal lengths (> 0) and principal point, pixels */
    int32_t *counts;         /* device, h: inliers of every hypothesis, -1 where there is no model */
    uint8_t *inliers;        /* device, n: 1 for the inliers of the best hypothesis, else 0 (nullable if n == 0) */
    int32_t *best;           /* device, 2: best hypothesis (-1: no model at all) and its inlier count */
    double *model;           /* device, 9, nullable: the best F, row-major, unit Frobenius norm (zeros: none) */
} lk_epi_set;

lk_result lk_epipolar_check(lk_context *ctx, const lk_epi_set *h_sets, int32_t n_sets, double threshold_px,
                            lk_stream stream);

/* ---- serving (continuous batching over many camera streams) --------------
 * A server owns, per camera stream, device frame buffers and two resident
 * pyramids (the previous frame's and the current one's) plus pinned host
 * staging.  Clients submit frames with their keypoints; a scheduler thread
 * forms a batch from whatever is ready whenever one of `inflight` device
 * streams is free, so frames that arrive while others are on the GPU join
 * the next launch and launches overlap on the device.  A camera stream has
 * at most one frame in flight (its previous pyramid is the dependency);
 * further frames wait in its FIFO.  The first frame of a stream only primes
 * its pyramid (its result has n = 0).  Streams are admitted while their
 * resident bytes fit the budget; otherwise lk_server_open_stream returns
 * LK_ERR_BUSY.  Results are bit-identical to lk_track on the same frames.
 * Entry points may be called from any thread. */
typedef struct {
    int32_t max_streams;          /* size of the stream table */
    int32_t max_points;           /* keypoints per frame, at most */
    int32_t levels;               /* pyramid levels kept per stream (>= params.levels) */
    int32_t storage;              /* LK_STORAGE_F32 or LK_STORAGE_F16 */
    lk_params params;             /* tracker parameters for every stream */
    int32_t max_batch;            /* frames per launch, at most */
    int32_t inflight;             /* launches (device streams) in flight, 1..8 */
    int32_t queue_depth;          /* frames per stream staged on the host (>= 1) */
    int32_t reserved;             /* must be 0 */
    uint64_t hbm_budget_bytes;    /* resident bytes of all streams (0: no limit) */
} lk_server_config;

typedef struct {
    uint64_t submit_ns;           /* host monotonic clock (CLOCK_MONOTONIC) */
    uint64_t launch_ns;           /* its batch was enqueued */
    uint64_t done_ns;             /* the scheduler saw the batch complete */
} lk_timing;

typedef struct {
    uint64_t frames;              /* frames completed */
    uint64_t batches;             /* launches completed */
    uint64_t points;              /* keypoints tracked */
    uint64_t resident_bytes;      /* device bytes held by open streams */
    int32_t open_streams;
    int32_t reserved;
} lk_server_stats;

lk_result lk_server_create(lk_context *ctx, const lk_server_config *cfg, lk_server **out);
lk_result lk_server_open_stream(lk_server *srv, int32_t w, int32_t h, uint32_t *id);
/* Copies the frame (h x pitch bytes, w used per row) and the points before
 * returning.  LK_ERR_BUSY: the stream's staging is full; poll and retry. */
lk_result lk_server_submit(lk_server *srv, uint32_t id, const uint8_t *h_frame, int32_t pitch, const float *h_pts,
                           const float *h_guess, int32_t n, uint64_t *ticket);
/* LK_SUCCESS: results copied out (n_out points) and the ticket retired;
 * LK_ERR_NOT_READY: still queued or running; LK_ERR_NOT_FOUND: unknown or
 * already retired ticket; LK_ERR_DEVICE: the batch failed. */
lk_result lk_server_poll(lk_server *srv, uint64_t ticket, float *h_out_pts, uint8_t *h_status, float *h_residual,
                         int32_t *n_out, lk_timing *timing);
/* Waits for the stream's running frame, drops its queued frames (their
 * tickets become unknown) and frees its resources. */
lk_result lk_server_close_stream(lk_server *srv, uint32_t id);
lk_result lk_server_get_stats(lk_server *srv, lk_server_stats *out);
/* Fault injection for tests of the failure path: the next n launches fail on
 * the host while staging their tables (after their frames' copies were
 * enqueued).  Their frames complete with LK_ERR_DEVICE from lk_server_poll;
 * each stream keeps its previous pyramid, so its next frame is tracked from
 * its last completed frame.  n = 0 clears it. */
lk_result lk_server_fail_next_launches(lk_server *srv, int32_t n);
void lk_server_destroy(lk_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* LKMI_LK_H */
