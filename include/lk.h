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
    LK_STORAGE_F16 = 1   /* binary16 levels (round to nearest even) and binary16 gradient
                            planes (Gx, Gy interleaved) for every level, built from the
                            stored levels; tracker arithmetic stays float32 */
};

/* Per-point status codes written to d_status (uint8). */
enum { LK_OK = 0, LK_LOST_EIG = 1, LK_LOST_OOB = 2, LK_LOST_FB = 3 };

#define LK_MAX_LEVELS 8

typedef struct lk_context lk_context;
typedef struct lk_pyramid lk_pyramid;
typedef struct lk_server lk_server;
typedef void *lk_stream;              /* hipStream_t */

/* Tracker parameters.  Valid ranges: win odd in [3, 63]; levels in
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
 * LK_STORAGE_F16, the gradient planes) in one device allocation.  Level 0 is
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
/* Copies level l (l >= 1) into d_dst as float32, row-major, width W_l
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

#ifdef __cplusplus
}
#endif
#endif /* LKMI_LK_H */
