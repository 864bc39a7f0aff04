// Internal types shared by the host runtime and the HIP kernels of liblkmi.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstdint>

#include "lk.h"

namespace lkmi {

// One pyramid level as the kernels see it.  Level 0 is the caller's 8-bit
// frame; levels >= 1 are float (LK_STORAGE_F32) or binary16 (LK_STORAGE_F16).
// For LK_STORAGE_F16 every level also has a (Gx, Gy) binary16 plane.
struct LevelDesc {
    const void *img;
    const __half2 *grad;   // nullptr for LK_STORAGE_F32
    int32_t pitch;         // elements per row of img
    int32_t gpitch;        // half2 elements per row of grad
    int32_t w, h;
};

struct PyrDesc {
    LevelDesc lv[LK_MAX_LEVELS];
    int32_t levels;
    int32_t storage;
};

struct TrackArgs {
    int32_t win, levels, max_iters, use_guess;
    float eps, min_eig, fb_thresh;
    int32_t n;                 // points (plain launch) or total points (batched)
    const float *pts;
    const float *guess;
    float *out_pts;
    uint8_t *status;
    float *residual;
    int32_t *iters;
};

// Item of a batched launch: points [pt_offset, pt_offset + n).  The
// descriptors live in device memory (each pyramid keeps its own).
struct BatchItem {
    const PyrDesc *prev;
    const PyrDesc *next;
    int64_t pt_offset;
    int32_t n;
    int32_t first_wave;        // prefix sum of n over earlier items
    const int32_t *limit;      // nullable: only the first *limit of the n points are live (a count on the device)
};

// A descriptor to be copied to device memory (by k_write_descs, or by the
// first workgroups of the fused level-1/2 pyramid launch).
struct PyrDescWrite {
    PyrDesc *dst;
    PyrDesc desc;
};

// One pyramid step (level l-1 -> level l) of one frame, tiled.
struct DownJob {
    const void *src;
    void *dst;
    int32_t spitch, dpitch;    // elements per row
    int32_t sw, sh, dw, dh;
    int32_t src_u8;            // source is the 8-bit level 0
    int32_t dst_f16;           // destination stored as binary16
    int32_t tiles_x, tile_begin;
};

// Levels 1 and 2 of one frame from its 8-bit level 0 in one pass: each
// workgroup makes a 32 x 16 tile of level 2 and the 64 x 32 tile of level 1
// under it (level 1 with a two-pixel halo stays in LDS).
struct Pyr12Job {
    const uint8_t *src;
    void *dst1, *dst2;
    __half2 *g1;                      // binary16 storage: gradient plane of level 1 (else null)
    int32_t spitch, pitch1, pitch2;   // elements per row
    int32_t gpitch1;                  // half2 elements per row of g1
    int32_t sw, sh, w1, h1, w2, h2;
    int32_t f16;                      // levels stored as binary16
    int32_t tiles_x, tile_begin;
};

// Gradient plane of one level of one frame (LK_STORAGE_F16 only).
struct GradJob {
    const void *src;
    __half2 *dst;
    int32_t spitch, dpitch;
    int32_t w, h;
    int32_t src_u8;
    int32_t tiles_x, tile_begin;
};

// Corner detection: one local maximum of the response (key = bits of R, which
// is > 0, then the raster index).
struct GfttPeak {
    unsigned long long rbits;
    uint32_t idx;
    uint32_t pad;
};

// One frame of a detection call, with its slices of the detector workspace.
struct GfttJob {
    const uint8_t *img;
    int32_t w, h, pitch;
    int32_t tiles_x, tile_begin;
    int32_t n_occupied;
    const float *occupied;
    const int32_t *n_occupied_dev;   // nullable: the number of occupied points, read on the device
    GfttPeak *peaks;                 // local maxima with R > 0; capacity w * h
    int32_t *n_peaks;
    GfttPeak *cand;                  // capacity w * h; n_cand: the peaks above the quality threshold that no
    int32_t *n_cand;                 // occupied point blocks.  With occupied points the compaction appends
                                     // them to cand and the bucket layout writes them to peaks; without, the
                                     // bucket layout writes the marked peaks to cand.  The selection reads the
                                     // bucket layout's list and uses the other as scratch.
    unsigned long long *max_bits;    // bits of max(0, max R)
    uint32_t *hist;                  // 256 bins: the candidates by the first byte of their R bits that the
                                     // threshold and the maximum leave open (their bucket; the compaction's)
    uint32_t *cursor;                // 256 fill counters of the buckets (the bucket layout's)
    uint32_t *keep;                  // 1 bit per peak: kept by the compaction's test (written by the
                                     // compaction, 64 peaks per wavefront store; capacity w h / 32 + 4)
    float *out_xy;
    int32_t *count;
    double *response;                // nullable
};

// One stream's track pool in one lifecycle step (all pointers are that
// stream's slices of the pool's device memory).
struct PoolJob {
    float *pts;                  // cap x 2: live tracks (read by the temporal pass, rewritten by the commit)
    int64_t *ids;                // cap
    float *right;                // cap x 2: stereo positions of the live tracks
    int32_t *count;              // live tracks
    int64_t *next_id;            // next unused identity
    const float *t_pts;          // temporal pass: end points and status of the live tracks
    const uint8_t *t_status;
    float *c_pts;                // candidates: survivors, then new corners
    int64_t *c_ids;
    int32_t *c_count;
    const float *d_xy;           // detector output on the new frame and its count
    const int32_t *d_count;
    const float *s_pts;          // cross-camera pass over the candidates
    const uint8_t *s_status;
    int32_t *stats;              // previous count, carried, new candidates, admitted
    int32_t tracked;             // the temporal pass ran for this stream
    int32_t gated;               // the cross-camera pass ran for this stream
    int32_t target;              // top up to this many tracks (<= cap)
    int32_t cap;                 // entries of every per-stream array
};

// One set of the epipolar check; its hypotheses are handled by the
// workgroups [wg_begin, wg_begin + ceil(h / 64)) of the first launch.
struct EpiJob {
    const float *p, *q;
    const int32_t *samples;
    int32_t *counts;
    uint8_t *inliers;
    int32_t *best;
    double *model;
    double fx, fy, cx, cy;
    int32_t n, h;
    int32_t wg_begin, pad;
};

constexpr int kGfttTileW = 64, kGfttTileH = 16;      // response tiles, block radius 2 and 3
// Response strips of one wavefront (block radius 0 and 1): 60 columns, 32
// rows, or 64 rows for calls of at least kGfttTallPixels level-0 pixels (about
// two strips per SIMD), where the shorter walks no longer shorten the launch
// and their extra halo rows cost.
constexpr int kGfttStripW = 60, kGfttStripH = 32, kGfttStripHTall = 64;
constexpr int64_t kGfttTallPixels = int64_t(8) << 20;
// Response tile (or strip) of a detection with block radius r over `pixels`
// level-0 pixels in all.
inline void gftt_tile_shape(int r, int64_t pixels, int *tw, int *th)
{
    *tw = r <= 1 ? kGfttStripW : kGfttTileW;
    *th = r <= 1 ? (pixels >= kGfttTallPixels ? kGfttStripHTall : kGfttStripH) : kGfttTileH;
}
constexpr int kGfttWindow = 2048;             // peaks sorted per selection window
constexpr int kGfttMaxCorners = LK_GFTT_MAX_CORNERS;

// Workgroups are dealt to the 8 XCDs of the chip round-robin (block b runs on
// XCD b mod 8).  Renumbering them so that XCD x takes one contiguous range of
// work items keeps neighbouring tiles (which share halo cache lines) and the
// keypoints of one frame in one L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Tile shapes of the pyramid kernels.
constexpr int kDownTileW = 64, kDownTileH = 16;
constexpr int kGradTileW = 64, kGradTileH = 16;
constexpr int kP12TileW = 32, kP12TileH = 16;   // level-2 tile of the fused build

// Window-to-lane layouts of the tracker (see lk_kernels.hip).
enum Layout { LAYOUT_NONE = -1, LAYOUT_W21 = 0, LAYOUT_W31 = 1 };
int choose_layout(int win);

// Launchers (lk_kernels.hip).  All enqueue on `stream` and return the launch status.
hipError_t launch_downsample(const DownJob &job, hipStream_t stream);
// Batched launches: workgroup t works on tile t - job.tile_begin of job
// d_tile_job[t].
hipError_t launch_downsample_batched(const DownJob *d_jobs, const int32_t *d_tile_job, int total_tiles,
                                     hipStream_t stream);
// ddst (nullable): also writes the pyramid's device descriptor (desc).
hipError_t launch_pyr12(const Pyr12Job &job, PyrDesc *ddst, const PyrDesc &desc, hipStream_t stream);
// d_descs / n_descs: descriptor writes folded into the launch (one per
// workgroup, n_descs <= total_tiles), or nullptr / 0
hipError_t launch_pyr12_batched(const Pyr12Job *d_jobs, const int32_t *d_tile_job, int total_tiles,
                                const PyrDescWrite *d_descs, int n_descs, hipStream_t stream);
hipError_t launch_grad(const GradJob &job, hipStream_t stream);
hipError_t launch_grad_batched(const GradJob *d_jobs, const int32_t *d_tile_job, int total_tiles,
                               hipStream_t stream);
hipError_t launch_track(const PyrDesc *d_prev, const PyrDesc *d_next, int storage, const TrackArgs &a,
                        hipStream_t stream);
hipError_t launch_write_desc(PyrDesc *d_dst, const PyrDesc &src, hipStream_t stream);
hipError_t launch_write_descs(const PyrDescWrite *d_w, int n, hipStream_t stream);
// waves_per_group: wavefronts per workgroup (0: the layout's default; other
// values only where track_waves_supported says the kernel is built).
hipError_t launch_track_batched(const BatchItem *d_items, int n_items, int total_points,
                                const TrackArgs &a, int storage, hipStream_t stream, int waves_per_group = 0);
bool track_waves_supported(int win, int waves_per_group);
// Persistent tracker grid: blocks_per_cu workgroups per compute unit, each
// wavefront taking `chunk` keypoints per fetch; 8 work counters at
// d_counters, kCounterStride ints apart (zeroed by the launch itself).
constexpr int kCounterStride = 64;
constexpr int kCounterBytes = 8 * kCounterStride * 4;
hipError_t launch_track_persistent(const BatchItem *d_items, int n_items, int total_points, const TrackArgs &a,
                                   int storage, int *d_counters, int blocks_per_cu, int num_cus, int chunk,
                                   hipStream_t stream);
// Detection of every frame in d_jobs (reset, peaks, compaction, bucket layout,
// selection: five launches).
hipError_t launch_gftt(const GfttJob *d_jobs, const int32_t *d_tile_job, int njobs, int total_tiles, int tile_h,
                       int radius, int border, double quality, int min_dist, int max_corners, hipStream_t stream);
// Track-pool lifecycle kernels (lk_pool_kernels.hip), one workgroup per stream.
hipError_t launch_pool_carry(const PoolJob *d_jobs, int n, hipStream_t stream);
hipError_t launch_pool_append(const PoolJob *d_jobs, int n, hipStream_t stream);
hipError_t launch_pool_commit(const PoolJob *d_jobs, int n, hipStream_t stream);
hipError_t launch_pool_reset(int32_t *d_count, int64_t *d_next_id, int n, hipStream_t stream);
// Epipolar check of every set (lk_epipolar_kernels.hip): hypotheses, then
// the best of each set.  d_wg_job[b] is the set of workgroup b.
hipError_t launch_epipolar(const EpiJob *d_jobs, const int32_t *d_wg_job, int n_jobs, int total_wgs, double threshold,
                           hipStream_t stream);
hipError_t launch_read_level(const LevelDesc &lv, int level, int storage, float *dst, float *dgrad,
                             hipStream_t stream);

}  // namespace lkmi
