// Corner detector objects and lk_detect_corners (lk.h): argument checks,
// the per-call job table and the detector workspace.
#include "lk_runtime.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

using namespace lkmi;

struct lk_detector {
    lk_context *ctx = nullptr;
    int32_t max_frames = 0;
    int64_t max_pixels = 0;
    void *d_ws = nullptr;            // per-frame counters, maxima and histograms, then peaks, then candidates
    size_t bytes = 0;
    int32_t *d_counts = nullptr;     // n_peaks of frame f at [2 f], n_cand at [2 f + 1]
    unsigned long long *d_max = nullptr;
    uint32_t *d_hist = nullptr;      // 256 bins, then 256 bucket counters, per frame
    GfttPeak *d_peaks = nullptr;
    GfttPeak *d_cand = nullptr;
    uint32_t *d_keep = nullptr;      // 1 bit per peak
};

namespace lkmi {

lk_result check_gftt_params(const lk_gftt_params *p)
{
    if (p->radius < 0 || p->radius > 3) return fail(LK_ERR_INVALID_ARG, "radius must be in [0, 3]");
    if (p->min_dist < 0 || p->min_dist > 32767) return fail(LK_ERR_INVALID_ARG, "min_dist must be in [0, 32767]");
    if (p->max_corners < 0 || p->max_corners > LK_GFTT_MAX_CORNERS)
        return fail(LK_ERR_INVALID_ARG, "max_corners must be in [0, %d]", LK_GFTT_MAX_CORNERS);
    if (p->border < 0) return fail(LK_ERR_INVALID_ARG, "border must be >= 0");
    if (!(p->quality >= 0.0) || !std::isfinite(p->quality))
        return fail(LK_ERR_INVALID_ARG, "quality must be finite and >= 0");
    return LK_SUCCESS;
}

lk_result detector_enqueue(lk_detector *det, std::vector<GfttJob> &jobs, const lk_gftt_params *p, hipStream_t s)
{
    lk_result r = check_gftt_params(p);
    if (r != LK_SUCCESS) return r;
    const int n_frames = (int)jobs.size();
    if (n_frames > det->max_frames)
        return fail(LK_ERR_INVALID_ARG, "%d frames exceed the detector's %d", n_frames, det->max_frames);
    if (n_frames == 0) return LK_SUCCESS;
    int64_t pixels = 0;
    for (int f = 0; f < n_frames; ++f) {
        const GfttJob &J = jobs[f];
        if (J.w < 3 || J.h < 3 || J.w > 32768 || J.h > 32768)
            return fail(LK_ERR_INVALID_ARG, "frame %d: size %dx%d not in [3, 32768]^2", f, J.w, J.h);
        if (J.pitch < J.w) return fail(LK_ERR_INVALID_ARG, "frame %d: pitch < width", f);
        pixels += (int64_t)J.w * J.h;
    }
    long long tiles = 0;
    int64_t keep_words = 0;
    int tw = 0, th = 0;
    gftt_tile_shape(p->radius, pixels, &tw, &th);
    pixels = 0;
    for (int f = 0; f < n_frames; ++f) {
        GfttJob &J = jobs[f];
        J.tiles_x = (J.w + tw - 1) / tw;
        J.tile_begin = (int32_t)tiles;
        J.peaks = det->d_peaks + pixels;
        J.n_peaks = det->d_counts + 2 * f;
        J.cand = det->d_cand + pixels;
        J.n_cand = det->d_counts + 2 * f + 1;
        J.max_bits = det->d_max + f;
        J.hist = det->d_hist + 512 * (size_t)f;
        J.cursor = J.hist + 256;
        J.keep = det->d_keep + keep_words;
        keep_words += ((int64_t)J.w * J.h + 63) / 64 * 2 + 2;
        pixels += (int64_t)J.w * J.h;
        tiles += (long long)J.tiles_x * ((J.h + th - 1) / th);
    }
    if (pixels > det->max_pixels)
        return fail(LK_ERR_INVALID_ARG, "%lld pixels exceed the detector's %lld", (long long)pixels,
                    (long long)det->max_pixels);
    if (tiles > 0x7FFFFFFFLL) return fail(LK_ERR_INVALID_ARG, "too many tiles");
    (void)hipSetDevice(det->ctx->device);
    // jobs, then the job of every tile
    std::vector<int32_t> tile_job((size_t)tiles);
    for (int f = 0; f < n_frames; ++f) {
        const long long n = (long long)jobs[f].tiles_x * ((jobs[f].h + th - 1) / th);
        std::fill(tile_job.begin() + jobs[f].tile_begin, tile_job.begin() + jobs[f].tile_begin + n, f);
    }
    StagingRing::Slot *slot = nullptr;
    const size_t jbytes = (jobs.size() * sizeof(GfttJob) + 15) & ~size_t(15);
    const size_t bytes = jbytes + tile_job.size() * sizeof(int32_t);
    r = det->ctx->staging.acquire(bytes, &slot);
    if (r != LK_SUCCESS) return r;
    std::memcpy(slot->host, jobs.data(), jobs.size() * sizeof(GfttJob));
    std::memcpy(static_cast<char *>(slot->host) + jbytes, tile_job.data(), tile_job.size() * sizeof(int32_t));
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(detector jobs)");
    e = launch_gftt(static_cast<const GfttJob *>(slot->dev),
                    reinterpret_cast<const int32_t *>(static_cast<const char *>(slot->dev) + jbytes), n_frames,
                    (int)tiles, th, p->radius, p->border, p->quality, p->min_dist, p->max_corners, s);
    (void)hipEventRecord(slot->done, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "detector launch");
}

}  // namespace lkmi

extern "C" {

lk_result lk_detector_create(lk_context *ctx, int32_t max_frames, int64_t max_pixels, lk_detector **out)
{
    if (!ctx || !out) return fail(LK_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    if (max_frames < 1 || max_frames > (1 << 20)) return fail(LK_ERR_INVALID_ARG, "max_frames must be in [1, 2^20]");
    if (max_pixels < 9 || max_pixels > (int64_t(1) << 34)) return fail(LK_ERR_INVALID_ARG, "max_pixels must be in [9, 2^34]");
    const size_t cnt_bytes = ((size_t)max_frames * 2 * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t max_off = cnt_bytes;
    const size_t max_bytes = ((size_t)max_frames * sizeof(unsigned long long) + 255) & ~size_t(255);
    const size_t hist_off = max_off + max_bytes;
    const size_t hist_bytes = (size_t)max_frames * 512 * sizeof(uint32_t);
    const size_t peaks_off = hist_off + hist_bytes;
    const size_t cand_off = peaks_off + (size_t)max_pixels * sizeof(GfttPeak);
    const size_t keep_off = cand_off + (size_t)max_pixels * sizeof(GfttPeak);
    const size_t bytes = keep_off + ((size_t)max_pixels / 32 + 4 * (size_t)max_frames + 64) * sizeof(uint32_t);
    if (ctx->budget && ctx->in_use.load() + bytes > ctx->budget)
        return fail(LK_ERR_OUT_OF_MEMORY, "detector workspace of %zu bytes exceeds the context budget", bytes);
    lk_detector *d = new (std::nothrow) lk_detector();
    if (!d) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipMalloc(&d->d_ws, bytes);
    if (e != hipSuccess) { delete d; return hip_fail(e, "hipMalloc(detector workspace)"); }
    d->ctx = ctx;
    d->max_frames = max_frames;
    d->max_pixels = max_pixels;
    d->bytes = bytes;
    d->d_counts = static_cast<int32_t *>(d->d_ws);
    d->d_max = reinterpret_cast<unsigned long long *>(static_cast<char *>(d->d_ws) + max_off);
    d->d_hist = reinterpret_cast<uint32_t *>(static_cast<char *>(d->d_ws) + hist_off);
    d->d_peaks = reinterpret_cast<GfttPeak *>(static_cast<char *>(d->d_ws) + peaks_off);
    d->d_cand = reinterpret_cast<GfttPeak *>(static_cast<char *>(d->d_ws) + cand_off);
    d->d_keep = reinterpret_cast<uint32_t *>(static_cast<char *>(d->d_ws) + keep_off);
    ctx->in_use += bytes;
    *out = d;
    return LK_SUCCESS;
}

lk_result lk_detect_corners(lk_detector *det, const lk_gftt_frame *h_frames, int32_t n_frames,
                            const lk_gftt_params *p, lk_stream stream)
{
    if (!det || !p) return fail(LK_ERR_INVALID_ARG, "detector or params is NULL");
    if (n_frames < 0 || n_frames > det->max_frames)
        return fail(LK_ERR_INVALID_ARG, "n_frames %d not in [0, %d]", n_frames, det->max_frames);
    if (n_frames == 0) return LK_SUCCESS;
    if (!h_frames) return fail(LK_ERR_INVALID_ARG, "h_frames is NULL");
    std::vector<GfttJob> jobs(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        const lk_gftt_frame &F = h_frames[f];
        if (!F.img || !F.out_xy || !F.count) return fail(LK_ERR_INVALID_ARG, "frame %d: NULL img, out_xy or count", f);
        if (F.n_occupied < 0 || (F.n_occupied > 0 && !F.occupied))
            return fail(LK_ERR_INVALID_ARG, "frame %d: bad occupied points", f);
        GfttJob &J = jobs[f];
        J.img = F.img;
        J.w = F.w;
        J.h = F.h;
        J.pitch = F.pitch;
        J.n_occupied = F.n_occupied;
        J.occupied = F.occupied;
        J.out_xy = F.out_xy;
        J.count = F.count;
        J.response = F.response;
    }
    return lkmi::detector_enqueue(det, jobs, p, static_cast<hipStream_t>(stream));
}

lk_result lk_detector_destroy(lk_detector *det)
{
    if (!det) return fail(LK_ERR_INVALID_ARG, "detector is NULL");
    (void)hipSetDevice(det->ctx->device);
    (void)hipDeviceSynchronize();
    if (det->d_ws) (void)hipFree(det->d_ws);
    det->ctx->in_use -= det->bytes;
    delete det;
    return LK_SUCCESS;
}

}  // extern "C"
