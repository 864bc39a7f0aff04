// lk_epipolar_check (lk.h): argument checks and the job tables of one call.
#include "lk_runtime.h"

#include <cmath>
#include <cstring>
#include <vector>

using namespace lkmi;

extern "C" {

lk_result lk_epipolar_check(lk_context *ctx, const lk_epi_set *h_sets, int32_t n_sets, double threshold_px,
                            lk_stream stream)
{
    if (!ctx) return fail(LK_ERR_INVALID_ARG, "ctx is NULL");
    if (n_sets < 0) return fail(LK_ERR_INVALID_ARG, "n_sets < 0");
    if (n_sets == 0) return LK_SUCCESS;
    if (!h_sets) return fail(LK_ERR_INVALID_ARG, "h_sets is NULL");
    if (!(threshold_px >= 0.0) || !std::isfinite(threshold_px))
        return fail(LK_ERR_INVALID_ARG, "threshold_px must be finite and >= 0");
    std::vector<EpiJob> jobs(n_sets);
    std::vector<int32_t> wg_job;
    for (int j = 0; j < n_sets; ++j) {
        const lk_epi_set &S = h_sets[j];
        if (S.n < 0 || S.h < 0) return fail(LK_ERR_INVALID_ARG, "set %d: negative n or h", j);
        if (S.n > 0 && (!S.p || !S.q || !S.inliers)) return fail(LK_ERR_INVALID_ARG, "set %d: NULL p, q or inliers", j);
        if (S.h > 0 && (!S.samples || !S.counts)) return fail(LK_ERR_INVALID_ARG, "set %d: NULL samples or counts", j);
        if (!S.best) return fail(LK_ERR_INVALID_ARG, "set %d: NULL best", j);
        if (!(S.fx > 0.0f) || !(S.fy > 0.0f) || !std::isfinite(S.fx) || !std::isfinite(S.fy) ||
            !std::isfinite(S.cx) || !std::isfinite(S.cy))
            return fail(LK_ERR_INVALID_ARG, "set %d: intrinsics must be finite with fx, fy > 0", j);
        EpiJob &J = jobs[j];
        J.p = S.p;
        J.q = S.q;
        J.samples = S.samples;
        J.counts = S.counts;
        J.inliers = S.inliers;
        J.best = S.best;
        J.model = S.model;
        J.fx = S.fx;
        J.fy = S.fy;
        J.cx = S.cx;
        J.cy = S.cy;
        J.n = S.n;
        J.h = S.h;
        J.wg_begin = (int32_t)wg_job.size();
        J.pad = 0;
        const long long wgs = ((long long)S.h + 63) / 64;
        if ((long long)wg_job.size() + wgs > 0x7FFFFFFFLL) return fail(LK_ERR_INVALID_ARG, "too many hypotheses");
        wg_job.insert(wg_job.end(), (size_t)wgs, j);
    }
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t jbytes = (jobs.size() * sizeof(EpiJob) + 255) & ~size_t(255);
    const size_t bytes = jbytes + wg_job.size() * sizeof(int32_t);
    StagingRing::Slot *slot = nullptr;
    lk_result r = ctx->staging.acquire(bytes, &slot);
    if (r != LK_SUCCESS) return r;
    std::memcpy(slot->host, jobs.data(), jobs.size() * sizeof(EpiJob));
    if (!wg_job.empty())
        std::memcpy(static_cast<char *>(slot->host) + jbytes, wg_job.data(), wg_job.size() * sizeof(int32_t));
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(epipolar jobs)");
    e = launch_epipolar(static_cast<const EpiJob *>(slot->dev),
                        reinterpret_cast<const int32_t *>(static_cast<const char *>(slot->dev) + jbytes), n_sets,
                        (int)wg_job.size(), threshold_px, s);
    (void)hipEventRecord(slot->done, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "epipolar check launch");
}

}  // extern "C"
