// Track pools (lk.h): argument checks, the pool's scratch memory and the
// launches of one lifecycle step (temporal pass, carry-over, detection,
// append, cross-camera pass, commit), all on the caller's stream.
#include "lk_runtime.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

using namespace lkmi;

struct lk_pool {
    lk_context *ctx = nullptr;
    int32_t n = 0, cap = 0;
    int64_t max_pixels = 0;
    lk_detector *det = nullptr;
    lk_pool_state st{};
    lk_pool_scratch sc{};
    // pool-owned device memory: scratch arrays the caller did not give, the
    // passes' residuals, the detector's output, statistics if not given
    void *d_mem = nullptr;
    size_t bytes = 0;
    float *t_res = nullptr, *s_res = nullptr, *d_xy = nullptr;
    int32_t *d_count = nullptr, *stats = nullptr;
};

namespace {

size_t carve(size_t *off, size_t bytes)
{
    const size_t at = *off;
    *off = (at + bytes + 255) & ~size_t(255);
    return at;
}

}  // namespace

extern "C" {

lk_result lk_pool_create(lk_context *ctx, int32_t n_streams, int32_t cap, int64_t max_pixels,
                         const lk_pool_state *state, const lk_pool_scratch *scratch, lk_pool **out)
{
    if (!ctx || !state || !out) return fail(LK_ERR_INVALID_ARG, "ctx, state or out is NULL");
    *out = nullptr;
    if (n_streams < 1 || cap < 1 || cap > LK_GFTT_MAX_CORNERS || (int64_t)n_streams * cap > (int64_t(1) << 26))
        return fail(LK_ERR_INVALID_ARG, "need n_streams >= 1, cap in [1, %d], n_streams x cap <= 2^26",
                    LK_GFTT_MAX_CORNERS);
    if (!state->pts || !state->ids || !state->count || !state->next_id)
        return fail(LK_ERR_INVALID_ARG, "state: NULL pts, ids, count or next_id");
    if (scratch && (!scratch->t_pts || !scratch->t_status || !scratch->c_pts || !scratch->c_ids ||
                    !scratch->c_count || !scratch->s_pts || !scratch->s_status))
        return fail(LK_ERR_INVALID_ARG, "scratch: every array must be given");
    lk_pool *p = new (std::nothrow) lk_pool();
    if (!p) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->ctx = ctx;
    p->n = n_streams;
    p->cap = cap;
    p->max_pixels = max_pixels;
    p->st = *state;
    const size_t pts = (size_t)n_streams * cap;
    size_t off = 0;
    const size_t o_tres = carve(&off, pts * 4), o_sres = carve(&off, pts * 4), o_dxy = carve(&off, pts * 8);
    const size_t o_dcnt = carve(&off, (size_t)n_streams * 4), o_stats = carve(&off, (size_t)n_streams * 16);
    size_t o_sc[7] = {0};
    if (!scratch) {
        o_sc[0] = carve(&off, pts * 8);                   // t_pts
        o_sc[1] = carve(&off, pts);                       // t_status
        o_sc[2] = carve(&off, pts * 8);                   // c_pts
        o_sc[3] = carve(&off, pts * 8);                   // c_ids
        o_sc[4] = carve(&off, (size_t)n_streams * 4);     // c_count
        o_sc[5] = carve(&off, pts * 8);                   // s_pts
        o_sc[6] = carve(&off, pts);                       // s_status
    }
    const size_t o_right = state->right ? 0 : carve(&off, pts * 8);
    if (ctx->budget && ctx->in_use.load() + off > ctx->budget) {
        delete p;
        return fail(LK_ERR_OUT_OF_MEMORY, "pool scratch of %zu bytes exceeds the context budget", off);
    }
    (void)hipSetDevice(ctx->device);
    hipError_t e = hipMalloc(&p->d_mem, off);
    if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc(pool scratch)"); }
    e = hipMemset(p->d_mem, 0, off);
    if (e != hipSuccess) { (void)hipFree(p->d_mem); delete p; return hip_fail(e, "hipMemset(pool scratch)"); }
    p->bytes = off;
    char *b = static_cast<char *>(p->d_mem);
    p->t_res = reinterpret_cast<float *>(b + o_tres);
    p->s_res = reinterpret_cast<float *>(b + o_sres);
    p->d_xy = reinterpret_cast<float *>(b + o_dxy);
    p->d_count = reinterpret_cast<int32_t *>(b + o_dcnt);
    p->stats = state->stats ? state->stats : reinterpret_cast<int32_t *>(b + o_stats);
    if (!state->right) p->st.right = reinterpret_cast<float *>(b + o_right);
    if (scratch) {
        p->sc = *scratch;
    } else {
        p->sc.t_pts = reinterpret_cast<float *>(b + o_sc[0]);
        p->sc.t_status = reinterpret_cast<uint8_t *>(b + o_sc[1]);
        p->sc.c_pts = reinterpret_cast<float *>(b + o_sc[2]);
        p->sc.c_ids = reinterpret_cast<int64_t *>(b + o_sc[3]);
        p->sc.c_count = reinterpret_cast<int32_t *>(b + o_sc[4]);
        p->sc.s_pts = reinterpret_cast<float *>(b + o_sc[5]);
        p->sc.s_status = reinterpret_cast<uint8_t *>(b + o_sc[6]);
    }
    lk_result r = lk_detector_create(ctx, n_streams, max_pixels, &p->det);
    if (r != LK_SUCCESS) { (void)hipFree(p->d_mem); delete p; return r; }
    ctx->in_use += off;
    *out = p;
    return LK_SUCCESS;
}

lk_result lk_pool_step(lk_pool *pool, const lk_pool_frame *h_frames, int32_t n_frames, const lk_params *temporal,
                       const lk_params *stereo, const lk_gftt_params *detect, lk_stream stream)
{
    if (!pool || !detect) return fail(LK_ERR_INVALID_ARG, "pool or detection parameters are NULL");
    if (n_frames < 0 || n_frames > pool->n) return fail(LK_ERR_INVALID_ARG, "n_frames %d not in [0, %d]", n_frames, pool->n);
    if (n_frames == 0) return LK_SUCCESS;
    if (!h_frames) return fail(LK_ERR_INVALID_ARG, "h_frames is NULL");
    lk_result r = check_gftt_params(detect);
    if (r != LK_SUCCESS) return r;
    if (detect->max_corners > pool->cap)
        return fail(LK_ERR_INVALID_ARG, "detect->max_corners %d exceeds the pool capacity %d", detect->max_corners,
                    pool->cap);
    const int cap = pool->cap;
    std::vector<char> seen((size_t)pool->n, 0);
    std::vector<lk_pair> tp, sp;
    std::vector<int> t_stream, s_stream;
    std::vector<GfttJob> gj(n_frames);
    std::vector<PoolJob> pj(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        const lk_pool_frame &F = h_frames[f];
        if (F.stream < 0 || F.stream >= pool->n) return fail(LK_ERR_INVALID_ARG, "frame %d: stream %d out of range", f, F.stream);
        if (seen[F.stream]) return fail(LK_ERR_INVALID_ARG, "frame %d: stream %d appears twice", f, F.stream);
        seen[F.stream] = 1;
        if (F.reserved != 0) return fail(LK_ERR_INVALID_ARG, "frame %d: reserved != 0", f);
        if (!F.next || F.next->ctx != pool->ctx || !F.next->built)
            return fail(LK_ERR_INVALID_ARG, "frame %d: next pyramid missing, of another context or never built", f);
        const int64_t so = (int64_t)F.stream * cap;
        if (F.prev) {
            if (!temporal) return fail(LK_ERR_INVALID_ARG, "frame %d: prev given without temporal parameters", f);
            r = check_pair(pool->ctx, F.prev, F.next, f);
            if (r != LK_SUCCESS) return r;
            tp.push_back(lk_pair{F.prev, F.next, so, cap, 0});
            t_stream.push_back(F.stream);
        }
        if (F.right) {
            if (!stereo) return fail(LK_ERR_INVALID_ARG, "frame %d: right given without stereo parameters", f);
            r = check_pair(pool->ctx, F.next, F.right, f);
            if (r != LK_SUCCESS) return r;
            sp.push_back(lk_pair{F.next, F.right, so, cap, 0});
            s_stream.push_back(F.stream);
        }
        const LevelDesc &L0 = F.next->desc.lv[0];
        GfttJob &G = gj[f];
        G.img = static_cast<const uint8_t *>(L0.img);
        G.w = L0.w;
        G.h = L0.h;
        G.pitch = L0.pitch;
        G.n_occupied = 0;
        G.occupied = pool->sc.c_pts + 2 * so;
        G.n_occupied_dev = pool->sc.c_count + F.stream;
        G.out_xy = pool->d_xy + 2 * so;
        G.count = pool->d_count + F.stream;
        G.response = nullptr;
        PoolJob &J = pj[f];
        J.pts = pool->st.pts + 2 * so;
        J.ids = pool->st.ids + so;
        J.right = pool->st.right + 2 * so;
        J.count = pool->st.count + F.stream;
        J.next_id = pool->st.next_id + F.stream;
        J.t_pts = pool->sc.t_pts + 2 * so;
        J.t_status = pool->sc.t_status + so;
        J.c_pts = pool->sc.c_pts + 2 * so;
        J.c_ids = pool->sc.c_ids + so;
        J.c_count = pool->sc.c_count + F.stream;
        J.d_xy = pool->d_xy + 2 * so;
        J.d_count = pool->d_count + F.stream;
        J.s_pts = pool->sc.s_pts + 2 * so;
        J.s_status = pool->sc.s_status + so;
        J.stats = pool->stats + 4 * F.stream;
        J.tracked = F.prev != nullptr;
        J.gated = F.right != nullptr;
        J.target = detect->max_corners;
        J.cap = cap;
    }
    int64_t pixels = 0;
    for (const GfttJob &G : gj) pixels += (int64_t)G.w * G.h;
    if (pixels > pool->max_pixels)      // checked here so that a rejected call enqueues nothing
        return fail(LK_ERR_INVALID_ARG, "%lld frame pixels exceed the pool's %lld", (long long)pixels,
                    (long long)pool->max_pixels);
    std::vector<BatchItem> ti, si;
    int t_storage = 0, s_storage = 0;
    long long t_total = 0, s_total = 0;
    if (!tp.empty()) {
        if (temporal->use_guess) return fail(LK_ERR_INVALID_ARG, "temporal: use_guess must be 0");
        r = plan_batch(pool->ctx, tp.data(), (int)tp.size(), temporal, &ti, &t_storage, &t_total);
        if (r != LK_SUCCESS) return r;
        for (size_t k = 0; k < ti.size(); ++k) ti[k].limit = pool->st.count + t_stream[k];
    }
    if (!sp.empty()) {
        if (stereo->use_guess) return fail(LK_ERR_INVALID_ARG, "stereo: use_guess must be 0");
        r = plan_batch(pool->ctx, sp.data(), (int)sp.size(), stereo, &si, &s_storage, &s_total);
        if (r != LK_SUCCESS) return r;
        for (size_t k = 0; k < si.size(); ++k) si[k].limit = pool->sc.c_count + s_stream[k];
    }
    (void)hipSetDevice(pool->ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one table copy: temporal items, cross-camera items, pool jobs
    const size_t o_si = (ti.size() * sizeof(BatchItem) + 255) & ~size_t(255);
    const size_t o_pj = o_si + ((si.size() * sizeof(BatchItem) + 255) & ~size_t(255));
    const size_t bytes = o_pj + pj.size() * sizeof(PoolJob);
    StagingRing::Slot *slot = nullptr;
    r = pool->ctx->staging.acquire(bytes, &slot);
    if (r != LK_SUCCESS) return r;
    char *h = static_cast<char *>(slot->host);
    if (!ti.empty()) std::memcpy(h, ti.data(), ti.size() * sizeof(BatchItem));
    if (!si.empty()) std::memcpy(h + o_si, si.data(), si.size() * sizeof(BatchItem));
    std::memcpy(h + o_pj, pj.data(), pj.size() * sizeof(PoolJob));
    const char *d = static_cast<const char *>(slot->dev);
    const PoolJob *d_pj = reinterpret_cast<const PoolJob *>(d + o_pj);
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(pool tables)");
    if (t_total > 0) {
        TrackArgs a = make_args(temporal, (int)t_total, pool->st.pts, nullptr, pool->sc.t_pts, pool->sc.t_status,
                                pool->t_res, nullptr);
        e = launch_track_batched(reinterpret_cast<const BatchItem *>(d), (int)ti.size(), (int)t_total, a, t_storage, s);
    }
    if (e == hipSuccess) e = launch_pool_carry(d_pj, n_frames, s);
    // the detector ships its own table through the next slot of the ring
    if (e == hipSuccess) {
        r = detector_enqueue(pool->det, gj, detect, s);
        if (r != LK_SUCCESS) {
            (void)hipEventRecord(slot->done, s);
            return r;
        }
        e = launch_pool_append(d_pj, n_frames, s);
    }
    if (e == hipSuccess && s_total > 0) {
        TrackArgs a = make_args(stereo, (int)s_total, pool->sc.c_pts, nullptr, pool->sc.s_pts, pool->sc.s_status,
                                pool->s_res, nullptr);
        e = launch_track_batched(reinterpret_cast<const BatchItem *>(d + o_si), (int)si.size(), (int)s_total, a,
                                 s_storage, s);
    }
    if (e == hipSuccess) e = launch_pool_commit(d_pj, n_frames, s);
    (void)hipEventRecord(slot->done, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "pool step");
}

lk_result lk_pool_reset(lk_pool *pool, lk_stream stream)
{
    if (!pool) return fail(LK_ERR_INVALID_ARG, "pool is NULL");
    (void)hipSetDevice(pool->ctx->device);
    hipError_t e = launch_pool_reset(pool->st.count, pool->st.next_id, pool->n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "pool reset");
}

lk_result lk_pool_destroy(lk_pool *pool)
{
    if (!pool) return fail(LK_ERR_INVALID_ARG, "pool is NULL");
    (void)hipSetDevice(pool->ctx->device);
    (void)hipDeviceSynchronize();
    if (pool->det) (void)lk_detector_destroy(pool->det);
    if (pool->d_mem) (void)hipFree(pool->d_mem);
    pool->ctx->in_use -= pool->bytes;
    delete pool;
    return LK_SUCCESS;
}

}  // extern "C"
