// Serving loop of liblkmi (lk_server_* in lk.h): the scheduler of
// lk_sched.cpp over the device backend defined here.
//
// Per camera stream the backend keeps, resident on the device, two 8-bit
// frame buffers and two pyramids used in turn (the previous frame's and the
// current one's); keypoint inputs and outputs live in pools with one fixed
// range per stream.  One launch, enqueued on one of `inflight` device
// streams, is: host-to-device copies of its frames and points from the
// scheduler's pinned staging slots, one batched pyramid build for all its
// frames, one batched tracker launch for all its pairs, device-to-host copies
// of the results into the slots, and an event the scheduler polls.
#include "lk_runtime.h"
#include "lk_sched.h"

#include <cstring>
#include <new>
#include <vector>

using namespace lkmi;

namespace {

class DeviceBackend final : public SchedBackend {
public:
    lk_result init(lk_context *ctx, const lk_server_config &cfg);
    void release();

    lk_result stream_bytes(int w, int h, uint64_t *bytes) override;
    lk_result open_stream(int stream, int w, int h) override;
    void close_stream(int stream) override;
    void *host_alloc(size_t bytes) override;
    void host_free(void *p) override;
    lk_result enqueue(int q, const std::vector<SchedFrame> &frames, bool inject_failure) override;
    int query(int q) override;
    void drain(int q) override;
    void thread_init() override { (void)hipSetDevice(ctx_->device); }

private:
    struct DevStream {
        int w = 0, h = 0, pitch = 0;
        uint8_t *d_frame[2] = {nullptr, nullptr};
        lk_pyramid *pyr[2] = {nullptr, nullptr};
    };
    struct Queue {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        StagingRing ring;                      // tables of this device stream
    };

    lk_context *ctx_ = nullptr;
    lk_server_config cfg_{};
    // keypoint pools: stream i owns entries [i * max_points, (i + 1) * max_points)
    void *d_pool_ = nullptr;
    float *d_pts_ = nullptr, *d_guess_ = nullptr, *d_out_ = nullptr, *d_res_ = nullptr;
    uint8_t *d_status_ = nullptr;
    std::vector<DevStream> streams_;
    std::vector<Queue> queues_;
};

lk_result DeviceBackend::init(lk_context *ctx, const lk_server_config &cfg)
{
    ctx_ = ctx;
    cfg_ = cfg;
    streams_.resize(cfg.max_streams);
    queues_.resize(cfg.inflight);
    (void)hipSetDevice(ctx->device);
    const size_t n = (size_t)cfg.max_streams * cfg.max_points;
    hipError_t e = hipMalloc(&d_pool_, n * (8 * 3 + 4 + 1) + 1024);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(keypoint pools)");
    d_pts_ = static_cast<float *>(d_pool_);
    d_guess_ = d_pts_ + 2 * n;
    d_out_ = d_guess_ + 2 * n;
    d_res_ = d_out_ + 2 * n;
    d_status_ = reinterpret_cast<uint8_t *>(d_res_ + n);
    for (auto &Q : queues_) {
        e = hipStreamCreateWithFlags(&Q.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&Q.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "server stream");
        lk_result r = Q.ring.init(4);
        if (r != LK_SUCCESS) return r;
    }
    return LK_SUCCESS;
}

void DeviceBackend::release()
{
    if (!ctx_) return;
    (void)hipSetDevice(ctx_->device);
    for (auto &Q : queues_)
        if (Q.stream) (void)hipStreamSynchronize(Q.stream);
    for (int i = 0; i < (int)streams_.size(); ++i) close_stream(i);
    for (auto &Q : queues_) {
        Q.ring.release();
        if (Q.done) (void)hipEventDestroy(Q.done);
        if (Q.stream) (void)hipStreamDestroy(Q.stream);
        Q = Queue{};
    }
    if (d_pool_) (void)hipFree(d_pool_);
    d_pool_ = nullptr;
}

lk_result DeviceBackend::stream_bytes(int w, int h, uint64_t *bytes)
{
    int32_t ws[LK_MAX_LEVELS], hs[LK_MAX_LEVELS];
    if (level_dims(w, h, cfg_.levels, ws, hs) != 0)
        return fail(LK_ERR_INVALID_ARG, "bad frame size %dx%d for %d levels", w, h, cfg_.levels);
    (void)hipSetDevice(ctx_->device);
    lk_pyramid *probe = nullptr;
    lk_result r = lk_pyramid_create(ctx_, w, h, cfg_.levels, cfg_.storage, &probe);
    if (r != LK_SUCCESS) return r;
    const uint64_t pyr_bytes = probe->bytes;
    lk_pyramid_destroy(probe);
    const uint64_t pitch = ((uint64_t)w + 255) & ~uint64_t(255);
    // two frames, two pyramids, the stream's share of the point pools
    *bytes = 2 * pitch * h + 2 * pyr_bytes + (uint64_t)cfg_.max_points * (8 * 3 + 4 + 1);
    return LK_SUCCESS;
}

lk_result DeviceBackend::open_stream(int stream, int w, int h)
{
    DevStream &c = streams_[stream];
    c = DevStream{};
    c.w = w; c.h = h;
    c.pitch = (w + 255) & ~255;
    (void)hipSetDevice(ctx_->device);
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc(&c.d_frame[k], (size_t)c.pitch * h);
        if (e != hipSuccess) {
            c.d_frame[k] = nullptr;
            close_stream(stream);
            return hip_fail(e, "hipMalloc(stream)");
        }
        lk_result r = lk_pyramid_create(ctx_, w, h, cfg_.levels, cfg_.storage, &c.pyr[k]);
        if (r != LK_SUCCESS) {
            c.pyr[k] = nullptr;
            close_stream(stream);
            return r;
        }
    }
    return LK_SUCCESS;
}

void DeviceBackend::close_stream(int stream)
{
    DevStream &c = streams_[stream];
    for (int k = 0; k < 2; ++k) {
        if (c.pyr[k]) lk_pyramid_destroy(c.pyr[k]);
        if (c.d_frame[k]) (void)hipFree(c.d_frame[k]);
    }
    c = DevStream{};
}

void *DeviceBackend::host_alloc(size_t bytes)
{
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void DeviceBackend::host_free(void *p) { (void)hipHostFree(p); }

lk_result DeviceBackend::enqueue(int q, const std::vector<SchedFrame> &frames, bool inject_failure)
{
    Queue &Q = queues_[q];
    hipStream_t st = Q.stream;
    const size_t P = (size_t)cfg_.max_points;
    std::vector<lk_pyramid *> build;
    std::vector<lk_pair> pairs;
    hipError_t e = hipSuccess;
    for (const SchedFrame &f : frames) {
        DevStream &c = streams_[f.stream];
        const SchedSlot &sl = *f.slot;
        const size_t base = (size_t)f.stream * P;
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(c.d_frame[f.cur], c.pitch, sl.frame, c.w, c.w, c.h, hipMemcpyHostToDevice, st);
        c.pyr[f.cur]->desc.lv[0].img = c.d_frame[f.cur];
        c.pyr[f.cur]->desc.lv[0].pitch = c.pitch;
        build.push_back(c.pyr[f.cur]);
        if (sl.n_out > 0) {
            // a missing guess is the point itself: zero initial flow, exactly
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_pts_ + 2 * base, sl.pts, (size_t)sl.n * 8, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_guess_ + 2 * base, sl.has_guess ? sl.guess : sl.pts, (size_t)sl.n * 8,
                                   hipMemcpyHostToDevice, st);
            pairs.push_back(lk_pair{c.pyr[f.cur ^ 1], c.pyr[f.cur], (int64_t)base, sl.n_out, 0});
        }
    }
    lk_result r = LK_SUCCESS;
    // one batched pyramid build for every frame of the launch
    if (e == hipSuccess) {
        BuildTables bt;
        make_build_tables(build.data(), (int)build.size(), &bt);
        StagingRing::Slot *rs = nullptr;
        if (inject_failure)
            r = fail(LK_ERR_OUT_OF_MEMORY, "pyramid table staging failed (injected)");
        else
            r = Q.ring.acquire(bt.bytes, &rs);
        if (r == LK_SUCCESS) {
            bt.pack(static_cast<char *>(rs->host));
            e = hipMemcpyAsync(rs->dev, rs->host, bt.bytes, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = launch_build_tables(bt, static_cast<const char *>(rs->dev), st);
            (void)hipEventRecord(rs->done, st);
            for (auto *p : build) p->built = true;
        }
    }
    // one tracker launch for every stream that has a previous pyramid
    if (e == hipSuccess && r == LK_SUCCESS && !pairs.empty()) {
        lk_params prm = cfg_.params;
        prm.use_guess = 1;
        std::vector<BatchItem> items;
        int storage = 0;
        long long total = 0;
        r = plan_batch(ctx_, pairs.data(), (int)pairs.size(), &prm, &items, &storage, &total);
        StagingRing::Slot *rs = nullptr;
        if (r == LK_SUCCESS) r = Q.ring.acquire(items.size() * sizeof(BatchItem), &rs);
        if (r == LK_SUCCESS) {
            std::memcpy(rs->host, items.data(), items.size() * sizeof(BatchItem));
            e = hipMemcpyAsync(rs->dev, rs->host, items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st);
            TrackArgs a = make_args(&prm, (int)total, d_pts_, d_guess_, d_out_, d_status_, d_res_, nullptr);
            if (e == hipSuccess)
                e = launch_track_batched(static_cast<const BatchItem *>(rs->dev), (int)items.size(), (int)total, a,
                                         storage, st);
            (void)hipEventRecord(rs->done, st);
        }
    }
    for (const SchedFrame &f : frames) {
        const SchedSlot &sl = *f.slot;
        const size_t base = (size_t)f.stream * P;
        if (sl.n_out > 0 && e == hipSuccess) {
            e = hipMemcpyAsync(sl.out, d_out_ + 2 * base, (size_t)sl.n_out * 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.status, d_status_ + base, (size_t)sl.n_out, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.residual, d_res_ + base, (size_t)sl.n_out * 4, hipMemcpyDeviceToHost, st);
        }
    }
    if (e == hipSuccess && r == LK_SUCCESS) e = hipEventRecord(Q.done, st);
    if (e != hipSuccess) return hip_fail(e, "server launch");
    return r;
}

int DeviceBackend::query(int q)
{
    const hipError_t e = hipEventQuery(queues_[q].done);
    if (e == hipErrorNotReady) return 0;
    return e == hipSuccess ? 1 : -1;
}

void DeviceBackend::drain(int q) { (void)hipStreamSynchronize(queues_[q].stream); }

}  // namespace

struct lk_server {
    Sched sched;
    DeviceBackend dev;
};

extern "C" {

lk_result lk_server_create(lk_context *ctx, const lk_server_config *cfg, lk_server **out)
{
    if (!ctx || !cfg || !out) return fail(LK_ERR_INVALID_ARG, "ctx, cfg or out is NULL");
    *out = nullptr;
    const lk_server_config &c = *cfg;
    lk_result r = sched_check_config(cfg);
    if (r != LK_SUCCESS) return r;
    if (c.storage != LK_STORAGE_F32 && c.storage != LK_STORAGE_F16) return fail(LK_ERR_INVALID_ARG, "bad storage");
    if (c.levels < 1 || c.levels > LK_MAX_LEVELS) return fail(LK_ERR_INVALID_ARG, "levels out of range");
    r = check_params(&c.params, c.levels);
    if (r != LK_SUCCESS) return r;
    lk_server *s = new (std::nothrow) lk_server();
    if (!s) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    r = s->dev.init(ctx, c);
    if (r == LK_SUCCESS) r = sched_start(&s->sched, c, &s->dev);
    if (r != LK_SUCCESS) {
        lk_server_destroy(s);
        return r;
    }
    *out = s;
    return LK_SUCCESS;
}

lk_result lk_server_open_stream(lk_server *s, int32_t w, int32_t h, uint32_t *id)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_open_stream(&s->sched, w, h, id);
}

lk_result lk_server_submit(lk_server *s, uint32_t id, const uint8_t *h_frame, int32_t pitch, const float *h_pts,
                           const float *h_guess, int32_t n, uint64_t *ticket)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_submit(&s->sched, id, h_frame, pitch, h_pts, h_guess, n, ticket);
}

lk_result lk_server_poll(lk_server *s, uint64_t ticket, float *h_out_pts, uint8_t *h_status, float *h_residual,
                         int32_t *n_out, lk_timing *timing)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_poll(&s->sched, ticket, h_out_pts, h_status, h_residual, n_out, timing);
}

lk_result lk_server_close_stream(lk_server *s, uint32_t id)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_close_stream(&s->sched, id);
}

lk_result lk_server_fail_next_launches(lk_server *s, int32_t n)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_fail_next(&s->sched, n);
}

lk_result lk_server_get_stats(lk_server *s, lk_server_stats *out)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    return sched_stats(&s->sched, out);
}

void lk_server_destroy(lk_server *s)
{
    if (!s) return;
    sched_stop(&s->sched);
    s->dev.release();
    delete s;
}

}  // extern "C"
