// Serving loop of liblkmi: continuous batching of frames from many camera
// streams (lk_server_* in lk.h).
//
// Per camera stream the server keeps, resident on the device, two 8-bit
// frame buffers and two pyramids used in turn (the previous frame's and the
// current one's), plus keypoint input/output arrays; on the host, a few
// pinned staging slots per stream (frame + keypoints in, results out).
//
// A scheduler thread loops: it retires launches whose completion event has
// fired (results are already in pinned memory), then, whenever one of the
// `inflight` device streams is free, it takes the head frame of every camera
// stream that has no frame in flight -- up to max_batch of them -- and
// enqueues one launch on that device stream: host-to-device copies, one
// batched pyramid build for all those frames, one batched tracker launch
// for all pairs, device-to-host copies of the results, and an event.  A
// frame that arrives while launches are running joins the next launch.
#include "lk_runtime.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include <time.h>

using namespace lkmi;

namespace {

uint64_t now_ns()
{
    timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

enum SlotState { SLOT_FREE = 0, SLOT_FILLING, SLOT_QUEUED, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED };

struct Slot {                 // pinned host staging of one frame
    uint8_t *frame = nullptr; // h x w, packed rows
    float *pts = nullptr;     // max_points x 2
    float *guess = nullptr;
    float *out = nullptr;     // results
    uint8_t *status = nullptr;
    float *residual = nullptr;
    int n = 0;
    int n_out = 0;
    bool has_guess = false;
    SlotState state = SLOT_FREE;
    uint64_t ticket = 0;
    lk_timing t{};
};

struct CamStream {
    bool open = false;
    bool closing = false;
    int w = 0, h = 0, pitch = 0;
    uint8_t *d_frame[2] = {nullptr, nullptr};
    lk_pyramid *pyr[2] = {nullptr, nullptr};
    int cur = 0;              // buffers of the next frame
    bool primed = false;      // pyr[cur ^ 1] holds the previous frame
    bool busy = false;        // a frame is in flight
    int fillers = 0;          // submits copying into a reserved slot right now
    uint32_t seq = 0;
    std::vector<Slot> slots;
    std::deque<int> fifo;     // queued slot indices
    uint64_t resident = 0;
    void *host_block = nullptr;
};

struct Launch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool failed = false;                       // some enqueue of this launch failed on the host
    std::vector<std::pair<int, int>> frames;   // (camera stream, slot)
    StagingRing ring;                          // tables of this device stream
};

}  // namespace

struct lk_server {
    lk_context *ctx = nullptr;
    lk_server_config cfg{};
    // keypoint pools: stream i owns entries [i * max_points, (i + 1) * max_points)
    void *d_pool = nullptr;
    float *d_pts = nullptr, *d_guess = nullptr, *d_out = nullptr, *d_res = nullptr;
    uint8_t *d_status = nullptr;
    std::vector<CamStream> cams;
    std::vector<Launch> launches;
    std::unordered_map<uint64_t, std::pair<int, int>> tickets;   // ticket -> (stream, slot)
    std::mutex mu;
    std::condition_variable cv;
    std::thread thread;
    bool stop = false;
    uint64_t resident = 0;
    lk_server_stats stats{};
    int fail_next = 0;        // launches whose table staging is made to fail (fault injection)
};

namespace {

size_t slot_bytes(const lk_server *s, int w, int h)
{
    const size_t P = (size_t)s->cfg.max_points;
    return (size_t)w * h + P * 8 * 3 + P + P * 4 + 64;
}

void free_stream(lk_server *s, CamStream &c)
{
    for (int k = 0; k < 2; ++k) {
        if (c.pyr[k]) lk_pyramid_destroy(c.pyr[k]);
        if (c.d_frame[k]) (void)hipFree(c.d_frame[k]);
    }
    if (c.host_block) (void)hipHostFree(c.host_block);
    s->resident -= c.resident;
    c = CamStream{};
}

// Completes launches whose event has fired.  A launch that failed on the
// host (its completion event may never have been recorded) is completed once
// the work it did enqueue has drained: its frames fail, and their streams
// keep their buffers and previous pyramid, so the next frame tracks from the
// last frame that completed.  Called with the lock held.
void retire(lk_server *s)
{
    for (auto &L : s->launches) {
        if (!L.busy) continue;
        hipError_t q;
        if (L.failed) {
            (void)hipStreamSynchronize(L.stream);   // the copies out of the pinned slots have finished
            q = hipErrorLaunchFailure;
            L.failed = false;
        } else {
            q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) continue;
        }
        const uint64_t t = now_ns();
        for (auto &fs : L.frames) {
            CamStream &c = s->cams[fs.first];
            Slot &sl = c.slots[fs.second];
            sl.state = q == hipSuccess ? SLOT_DONE : SLOT_FAILED;
            sl.t.done_ns = t;
            c.busy = false;
            if (q == hipSuccess) {
                c.primed = true;
                c.cur ^= 1;
                s->stats.frames += 1;
                s->stats.points += (uint64_t)sl.n_out;
            }
        }
        if (q == hipSuccess) s->stats.batches += 1;
        L.frames.clear();
        L.busy = false;
    }
}

// Enqueues one launch with the ready head frames.  Called with the lock held.
lk_result launch_ready(lk_server *s, Launch &L)
{
    std::vector<std::pair<int, int>> take;
    for (int i = 0; i < (int)s->cams.size() && (int)take.size() < s->cfg.max_batch; ++i) {
        CamStream &c = s->cams[i];
        if (!c.open || c.closing || c.busy || c.fifo.empty()) continue;
        take.push_back({i, c.fifo.front()});
    }
    if (take.empty()) return LK_SUCCESS;
    hipStream_t st = L.stream;
    const uint64_t t = now_ns();
    const size_t P = (size_t)s->cfg.max_points;
    std::vector<lk_pyramid *> build;
    std::vector<lk_pair> pairs;
    hipError_t e = hipSuccess;
    for (auto &fs : take) {
        CamStream &c = s->cams[fs.first];
        Slot &sl = c.slots[fs.second];
        c.fifo.pop_front();
        c.busy = true;
        sl.state = SLOT_RUNNING;
        sl.t.launch_ns = t;
        const size_t base = (size_t)fs.first * P;
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(c.d_frame[c.cur], c.pitch, sl.frame, c.w, c.w, c.h, hipMemcpyHostToDevice, st);
        c.pyr[c.cur]->desc.lv[0].img = c.d_frame[c.cur];
        c.pyr[c.cur]->desc.lv[0].pitch = c.pitch;
        build.push_back(c.pyr[c.cur]);
        sl.n_out = c.primed ? sl.n : 0;
        if (sl.n_out > 0) {
            // a missing guess is the point itself: zero initial flow, exactly
            if (e == hipSuccess) e = hipMemcpyAsync(s->d_pts + 2 * base, sl.pts, (size_t)sl.n * 8, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->d_guess + 2 * base, sl.has_guess ? sl.guess : sl.pts, (size_t)sl.n * 8,
                                   hipMemcpyHostToDevice, st);
            pairs.push_back(lk_pair{c.pyr[c.cur ^ 1], c.pyr[c.cur], (int64_t)base, sl.n_out, 0});
        }
    }
    lk_result r = LK_SUCCESS;
    // one batched pyramid build for every frame of the launch
    if (e == hipSuccess) {
        BuildTables bt;
        make_build_tables(build.data(), (int)build.size(), &bt);
        StagingRing::Slot *rs = nullptr;
        if (s->fail_next > 0) {
            --s->fail_next;
            r = fail(LK_ERR_OUT_OF_MEMORY, "pyramid table staging failed (injected)");
        } else {
            r = L.ring.acquire(bt.bytes, &rs);
        }
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
        lk_params prm = s->cfg.params;
        prm.use_guess = 1;
        std::vector<BatchItem> items;
        int storage = 0;
        long long total = 0;
        r = plan_batch(s->ctx, pairs.data(), (int)pairs.size(), &prm, &items, &storage, &total);
        StagingRing::Slot *rs = nullptr;
        if (r == LK_SUCCESS) r = L.ring.acquire(items.size() * sizeof(BatchItem), &rs);
        if (r == LK_SUCCESS) {
            std::memcpy(rs->host, items.data(), items.size() * sizeof(BatchItem));
            e = hipMemcpyAsync(rs->dev, rs->host, items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st);
            TrackArgs a = make_args(&prm, (int)total, s->d_pts, s->d_guess, s->d_out, s->d_status, s->d_res, nullptr);
            if (e == hipSuccess)
                e = launch_track_batched(static_cast<const BatchItem *>(rs->dev), (int)items.size(), (int)total, a,
                                         storage, st);
            (void)hipEventRecord(rs->done, st);
        }
    }
    for (auto &fs : take) {
        Slot &sl = s->cams[fs.first].slots[fs.second];
        const size_t base = (size_t)fs.first * P;
        if (sl.n_out > 0 && e == hipSuccess) {
            e = hipMemcpyAsync(sl.out, s->d_out + 2 * base, (size_t)sl.n_out * 8, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.status, s->d_status + base, (size_t)sl.n_out, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sl.residual, s->d_res + base, (size_t)sl.n_out * 4, hipMemcpyDeviceToHost, st);
        }
    }
    if (e == hipSuccess && r == LK_SUCCESS) e = hipEventRecord(L.done, st);
    L.frames = take;
    L.busy = true;
    L.failed = e != hipSuccess || r != LK_SUCCESS;
    if (e != hipSuccess) return hip_fail(e, "server launch");
    return r;
}

void scheduler(lk_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        retire(s);
        bool any_busy = false, launched = false;
        for (auto &L : s->launches) {
            if (!L.busy) {
                lk_result r = launch_ready(s, L);
                if (r != LK_SUCCESS) {
                    // mark what this launch took as failed; the device state is unknown
                    for (auto &fs : L.frames) s->cams[fs.first].slots[fs.second].state = SLOT_FAILED;
                }
                launched |= L.busy;
            }
            any_busy |= L.busy;
        }
        s->cv.notify_all();
        if (any_busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(launched ? 5 : 20));
            lk.lock();
        } else {
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

extern "C" {

lk_result lk_server_create(lk_context *ctx, const lk_server_config *cfg, lk_server **out)
{
    if (!ctx || !cfg || !out) return fail(LK_ERR_INVALID_ARG, "ctx, cfg or out is NULL");
    *out = nullptr;
    const lk_server_config &c = *cfg;
    if (c.max_streams < 1 || c.max_streams > (1 << 20)) return fail(LK_ERR_INVALID_ARG, "max_streams out of range");
    if (c.max_points < 1 || c.max_points > (1 << 20)) return fail(LK_ERR_INVALID_ARG, "max_points out of range");
    if (c.storage != LK_STORAGE_F32 && c.storage != LK_STORAGE_F16) return fail(LK_ERR_INVALID_ARG, "bad storage");
    if (c.levels < 1 || c.levels > LK_MAX_LEVELS) return fail(LK_ERR_INVALID_ARG, "levels out of range");
    lk_result r = check_params(&c.params, c.levels);
    if (r != LK_SUCCESS) return r;
    if (c.max_batch < 1 || c.inflight < 1 || c.inflight > 8 || c.queue_depth < 1 || c.queue_depth > 64 || c.reserved)
        return fail(LK_ERR_INVALID_ARG, "max_batch, inflight (1..8), queue_depth (1..64) or reserved invalid");
    lk_server *s = new (std::nothrow) lk_server();
    if (!s) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->ctx = ctx;
    s->cfg = c;
    s->cams.resize(c.max_streams);
    s->launches.resize(c.inflight);
    (void)hipSetDevice(ctx->device);
    {
        const size_t n = (size_t)c.max_streams * c.max_points;
        hipError_t e = hipMalloc(&s->d_pool, n * (8 * 3 + 4 + 1) + 1024);
        if (e != hipSuccess) { lk_server_destroy(s); return hip_fail(e, "hipMalloc(keypoint pools)"); }
        s->d_pts = static_cast<float *>(s->d_pool);
        s->d_guess = s->d_pts + 2 * n;
        s->d_out = s->d_guess + 2 * n;
        s->d_res = s->d_out + 2 * n;
        s->d_status = reinterpret_cast<uint8_t *>(s->d_res + n);
    }
    for (auto &L : s->launches) {
        hipError_t e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e != hipSuccess) { lk_server_destroy(s); return hip_fail(e, "server stream"); }
        r = L.ring.init(4);
        if (r != LK_SUCCESS) { lk_server_destroy(s); return r; }
    }
    s->thread = std::thread(scheduler, s);
    *out = s;
    return LK_SUCCESS;
}

lk_result lk_server_open_stream(lk_server *s, int32_t w, int32_t h, uint32_t *id)
{
    if (!s || !id) return fail(LK_ERR_INVALID_ARG, "srv or id is NULL");
    int32_t ws[LK_MAX_LEVELS], hs[LK_MAX_LEVELS];
    if (w > (1 << 15) || h > (1 << 15) || level_dims(w, h, s->cfg.levels, ws, hs) != 0)
        return fail(LK_ERR_INVALID_ARG, "bad frame size %dx%d for %d levels", w, h, s->cfg.levels);
    std::lock_guard<std::mutex> g(s->mu);
    int slot = -1;
    for (int i = 0; i < (int)s->cams.size(); ++i)
        if (!s->cams[i].open) { slot = i; break; }
    if (slot < 0) return fail(LK_ERR_BUSY, "all %d stream slots are in use", s->cfg.max_streams);
    CamStream &c = s->cams[slot];
    c = CamStream{};
    c.w = w; c.h = h;
    c.pitch = (w + 255) & ~255;
    const size_t P = (size_t)s->cfg.max_points;
    (void)hipSetDevice(s->ctx->device);
    // resident bytes of this stream: two frames, two pyramids, point arrays
    lk_pyramid *probe = nullptr;
    lk_result r = lk_pyramid_create(s->ctx, w, h, s->cfg.levels, s->cfg.storage, &probe);
    if (r != LK_SUCCESS) return r;
    const uint64_t pyr_bytes = probe->bytes;
    lk_pyramid_destroy(probe);
    const uint64_t need = 2 * (uint64_t)c.pitch * h + 2 * pyr_bytes + P * (8 * 3 + 4 + 1);   // incl. its pool share
    if (s->cfg.hbm_budget_bytes && s->resident + need > s->cfg.hbm_budget_bytes)
        return fail(LK_ERR_BUSY, "stream needs %llu resident bytes, %llu of %llu in use",
                    (unsigned long long)need, (unsigned long long)s->resident,
                    (unsigned long long)s->cfg.hbm_budget_bytes);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipMalloc(&c.d_frame[k], (size_t)c.pitch * h);
        if (e == hipSuccess) {
            r = lk_pyramid_create(s->ctx, w, h, s->cfg.levels, s->cfg.storage, &c.pyr[k]);
            if (r != LK_SUCCESS) { free_stream(s, c); return r; }
        }
    }
    if (e != hipSuccess) { free_stream(s, c); return hip_fail(e, "hipMalloc(stream)"); }
    // pinned staging
    const size_t sb = (slot_bytes(s, w, h) + 255) & ~size_t(255);
    e = hipHostMalloc(&c.host_block, sb * s->cfg.queue_depth, hipHostMallocDefault);
    if (e != hipSuccess) { free_stream(s, c); return hip_fail(e, "hipHostMalloc(stream staging)"); }
    c.slots.resize(s->cfg.queue_depth);
    for (int k = 0; k < s->cfg.queue_depth; ++k) {
        char *b = static_cast<char *>(c.host_block) + k * sb;
        Slot &sl = c.slots[k];
        sl.pts = reinterpret_cast<float *>(b);
        sl.guess = sl.pts + 2 * P;
        sl.out = sl.guess + 2 * P;
        sl.residual = sl.out + 2 * P;
        sl.status = reinterpret_cast<uint8_t *>(sl.residual + P);
        sl.frame = sl.status + ((P + 63) & ~size_t(63));
    }
    c.resident = need;
    c.open = true;
    s->resident += need;
    *id = (uint32_t)slot;
    return LK_SUCCESS;
}

lk_result lk_server_submit(lk_server *s, uint32_t id, const uint8_t *h_frame, int32_t pitch, const float *h_pts,
                           const float *h_guess, int32_t n, uint64_t *ticket)
{
    if (!s || !h_frame || !ticket) return fail(LK_ERR_INVALID_ARG, "NULL argument");
    const uint64_t t0 = now_ns();
    std::unique_lock<std::mutex> g(s->mu);
    if (id >= s->cams.size() || !s->cams[id].open || s->cams[id].closing)
        return fail(LK_ERR_NOT_FOUND, "stream %u is not open", id);
    CamStream &c = s->cams[id];
    if (pitch < c.w) return fail(LK_ERR_INVALID_ARG, "pitch < width");
    if (n < 0 || n > s->cfg.max_points) return fail(LK_ERR_INVALID_ARG, "n must be in [0, %d]", s->cfg.max_points);
    if (n > 0 && !h_pts) return fail(LK_ERR_INVALID_ARG, "h_pts is NULL");
    int k = -1;
    for (int i = 0; i < (int)c.slots.size(); ++i)
        if (c.slots[i].state == SLOT_FREE) { k = i; break; }
    if (k < 0) return fail(LK_ERR_BUSY, "stream %u: all %zu staging slots hold frames", id, c.slots.size());
    Slot &sl = c.slots[k];
    sl.state = SLOT_FILLING;
    ++c.fillers;              // lk_server_close_stream waits for this copy to end
    g.unlock();
    // the slot is reserved: only this call writes it until it is queued
    for (int y = 0; y < c.h; ++y) std::memcpy(sl.frame + (size_t)y * c.w, h_frame + (size_t)y * pitch, c.w);
    if (n > 0) std::memcpy(sl.pts, h_pts, (size_t)n * 8);
    if (n > 0 && h_guess) std::memcpy(sl.guess, h_guess, (size_t)n * 8);
    g.lock();
    --c.fillers;
    s->cv.notify_all();
    if (!c.open || c.closing) {
        if (c.open) sl.state = SLOT_FREE;
        return fail(LK_ERR_NOT_FOUND, "stream %u was closed", id);
    }
    sl.n = n;
    sl.has_guess = h_guess != nullptr && n > 0;
    sl.t = lk_timing{t0, 0, 0};
    sl.ticket = ((uint64_t)id << 40) | ((uint64_t)(c.seq++) << 8) | (uint64_t)k;
    sl.state = SLOT_QUEUED;
    c.fifo.push_back(k);
    s->tickets[sl.ticket] = {(int)id, k};
    *ticket = sl.ticket;
    s->cv.notify_all();
    return LK_SUCCESS;
}

lk_result lk_server_poll(lk_server *s, uint64_t ticket, float *h_out_pts, uint8_t *h_status, float *h_residual,
                         int32_t *n_out, lk_timing *timing)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    retire(s);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(LK_ERR_NOT_FOUND, "unknown ticket");
    CamStream &c = s->cams[it->second.first];
    Slot &sl = c.slots[it->second.second];
    if (sl.state == SLOT_QUEUED || sl.state == SLOT_RUNNING || sl.state == SLOT_FILLING) return LK_ERR_NOT_READY;
    const bool ok = sl.state == SLOT_DONE;
    if (ok && sl.n_out > 0) {
        if (h_out_pts) std::memcpy(h_out_pts, sl.out, (size_t)sl.n_out * 8);
        if (h_status) std::memcpy(h_status, sl.status, (size_t)sl.n_out);
        if (h_residual) std::memcpy(h_residual, sl.residual, (size_t)sl.n_out * 4);
    }
    if (n_out) *n_out = ok ? sl.n_out : 0;
    if (timing) *timing = sl.t;
    sl.state = SLOT_FREE;
    s->tickets.erase(it);
    if (!ok) return fail(LK_ERR_DEVICE, "the launch of this frame failed");
    return LK_SUCCESS;
}

lk_result lk_server_close_stream(lk_server *s, uint32_t id)
{
    if (!s) return fail(LK_ERR_INVALID_ARG, "srv is NULL");
    std::unique_lock<std::mutex> g(s->mu);
    if (id >= s->cams.size() || !s->cams[id].open) return fail(LK_ERR_NOT_FOUND, "stream %u is not open", id);
    CamStream &c = s->cams[id];
    c.closing = true;
    // the running frame has completed and no submit is still copying into
    // one of the stream's staging slots
    s->cv.wait(g, [&] {
        retire(s);
        return !c.busy && c.fillers == 0;
    });
    for (auto it = s->tickets.begin(); it != s->tickets.end();)
        if (it->second.first == (int)id) it = s->tickets.erase(it); else ++it;
    free_stream(s, c);
    return LK_SUCCESS;
}

lk_result lk_server_fail_next_launches(lk_server *s, int32_t n)
{
    if (!s || n < 0) return fail(LK_ERR_INVALID_ARG, "srv is NULL or n < 0");
    std::lock_guard<std::mutex> g(s->mu);
    s->fail_next = n;
    return LK_SUCCESS;
}

lk_result lk_server_get_stats(lk_server *s, lk_server_stats *out)
{
    if (!s || !out) return fail(LK_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->resident_bytes = s->resident;
    int open = 0;
    for (auto &c : s->cams) open += c.open ? 1 : 0;
    out->open_streams = open;
    return LK_SUCCESS;
}

void lk_server_destroy(lk_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto &L : s->launches)
        if (L.stream) (void)hipStreamSynchronize(L.stream);
    for (auto &c : s->cams)
        if (c.open) free_stream(s, c);
    for (auto &L : s->launches) {
        L.ring.release();
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    if (s->d_pool) (void)hipFree(s->d_pool);
    delete s;
}

}  // extern "C"
