// Scheduler of the serving loop: stream table, staging slots, tickets,
// admission by resident bytes and continuous batching (lk_sched.h).  No
// device code: the device work goes through the SchedBackend.
#include "lk_sched.h"

#include <chrono>
#include <cstring>

#include <time.h>

#include "lk_error.h"

namespace lkmi {

namespace {

uint64_t now_ns()
{
    timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

// Host bytes of one staging slot of a w x h stream: points, guesses and
// results (x, y as float), residuals, status bytes and the frame.
size_t slot_bytes(const Sched *s, int w, int h)
{
    const size_t P = (size_t)s->cfg.max_points;
    return (size_t)w * h + P * 8 * 3 + P + P * 4 + 64;
}

void free_stream(Sched *s, int id)
{
    SchedStream &c = s->cams[id];
    s->be->close_stream(id);
    if (c.host_block) s->be->host_free(c.host_block);
    s->resident -= c.resident;
    c = SchedStream{};
}

// Completes launches that have finished.  A launch that could not be
// enqueued completely is completed once what it did enqueue has drained: its
// frames fail, and their streams keep their buffers and previous frame, so
// the next frame is tracked from the last frame that completed.  Called with
// the lock held.
void retire(Sched *s)
{
    for (int q = 0; q < (int)s->queues.size(); ++q) {
        SchedQueue &Q = s->queues[q];
        if (!Q.busy) continue;
        bool ok;
        if (Q.failed) {
            s->be->drain(q);      // the copies out of the staging slots have finished
            ok = false;
            Q.failed = false;
        } else {
            const int st = s->be->query(q);
            if (st == 0) continue;
            ok = st > 0;
        }
        const uint64_t t = now_ns();
        for (auto &fs : Q.frames) {
            SchedStream &c = s->cams[fs.first];
            SchedSlot &sl = c.slots[fs.second];
            sl.state = ok ? SLOT_DONE : SLOT_FAILED;
            sl.t.done_ns = t;
            c.busy = false;
            if (ok) {
                c.primed = true;
                c.cur ^= 1;
                s->stats.frames += 1;
                s->stats.points += (uint64_t)sl.n_out;
            }
        }
        if (ok) s->stats.batches += 1;
        Q.frames.clear();
        Q.busy = false;
    }
}

// Hands the ready head frames to the backend as one launch on queue q.
// Called with the lock held.
lk_result launch_ready(Sched *s, int q)
{
    SchedQueue &Q = s->queues[q];
    std::vector<std::pair<int, int>> take;
    for (int i = 0; i < (int)s->cams.size() && (int)take.size() < s->cfg.max_batch; ++i) {
        SchedStream &c = s->cams[i];
        if (!c.open || c.closing || c.busy || c.fifo.empty()) continue;
        take.push_back({i, c.fifo.front()});
    }
    if (take.empty()) return LK_SUCCESS;
    const uint64_t t = now_ns();
    std::vector<SchedFrame> frames;
    frames.reserve(take.size());
    for (auto &fs : take) {
        SchedStream &c = s->cams[fs.first];
        SchedSlot &sl = c.slots[fs.second];
        c.fifo.pop_front();
        c.busy = true;
        sl.state = SLOT_RUNNING;
        sl.t.launch_ns = t;
        sl.n_out = c.primed ? sl.n : 0;
        frames.push_back(SchedFrame{fs.first, c.cur, &sl});
    }
    const bool inject = s->fail_next > 0;
    if (inject) --s->fail_next;
    const lk_result r = s->be->enqueue(q, frames, inject);
    Q.frames = take;
    Q.busy = true;
    Q.failed = r != LK_SUCCESS;
    return r;
}

void scheduler(Sched *s)
{
    s->be->thread_init();
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        retire(s);
        bool any_busy = false, launched = false;
        for (int q = 0; q < (int)s->queues.size(); ++q) {
            SchedQueue &Q = s->queues[q];
            if (!Q.busy) {
                const lk_result r = launch_ready(s, q);
                if (r != LK_SUCCESS) {
                    // what this launch took has failed; the device state is unknown
                    for (auto &fs : Q.frames) s->cams[fs.first].slots[fs.second].state = SLOT_FAILED;
                }
                launched |= Q.busy;
            }
            any_busy |= Q.busy;
        }
        s->cv.notify_all();
        if (any_busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(launched ? 5 : 20));
            lk.lock();
        } else {
            // idle: only a submit (or stop) makes work, and both notify under
            // the lock, so no wake-up is lost between the check and the wait
            s->cv.wait(lk);
        }
    }
}

}  // namespace

lk_result sched_check_config(const lk_server_config *cfg)
{
    if (!cfg) return fail(LK_ERR_INVALID_ARG, "cfg is NULL");
    const lk_server_config &c = *cfg;
    if (c.max_streams < 1 || c.max_streams > (1 << 20)) return fail(LK_ERR_INVALID_ARG, "max_streams out of range");
    if (c.max_points < 1 || c.max_points > (1 << 20)) return fail(LK_ERR_INVALID_ARG, "max_points out of range");
    if (c.max_batch < 1 || c.inflight < 1 || c.inflight > 8 || c.queue_depth < 1 || c.queue_depth > 64 || c.reserved)
        return fail(LK_ERR_INVALID_ARG, "max_batch, inflight (1..8), queue_depth (1..64) or reserved invalid");
    return LK_SUCCESS;
}

lk_result sched_start(Sched *s, const lk_server_config &cfg, SchedBackend *be)
{
    s->cfg = cfg;
    s->be = be;
    s->cams.resize(cfg.max_streams);
    s->queues.resize(cfg.inflight);
    try {
        s->thread = std::thread(scheduler, s);
    } catch (...) {
        return fail(LK_ERR_OUT_OF_MEMORY, "scheduler thread could not be started");
    }
    return LK_SUCCESS;
}

lk_result sched_open_stream(Sched *s, int32_t w, int32_t h, uint32_t *id)
{
    if (!id) return fail(LK_ERR_INVALID_ARG, "id is NULL");
    if (w < 1 || h < 1 || w > (1 << 15) || h > (1 << 15))
        return fail(LK_ERR_INVALID_ARG, "bad frame size %dx%d", w, h);
    std::lock_guard<std::mutex> g(s->mu);
    int slot = -1;
    for (int i = 0; i < (int)s->cams.size(); ++i)
        if (!s->cams[i].open) { slot = i; break; }
    if (slot < 0) return fail(LK_ERR_BUSY, "all %d stream slots are in use", s->cfg.max_streams);
    uint64_t need = 0;
    lk_result r = s->be->stream_bytes(w, h, &need);
    if (r != LK_SUCCESS) return r;
    if (s->cfg.hbm_budget_bytes && s->resident + need > s->cfg.hbm_budget_bytes)
        return fail(LK_ERR_BUSY, "stream needs %llu resident bytes, %llu of %llu in use",
                    (unsigned long long)need, (unsigned long long)s->resident,
                    (unsigned long long)s->cfg.hbm_budget_bytes);
    SchedStream &c = s->cams[slot];
    c = SchedStream{};
    c.w = w; c.h = h;
    r = s->be->open_stream(slot, w, h);
    if (r != LK_SUCCESS) return r;
    const size_t P = (size_t)s->cfg.max_points;
    const size_t sb = (slot_bytes(s, w, h) + 255) & ~size_t(255);
    c.host_block = s->be->host_alloc(sb * s->cfg.queue_depth);
    if (!c.host_block) {
        s->be->close_stream(slot);
        c = SchedStream{};
        return fail(LK_ERR_OUT_OF_MEMORY, "stream staging (%zu bytes) could not be allocated",
                    sb * s->cfg.queue_depth);
    }
    c.slots.resize(s->cfg.queue_depth);
    for (int k = 0; k < s->cfg.queue_depth; ++k) {
        char *b = static_cast<char *>(c.host_block) + k * sb;
        SchedSlot &sl = c.slots[k];
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

lk_result sched_submit(Sched *s, uint32_t id, const uint8_t *h_frame, int32_t pitch, const float *h_pts,
                       const float *h_guess, int32_t n, uint64_t *ticket)
{
    if (!h_frame || !ticket) return fail(LK_ERR_INVALID_ARG, "NULL argument");
    const uint64_t t0 = now_ns();
    std::unique_lock<std::mutex> g(s->mu);
    if (id >= s->cams.size() || !s->cams[id].open || s->cams[id].closing)
        return fail(LK_ERR_NOT_FOUND, "stream %u is not open", id);
    SchedStream &c = s->cams[id];
    if (pitch < c.w) return fail(LK_ERR_INVALID_ARG, "pitch < width");
    if (n < 0 || n > s->cfg.max_points) return fail(LK_ERR_INVALID_ARG, "n must be in [0, %d]", s->cfg.max_points);
    if (n > 0 && !h_pts) return fail(LK_ERR_INVALID_ARG, "h_pts is NULL");
    int k = -1;
    for (int i = 0; i < (int)c.slots.size(); ++i)
        if (c.slots[i].state == SLOT_FREE) { k = i; break; }
    if (k < 0) return fail(LK_ERR_BUSY, "stream %u: all %zu staging slots hold frames", id, c.slots.size());
    SchedSlot &sl = c.slots[k];
    sl.state = SLOT_FILLING;
    ++c.fillers;              // sched_close_stream waits for this copy to end
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

lk_result sched_poll(Sched *s, uint64_t ticket, float *h_out_pts, uint8_t *h_status, float *h_residual,
                     int32_t *n_out, lk_timing *timing)
{
    std::lock_guard<std::mutex> g(s->mu);
    retire(s);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(LK_ERR_NOT_FOUND, "unknown ticket");
    SchedStream &c = s->cams[it->second.first];
    SchedSlot &sl = c.slots[it->second.second];
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

lk_result sched_close_stream(Sched *s, uint32_t id)
{
    std::unique_lock<std::mutex> g(s->mu);
    if (id >= s->cams.size() || !s->cams[id].open) return fail(LK_ERR_NOT_FOUND, "stream %u is not open", id);
    SchedStream &c = s->cams[id];
    c.closing = true;
    // the running frame has completed and no submit is still copying into
    // one of the stream's staging slots
    s->cv.wait(g, [&] {
        retire(s);
        return !c.busy && c.fillers == 0;
    });
    for (auto it = s->tickets.begin(); it != s->tickets.end();)
        if (it->second.first == (int)id) it = s->tickets.erase(it); else ++it;
    free_stream(s, (int)id);
    return LK_SUCCESS;
}

lk_result sched_fail_next(Sched *s, int32_t n)
{
    if (n < 0) return fail(LK_ERR_INVALID_ARG, "n < 0");
    std::lock_guard<std::mutex> g(s->mu);
    s->fail_next = n;
    return LK_SUCCESS;
}

lk_result sched_stats(Sched *s, lk_server_stats *out)
{
    if (!out) return fail(LK_ERR_INVALID_ARG, "out is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->resident_bytes = s->resident;
    int open = 0;
    for (auto &c : s->cams) open += c.open ? 1 : 0;
    out->open_streams = open;
    return LK_SUCCESS;
}

void sched_stop(Sched *s)
{
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    if (!s->be) return;
    std::lock_guard<std::mutex> g(s->mu);
    for (int q = 0; q < (int)s->queues.size(); ++q) s->be->drain(q);
    for (int i = 0; i < (int)s->cams.size(); ++i)
        if (s->cams[i].open) free_stream(s, i);
}

}  // namespace lkmi
