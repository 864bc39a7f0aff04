// Scheduler of the serving loop (lk_server_* in lk.h), free of device code.
//
// It owns the camera-stream table, each stream's staging slots and frame
// queue, the tickets, admission by resident bytes, and the scheduler thread:
// the thread retires launches that have completed, then, whenever one of the
// `inflight` launch queues is free, takes the head frame of every stream that
// has no frame in flight -- up to max_batch of them -- and hands them to the
// backend as one launch.  A frame that arrives while launches run joins the
// next one.  Everything the device does -- resident buffers, copies, the
// batched pyramid build and tracker launch, completion -- is behind
// SchedBackend: the HIP backend of the library, or a CPU executor in the
// scheduler's own tests.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "lk.h"

namespace lkmi {

enum SlotState { SLOT_FREE = 0, SLOT_FILLING, SLOT_QUEUED, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED };

// Host staging of one frame: inputs copied in by submit, results written by
// the backend's launch, copied out by poll.
struct SchedSlot {
    uint8_t *frame = nullptr;   // h x w, packed rows
    float *pts = nullptr;       // max_points x 2
    float *guess = nullptr;     // max_points x 2
    float *out = nullptr;       // max_points x 2
    uint8_t *status = nullptr;  // max_points
    float *residual = nullptr;  // max_points
    int n = 0;                  // points submitted
    int n_out = 0;              // points tracked: n, or 0 for a stream's first frame
    bool has_guess = false;
    SlotState state = SLOT_FREE;
    uint64_t ticket = 0;
    lk_timing t{};
};

// One frame of a launch, as the backend sees it.
struct SchedFrame {
    int stream;                 // camera stream index
    int cur;                    // the stream's buffer (0 or 1) that receives this frame
    const SchedSlot *slot;      // inputs and result buffers; slot->n_out == 0: build only
};

class SchedBackend {
public:
    virtual ~SchedBackend() = default;
    // Device bytes a w x h stream holds while open (frames, pyramids, its
    // share of the point arrays); LK_ERR_INVALID_ARG for a size the
    // configured level count does not allow.
    virtual lk_result stream_bytes(int w, int h, uint64_t *bytes) = 0;
    virtual lk_result open_stream(int stream, int w, int h) = 0;
    // Frees what open_stream took; the stream has no frame in flight.
    virtual void close_stream(int stream) = 0;
    // Staging memory of a stream's slots (pinned host memory for a device
    // backend); NULL on failure.
    virtual void *host_alloc(size_t bytes) = 0;
    virtual void host_free(void *p) = 0;
    // Enqueues one launch on queue q: every frame into its stream's buffer
    // `cur` and its pyramid; for every frame with n_out > 0, tracking from
    // the stream's other buffer (its previous frame) with the slot's points
    // (and guesses), results into the slot.  inject_failure: fail as a
    // host-side staging error would, after the frames' copies are enqueued.
    // An error return means the launch is incomplete: the scheduler drains
    // the queue and fails its frames.
    virtual lk_result enqueue(int q, const std::vector<SchedFrame> &frames, bool inject_failure) = 0;
    // The last launch on q: 1 complete, 0 still running, -1 failed.
    virtual int query(int q) = 0;
    // Waits until everything enqueued on q has finished.
    virtual void drain(int q) = 0;
    // Called first on the scheduler thread (device selection).
    virtual void thread_init() {}
};

struct SchedStream {
    bool open = false;
    bool closing = false;
    int w = 0, h = 0;
    int cur = 0;                // buffer of the next frame
    bool primed = false;        // buffer cur ^ 1 holds the previous frame
    bool busy = false;          // a frame is in flight
    int fillers = 0;            // submits copying into a reserved slot right now
    uint32_t seq = 0;
    std::vector<SchedSlot> slots;
    std::deque<int> fifo;       // queued slot indices
    uint64_t resident = 0;
    void *host_block = nullptr;
};

struct SchedQueue {
    bool busy = false;
    bool failed = false;                       // the launch could not be enqueued completely
    std::vector<std::pair<int, int>> frames;   // (stream, slot)
};

struct Sched {
    lk_server_config cfg{};
    SchedBackend *be = nullptr;
    std::vector<SchedStream> cams;
    std::vector<SchedQueue> queues;
    std::unordered_map<uint64_t, std::pair<int, int>> tickets;   // ticket -> (stream, slot)
    std::mutex mu;
    std::condition_variable cv;
    std::thread thread;
    bool stop = false;
    uint64_t resident = 0;
    lk_server_stats stats{};
    int fail_next = 0;          // launches made to fail on the host (fault injection)
};

// Checks the scheduler's part of a server configuration (stream, point,
// batch, queue and slot counts).
lk_result sched_check_config(const lk_server_config *cfg);
// Starts the scheduler thread; cfg must have passed sched_check_config.
lk_result sched_start(Sched *s, const lk_server_config &cfg, SchedBackend *be);
lk_result sched_open_stream(Sched *s, int32_t w, int32_t h, uint32_t *id);
lk_result sched_submit(Sched *s, uint32_t id, const uint8_t *h_frame, int32_t pitch, const float *h_pts,
                       const float *h_guess, int32_t n, uint64_t *ticket);
lk_result sched_poll(Sched *s, uint64_t ticket, float *h_out_pts, uint8_t *h_status, float *h_residual,
                     int32_t *n_out, lk_timing *timing);
lk_result sched_close_stream(Sched *s, uint32_t id);
lk_result sched_fail_next(Sched *s, int32_t n);
lk_result sched_stats(Sched *s, lk_server_stats *out);
// Stops the thread, waits for every queue, closes every open stream.
void sched_stop(Sched *s);

}  // namespace lkmi
