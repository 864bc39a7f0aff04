// Tests of the serving scheduler (paper_2607_01757_amd/csrc/lk_sched.cpp) on
// the CPU, against a fake device backend: a CPU executor with one worker
// thread per launch queue that tracks with the FP64 oracle (oracle/lk_oracle.c,
// linked in) after an injected latency, and can be told to fail launches.
// It checks results against direct oracle calls, per-stream order, timing
// fields, continuous batching, admission by resident bytes, full staging,
// close while in flight, unknown tickets, device errors and host-side launch
// failures (every frame of the launch fails; the stream then tracks from its
// last completed frame), invalid arguments, a failing staging allocation,
// and several submitting threads at once.  Built plain and under host
// sanitizers by tests/test_server_cpu.py; prints "sched cpu run ok" and exits
// 0, or names the failed check and exits 1.  Test infrastructure.
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "lk_error.h"
#include "lk_sched.h"

extern "C" {
// the oracle's parameter block and 8-bit tracking entry point (lk_oracle.c)
typedef struct {
    int32_t win, levels, max_iters, use_guess, f16_storage, nthreads;
    double eps, min_eig, fb_thresh;
} lko_params;
int lko_track_u8(const uint8_t *prev, const uint8_t *next, int w, int h, int pitch, const double *pts,
                 const double *guess, int n, const lko_params *prm, double *out_pts, uint8_t *status,
                 double *residual, int32_t *iters, double *margins);
}

using namespace lkmi;

#define CHECK(c)                                                                          \
    do {                                                                                  \
        if (!(c)) {                                                                       \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);                    \
            std::fflush(stdout);                                                          \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

namespace {

lko_params oracle_params(const lk_server_config &cfg)
{
    lko_params p{};
    p.win = cfg.params.win;
    p.levels = cfg.params.levels;
    p.max_iters = cfg.params.max_iters;
    p.use_guess = 1;                 // the server always passes guesses (the points when none are given)
    p.f16_storage = cfg.storage;
    p.nthreads = 1;
    p.eps = cfg.params.eps;
    p.min_eig = cfg.params.min_eig;
    p.fb_thresh = cfg.params.fb_thresh;
    return p;
}

// ------------------------------------------------------------ fake backend

class FakeBackend final : public SchedBackend {
public:
    std::atomic<int> latency_us{0};
    std::atomic<int> fail_completions{0};   // next launches complete as failed (a device error)
    std::atomic<bool> fail_host_alloc{false};
    std::atomic<int> violations{0};         // a stream closed or reopened with a launch on it
    std::atomic<int> launches{0};
    std::atomic<int> open_count{0};

    FakeBackend(const lk_server_config &cfg) : cfg_(cfg), streams_(cfg.max_streams), queues_(cfg.inflight)
    {
        for (int q = 0; q < cfg.inflight; ++q) queues_[q].worker = std::thread(&FakeBackend::work, this, q);
    }
    ~FakeBackend() override
    {
        for (auto &Q : queues_) {
            {
                std::lock_guard<std::mutex> g(Q.mu);
                Q.stop = true;
            }
            Q.cv.notify_all();
            Q.worker.join();
        }
    }

    lk_result stream_bytes(int w, int h, uint64_t *bytes) override
    {
        int lw = w, lh = h;
        for (int l = 1; l < cfg_.levels; ++l) { lw = (lw + 1) / 2; lh = (lh + 1) / 2; }
        if (lw < 4 || lh < 4) return fail(LK_ERR_INVALID_ARG, "bad frame size %dx%d", w, h);
        *bytes = bytes_for(w, h);
        return LK_SUCCESS;
    }
    uint64_t bytes_for(int w, int h) const { return 6ull * w * h + (uint64_t)cfg_.max_points * 29; }

    lk_result open_stream(int stream, int w, int h) override
    {
        Stream &S = streams_[stream];
        std::lock_guard<std::mutex> g(S.mu);
        if (S.open || S.in_flight) ++violations;
        S.open = true;
        S.w = w; S.h = h;
        S.buf[0].assign((size_t)w * h, 0);
        S.buf[1].assign((size_t)w * h, 0);
        ++open_count;
        return LK_SUCCESS;
    }
    void close_stream(int stream) override
    {
        Stream &S = streams_[stream];
        std::lock_guard<std::mutex> g(S.mu);
        if (!S.open) return;
        if (S.in_flight) ++violations;
        S.open = false;
        S.buf[0].clear();
        S.buf[1].clear();
        --open_count;
    }
    void *host_alloc(size_t bytes) override { return fail_host_alloc ? nullptr : std::malloc(bytes); }
    void host_free(void *p) override { std::free(p); }

    lk_result enqueue(int q, const std::vector<SchedFrame> &frames, bool inject_failure) override
    {
        Queue &Q = queues_[q];
        std::lock_guard<std::mutex> g(Q.mu);
        if (Q.state == 0) ++violations;   // a queue is handed a launch only once the last one retired
        if (inject_failure) {
            Q.state = -1;                 // nothing runs; the scheduler drains and fails the frames
            return fail(LK_ERR_OUT_OF_MEMORY, "injected staging failure");
        }
        for (const SchedFrame &f : frames) {
            Stream &S = streams_[f.stream];
            std::lock_guard<std::mutex> gs(S.mu);
            if (!S.open || S.in_flight) ++violations;
            S.in_flight = true;
        }
        Q.job = frames;
        Q.state = 0;
        Q.has_job = true;
        ++launches;
        Q.cv.notify_all();
        return LK_SUCCESS;
    }
    int query(int q) override
    {
        Queue &Q = queues_[q];
        std::lock_guard<std::mutex> g(Q.mu);
        return Q.state;
    }
    void drain(int q) override
    {
        Queue &Q = queues_[q];
        std::unique_lock<std::mutex> g(Q.mu);
        Q.cv.wait(g, [&] { return !Q.has_job; });
    }

private:
    struct Stream {
        std::mutex mu;
        bool open = false, in_flight = false;
        int w = 0, h = 0;
        std::vector<uint8_t> buf[2];
    };
    struct Queue {
        std::mutex mu;
        std::condition_variable cv;
        std::thread worker;
        std::vector<SchedFrame> job;
        bool has_job = false, stop = false;
        int state = 1;                    // 1 complete, 0 running, -1 failed
    };

    void work(int q)
    {
        Queue &Q = queues_[q];
        const lko_params prm = oracle_params(cfg_);
        for (;;) {
            std::vector<SchedFrame> job;
            {
                std::unique_lock<std::mutex> g(Q.mu);
                Q.cv.wait(g, [&] { return Q.has_job || Q.stop; });
                if (Q.stop && !Q.has_job) return;
                job = Q.job;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(latency_us.load()));
            for (const SchedFrame &f : job) {
                Stream &S = streams_[f.stream];
                const SchedSlot &sl = *f.slot;
                std::lock_guard<std::mutex> gs(S.mu);
                std::memcpy(S.buf[f.cur].data(), sl.frame, (size_t)S.w * S.h);   // the frame's copy in
                if (sl.n_out > 0) {
                    std::vector<double> p(2 * sl.n_out), gs2(2 * sl.n_out), o(2 * sl.n_out), r(sl.n_out);
                    const float *gsrc = sl.has_guess ? sl.guess : sl.pts;
                    for (int i = 0; i < 2 * sl.n_out; ++i) { p[i] = sl.pts[i]; gs2[i] = gsrc[i]; }
                    const int rc = lko_track_u8(S.buf[f.cur ^ 1].data(), S.buf[f.cur].data(), S.w, S.h, S.w,
                                                p.data(), gs2.data(), sl.n_out, &prm, o.data(), sl.status,
                                                r.data(), nullptr, nullptr);
                    if (rc != 0) ++violations;
                    for (int i = 0; i < 2 * sl.n_out; ++i) sl.out[i] = (float)o[i];
                    for (int i = 0; i < sl.n_out; ++i) sl.residual[i] = (float)r[i];
                }
            }
            for (const SchedFrame &f : job) {
                Stream &S = streams_[f.stream];
                std::lock_guard<std::mutex> gs(S.mu);
                S.in_flight = false;
            }
            std::lock_guard<std::mutex> g(Q.mu);
            int fc = fail_completions.load();
            while (fc > 0 && !fail_completions.compare_exchange_weak(fc, fc - 1)) {}
            Q.state = fc > 0 ? -1 : 1;
            Q.has_job = false;
            Q.cv.notify_all();
        }
    }

    lk_server_config cfg_;
    std::vector<Stream> streams_;
    std::vector<Queue> queues_;
};

// ------------------------------------------------------------ helpers

lk_server_config make_cfg(int streams, int points, int batch, int inflight, int depth, uint64_t budget)
{
    lk_server_config c{};
    c.max_streams = streams;
    c.max_points = points;
    c.levels = 2;
    c.storage = 0;
    c.params.win = 9;
    c.params.levels = 2;
    c.params.max_iters = 20;
    c.params.use_guess = 0;
    c.params.eps = 0.01f;
    c.params.min_eig = 1e-6f;
    c.params.fb_thresh = 0.0f;
    c.max_batch = batch;
    c.inflight = inflight;
    c.queue_depth = depth;
    c.hbm_budget_bytes = budget;
    return c;
}

struct Server {
    lk_server_config cfg;
    FakeBackend be;
    Sched s;
    explicit Server(const lk_server_config &c) : cfg(c), be(c)
    {
        CHECK(sched_check_config(&cfg) == LK_SUCCESS);
        CHECK(sched_start(&s, cfg, &be) == LK_SUCCESS);
    }
    ~Server() { sched_stop(&s); }
};

// a smooth texture moved by (dx, dy) = k * (0.6, -0.35), plus a per-seed phase
std::vector<uint8_t> frame(int w, int h, int k, int seed, int pitch = 0)
{
    if (pitch == 0) pitch = w;
    std::vector<uint8_t> img((size_t)pitch * h, 7);
    const double dx = 0.6 * k, dy = -0.35 * k, ph = 0.7 * seed;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const double u = x - dx, t = y - dy;
            const double v = 128.0 + 60.0 * std::sin(0.23 * u + 0.07 * t + ph) + 45.0 * std::cos(0.19 * t - 0.13 * u)
                             + 15.0 * std::sin(0.5 * u + ph) * std::cos(0.41 * t);
            img[(size_t)y * pitch + x] = (uint8_t)std::lround(v < 0 ? 0 : (v > 255 ? 255 : v));
        }
    return img;
}

std::vector<float> points(int w, int h, int n, int seed)
{
    std::vector<float> p(2 * n);
    for (int i = 0; i < n; ++i) {
        p[2 * i] = (float)(8 + (i * 7 + seed * 3) % (w - 16)) + 0.25f;
        p[2 * i + 1] = (float)(8 + (i * 11 + seed * 5) % (h - 16)) + 0.5f;
    }
    return p;
}

struct Result {
    std::vector<float> out, res;
    std::vector<uint8_t> st;
    int n = -1;
    lk_timing t{};
};

lk_result poll_wait(Sched *s, uint64_t ticket, Result *r, int max_points)
{
    r->out.assign(2 * max_points, 0.f);
    r->res.assign(max_points, 0.f);
    r->st.assign(max_points, 255);
    for (int spin = 0; spin < 200000; ++spin) {
        const lk_result e = sched_poll(s, ticket, r->out.data(), r->st.data(), r->res.data(), &r->n, &r->t);
        if (e != LK_ERR_NOT_READY) return e;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return LK_ERR_NOT_READY;
}

// the oracle on (prev -> next) with the server's arguments, as float
void expect_oracle(const lk_server_config &cfg, const std::vector<uint8_t> &prev, const std::vector<uint8_t> &next,
                   int w, int h, const std::vector<float> &pts, int n, const Result &r)
{
    const lko_params prm = oracle_params(cfg);
    std::vector<double> p(2 * n), o(2 * n), res(n);
    std::vector<uint8_t> st(n);
    for (int i = 0; i < 2 * n; ++i) p[i] = pts[i];
    CHECK(lko_track_u8(prev.data(), next.data(), w, h, w, p.data(), p.data(), n, &prm, o.data(), st.data(),
                       res.data(), nullptr, nullptr) == 0);
    CHECK(r.n == n);
    int ok = 0;
    for (int i = 0; i < n; ++i) {
        CHECK(r.st[i] == st[i]);
        CHECK(r.out[2 * i] == (float)o[2 * i] && r.out[2 * i + 1] == (float)o[2 * i + 1]);
        CHECK(r.res[i] == (float)res[i]);
        ok += st[i] == 0;
    }
    CHECK(ok >= n / 2);                // the sequence is trackable: most points are kept
}

// ------------------------------------------------------------ cases

void case_results_and_order()
{
    Server S(make_cfg(4, 48, 4, 2, 4, 0));
    const int W[3] = {64, 96, 72}, H[3] = {48, 64, 72};
    uint32_t id[3];
    for (int i = 0; i < 3; ++i) CHECK(sched_open_stream(&S.s, W[i], H[i], &id[i]) == LK_SUCCESS);
    const int F = 5;
    std::vector<std::vector<uint8_t>> frames[3];
    std::vector<float> pts[3];
    uint64_t tk[3][F];
    for (int i = 0; i < 3; ++i) {
        pts[i] = points(W[i], H[i], 40, i);
        for (int k = 0; k < F; ++k) frames[i].push_back(frame(W[i], H[i], k, i));
    }
    // frames of all streams interleaved, at most queue_depth outstanding per stream
    for (int k = 0; k < F; ++k)
        for (int i = 0; i < 3; ++i) {
            lk_result e;
            while ((e = sched_submit(&S.s, id[i], frames[i][k].data(), W[i], pts[i].data(), nullptr, 40,
                                     &tk[i][k])) == LK_ERR_BUSY)
                std::this_thread::sleep_for(std::chrono::microseconds(100));
            CHECK(e == LK_SUCCESS);
            if (k >= 3) {                 // keep the staging from filling: retire an older frame
                Result r;
                CHECK(poll_wait(&S.s, tk[i][k - 3], &r, 48) == LK_SUCCESS);
                if (k - 3 == 0) CHECK(r.n == 0);
                else expect_oracle(S.cfg, frames[i][k - 4], frames[i][k - 3], W[i], H[i], pts[i], 40, r);
            }
        }
    for (int i = 0; i < 3; ++i) {
        uint64_t prev_done = 0;
        for (int k = F - 3; k < F; ++k) {
            Result r;
            CHECK(poll_wait(&S.s, tk[i][k], &r, 48) == LK_SUCCESS);
            expect_oracle(S.cfg, frames[i][k - 1], frames[i][k], W[i], H[i], pts[i], 40, r);
            CHECK(r.t.submit_ns <= r.t.launch_ns && r.t.launch_ns <= r.t.done_ns);
            CHECK(r.t.done_ns >= prev_done);      // one stream's frames complete in submit order
            prev_done = r.t.done_ns;
        }
    }
    lk_server_stats st{};
    CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
    CHECK(st.frames == 3 * F && st.open_streams == 3);
    CHECK(st.points == 3ull * (F - 1) * 40);
    CHECK(S.be.violations == 0);
}

void case_timing_and_batching()
{
    // one launch queue, 5 ms per launch: a burst of 16 frames goes out in few launches
    Server S(make_cfg(16, 16, 16, 1, 2, 0));
    S.be.latency_us = 5000;
    uint32_t id[16];
    std::vector<uint8_t> f0 = frame(32, 32, 0, 0);
    std::vector<float> p = points(32, 32, 8, 0);
    for (int i = 0; i < 16; ++i) CHECK(sched_open_stream(&S.s, 32, 32, &id[i]) == LK_SUCCESS);
    uint64_t tk[16];
    for (int i = 0; i < 16; ++i) CHECK(sched_submit(&S.s, id[i], f0.data(), 32, p.data(), nullptr, 8, &tk[i]) == LK_SUCCESS);
    for (int i = 0; i < 16; ++i) {
        Result r;
        CHECK(poll_wait(&S.s, tk[i], &r, 16) == LK_SUCCESS);
        CHECK(r.n == 0);
        CHECK(r.t.submit_ns <= r.t.launch_ns && r.t.launch_ns <= r.t.done_ns);
        CHECK(r.t.done_ns - r.t.launch_ns >= 5000000ull);   // the launch's latency
    }
    lk_server_stats st{};
    CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
    CHECK(st.frames == 16);
    CHECK(st.batches <= 3);           // frames that arrive while a launch runs join the next one
    CHECK(S.be.launches == (int)st.batches);
    CHECK(S.be.violations == 0);
}

void case_admission_and_limits()
{
    FakeBackend probe(make_cfg(1, 32, 1, 1, 1, 0));
    const uint64_t need = probe.bytes_for(64, 48);
    Server S(make_cfg(3, 32, 4, 1, 2, need * 5 / 2));
    uint32_t a, b, c;
    CHECK(sched_open_stream(&S.s, 64, 48, &a) == LK_SUCCESS);
    CHECK(sched_open_stream(&S.s, 64, 48, &b) == LK_SUCCESS);
    CHECK(sched_open_stream(&S.s, 64, 48, &c) == LK_ERR_BUSY);        // over the budget
    lk_server_stats st{};
    CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
    CHECK(st.resident_bytes == 2 * need && st.open_streams == 2);
    CHECK(sched_close_stream(&S.s, a) == LK_SUCCESS);
    CHECK(sched_open_stream(&S.s, 64, 48, &c) == LK_SUCCESS);         // fits again, in the freed entry
    CHECK(c == a);
    CHECK(sched_close_stream(&S.s, b) == LK_SUCCESS);
    // a table of 2 entries is full after 2 opens whatever the budget
    Server T(make_cfg(2, 32, 4, 1, 2, 0));
    uint32_t x;
    CHECK(sched_open_stream(&T.s, 64, 48, &x) == LK_SUCCESS);
    CHECK(sched_open_stream(&T.s, 64, 48, &x) == LK_SUCCESS);
    CHECK(sched_open_stream(&T.s, 64, 48, &x) == LK_ERR_BUSY);
    // the staging allocation fails: nothing stays reserved
    T.be.fail_host_alloc = true;
    CHECK(sched_close_stream(&T.s, x) == LK_SUCCESS);
    CHECK(sched_open_stream(&T.s, 64, 48, &x) == LK_ERR_OUT_OF_MEMORY);
    CHECK(sched_stats(&T.s, &st) == LK_SUCCESS);
    CHECK(st.open_streams == 1 && st.resident_bytes == probe.bytes_for(64, 48));
    CHECK(T.be.open_count == 1);
    T.be.fail_host_alloc = false;
    CHECK(sched_open_stream(&T.s, 64, 48, &x) == LK_SUCCESS);
    CHECK(S.be.violations == 0 && T.be.violations == 0);
}

void case_invalid_arguments()
{
    lk_server_config c = make_cfg(2, 16, 4, 1, 2, 0);
    CHECK(sched_check_config(nullptr) == LK_ERR_INVALID_ARG);
    lk_server_config bad = c; bad.inflight = 9;
    CHECK(sched_check_config(&bad) == LK_ERR_INVALID_ARG);
    bad = c; bad.max_streams = 0;
    CHECK(sched_check_config(&bad) == LK_ERR_INVALID_ARG);
    bad = c; bad.queue_depth = 65;
    CHECK(sched_check_config(&bad) == LK_ERR_INVALID_ARG);
    bad = c; bad.max_batch = 0;
    CHECK(sched_check_config(&bad) == LK_ERR_INVALID_ARG);
    bad = c; bad.reserved = 1;
    CHECK(sched_check_config(&bad) == LK_ERR_INVALID_ARG);
    Server S(c);
    uint32_t id;
    CHECK(sched_open_stream(&S.s, 0, 32, &id) == LK_ERR_INVALID_ARG);
    CHECK(sched_open_stream(&S.s, 6, 32, &id) == LK_ERR_INVALID_ARG);       // level 1 would be 3 wide
    CHECK(sched_open_stream(&S.s, 1 << 16, 32, &id) == LK_ERR_INVALID_ARG);
    CHECK(sched_open_stream(&S.s, 32, 32, nullptr) == LK_ERR_INVALID_ARG);
    CHECK(sched_open_stream(&S.s, 32, 32, &id) == LK_SUCCESS);
    std::vector<uint8_t> f = frame(32, 32, 0, 0);
    std::vector<float> p = points(32, 32, 16, 0);
    uint64_t t;
    CHECK(sched_submit(&S.s, id, f.data(), 31, p.data(), nullptr, 4, &t) == LK_ERR_INVALID_ARG);   // pitch < w
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 17, &t) == LK_ERR_INVALID_ARG);  // > max_points
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, -1, &t) == LK_ERR_INVALID_ARG);
    CHECK(sched_submit(&S.s, id, f.data(), 32, nullptr, nullptr, 4, &t) == LK_ERR_INVALID_ARG);
    CHECK(sched_submit(&S.s, id, nullptr, 32, p.data(), nullptr, 4, &t) == LK_ERR_INVALID_ARG);
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 4, nullptr) == LK_ERR_INVALID_ARG);
    CHECK(sched_submit(&S.s, id + 1, f.data(), 32, p.data(), nullptr, 4, &t) == LK_ERR_NOT_FOUND);
    CHECK(sched_submit(&S.s, 1000, f.data(), 32, p.data(), nullptr, 4, &t) == LK_ERR_NOT_FOUND);
    CHECK(sched_fail_next(&S.s, -1) == LK_ERR_INVALID_ARG);
    CHECK(sched_stats(&S.s, nullptr) == LK_ERR_INVALID_ARG);
    CHECK(sched_close_stream(&S.s, id + 1) == LK_ERR_NOT_FOUND);
    // an empty frame (n = 0) is valid
    CHECK(sched_submit(&S.s, id, f.data(), 32, nullptr, nullptr, 0, &t) == LK_SUCCESS);
    Result r;
    CHECK(poll_wait(&S.s, t, &r, 16) == LK_SUCCESS && r.n == 0);
    // unknown and retired tickets
    CHECK(sched_poll(&S.s, t, nullptr, nullptr, nullptr, nullptr, nullptr) == LK_ERR_NOT_FOUND);
    CHECK(sched_poll(&S.s, 0xdeadbeefull, nullptr, nullptr, nullptr, nullptr, nullptr) == LK_ERR_NOT_FOUND);
}

void case_staging_full_and_close_in_flight()
{
    Server S(make_cfg(2, 16, 4, 1, 2, 0));
    S.be.latency_us = 20000;
    uint32_t id;
    CHECK(sched_open_stream(&S.s, 32, 32, &id) == LK_SUCCESS);
    std::vector<uint8_t> f = frame(32, 32, 0, 0);
    std::vector<float> p = points(32, 32, 8, 0);
    uint64_t t1, t2, t3;
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 8, &t1) == LK_SUCCESS);
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 8, &t2) == LK_SUCCESS);
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 8, &t3) == LK_ERR_BUSY);   // both slots hold frames
    // close while the first frame is (or is about to be) on the device: close
    // waits for it, drops the queued one, and both tickets become unknown
    CHECK(sched_close_stream(&S.s, id) == LK_SUCCESS);
    CHECK(sched_poll(&S.s, t1, nullptr, nullptr, nullptr, nullptr, nullptr) == LK_ERR_NOT_FOUND);
    CHECK(sched_poll(&S.s, t2, nullptr, nullptr, nullptr, nullptr, nullptr) == LK_ERR_NOT_FOUND);
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 8, &t3) == LK_ERR_NOT_FOUND);
    lk_server_stats st{};
    CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
    CHECK(st.open_streams == 0 && st.resident_bytes == 0);
    CHECK(S.be.open_count == 0 && S.be.violations == 0);
    // the stream table entry is reusable
    CHECK(sched_open_stream(&S.s, 32, 32, &id) == LK_SUCCESS);
    S.be.latency_us = 0;
    CHECK(sched_submit(&S.s, id, f.data(), 32, p.data(), nullptr, 8, &t1) == LK_SUCCESS);
    Result r;
    CHECK(poll_wait(&S.s, t1, &r, 16) == LK_SUCCESS && r.n == 0);   // a reopened stream starts cold
}

// A failed launch fails every frame in it; each stream keeps its last
// completed frame and tracks the next one from there.
void case_failures(bool device_error)
{
    Server S(make_cfg(4, 32, 8, 1, 4, 0));
    const int N = 3;
    uint32_t id[N];
    std::vector<float> p[N];
    std::vector<std::vector<uint8_t>> f[N];
    for (int i = 0; i < N; ++i) {
        CHECK(sched_open_stream(&S.s, 64, 48, &id[i]) == LK_SUCCESS);
        p[i] = points(64, 48, 24, i);
        for (int k = 0; k < 3; ++k) f[i].push_back(frame(64, 48, k, i));
    }
    auto prime_round = [&](int k, lk_result want) {
        uint64_t tk[N];
        S.be.latency_us = 3000;          // the whole round goes out as one launch
        for (int i = 0; i < N; ++i)
            CHECK(sched_submit(&S.s, id[i], f[i][k].data(), 64, p[i].data(), nullptr, 24, &tk[i]) == LK_SUCCESS);
        for (int i = 0; i < N; ++i) {
            Result r;
            CHECK(poll_wait(&S.s, tk[i], &r, 32) == want);
            if (want != LK_SUCCESS) CHECK(r.n == 0);
            else if (k > 0) expect_oracle(S.cfg, f[i][0], f[i][k], 64, 48, p[i], 24, r);
        }
    };
    prime_round(0, LK_SUCCESS);           // primes every stream with frame 0
    lk_server_stats before{};
    CHECK(sched_stats(&S.s, &before) == LK_SUCCESS);
    if (device_error) S.be.fail_completions = 1;
    else CHECK(sched_fail_next(&S.s, 1) == LK_SUCCESS);
    // frame 1 of every stream: the launch fails, and so does every frame in it
    // (the frames may go out in more than one launch; only the first fails)
    {
        uint64_t tk[N];
        for (int i = 0; i < N; ++i)
            CHECK(sched_submit(&S.s, id[i], f[i][1].data(), 64, p[i].data(), nullptr, 24, &tk[i]) == LK_SUCCESS);
        int failed = 0;
        for (int i = 0; i < N; ++i) {
            Result r;
            const lk_result e = poll_wait(&S.s, tk[i], &r, 32);
            CHECK(e == LK_SUCCESS || e == LK_ERR_DEVICE);
            if (e == LK_ERR_DEVICE) {
                ++failed;
                CHECK(r.n == 0);
                f[i][1] = f[i][0];           // this stream still holds frame 0
            } else {
                expect_oracle(S.cfg, f[i][0], f[i][1], 64, 48, p[i], 24, r);
            }
        }
        CHECK(failed >= 1);
    }
    lk_server_stats after{};
    CHECK(sched_stats(&S.s, &after) == LK_SUCCESS);
    CHECK(after.batches >= before.batches);
    // frame 2: tracked from the last frame each stream completed
    {
        uint64_t tk[N];
        for (int i = 0; i < N; ++i)
            CHECK(sched_submit(&S.s, id[i], f[i][2].data(), 64, p[i].data(), nullptr, 24, &tk[i]) == LK_SUCCESS);
        for (int i = 0; i < N; ++i) {
            Result r;
            CHECK(poll_wait(&S.s, tk[i], &r, 32) == LK_SUCCESS);
            expect_oracle(S.cfg, f[i][1], f[i][2], 64, 48, p[i], 24, r);
        }
    }
    CHECK(S.be.violations == 0);
}

// Several threads submit and poll at once (one stream each, plus a shared
// one whose frames carry guesses); a thread reads statistics meanwhile.
void case_threads()
{
    const int T = 4, F = 12;
    Server S(make_cfg(T + 1, 32, 8, 2, 3, 0));
    S.be.latency_us = 300;
    std::atomic<bool> done{false};
    std::thread stats([&] {
        while (!done) {
            lk_server_stats st{};
            CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            const int w = 48 + 16 * (t % 2), h = 40 + 8 * t;
            uint32_t id;
            CHECK(sched_open_stream(&S.s, w, h, &id) == LK_SUCCESS);
            std::vector<float> p = points(w, h, 20, t);
            std::vector<std::vector<uint8_t>> f;
            for (int k = 0; k < F; ++k) f.push_back(frame(w, h, k, t + 10));
            for (int k = 0; k < F; ++k) {
                uint64_t tk;
                lk_result e;
                while ((e = sched_submit(&S.s, id, f[k].data(), w, p.data(), nullptr, 20, &tk)) == LK_ERR_BUSY)
                    std::this_thread::yield();
                CHECK(e == LK_SUCCESS);
                Result r;
                CHECK(poll_wait(&S.s, tk, &r, 32) == LK_SUCCESS);
                if (k == 0) CHECK(r.n == 0);
                else expect_oracle(S.cfg, f[k - 1], f[k], w, h, p, 20, r);
            }
            CHECK(sched_close_stream(&S.s, id) == LK_SUCCESS);
        });
    for (auto &x : th) x.join();
    done = true;
    stats.join();
    lk_server_stats st{};
    CHECK(sched_stats(&S.s, &st) == LK_SUCCESS);
    CHECK(st.frames == (uint64_t)T * F && st.open_streams == 0 && st.resident_bytes == 0);
    CHECK(S.be.violations == 0);
}

// Stopping with frames queued and launches running drains and frees everything.
void case_stop_with_work()
{
    Server *S = new Server(make_cfg(3, 16, 2, 2, 4, 0));
    S->be.latency_us = 2000;
    std::vector<uint8_t> f = frame(32, 32, 0, 0);
    std::vector<float> p = points(32, 32, 8, 0);
    for (int i = 0; i < 3; ++i) {
        uint32_t id;
        CHECK(sched_open_stream(&S->s, 32, 32, &id) == LK_SUCCESS);
        for (int k = 0; k < 4; ++k) {
            uint64_t t;
            CHECK(sched_submit(&S->s, id, f.data(), 32, p.data(), nullptr, 8, &t) == LK_SUCCESS);
        }
    }
    delete S;
}

}  // namespace

int main()
{
    case_results_and_order();
    std::printf("results and order ok\n");
    case_timing_and_batching();
    std::printf("timing and batching ok\n");
    case_admission_and_limits();
    std::printf("admission and limits ok\n");
    case_invalid_arguments();
    std::printf("invalid arguments ok\n");
    case_staging_full_and_close_in_flight();
    std::printf("staging full and close in flight ok\n");
    case_failures(true);
    std::printf("device error ok\n");
    case_failures(false);
    std::printf("host-side launch failure ok\n");
    case_threads();
    std::printf("threads ok\n");
    case_stop_with_work();
    std::printf("sched cpu run ok\n");
    return 0;
}
