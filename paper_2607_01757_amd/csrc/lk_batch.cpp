// Prepared batched steps: device-resident job tables, optional HIP graph
// capture, persistent tracker launch, and the autotuner over execution
// shapes (lk_batch_* in lk.h).
#include "lk_runtime.h"

#include <cstring>
#include <new>
#include <vector>

using namespace lkmi;

struct lk_batch {
    lk_context *ctx = nullptr;
    BuildTables build;
    void *d_tab = nullptr;           // build tables, batch items, work counters
    const char *d_build = nullptr;
    const BatchItem *d_items = nullptr;
    int *d_counters = nullptr;
    int n_items = 0;
    long long total = 0;
    int storage = 0;
    TrackArgs args{};
    lk_exec_config cfg{};
    int num_cus = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

hipError_t enqueue_step(lk_batch *b, hipStream_t s)
{
    hipError_t e = launch_build_tables(b->build, b->d_build, s);
    if (e != hipSuccess || b->total == 0) return e;
    if (b->cfg.persistent)
        return launch_track_persistent(b->d_items, b->n_items, (int)b->total, b->args, b->storage, b->d_counters,
                                       b->cfg.blocks_per_cu, b->num_cus, s);
    return launch_track_batched(b->d_items, b->n_items, (int)b->total, b->args, b->storage, s);
}

void drop_graph(lk_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

lk_result capture(lk_batch *b)
{
    drop_graph(b);
    if (!b->cfg.use_graph) return LK_SUCCESS;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = enqueue_step(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) return hip_fail(le, "launch during capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return LK_SUCCESS;
}

lk_result check_cfg(const lk_exec_config *c)
{
    if (c->persistent != 0 && c->persistent != 1) return fail(LK_ERR_INVALID_ARG, "persistent must be 0 or 1");
    if (c->persistent && (c->blocks_per_cu < 1 || c->blocks_per_cu > 64))
        return fail(LK_ERR_INVALID_ARG, "blocks_per_cu must be in [1, 64]");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(LK_ERR_INVALID_ARG, "use_graph must be 0 or 1");
    if (c->reserved != 0) return fail(LK_ERR_INVALID_ARG, "reserved must be 0");
    return LK_SUCCESS;
}

}  // namespace

extern "C" {

lk_result lk_batch_create(lk_context *ctx, const lk_batch_desc *d, const lk_exec_config *cfg, lk_batch **out)
{
    if (!ctx || !d || !out) return fail(LK_ERR_INVALID_ARG, "ctx, desc or out is NULL");
    *out = nullptr;
    lk_exec_config c = cfg ? *cfg : lk_exec_config{0, 4, 1, 0};
    lk_result r = check_cfg(&c);
    if (r != LK_SUCCESS) return r;
    if (d->n_builds < 0 || d->n_pairs < 0) return fail(LK_ERR_INVALID_ARG, "negative counts");
    if (d->n_builds > 0 && (!d->build_pyrs || !d->build_imgs || !d->build_pitches))
        return fail(LK_ERR_INVALID_ARG, "NULL build arrays");
    if (d->n_pairs > 0 && !d->pairs) return fail(LK_ERR_INVALID_ARG, "NULL pairs");
    for (int i = 0; i < d->n_builds; ++i) {
        lk_pyramid *p = d->build_pyrs[i];
        if (!p || !d->build_imgs[i]) return fail(LK_ERR_INVALID_ARG, "build %d: NULL pyramid or image", i);
        if (p->ctx != ctx) return fail(LK_ERR_INVALID_ARG, "build %d: pyramid of another context", i);
        if (d->build_pitches[i] < p->desc.lv[0].w) return fail(LK_ERR_INVALID_ARG, "build %d: pitch < width", i);
    }
    // record level 0 of the rebuilt pyramids before the pairs are checked (a
    // pair may use a pyramid that only this step builds)
    std::vector<std::pair<const void *, int32_t>> saved(d->n_builds);
    std::vector<bool> was_built(d->n_builds);
    for (int i = 0; i < d->n_builds; ++i) {
        lk_pyramid *p = d->build_pyrs[i];
        saved[i] = {p->desc.lv[0].img, p->desc.lv[0].pitch};
        was_built[i] = p->built;
        p->desc.lv[0].img = d->build_imgs[i];
        p->desc.lv[0].pitch = d->build_pitches[i];
        p->built = true;
    }
    auto restore = [&]() {
        for (int i = 0; i < d->n_builds; ++i) {
            d->build_pyrs[i]->desc.lv[0].img = saved[i].first;
            d->build_pyrs[i]->desc.lv[0].pitch = saved[i].second;
            d->build_pyrs[i]->built = was_built[i];
        }
    };
    std::vector<BatchItem> items;
    int storage = LK_STORAGE_F32;
    long long total = 0;
    if (d->n_pairs > 0) {
        r = plan_batch(ctx, d->pairs, d->n_pairs, &d->params, &items, &storage, &total);
        if (r != LK_SUCCESS) { restore(); return r; }
        if (total > 0 && (!d->d_pts || !d->d_out_pts || !d->d_status || !d->d_residual)) {
            restore();
            return fail(LK_ERR_INVALID_ARG, "NULL point or output array");
        }
        if (d->params.use_guess && !d->d_guess) { restore(); return fail(LK_ERR_INVALID_ARG, "use_guess without d_guess"); }
    }
    lk_batch *b = new (std::nothrow) lk_batch();
    if (!b) { restore(); return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed"); }
    b->ctx = ctx;
    b->cfg = c;
    b->storage = storage;
    b->total = total;
    b->n_items = (int)items.size();
    make_build_tables(d->build_pyrs, d->n_builds, &b->build);
    const size_t items_off = (b->build.bytes + 255) & ~size_t(255);
    const size_t cnt_off = (items_off + items.size() * sizeof(BatchItem) + 255) & ~size_t(255);
    const size_t bytes = cnt_off + 8 * sizeof(int);
    (void)hipSetDevice(ctx->device);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) { delete b; return hip_fail(e, "hipGetDeviceProperties"); }
    b->num_cus = prop.multiProcessorCount;
    e = hipMalloc(&b->d_tab, bytes);
    if (e != hipSuccess) { delete b; return hip_fail(e, "hipMalloc(batch tables)"); }
    std::vector<char> host(bytes, 0);
    b->build.pack(host.data());
    if (!items.empty()) std::memcpy(host.data() + items_off, items.data(), items.size() * sizeof(BatchItem));
    e = hipMemcpy(b->d_tab, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(b->d_tab); delete b; return hip_fail(e, "hipMemcpy(batch tables)"); }
    b->d_build = static_cast<const char *>(b->d_tab);
    b->d_items = reinterpret_cast<const BatchItem *>(static_cast<char *>(b->d_tab) + items_off);
    b->d_counters = reinterpret_cast<int *>(static_cast<char *>(b->d_tab) + cnt_off);
    b->args = make_args(&d->params, (int)total, d->d_pts, d->d_guess, d->d_out_pts, d->d_status, d->d_residual,
                        d->d_iters);
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { (void)hipFree(b->d_tab); delete b; return hip_fail(e, "hipStreamCreate"); }
    r = capture(b);
    if (r != LK_SUCCESS) { lk_batch_destroy(b); return r; }
    *out = b;
    return LK_SUCCESS;
}

lk_result lk_batch_run(lk_batch *b, lk_stream stream)
{
    if (!b) return fail(LK_ERR_INVALID_ARG, "batch is NULL");
    (void)hipSetDevice(b->ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = b->exec ? hipGraphLaunch(b->exec, s) : enqueue_step(b, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "batch launch");
}

lk_result lk_batch_config(const lk_batch *b, lk_exec_config *cfg)
{
    if (!b || !cfg) return fail(LK_ERR_INVALID_ARG, "NULL argument");
    *cfg = b->cfg;
    return LK_SUCCESS;
}

lk_result lk_batch_tune(lk_batch *b, lk_stream stream, int32_t reps, lk_exec_config *best, float *best_ms)
{
    if (!b) return fail(LK_ERR_INVALID_ARG, "batch is NULL");
    if (reps < 1) return fail(LK_ERR_INVALID_ARG, "reps must be >= 1");
    (void)hipSetDevice(b->ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int use_graph = b->cfg.use_graph;
    static const lk_exec_config cands[] = {
        {0, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 0, 0}, {1, 3, 0, 0}, {1, 4, 0, 0}, {1, 8, 0, 0}, {1, 16, 0, 0}};
    hipEvent_t a, z;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&z) != hipSuccess)
        return fail(LK_ERR_DEVICE, "hipEventCreate failed");
    drop_graph(b);
    float bt = 1e30f;
    lk_exec_config bc = b->cfg;
    hipError_t e = hipSuccess;
    for (const auto &c : cands) {
        b->cfg = c;
        e = enqueue_step(b, s);                    // warm-up
        for (int i = 0; i < reps && e == hipSuccess; ++i) {
            if (i == 0) e = hipEventRecord(a, s);
            if (e == hipSuccess) e = enqueue_step(b, s);
        }
        if (e == hipSuccess) e = hipEventRecord(z, s);
        if (e == hipSuccess) e = hipEventSynchronize(z);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, z);
        if (e != hipSuccess) break;
        ms /= reps;
        if (ms < bt) { bt = ms; bc = c; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    bc.use_graph = use_graph;
    b->cfg = bc;
    if (e != hipSuccess) return hip_fail(e, "tuning launch");
    lk_result r = capture(b);
    if (r != LK_SUCCESS) return r;
    if (best) *best = bc;
    if (best_ms) *best_ms = bt;
    return LK_SUCCESS;
}

lk_result lk_batch_destroy(lk_batch *b)
{
    if (!b) return fail(LK_ERR_INVALID_ARG, "batch is NULL");
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_tab) (void)hipFree(b->d_tab);
    delete b;
    return LK_SUCCESS;
}

}  // extern "C"
