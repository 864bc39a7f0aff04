// Prepared batched steps: device-resident job tables, optional HIP graph
// capture, persistent tracker launch, and the autotuner over execution
// shapes (lk_batch_* in lk.h).
#include "lk_runtime.h"

#include <dlfcn.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
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
    int win = 0;
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
                                       b->cfg.blocks_per_cu, b->num_cus, b->cfg.chunk > 0 ? b->cfg.chunk : 16, s);
    return launch_track_batched(b->d_items, b->n_items, (int)b->total, b->args, b->storage, s,
                                b->cfg.waves_per_group);
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

lk_result check_cfg(const lk_exec_config *c, int win)
{
    if (c->persistent != 0 && c->persistent != 1) return fail(LK_ERR_INVALID_ARG, "persistent must be 0 or 1");
    if (c->persistent && (c->blocks_per_cu < 1 || c->blocks_per_cu > 64))
        return fail(LK_ERR_INVALID_ARG, "blocks_per_cu must be in [1, 64]");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(LK_ERR_INVALID_ARG, "use_graph must be 0 or 1");
    if (c->chunk < 0 || c->chunk > 1024) return fail(LK_ERR_INVALID_ARG, "chunk must be in [0, 1024]");
    if (c->waves_per_group != 0 && (c->persistent || !track_waves_supported(win, c->waves_per_group)))
        return fail(LK_ERR_INVALID_ARG, "waves_per_group %d is not built for win %d%s", c->waves_per_group, win,
                    c->persistent ? " (or the grid is persistent)" : "");
    if (c->reserved != 0) return fail(LK_ERR_INVALID_ARG, "reserved must be 0");
    return LK_SUCCESS;
}

// ------------------------------------------------------------ shape table

struct TableRow {
    std::string arch;
    int win, levels, storage, res, kp;
    lk_exec_config cfg;
};

std::mutex g_table_mu;
std::string g_table_file;            // the file g_table was read from ("" : never read)
bool g_table_read = false;
std::vector<TableRow> g_table;

std::string table_path()
{
    if (const char *env = std::getenv("LKMI_EXEC_TABLE")) return env;
    Dl_info info{};
    if (dladdr(reinterpret_cast<void *>(&lk_exec_buckets), &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/lk_exec_table.txt";
    }
    return "lk_exec_table.txt";
}

// (Re)reads the table when its path differs from the last read one; the
// caller holds g_table_mu.
void load_table()
{
    const std::string path = table_path();
    if (g_table_read && path == g_table_file) return;
    g_table_read = true;
    g_table_file = path;
    g_table.clear();
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (char *hash = std::strchr(line, '#')) *hash = 0;
        char arch[64];
        TableRow r{};
        const int got = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d", arch, &r.win, &r.levels, &r.storage,
                                    &r.res, &r.kp, &r.cfg.persistent, &r.cfg.blocks_per_cu, &r.cfg.use_graph,
                                    &r.cfg.chunk, &r.cfg.waves_per_group);
        if (got != 11) continue;                  // blank, comment or malformed line
        if (check_cfg(&r.cfg, r.win) != LK_SUCCESS) continue;
        r.arch = arch;
        g_table.push_back(r);
    }
    std::fclose(f);
    clear_error();
}

std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// The table's shape for desc (pairs already checked), or the default.
lk_exec_config table_shape(lk_context *ctx, const lk_batch_desc *d, int *found)
{
    lk_exec_config c{0, 0, 1, 0, 0, 0};
    *found = 0;
    if (d->n_pairs <= 0) return c;
    long long px = 0, kp = 0;
    for (int i = 0; i < d->n_pairs; ++i) {
        px += (long long)d->pairs[i].prev->desc.lv[0].w * d->pairs[i].prev->desc.lv[0].h;
        kp += d->pairs[i].n;
    }
    int rb = 0, kb = 0;
    (void)lk_exec_buckets(px / d->n_pairs, (int32_t)(kp / d->n_pairs), &rb, &kb);
    const std::string arch = device_arch(ctx->device);
    const int storage = d->pairs[0].prev->desc.storage;
    std::lock_guard<std::mutex> lock(g_table_mu);
    load_table();
    for (const TableRow &r : g_table)
        if (r.arch == arch && r.win == d->params.win && r.levels == d->params.levels && r.storage == storage &&
            r.res == rb && r.kp == kb) {
            *found = 1;
            return r.cfg;
        }
    return c;
}

}  // namespace

extern "C" {

lk_result lk_batch_create(lk_context *ctx, const lk_batch_desc *d, const lk_exec_config *cfg, lk_batch **out)
{
    if (!ctx || !d || !out) return fail(LK_ERR_INVALID_ARG, "ctx, desc or out is NULL");
    *out = nullptr;
    lk_exec_config c = cfg ? *cfg : lk_exec_config{0, 0, 1, 0, 0, 0};
    lk_result r = check_cfg(&c, d->params.win);
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
    if (!cfg && d->n_pairs > 0) {
        int found = 0;
        c = table_shape(ctx, d, &found);
    }
    lk_batch *b = new (std::nothrow) lk_batch();
    if (!b) { restore(); return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed"); }
    b->ctx = ctx;
    b->cfg = c;
    b->win = d->params.win;
    b->storage = storage;
    b->total = total;
    b->n_items = (int)items.size();
    make_build_tables(d->build_pyrs, d->n_builds, &b->build);
    const size_t items_off = (b->build.bytes + 255) & ~size_t(255);
    const size_t cnt_off = (items_off + items.size() * sizeof(BatchItem) + 255) & ~size_t(255);
    const size_t bytes = cnt_off + kCounterBytes;
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
    // candidates: hardware dispatch with every built workgroup size, and
    // persistent grids (half and full residency of the 5-wave build, fine
    // and coarse work fetches)
    std::vector<lk_exec_config> cands;
    for (int w : {0, 2, 4})
        if (track_waves_supported(b->win, w)) cands.push_back({0, 0, 0, 0, w, 0});
    for (int bpc : {10, 20})
        for (int chunk : {8, 32}) cands.push_back({1, bpc, 0, chunk, 0, 0});
    hipEvent_t a, z;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&z) != hipSuccess)
        return fail(LK_ERR_DEVICE, "hipEventCreate failed");
    drop_graph(b);
    hipError_t e = hipSuccess;
    // untimed steps until the device has run about 20 ms of them: its clock
    // rises over the first tens of milliseconds of sustained work, and the
    // first candidates would otherwise be timed at a lower one
    b->cfg = cands[0];
    const auto t0 = std::chrono::steady_clock::now();
    while (e == hipSuccess && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(20)) {
        for (int i = 0; i < 4 && e == hipSuccess; ++i) e = enqueue_step(b, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    float bt = 1e30f;
    lk_exec_config bc = b->cfg;
    for (const auto &c : cands) {
        if (e != hipSuccess) break;
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

lk_result lk_exec_buckets(int64_t mean_pixels, int32_t mean_points, int32_t *res_bucket, int32_t *kp_bucket)
{
    if (!res_bucket || !kp_bucket) return fail(LK_ERR_INVALID_ARG, "NULL output");
    if (mean_pixels < 0 || mean_points < 0) return fail(LK_ERR_INVALID_ARG, "negative mean");
    static const int64_t px_edges[] = {400000, 700000, 1500000, 3000000};
    static const int32_t kp_edges[] = {256, 512, 1024, 2048};
    int rb = 0, kb = 0;
    while (rb < 4 && mean_pixels >= px_edges[rb]) ++rb;
    while (kb < 4 && mean_points >= kp_edges[kb]) ++kb;
    *res_bucket = rb;
    *kp_bucket = kb;
    return LK_SUCCESS;
}

lk_result lk_exec_table_lookup(lk_context *ctx, const lk_batch_desc *d, lk_exec_config *out, int32_t *found)
{
    if (!ctx || !d || !out || !found) return fail(LK_ERR_INVALID_ARG, "NULL argument");
    if (d->n_pairs < 0 || (d->n_pairs > 0 && !d->pairs)) return fail(LK_ERR_INVALID_ARG, "bad pairs");
    for (int i = 0; i < d->n_pairs; ++i) {
        lk_result r = check_pair(ctx, d->pairs[i].prev, d->pairs[i].next, i);
        if (r != LK_SUCCESS) return r;
    }
    int f = 0;
    *out = table_shape(ctx, d, &f);
    *found = f;
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
