// Host runtime of liblkmi: contexts, pyramid objects, argument checks, the
// C ABI of lk.h, and the staging of batch tables.
#include "lk_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace lkmi;

// ------------------------------------------------------------------ errors

namespace lkmi {

lk_result hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? LK_ERR_OUT_OF_MEMORY : LK_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// ------------------------------------------------------------------ staging

lk_result StagingRing::init(int nslots)
{
    slots.resize(nslots);
    for (auto &s : slots) {
        hipError_t e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    return LK_SUCCESS;
}

void StagingRing::release()
{
    for (auto &s : slots) {
        if (s.done) (void)hipEventSynchronize(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.done) (void)hipEventDestroy(s.done);
        s = Slot{};
    }
}

lk_result StagingRing::acquire(size_t bytes, Slot **out)
{
    Slot &s = slots[next];
    next = (next + 1) % (int)slots.size();
    hipError_t e = hipEventSynchronize(s.done);   // previous user of this slot has finished
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    if (bytes > s.cap) {
        size_t cap = std::max<size_t>(bytes, 2 * s.cap);
        cap = (cap + 4095) & ~size_t(4095);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        s.host = nullptr; s.dev = nullptr; s.cap = 0;
        e = hipHostMalloc(&s.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
        e = hipMalloc(&s.dev, cap);
        if (e != hipSuccess) { (void)hipHostFree(s.host); s.host = nullptr; return hip_fail(e, "hipMalloc"); }
        s.cap = cap;
    }
    *out = &s;
    return LK_SUCCESS;
}

// ------------------------------------------------- fixed batch-table array
//
// lk_track_batched_noalloc keeps its batch table here instead of in memory
// the library allocates on demand: LK_NOALLOC_MAX_PAIRS items, one copy per
// device, held until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code it is a stand-in, not a device
// address): it uses the address hipGetSymbolAddress returns for the current
// device, taken once per device at context creation.

static_assert(sizeof(BatchItem) == 40, "LK_NOALLOC_MAX_PAIRS entries take 160 KiB");
static __device__ __align__(256) unsigned char scratch[LK_NOALLOC_MAX_PAIRS * sizeof(BatchItem)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of this device's array; the device must be current.
lk_result scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(LK_ERR_INVALID_ARG, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(batch-table array)");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return LK_SUCCESS;
}

}  // namespace

// ------------------------------------------------------------------ checks

int level_dims(int w, int h, int levels, int32_t *ws, int32_t *hs)
{
    if (levels < 1 || levels > LK_MAX_LEVELS || w < 1 || h < 1) return -1;
    ws[0] = w; hs[0] = h;
    for (int l = 1; l < levels; ++l) {
        ws[l] = (ws[l - 1] + 1) / 2;
        hs[l] = (hs[l - 1] + 1) / 2;
    }
    return (ws[levels - 1] >= 4 && hs[levels - 1] >= 4) ? 0 : -1;
}

lk_result check_params(const lk_params *p, int pyr_levels)
{
    if (!p) return fail(LK_ERR_INVALID_ARG, "params is NULL");
    // windows above 31 would need the four-column lane layout, which is not
    // built (an earlier build of it faulted on the GPU and no cause was shown)
    if (p->win < 3 || p->win > LK_MAX_WIN || (p->win & 1) == 0)
        return fail(LK_ERR_INVALID_ARG, "win must be odd in [3, %d] (got %d)", LK_MAX_WIN, p->win);
    if (p->levels < 1 || p->levels > pyr_levels)
        return fail(LK_ERR_INVALID_ARG, "levels must be in [1, %d] (got %d)", pyr_levels, p->levels);
    if (p->max_iters < 1 || p->max_iters > 1000)
        return fail(LK_ERR_INVALID_ARG, "max_iters must be in [1, 1000] (got %d)", p->max_iters);
    if (!(p->eps > 0.0f) || !std::isfinite(p->eps)) return fail(LK_ERR_INVALID_ARG, "eps must be > 0");
    if (!(p->min_eig >= 0.0f) || !std::isfinite(p->min_eig)) return fail(LK_ERR_INVALID_ARG, "min_eig must be >= 0");
    if (!(p->fb_thresh >= 0.0f) || !std::isfinite(p->fb_thresh))
        return fail(LK_ERR_INVALID_ARG, "fb_thresh must be >= 0");
    if (p->use_guess != 0 && p->use_guess != 1) return fail(LK_ERR_INVALID_ARG, "use_guess must be 0 or 1");
    if (p->reserved != 0) return fail(LK_ERR_INVALID_ARG, "reserved must be 0");
    return LK_SUCCESS;
}

TrackArgs make_args(const lk_params *p, int n, const float *pts, const float *guess, float *out, uint8_t *st,
                    float *res, int32_t *iters)
{
    TrackArgs a;
    a.win = p->win; a.levels = p->levels; a.max_iters = p->max_iters; a.use_guess = p->use_guess;
    a.eps = p->eps; a.min_eig = p->min_eig; a.fb_thresh = p->fb_thresh;
    a.n = n; a.pts = pts; a.guess = p->use_guess ? guess : nullptr;
    a.out_pts = out; a.status = st; a.residual = res; a.iters = iters;
    return a;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Down/grad jobs that build one pyramid from its recorded level 0.
void pyramid_jobs(const lk_pyramid *p, std::vector<Pyr12Job> *p12, std::vector<DownJob> *down_by_level,
                  std::vector<GradJob> *grads)
{
    const PyrDesc &d = p->desc;
    const bool f16 = d.storage == LK_STORAGE_F16;
    int first = 1;
    if (d.levels >= 3) {
        Pyr12Job j{};
        j.src = static_cast<const uint8_t *>(d.lv[0].img);
        j.dst1 = const_cast<void *>(d.lv[1].img);
        j.dst2 = const_cast<void *>(d.lv[2].img);
        j.spitch = d.lv[0].pitch; j.pitch1 = d.lv[1].pitch; j.pitch2 = d.lv[2].pitch;
        j.sw = d.lv[0].w; j.sh = d.lv[0].h; j.w1 = d.lv[1].w; j.h1 = d.lv[1].h; j.w2 = d.lv[2].w; j.h2 = d.lv[2].h;
        j.f16 = f16;
        if (f16) {      // the fused launch also writes the gradient plane of level 1
            j.g1 = const_cast<__half2 *>(d.lv[1].grad); j.gpitch1 = d.lv[1].gpitch;
        }
        j.tiles_x = (j.w2 + kP12TileW - 1) / kP12TileW;
        j.tile_begin = 0;
        p12->push_back(j);
        first = 3;
    }
    for (int l = first; l < d.levels; ++l) {
        DownJob j{};
        j.src = d.lv[l - 1].img; j.dst = const_cast<void *>(d.lv[l].img);
        j.spitch = d.lv[l - 1].pitch; j.dpitch = d.lv[l].pitch;
        j.sw = d.lv[l - 1].w; j.sh = d.lv[l - 1].h; j.dw = d.lv[l].w; j.dh = d.lv[l].h;
        j.src_u8 = l == 1; j.dst_f16 = f16;
        j.tiles_x = (j.dw + kDownTileW - 1) / kDownTileW;
        j.tile_begin = 0;
        down_by_level[l].push_back(j);
    }
    if (f16)   // level 0 has no stored plane: the tracker forms its gradients from the frame
        for (int l = first == 3 ? 2 : 1; l < d.levels; ++l) {
            GradJob g{};
            g.src = d.lv[l].img; g.dst = const_cast<__half2 *>(d.lv[l].grad);
            g.spitch = d.lv[l].pitch; g.dpitch = d.lv[l].gpitch;
            g.w = d.lv[l].w; g.h = d.lv[l].h; g.src_u8 = l == 0;
            g.tiles_x = (g.w + kGradTileW - 1) / kGradTileW;
            g.tile_begin = 0;
            grads->push_back(g);
        }
}

}  // namespace lkmi

// ====================================================================== ABI

extern "C" {

lk_result lk_params_check(const lk_params *params, int32_t pyr_levels)
{
    if (pyr_levels < 1 || pyr_levels > LK_MAX_LEVELS)
        return fail(LK_ERR_INVALID_ARG, "pyr_levels must be in [1, %d] (got %d)", LK_MAX_LEVELS, pyr_levels);
    lk_result r = check_params(params, pyr_levels);
    if (r == LK_SUCCESS) clear_error();
    return r;
}

lk_params lk_params_default(void)
{
    lk_params p;
    p.win = 21; p.levels = 3; p.max_iters = 30; p.use_guess = 0;
    p.eps = 0.01f; p.min_eig = 1e-6f; p.fb_thresh = 0.0f; p.reserved = 0;
    return p;
}

lk_result lk_context_create(int32_t device, uint64_t hbm_budget_bytes, lk_context **out)
{
    if (!out) return fail(LK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(LK_ERR_INVALID_ARG, "device %d not in [0, %d)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    lk_context *c = new (std::nothrow) lk_context();
    if (!c) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->device = device;
    c->budget = hbm_budget_bytes;
    lk_result r = c->staging.init(8);
    if (r == LK_SUCCESS) r = scratch_address(device, &c->table_dev);
    if (r == LK_SUCCESS) {
        e = hipHostMalloc(&c->table_host, LK_NOALLOC_MAX_PAIRS * sizeof(BatchItem), hipHostMallocDefault);
        if (e != hipSuccess) { c->table_host = nullptr; r = hip_fail(e, "hipHostMalloc(batch table)"); }
    }
    if (r == LK_SUCCESS) {
        e = hipEventCreateWithFlags(&c->table_done, hipEventDisableTiming);
        if (e != hipSuccess) { c->table_done = nullptr; r = hip_fail(e, "hipEventCreate"); }
    }
    if (r != LK_SUCCESS) {
        c->staging.release();
        if (c->table_host) (void)hipHostFree(c->table_host);
        delete c;
        return r;
    }
    *out = c;
    clear_error();
    return LK_SUCCESS;
}

void lk_context_destroy(lk_context *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->graphs_release();
    ctx->staging.release();
    if (ctx->table_done) (void)hipEventDestroy(ctx->table_done);
    if (ctx->table_host) (void)hipHostFree(ctx->table_host);
    delete ctx;
}

uint64_t lk_context_bytes_in_use(const lk_context *ctx) { return ctx ? ctx->in_use.load() : 0; }

lk_result lk_pyramid_create(lk_context *ctx, int32_t w, int32_t h, int32_t levels, int32_t storage, lk_pyramid **out)
{
    if (!ctx || !out) return fail(LK_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    if (storage != LK_STORAGE_F32 && storage != LK_STORAGE_F16)
        return fail(LK_ERR_INVALID_ARG, "storage must be LK_STORAGE_F32 or LK_STORAGE_F16");
    int32_t ws[LK_MAX_LEVELS], hs[LK_MAX_LEVELS];
    if (w > (1 << 15) || h > (1 << 15) || level_dims(w, h, levels, ws, hs) != 0)
        return fail(LK_ERR_INVALID_ARG, "bad pyramid shape %dx%d with %d levels (1..8 levels, coarsest >= 4x4, "
                    "sides <= 32768)", w, h, levels);
    lk_pyramid *p = new (std::nothrow) lk_pyramid();
    if (!p) return fail(LK_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->ctx = ctx;
    PyrDesc &d = p->desc;
    std::memset(&d, 0, sizeof d);
    d.levels = levels;
    d.storage = storage;
    const size_t es = storage == LK_STORAGE_F16 ? 2 : 4;
    size_t off[LK_MAX_LEVELS] = {0}, goff[LK_MAX_LEVELS] = {0};
    size_t total = align_up(sizeof(PyrDesc), 256);   // the device copy of the descriptor comes first
    for (int l = 0; l < levels; ++l) {
        d.lv[l].w = ws[l]; d.lv[l].h = hs[l];
        if (l > 0) {
            d.lv[l].pitch = (int32_t)align_up(ws[l], 256 / es);
            off[l] = total;
            total = align_up(total + (size_t)d.lv[l].pitch * hs[l] * es, 256);
        }
        if (storage == LK_STORAGE_F16 && l > 0) {
            d.lv[l].gpitch = (int32_t)align_up(ws[l], 64);
            goff[l] = total;
            total = align_up(total + (size_t)d.lv[l].gpitch * hs[l] * 4, 256);
        }
    }
    if (ctx->budget && ctx->in_use.load() + total > ctx->budget) {
        delete p;
        return fail(LK_ERR_OUT_OF_MEMORY, "pyramid of %zu bytes exceeds the context budget", total);
    }
    (void)hipSetDevice(ctx->device);
    {
        hipError_t e = hipMalloc(&p->base, total);
        if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc(pyramid)"); }
    }
    p->bytes = total;
    ctx->in_use += total;
    char *b = static_cast<char *>(p->base);
    p->d_desc = reinterpret_cast<PyrDesc *>(b);
    for (int l = 0; l < levels; ++l) {
        if (l > 0) d.lv[l].img = b + off[l];
        if (storage == LK_STORAGE_F16 && l > 0) d.lv[l].grad = reinterpret_cast<const __half2 *>(b + goff[l]);
    }
    *out = p;
    return LK_SUCCESS;
}

lk_result lk_pyramid_destroy(lk_pyramid *pyr)
{
    if (!pyr) return fail(LK_ERR_INVALID_ARG, "pyr is NULL");
    if (pyr->base) {
        (void)hipSetDevice(pyr->ctx->device);
        hipError_t e = hipFree(pyr->base);
        pyr->ctx->in_use -= pyr->bytes;
        delete pyr;
        if (e != hipSuccess) return hip_fail(e, "hipFree(pyramid)");
        return LK_SUCCESS;
    }
    delete pyr;
    return LK_SUCCESS;
}

lk_result lk_pyramid_info(const lk_pyramid *pyr, int32_t *w, int32_t *h, int32_t *levels, int32_t *storage)
{
    if (!pyr) return fail(LK_ERR_INVALID_ARG, "pyr is NULL");
    if (w) *w = pyr->desc.lv[0].w;
    if (h) *h = pyr->desc.lv[0].h;
    if (levels) *levels = pyr->desc.levels;
    if (storage) *storage = pyr->desc.storage;
    return LK_SUCCESS;
}

lk_result lk_build_pyramid(lk_context *ctx, lk_pyramid *pyr, const uint8_t *d_img, int32_t pitch, lk_stream stream)
{
    if (!ctx || !pyr || !d_img) return fail(LK_ERR_INVALID_ARG, "ctx, pyr or d_img is NULL");
    if (pyr->ctx != ctx) return fail(LK_ERR_INVALID_ARG, "pyramid belongs to another context");
    if (pitch < pyr->desc.lv[0].w) return fail(LK_ERR_INVALID_ARG, "pitch %d < width %d", pitch, pyr->desc.lv[0].w);
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    pyr->desc.lv[0].img = d_img;
    pyr->desc.lv[0].pitch = pitch;
    std::vector<Pyr12Job> p12;
    std::vector<DownJob> down[LK_MAX_LEVELS];
    std::vector<GradJob> grads;
    pyramid_jobs(pyr, &p12, down, &grads);
    // the device descriptor rides on the fused level-1/2 launch when there is
    // one (a pyramid of three or more levels), else it takes a launch of its own
    if (p12.empty()) {
        hipError_t e = launch_write_desc(pyr->d_desc, pyr->desc, s);
        if (e != hipSuccess) return hip_fail(e, "descriptor write launch");
    }
    for (size_t i = 0; i < p12.size(); ++i) {
        hipError_t e = launch_pyr12(p12[i], i == 0 ? pyr->d_desc : nullptr, pyr->desc, s);
        if (e != hipSuccess) return hip_fail(e, "pyramid kernel launch");
    }
    for (int l = 1; l < pyr->desc.levels; ++l)
        for (auto &j : down[l]) {
            hipError_t e = launch_downsample(j, s);
            if (e != hipSuccess) return hip_fail(e, "pyramid kernel launch");
        }
    for (auto &g : grads) {
        hipError_t e = launch_grad(g, s);
        if (e != hipSuccess) return hip_fail(e, "gradient kernel launch");
    }
    pyr->built = true;
    return LK_SUCCESS;
}

lk_result lk_build_pyramids(lk_context *ctx, lk_pyramid *const *h_pyrs, const uint8_t *const *h_imgs,
                            const int32_t *h_pitches, int32_t n, lk_stream stream)
{
    if (!ctx) return fail(LK_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0) return fail(LK_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return LK_SUCCESS;
    if (!h_pyrs || !h_imgs || !h_pitches) return fail(LK_ERR_INVALID_ARG, "NULL array");
    for (int i = 0; i < n; ++i) {
        if (!h_pyrs[i] || !h_imgs[i]) return fail(LK_ERR_INVALID_ARG, "item %d: NULL pyramid or image", i);
        if (h_pyrs[i]->ctx != ctx) return fail(LK_ERR_INVALID_ARG, "item %d: pyramid of another context", i);
        if (h_pitches[i] < h_pyrs[i]->desc.lv[0].w) return fail(LK_ERR_INVALID_ARG, "item %d: pitch < width", i);
    }
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
        h_pyrs[i]->desc.lv[0].img = h_imgs[i];
        h_pyrs[i]->desc.lv[0].pitch = h_pitches[i];
    }
    return enqueue_build(ctx, h_pyrs, n, s);
}

lk_result lk_pyramid_read_level(lk_context *ctx, const lk_pyramid *pyr, int32_t level, float *d_dst, float *d_grad,
                                lk_stream stream)
{
    if (!ctx || !pyr || !d_dst) return fail(LK_ERR_INVALID_ARG, "ctx, pyr or d_dst is NULL");
    if (level < 0 || level >= pyr->desc.levels) return fail(LK_ERR_INVALID_ARG, "level must be in [0, levels)");
    if (!pyr->built) return fail(LK_ERR_INVALID_ARG, "pyramid was never built");
    (void)hipSetDevice(ctx->device);
    hipError_t e = launch_read_level(pyr->desc.lv[level], level, pyr->desc.storage, d_dst, d_grad,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "read level launch");
}

lk_result lk_track(lk_context *ctx, const lk_pyramid *prev, const lk_pyramid *next, const float *d_pts,
                   const float *d_guess, int32_t n, const lk_params *params, float *d_out_pts, uint8_t *d_status,
                   float *d_residual, int32_t *d_iters, lk_stream stream)
{
    if (!ctx || !prev || !next) return fail(LK_ERR_INVALID_ARG, "ctx, prev or next is NULL");
    lk_result r = check_pair(ctx, prev, next, -1);
    if (r != LK_SUCCESS) return r;
    r = check_params(params, std::min(prev->desc.levels, next->desc.levels));
    if (r != LK_SUCCESS) return r;
    if (n < 0) return fail(LK_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return LK_SUCCESS;
    if (!d_pts || !d_out_pts || !d_status || !d_residual)
        return fail(LK_ERR_INVALID_ARG, "NULL point or output array");
    if (params->use_guess && !d_guess) return fail(LK_ERR_INVALID_ARG, "use_guess set but d_guess is NULL");
    (void)hipSetDevice(ctx->device);
    TrackArgs a = make_args(params, n, d_pts, d_guess, d_out_pts, d_status, d_residual, d_iters);
    hipError_t e = launch_track(prev->d_desc, next->d_desc, prev->desc.storage, a, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "tracker launch");
}

lk_result lk_track_batched(lk_context *ctx, const lk_pair *h_pairs, int32_t n_pairs, const float *d_pts,
                           const float *d_guess, const lk_params *params, float *d_out_pts, uint8_t *d_status,
                           float *d_residual, int32_t *d_iters, lk_stream stream)
{
    if (!ctx) return fail(LK_ERR_INVALID_ARG, "ctx is NULL");
    if (n_pairs < 0) return fail(LK_ERR_INVALID_ARG, "n_pairs < 0");
    if (n_pairs == 0) return LK_SUCCESS;
    if (!h_pairs) return fail(LK_ERR_INVALID_ARG, "h_pairs is NULL");
    std::vector<BatchItem> items;
    int storage = -1;
    long long total = 0;
    lk_result r = plan_batch(ctx, h_pairs, n_pairs, params, &items, &storage, &total);
    if (r != LK_SUCCESS) return r;
    if (total == 0) return LK_SUCCESS;
    if (!d_pts || !d_out_pts || !d_status || !d_residual)
        return fail(LK_ERR_INVALID_ARG, "NULL point or output array");
    if (params->use_guess && !d_guess) return fail(LK_ERR_INVALID_ARG, "use_guess set but d_guess is NULL");
    (void)hipSetDevice(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StagingRing::Slot *slot = nullptr;
    const size_t bytes = items.size() * sizeof(BatchItem);
    r = ctx->staging.acquire(bytes, &slot);
    if (r != LK_SUCCESS) return r;
    std::memcpy(slot->host, items.data(), bytes);
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch table)");
    TrackArgs a = make_args(params, (int)total, d_pts, d_guess, d_out_pts, d_status, d_residual, d_iters);
    e = launch_track_batched(static_cast<const BatchItem *>(slot->dev), (int)items.size(), (int)total, a, storage, s);
    (void)hipEventRecord(slot->done, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "batched tracker launch");
}

lk_result lk_track_batched_noalloc(lk_context *ctx, const lk_pair *h_pairs, int32_t n_pairs, const float *d_pts,
                                   const float *d_guess, const lk_params *params, float *d_out_pts,
                                   uint8_t *d_status, float *d_residual, int32_t *d_iters, lk_stream stream)
{
    if (!ctx) return fail(LK_ERR_INVALID_ARG, "ctx is NULL");
    if (n_pairs < 0) return fail(LK_ERR_INVALID_ARG, "n_pairs < 0");
    if (n_pairs > LK_NOALLOC_MAX_PAIRS)
        return fail(LK_ERR_INVALID_ARG, "n_pairs %d exceeds the fixed batch table (%d pairs)", n_pairs,
                    LK_NOALLOC_MAX_PAIRS);
    if (n_pairs == 0) return LK_SUCCESS;
    if (!h_pairs) return fail(LK_ERR_INVALID_ARG, "h_pairs is NULL");
    if (!ctx->table_dev || !ctx->table_host || !ctx->table_done)
        return fail(LK_ERR_DEVICE, "the context has no batch-table array");
    (void)hipSetDevice(ctx->device);
    // the pinned table is rewritten only after the previous upload from it ended
    hipError_t e = hipEventSynchronize(ctx->table_done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    BatchItem *items = static_cast<BatchItem *>(ctx->table_host);
    int storage = -1;
    long long total = 0;
    lk_result r = plan_batch_into(ctx, h_pairs, n_pairs, params, items, &storage, &total);
    if (r != LK_SUCCESS) return r;
    if (total == 0) return LK_SUCCESS;
    if (!d_pts || !d_out_pts || !d_status || !d_residual)
        return fail(LK_ERR_INVALID_ARG, "NULL point or output array");
    if (params->use_guess && !d_guess) return fail(LK_ERR_INVALID_ARG, "use_guess set but d_guess is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)n_pairs * sizeof(BatchItem);
    e = hipMemcpyAsync(ctx->table_dev, items, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch table)");
    (void)hipEventRecord(ctx->table_done, s);
    TrackArgs a = make_args(params, (int)total, d_pts, d_guess, d_out_pts, d_status, d_residual, d_iters);
    e = launch_track_batched(static_cast<const BatchItem *>(ctx->table_dev), n_pairs, (int)total, a, storage, s);
    return e == hipSuccess ? LK_SUCCESS : hip_fail(e, "batched tracker launch");
}

}  // extern "C"

// ------------------------------------------------------------- shared helpers

namespace lkmi {

lk_result check_pair(const lk_context *ctx, const lk_pyramid *prev, const lk_pyramid *next, int idx)
{
    char tag[32] = "";
    if (idx >= 0) snprintf(tag, sizeof tag, "pair %d: ", idx);
    if (!prev || !next) return fail(LK_ERR_INVALID_ARG, "%sNULL pyramid", tag);
    if (prev->ctx != ctx || next->ctx != ctx) return fail(LK_ERR_INVALID_ARG, "%spyramid of another context", tag);
    if (!prev->built || !next->built) return fail(LK_ERR_INVALID_ARG, "%spyramid was never built", tag);
    if (prev->desc.lv[0].w != next->desc.lv[0].w || prev->desc.lv[0].h != next->desc.lv[0].h)
        return fail(LK_ERR_INVALID_ARG, "%sframes differ in size", tag);
    if (prev->desc.storage != next->desc.storage) return fail(LK_ERR_INVALID_ARG, "%sstorages differ", tag);
    return LK_SUCCESS;
}

lk_result plan_batch_into(lk_context *ctx, const lk_pair *pairs, int n_pairs, const lk_params *params,
                          BatchItem *items, int *storage, long long *total)
{
    int min_levels = LK_MAX_LEVELS;
    *storage = -1;
    *total = 0;
    for (int i = 0; i < n_pairs; ++i) {
        const lk_pair &p = pairs[i];
        lk_result r = check_pair(ctx, p.prev, p.next, i);
        if (r != LK_SUCCESS) return r;
        if (p.n < 0 || p.pt_offset < 0 || p.reserved != 0)
            return fail(LK_ERR_INVALID_ARG, "pair %d: negative n or offset, or reserved != 0", i);
        // the kernels index points with 32-bit integers (2 idx + 1 < 2^31)
        if (p.pt_offset + (int64_t)p.n > (int64_t(1) << 30))
            return fail(LK_ERR_INVALID_ARG, "pair %d: pt_offset + n exceeds 2^30", i);
        if (*storage >= 0 && p.prev->desc.storage != *storage)
            return fail(LK_ERR_INVALID_ARG, "pair %d: all pairs of one batch must share a storage", i);
        *storage = p.prev->desc.storage;
        min_levels = std::min(min_levels, std::min(p.prev->desc.levels, p.next->desc.levels));
        BatchItem it{};
        it.prev = p.prev->d_desc;
        it.next = p.next->d_desc;
        it.pt_offset = p.pt_offset;
        it.n = p.n;
        it.first_wave = (int32_t)*total;
        *total += p.n;
        if (*total > (1LL << 30)) return fail(LK_ERR_INVALID_ARG, "more than 2^30 points in one batch");
        items[i] = it;
    }
    return check_params(params, min_levels);
}

lk_result plan_batch(lk_context *ctx, const lk_pair *pairs, int n_pairs, const lk_params *params,
                     std::vector<BatchItem> *items, int *storage, long long *total)
{
    items->assign((size_t)std::max(n_pairs, 0), BatchItem{});
    return plan_batch_into(ctx, pairs, n_pairs, params, items->data(), storage, total);
}

namespace {

// Tile numbering of one launch: job k owns tiles [tile_begin, tile_begin +
// tiles); tj[t] is the job of tile t.
template <class J>
void number_tiles(std::vector<J> &jobs, std::vector<int32_t> &tj, int tile_h, int (*rows)(const J &))
{
    tj.clear();
    for (size_t k = 0; k < jobs.size(); ++k) {
        J &j = jobs[k];
        j.tile_begin = (int32_t)tj.size();
        const long long tiles = (long long)j.tiles_x * ((rows(j) + tile_h - 1) / tile_h);
        tj.insert(tj.end(), (size_t)tiles, (int32_t)k);
    }
}

size_t place(size_t *o, size_t bytes)
{
    const size_t at = *o;
    *o = (at + bytes + 15) & ~size_t(15);
    return at;
}

}  // namespace

void make_build_tables(lk_pyramid *const *pyrs, int n, BuildTables *t)
{
    *t = BuildTables{};
    t->descs.resize(n);
    for (int i = 0; i < n; ++i) {
        t->descs[i].dst = pyrs[i]->d_desc;
        t->descs[i].desc = pyrs[i]->desc;
        pyramid_jobs(pyrs[i], &t->p12, t->down, &t->grads);
    }
    number_tiles<Pyr12Job>(t->p12, t->tj_p12, kP12TileH, [](const Pyr12Job &j) { return (int)j.h2; });
    for (int l = 1; l < LK_MAX_LEVELS; ++l)
        number_tiles<DownJob>(t->down[l], t->tj_down[l], kDownTileH, [](const DownJob &j) { return (int)j.dh; });
    number_tiles<GradJob>(t->grads, t->tj_grad, kGradTileH, [](const GradJob &j) { return (int)j.h; });
    size_t o = 0;
    place(&o, t->descs.size() * sizeof(PyrDescWrite));
    t->off_p12 = place(&o, t->p12.size() * sizeof(Pyr12Job));
    for (int l = 1; l < LK_MAX_LEVELS; ++l) t->off_down[l] = place(&o, t->down[l].size() * sizeof(DownJob));
    t->off_grad = place(&o, t->grads.size() * sizeof(GradJob));
    t->off_tj_p12 = place(&o, t->tj_p12.size() * sizeof(int32_t));
    for (int l = 1; l < LK_MAX_LEVELS; ++l) t->off_tj_down[l] = place(&o, t->tj_down[l].size() * sizeof(int32_t));
    t->off_tj_grad = place(&o, t->tj_grad.size() * sizeof(int32_t));
    t->bytes = o;
}

void BuildTables::pack(char *host) const
{
    auto put = [&](size_t off, const void *src, size_t bytes) { if (bytes) std::memcpy(host + off, src, bytes); };
    put(0, descs.data(), descs.size() * sizeof(PyrDescWrite));
    put(off_p12, p12.data(), p12.size() * sizeof(Pyr12Job));
    for (int l = 1; l < LK_MAX_LEVELS; ++l) put(off_down[l], down[l].data(), down[l].size() * sizeof(DownJob));
    put(off_grad, grads.data(), grads.size() * sizeof(GradJob));
    put(off_tj_p12, tj_p12.data(), tj_p12.size() * sizeof(int32_t));
    for (int l = 1; l < LK_MAX_LEVELS; ++l) put(off_tj_down[l], tj_down[l].data(), tj_down[l].size() * sizeof(int32_t));
    put(off_tj_grad, tj_grad.data(), tj_grad.size() * sizeof(int32_t));
}

hipError_t launch_build_tables(const BuildTables &t, const char *d_base, hipStream_t s)
{
    // the descriptor writes ride on the fused level-1/2 launch when it has a
    // workgroup for each of them, else they take a launch of their own
    const PyrDescWrite *d_descs = reinterpret_cast<const PyrDescWrite *>(d_base);
    const int nd = (int)t.descs.size();
    const bool fold = !t.p12.empty() && nd <= (int)t.tj_p12.size();
    hipError_t e = fold ? hipSuccess : launch_write_descs(d_descs, nd, s);
    if (e == hipSuccess && !t.p12.empty())
        e = launch_pyr12_batched(reinterpret_cast<const Pyr12Job *>(d_base + t.off_p12),
                                 reinterpret_cast<const int32_t *>(d_base + t.off_tj_p12), (int)t.tj_p12.size(),
                                 fold ? d_descs : nullptr, fold ? nd : 0, s);
    for (int l = 1; l < LK_MAX_LEVELS && e == hipSuccess; ++l)
        if (!t.down[l].empty())
            e = launch_downsample_batched(reinterpret_cast<const DownJob *>(d_base + t.off_down[l]),
                                          reinterpret_cast<const int32_t *>(d_base + t.off_tj_down[l]),
                                          (int)t.tj_down[l].size(), s);
    if (e == hipSuccess && !t.grads.empty())
        e = launch_grad_batched(reinterpret_cast<const GradJob *>(d_base + t.off_grad),
                                reinterpret_cast<const int32_t *>(d_base + t.off_tj_grad), (int)t.tj_grad.size(), s);
    return e;
}

lk_result enqueue_build(lk_context *ctx, lk_pyramid *const *pyrs, int n, hipStream_t s)
{
    BuildTables t;
    make_build_tables(pyrs, n, &t);
    StagingRing::Slot *slot = nullptr;
    lk_result r = ctx->staging.acquire(t.bytes, &slot);
    if (r != LK_SUCCESS) return r;
    t.pack(static_cast<char *>(slot->host));
    hipError_t e = hipMemcpyAsync(slot->dev, slot->host, t.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(pyramid table)");
    e = launch_build_tables(t, static_cast<const char *>(slot->dev), s);
    (void)hipEventRecord(slot->done, s);
    if (e != hipSuccess) return hip_fail(e, "batched pyramid launch");
    for (int i = 0; i < n; ++i) pyrs[i]->built = true;
    return LK_SUCCESS;
}

}  // namespace lkmi

void lk_context::graphs_release() {}
