// Host-side objects of liblkmi (context, pyramid, staging ring) and the
// helpers shared by the ABI, the batched path and the server.
#pragma once

#include <atomic>
#include <cstddef>
#include <vector>

#include "lk_error.h"
#include "lk_internal.h"

// Pinned host + device buffer pairs used to ship small tables (batch items,
// pyramid jobs) to the device with one asynchronous copy.  A slot is reused
// only after the event recorded behind its last user has completed.
namespace lkmi {
struct StagingRing {
    struct Slot {
        void *host = nullptr;
        void *dev = nullptr;
        size_t cap = 0;
        hipEvent_t done = nullptr;
    };
    std::vector<Slot> slots;
    int next = 0;
    lk_result init(int nslots);
    void release();
    lk_result acquire(size_t bytes, Slot **out);
};
}  // namespace lkmi

struct lk_context {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> in_use{0};
    lkmi::StagingRing staging;
    // lk_track_batched_noalloc: the device's fixed batch-table array (set up
    // at creation), a pinned host copy of the table and the event of its last
    // upload
    void *table_dev = nullptr;
    void *table_host = nullptr;
    hipEvent_t table_done = nullptr;
    void graphs_release();
};

struct lk_pyramid {
    lk_context *ctx = nullptr;
    lkmi::PyrDesc desc{};
    lkmi::PyrDesc *d_desc = nullptr;   // device copy of desc, rewritten by every build
    void *base = nullptr;      // descriptor, levels >= 1 and gradient planes, one allocation
    size_t bytes = 0;
    bool built = false;
};

namespace lkmi {

// Job tables of a batched pyramid build, laid out for one device buffer:
// descriptor writes, fused level-1+2 jobs, down jobs level by level (levels
// >= 3, or level 1 of two-level pyramids), gradient jobs, then one
// tile-to-job table per launch.
struct BuildTables {
    std::vector<PyrDescWrite> descs;
    std::vector<Pyr12Job> p12;
    std::vector<DownJob> down[LK_MAX_LEVELS];
    std::vector<GradJob> grads;
    std::vector<int32_t> tj_p12, tj_down[LK_MAX_LEVELS], tj_grad;
    size_t off_p12 = 0, off_down[LK_MAX_LEVELS] = {0}, off_grad = 0;
    size_t off_tj_p12 = 0, off_tj_down[LK_MAX_LEVELS] = {0}, off_tj_grad = 0, bytes = 0;
    void pack(char *host) const;
};
void make_build_tables(lk_pyramid *const *pyrs, int n, BuildTables *t);
// Enqueues the build from tables already in device memory at d_base.
hipError_t launch_build_tables(const BuildTables &t, const char *d_base, hipStream_t s);

lk_result hip_fail(hipError_t e, const char *what);
int level_dims(int w, int h, int levels, int32_t *ws, int32_t *hs);
lk_result check_params(const lk_params *p, int pyr_levels);
lk_result check_pair(const lk_context *ctx, const lk_pyramid *prev, const lk_pyramid *next, int idx);
TrackArgs make_args(const lk_params *p, int n, const float *pts, const float *guess, float *out, uint8_t *st,
                    float *res, int32_t *iters);
lk_result plan_batch(lk_context *ctx, const lk_pair *pairs, int n_pairs, const lk_params *params,
                     std::vector<BatchItem> *items, int *storage, long long *total);
// plan_batch into a caller array of n_pairs items (no host allocation)
lk_result plan_batch_into(lk_context *ctx, const lk_pair *pairs, int n_pairs, const lk_params *params,
                          BatchItem *items, int *storage, long long *total);
lk_result enqueue_build(lk_context *ctx, lk_pyramid *const *pyrs, int n, hipStream_t s);
// Jobs of one pyramid build: levels 1+2 fused when the pyramid has three or
// more levels, one down job per remaining level, gradient planes (binary16).
void pyramid_jobs(const lk_pyramid *p, std::vector<Pyr12Job> *p12, std::vector<DownJob> *down_by_level,
                  std::vector<GradJob> *grads);
lk_result check_gftt_params(const lk_gftt_params *p);
// Detection of every job (img, w, h, pitch, occupied points, out_xy, count,
// response filled in by the caller; tiles and workspace slices here).
lk_result detector_enqueue(lk_detector *det, std::vector<GfttJob> &jobs, const lk_gftt_params *p, hipStream_t s);
}  // namespace lkmi
