// Track-pool lifecycle kernels: carry-over of the tracks that survive the
// temporal pass, the append of new corners, and the commit (cross-camera
// gate, new identities).  Associated features keep their identity, unmatched
// new detections start new tracks (Sec. III-C); in stereo mode only points
// that pass the cross-camera check enter the pool (Sec. V).  One workgroup
// per stream walks its list in chunks of kPoolThreads; ranks come from
// wavefront ballots, so the order of a list is kept exactly.
#include "lk_internal.h"

namespace lkmi {
namespace {

constexpr int kPoolThreads = 256;
constexpr int kPoolWaves = kPoolThreads / 64;

// Rank of this thread among the threads of the workgroup whose flag is set
// (threads in index order) and, in *total, how many flags are set.  Every
// thread of the workgroup must call it.
__device__ int group_rank(bool flag, int *s_waves, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long m = __ballot(flag);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_waves[w] = __popcll(m);
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kPoolWaves; ++k) {
        const int c = s_waves[k];
        base += k < w ? c : 0;
        tot += c;
    }
    __syncthreads();   // s_waves is rewritten by the next call
    *total = tot;
    return base + below;
}

// Survivors of the temporal pass (status LK_OK), in pool order, with their
// end points and identities -> candidates.
__global__ __launch_bounds__(kPoolThreads) void k_pool_carry(const PoolJob *jobs)
{
    __shared__ int s_waves[kPoolWaves];
    const PoolJob &J = jobs[blockIdx.x];
    const int n_prev = min(max(*J.count, 0), J.cap);   // a corrupt count cannot reach past the slice
    const int n = J.tracked ? n_prev : 0;               // no temporal pass: every track ends
    int base = 0;
    for (int i0 = 0; i0 < n; i0 += kPoolThreads) {
        const int i = i0 + (int)threadIdx.x;
        const bool keep = i < n && J.t_status[i] == LK_OK;
        int tot;
        const int r = group_rank(keep, s_waves, &tot);
        if (keep) {
            const int o = base + r;
            J.c_pts[2 * o] = J.t_pts[2 * i];
            J.c_pts[2 * o + 1] = J.t_pts[2 * i + 1];
            J.c_ids[o] = J.ids[i];
        }
        base += tot;
    }
    if (threadIdx.x == 0) {
        *J.c_count = base;
        J.stats[0] = n_prev;
        J.stats[1] = base;
    }
}

// New corners after the survivors until the target.  The detector ran with
// the target as its corner limit; greedy selection in rank order makes its
// first (target - survivors) corners the corners of a run with that limit.
__global__ __launch_bounds__(kPoolThreads) void k_pool_append(const PoolJob *jobs)
{
    const PoolJob &J = jobs[blockIdx.x];
    const int s = *J.c_count;
    const int k = *J.d_count;
    const int m = max(0, min(k, J.target - s));
    for (int j = threadIdx.x; j < m; j += kPoolThreads) {
        J.c_pts[2 * (s + j)] = J.d_xy[2 * j];
        J.c_pts[2 * (s + j) + 1] = J.d_xy[2 * j + 1];
        J.c_ids[s + j] = -1;
    }
    __syncthreads();   // every thread has read c_count
    if (threadIdx.x == 0) {
        *J.c_count = s + m;
        J.stats[2] = m;
    }
}

// Candidates -> the pool: all of them, or with the gate those whose
// cross-camera status is LK_OK (with their right-camera positions); new
// ones take the next identities in order.
__global__ __launch_bounds__(kPoolThreads) void k_pool_commit(const PoolJob *jobs)
{
    __shared__ int s_waves[kPoolWaves];
    const PoolJob &J = jobs[blockIdx.x];
    const int c = *J.c_count;
    const long long nid = *J.next_id;
    int base = 0, base_new = 0;
    for (int i0 = 0; i0 < c; i0 += kPoolThreads) {
        const int i = i0 + (int)threadIdx.x;
        const bool keep = i < c && (!J.gated || J.s_status[i] == LK_OK);
        const long long cid = keep ? J.c_ids[i] : 0;
        const bool fresh = keep && cid < 0;
        int tot, tot_new;
        const int r = group_rank(keep, s_waves, &tot);
        const int rn = group_rank(fresh, s_waves, &tot_new);
        if (keep) {
            const int o = base + r;
            J.pts[2 * o] = J.c_pts[2 * i];
            J.pts[2 * o + 1] = J.c_pts[2 * i + 1];
            J.ids[o] = fresh ? nid + base_new + rn : cid;
            if (J.gated) {
                J.right[2 * o] = J.s_pts[2 * i];
                J.right[2 * o + 1] = J.s_pts[2 * i + 1];
            }
        }
        base += tot;
        base_new += tot_new;
    }
    __syncthreads();   // every thread has read next_id
    if (threadIdx.x == 0) {
        *J.count = base;
        *J.next_id = nid + base_new;
        J.stats[3] = base;
    }
}

// Every stream empty, identities from 0.
__global__ __launch_bounds__(kPoolThreads) void k_pool_reset(int32_t *count, int64_t *next_id, int n)
{
    const int i = blockIdx.x * kPoolThreads + threadIdx.x;
    if (i < n) {
        count[i] = 0;
        next_id[i] = 0;
    }
}

}  // namespace

hipError_t launch_pool_reset(int32_t *d_count, int64_t *d_next_id, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_reset, dim3((n + kPoolThreads - 1) / kPoolThreads), dim3(kPoolThreads), 0, s, d_count,
                       d_next_id, n);
    return hipGetLastError();
}

hipError_t launch_pool_carry(const PoolJob *d_jobs, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_carry, dim3(n), dim3(kPoolThreads), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_pool_append(const PoolJob *d_jobs, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_append, dim3(n), dim3(kPoolThreads), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_pool_commit(const PoolJob *d_jobs, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pool_commit, dim3(n), dim3(kPoolThreads), 0, s, d_jobs);
    return hipGetLastError();
}

}  // namespace lkmi
