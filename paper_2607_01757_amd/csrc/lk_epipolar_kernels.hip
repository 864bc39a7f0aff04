// Epipolar check after LK (the geometric verification of temporal
// correspondences, Sec. III-C): eight-point models from caller-drawn
// samples, scored by the point-to-epipolar-line distance in pixels.
//
//   k_epi_hypotheses  one lane per hypothesis: the 8 x 9 system on the
//                     normalized plane is reduced by Gaussian elimination
//                     with complete pivoting (binary64) in a lane-private
//                     LDS slab (entry (r, c) of lane l at [(9 r + c) 64 + l],
//                     so the lanes of a wavefront hit distinct banks), the
//                     null vector is mapped to pixel space and every
//                     correspondence of the set is scored; the set's
//                     correspondences are staged in LDS, 512 at a time, by
//                     the whole wavefront, and every lane reads each one
//                     from there (one broadcast read, no memory round trip
//                     per correspondence);
//   k_epi_best        one workgroup per set: the best hypothesis (most
//                     inliers, lowest index on ties), its model solved again
//                     by the same code (same bits), and its inlier mask.
//
// Neither function contracts multiply-adds, so the count of a hypothesis in
// the first kernel and its mask in the second come from identical arithmetic.
#include "lk_internal.h"

namespace lkmi {
namespace {

constexpr int kEpiLanes = 64;
constexpr int kEpiChunk = 512;             // correspondences staged in LDS at a time
constexpr double kEpiRankTol = 1e-10;

__device__ __forceinline__ double &slab(double *sa, int r, int c, int lane)
{
    return sa[(9 * r + c) * kEpiLanes + lane];
}

// Pixel-space F (unit Frobenius norm) of the samples s[0..7] of job J, or
// false when the samples are invalid or the system has numerical rank < 8.
__device__ bool epi_model(const EpiJob &J, const int32_t *s, double *sa, int *scol, int lane, double (&F)[9])
{
#pragma clang fp contract(off)
    int idx[8];
    bool bad = false;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        idx[a] = s[a];
        bad |= idx[a] < 0 || idx[a] >= J.n;
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = a + 1; b < 8; ++b) bad |= idx[a] == idx[b];
    if (bad) return false;
    const double ifx = 1.0 / J.fx, ify = 1.0 / J.fy;
    // rows x_q (x) x_p on the normalized plane
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int i = idx[r];
        const double xp = ((double)J.p[2 * i] - J.cx) * ifx, yp = ((double)J.p[2 * i + 1] - J.cy) * ify;
        const double xq = ((double)J.q[2 * i] - J.cx) * ifx, yq = ((double)J.q[2 * i + 1] - J.cy) * ify;
        slab(sa, r, 0, lane) = xq * xp;
        slab(sa, r, 1, lane) = xq * yp;
        slab(sa, r, 2, lane) = xq;
        slab(sa, r, 3, lane) = yq * xp;
        slab(sa, r, 4, lane) = yq * yp;
        slab(sa, r, 5, lane) = yq;
        slab(sa, r, 6, lane) = xp;
        slab(sa, r, 7, lane) = yp;
        slab(sa, r, 8, lane) = 1.0;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) scol[c * kEpiLanes + lane] = c;
    double amax = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        // complete pivoting: the largest entry of the remaining block
        double best = -1.0;
        int br = k, bc = k;
#pragma unroll
        for (int r = k; r < 8; ++r)
#pragma unroll
            for (int c = k; c < 9; ++c) {
                const double v = fabs(slab(sa, r, c, lane));
                if (v > best) { best = v; br = r; bc = c; }
            }
        if (k == 0) amax = best;
        if (!(best > kEpiRankTol * amax)) return false;     // also catches NaN
        if (br != k)
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const double t = slab(sa, k, c, lane);
                slab(sa, k, c, lane) = slab(sa, br, c, lane);
                slab(sa, br, c, lane) = t;
            }
        if (bc != k) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const double t = slab(sa, r, k, lane);
                slab(sa, r, k, lane) = slab(sa, r, bc, lane);
                slab(sa, r, bc, lane) = t;
            }
            const int t = scol[k * kEpiLanes + lane];
            scol[k * kEpiLanes + lane] = scol[bc * kEpiLanes + lane];
            scol[bc * kEpiLanes + lane] = t;
        }
        const double piv = slab(sa, k, k, lane);
#pragma unroll
        for (int r = k + 1; r < 8; ++r) {
            const double f = slab(sa, r, k, lane) / piv;
#pragma unroll
            for (int c = k + 1; c < 9; ++c) slab(sa, r, c, lane) = slab(sa, r, c, lane) - f * slab(sa, k, c, lane);
        }
    }
    // null vector in the permuted columns (free column last), back substitution
    double y[9];
    y[8] = 1.0;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        double acc = 0.0;
#pragma unroll
        for (int c = k + 1; c < 9; ++c) acc = acc + slab(sa, k, c, lane) * y[c];
        y[k] = -acc / slab(sa, k, k, lane);
    }
    // undo the column permutation (through row 0 of the slab)
#pragma unroll
    for (int c = 0; c < 9; ++c) slab(sa, 0, scol[c * kEpiLanes + lane], lane) = y[c];
    double e[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) e[c] = slab(sa, 0, c, lane);
    // F = K^-T E K^-1
    const double ax = -J.cx * ifx, ay = -J.cy * ify;
    double m[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        m[3 * i] = e[3 * i] * ifx;
        m[3 * i + 1] = e[3 * i + 1] * ify;
        m[3 * i + 2] = e[3 * i] * ax + e[3 * i + 1] * ay + e[3 * i + 2];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[j] = ifx * m[j];
        F[3 + j] = ify * m[3 + j];
        F[6 + j] = ax * m[j] + ay * m[3 + j] + m[6 + j];
    }
    double nn = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) nn = nn + F[j] * F[j];
    const double inv = 1.0 / sqrt(nn);
#pragma unroll
    for (int j = 0; j < 9; ++j) F[j] = F[j] * inv;
    return true;
}

// Correspondence (p, q) is an inlier of F: the distance of q to the line
// F (p, 1) is at most the threshold (thr2 = threshold^2).
__device__ __forceinline__ bool epi_inlier(const double (&F)[9], float px, float py, float qx, float qy, double thr2)
{
#pragma clang fp contract(off)
    const double x = px, y = py;
    const double l0 = F[0] * x + F[1] * y + F[2];
    const double l1 = F[3] * x + F[4] * y + F[5];
    const double l2 = F[6] * x + F[7] * y + F[8];
    const double num = (double)qx * l0 + (double)qy * l1 + l2;
    const double den = l0 * l0 + l1 * l1;
    return (den > 0.0) & (num * num <= thr2 * den);
}

__global__ __launch_bounds__(kEpiLanes) void k_epi_hypotheses(const EpiJob *__restrict__ jobs,
                                                              const int32_t *__restrict__ wg_job, double thr2)
{
    __shared__ double sa[72 * kEpiLanes];
    __shared__ int scol[9 * kEpiLanes];
    __shared__ float4 spq[kEpiChunk];
    const int lane = threadIdx.x;
    const EpiJob &J = jobs[__builtin_amdgcn_readfirstlane(wg_job[blockIdx.x])];
    const int n = __builtin_amdgcn_readfirstlane(J.n);
    const int k = (blockIdx.x - J.wg_begin) * kEpiLanes + lane;
    const bool live = k < J.h;
    double F[9];
    // every lane stays to the end: the whole wavefront stages the correspondences
    const bool ok = live && epi_model(J, J.samples + 8 * k, sa, scol, lane, F);
    int cnt = 0;
    for (int i0 = 0; i0 < n; i0 += kEpiChunk) {
        const int m = min(kEpiChunk, n - i0);
        __syncthreads();                       // every lane has read the previous chunk
        for (int i = lane; i < m; i += kEpiLanes) {
            const int g = i0 + i;
            spq[i] = make_float4(J.p[2 * g], J.p[2 * g + 1], J.q[2 * g], J.q[2 * g + 1]);
        }
        __syncthreads();
        if (ok) {
#pragma unroll 4
            for (int i = 0; i < m; ++i) {
                const float4 v = spq[i];
                cnt += epi_inlier(F, v.x, v.y, v.z, v.w, thr2);
            }
        }
    }
    if (live) J.counts[k] = ok ? cnt : -1;
}

__global__ __launch_bounds__(kEpiLanes) void k_epi_best(const EpiJob *__restrict__ jobs, double thr2)
{
    __shared__ double sa[72 * kEpiLanes];
    __shared__ int scol[9 * kEpiLanes];
    __shared__ double sF[9];
    __shared__ int s_ok;
    const int lane = threadIdx.x;
    const EpiJob &J = jobs[blockIdx.x];
    // most inliers, then the lowest index: key = (count + 1) << 32 | ~index
    unsigned long long key = 0;
    for (int k = lane; k < J.h; k += kEpiLanes) {
        const int c = J.counts[k];
        if (c >= 0) {
            const unsigned long long v = ((unsigned long long)(c + 1) << 32) | (0xFFFFFFFFu - (uint32_t)k);
            key = v > key ? v : key;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = __shfl_xor(key, o, kEpiLanes);
        key = v > key ? v : key;
    }
    const int bk = key ? (int)(0xFFFFFFFFu - (uint32_t)key) : -1;
    const int bc = key ? (int)(key >> 32) - 1 : 0;
    if (lane == 0) {
        double F[9];
        const bool ok = bk >= 0 && epi_model(J, J.samples + 8 * bk, sa, scol, 0, F);
#pragma unroll
        for (int j = 0; j < 9; ++j) sF[j] = ok ? F[j] : 0.0;
        s_ok = ok;
    }
    __syncthreads();
    double F[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) F[j] = sF[j];
    const bool ok = s_ok != 0;
    for (int i = lane; i < J.n; i += kEpiLanes)
        J.inliers[i] = ok && epi_inlier(F, J.p[2 * i], J.p[2 * i + 1], J.q[2 * i], J.q[2 * i + 1], thr2) ? 1 : 0;
    if (lane == 0) {
        J.best[0] = bk;
        J.best[1] = bc;
    }
    if (J.model && lane < 9) J.model[lane] = sF[lane];
}

}  // namespace

hipError_t launch_epipolar(const EpiJob *d_jobs, const int32_t *d_wg_job, int n_jobs, int total_wgs, double threshold,
                           hipStream_t s)
{
    const double thr2 = threshold * threshold;
    if (total_wgs > 0) {
        hipLaunchKernelGGL(k_epi_hypotheses, dim3(total_wgs), dim3(kEpiLanes), 0, s, d_jobs, d_wg_job, thr2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_jobs > 0) hipLaunchKernelGGL(k_epi_best, dim3(n_jobs), dim3(kEpiLanes), 0, s, d_jobs, thr2);
    return hipGetLastError();
}

}  // namespace lkmi
