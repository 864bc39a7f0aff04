// Shi-Tomasi corner detection ("good features to track") for gfx950: the
// detector that seeds and replenishes LK tracks in the paper's GFTT+LK
// front-end (Sec. IV, Sec. V-E).  The definition computed (integer Scharr
// structure tensor, binary64 smaller eigenvalue, 3x3 non-maximum suppression,
// quality threshold, greedy minimum-distance selection in rank order) is the
// one stated in lk.h; results are exact, not approximations of it.
//
// Three launches per call, all frames of the call at once:
//   k_gftt_reset   zero the per-frame peak counters and maxima (a fill kernel,
//                  safe under graph capture);
//   k_gftt_peaks   one 64x16 tile per workgroup: the frame window with a halo
//                  is staged in LDS, gradients, box sums and the response are
//                  formed there, every in-frame 3x3 local maximum with R > 0
//                  is appended to the frame's peak list and the frame maximum
//                  is raised with one atomic per workgroup;
//   k_gftt_select  one workgroup per frame: the quality threshold follows
//                  from the maximum; windows of the best remaining peaks are
//                  found by radix selection on the 96-bit rank key (R bits,
//                  then the complemented raster index), sorted in LDS, and
//                  accepted 256 at a time against the corners taken so far
//                  and the occupied points.  The acceptance within a chunk
//                  resolves the greedy rule exactly (a candidate is taken
//                  iff no better candidate that is taken lies too close).
#include "lk_internal.h"

namespace lkmi {

namespace {

constexpr int TW = kGfttTileW, TH = kGfttTileH;
constexpr int BLOCK = 256;

__device__ __forceinline__ int reflect101(int i, int n)
{
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

// Smaller eigenvalue of [a b; b c] in binary64, one rounding per operation in
// the order fixed by the definition (contraction into fused operations is
// switched off for this function).
__device__ __forceinline__ double min_eig(int32_t a, int32_t b, int32_t c)
{
#pragma clang fp contract(off)
    const double t = (double)(a - c);
    const double u = (double)b;
    const double d1 = t * t;
    const double d2 = (4.0 * u) * u;
    const double disc = d1 + d2;
    const double s = __builtin_sqrt(disc);
    const double tr = (double)(a + c);
    return (tr - s) * 0.5;
}

__device__ __forceinline__ int find_job(const GfttJob *jobs, int njobs, int tile)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int R>
struct PeakSmem {
    static constexpr int IW = TW + 4 + 2 * R, IH = TH + 4 + 2 * R;   // image window
    static constexpr int GW = TW + 2 + 2 * R, GH = TH + 2 + 2 * R;   // gradients
    static constexpr int RW = TW + 2, RH = TH + 2;                   // response
    uint8_t img[IH][IW + 4];
    int16_t gx[GH][GW], gy[GH][GW];
    int32_t ha[GH][RW], hb[GH][RW], hc[GH][RW];
    double r[RH][RW];
    uint32_t n_local;
    uint32_t base;
    unsigned long long wmax[BLOCK / 64];
};

template <int R>
__global__ __launch_bounds__(BLOCK) void k_gftt_peaks(const GfttJob *__restrict__ jobs, int njobs, int border)
{
    using S = PeakSmem<R>;
    __shared__ S sm;
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const GfttJob &J = jobs[find_job(jobs, njobs, tile)];
    const int t = tile - J.tile_begin;
    const int W = J.w, H = J.h;
    const int x0 = (t % J.tiles_x) * TW, y0 = (t / J.tiles_x) * TH;
    const uint8_t *img = J.img;

    if (tid == 0) sm.n_local = 0;
    // 1. frame window [x0-2-R, x0+TW+2+R) x [y0-2-R, ...): in-frame samples only
    for (int e = tid; e < S::IH * S::IW; e += BLOCK) {
        const int j = e / S::IW, i = e - j * S::IW;
        const int X = x0 - 2 - R + i, Y = y0 - 2 - R + j;
        uint8_t v = 0;
        if (X >= 0 && X < W && Y >= 0 && Y < H) v = img[(size_t)Y * J.pitch + X];
        sm.img[j][i] = v;
    }
    __syncthreads();
    // 2. Scharr gradients at the in-frame samples of [x0-1-R, x0+TW+1+R) x ...;
    //    neighbours outside the frame are reflected (reflect-101) into it
    for (int e = tid; e < S::GH * S::GW; e += BLOCK) {
        const int j = e / S::GW, i = e - j * S::GW;
        const int X = x0 - 1 - R + i, Y = y0 - 1 - R + j;
        int16_t vx = 0, vy = 0;
        if (X >= 0 && X < W && Y >= 0 && Y < H) {
            const int ox = x0 - 2 - R, oy = y0 - 2 - R;
            const int xm = reflect101(X - 1, W) - ox, xp = reflect101(X + 1, W) - ox, xc = X - ox;
            const int ym = reflect101(Y - 1, H) - oy, yp = reflect101(Y + 1, H) - oy, yc = Y - oy;
            const int a00 = sm.img[ym][xm], a01 = sm.img[ym][xc], a02 = sm.img[ym][xp];
            const int a10 = sm.img[yc][xm], a12 = sm.img[yc][xp];
            const int a20 = sm.img[yp][xm], a21 = sm.img[yp][xc], a22 = sm.img[yp][xp];
            vx = (int16_t)(3 * (a02 - a00) + 10 * (a12 - a10) + 3 * (a22 - a20));
            vy = (int16_t)(3 * (a20 - a00) + 10 * (a21 - a01) + 3 * (a22 - a02));
        }
        sm.gx[j][i] = vx;
        sm.gy[j][i] = vy;
    }
    __syncthreads();
    // 3. horizontal block sums at the response columns, every in-frame gradient row
    for (int e = tid; e < S::GH * S::RW; e += BLOCK) {
        const int j = e / S::RW, i = e - j * S::RW;
        const int X = x0 - 1 + i, Yg = y0 - 1 - R + j;
        int32_t a = 0, b = 0, c = 0;
        if (X >= 0 && X < W && Yg >= 0 && Yg < H) {
#pragma unroll
            for (int k = -R; k <= R; ++k) {
                const int gi = reflect101(X + k, W) - (x0 - 1 - R);
                const int32_t gx = sm.gx[j][gi], gy = sm.gy[j][gi];
                a += gx * gx;
                b += gx * gy;
                c += gy * gy;
            }
        }
        sm.ha[j][i] = a;
        sm.hb[j][i] = b;
        sm.hc[j][i] = c;
    }
    __syncthreads();
    // 4. vertical sums and the response on [x0-1, x0+TW+1) x [y0-1, y0+TH+1);
    //    positions outside the frame never win a comparison
    for (int e = tid; e < S::RH * S::RW; e += BLOCK) {
        const int j = e / S::RW, i = e - j * S::RW;
        const int X = x0 - 1 + i, Y = y0 - 1 + j;
        double v = -__builtin_inf();
        if (X >= 0 && X < W && Y >= 0 && Y < H) {
            int32_t a = 0, b = 0, c = 0;
#pragma unroll
            for (int k = -R; k <= R; ++k) {
                const int hj = reflect101(Y + k, H) - (y0 - 1 - R);
                a += sm.ha[hj][i];
                b += sm.hb[hj][i];
                c += sm.hc[hj][i];
            }
            v = min_eig(a, b, c);
        }
        sm.r[j][i] = v;
    }
    __syncthreads();
    // 5. maximum, optional response map, peaks
    double vmax = 0.0;
    int my_n = 0;
    int my_idx[TW * TH / BLOCK];
    double my_r[TW * TH / BLOCK];
    uint32_t my_slot[TW * TH / BLOCK];
#pragma unroll
    for (int q = 0; q < TW * TH / BLOCK; ++q) {
        const int e = tid + q * BLOCK;
        const int j = e / TW, i = e - j * TW;
        const int X = x0 + i, Y = y0 + j;
        if (X >= W || Y >= H) continue;
        const double v = sm.r[j + 1][i + 1];
        if (J.response) J.response[(size_t)Y * W + X] = v;
        if (v > vmax) vmax = v;
        if (!(v > 0.0) || X < border || Y < border || X >= W - border || Y >= H - border) continue;
        bool peak = true;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di)
                if ((di != 1 || dj != 1) && sm.r[j + dj][i + di] > v) peak = false;
        if (!peak) continue;
        my_idx[my_n] = Y * W + X;
        my_r[my_n] = v;
        my_slot[my_n] = atomicAdd(&sm.n_local, 1u);
        ++my_n;
    }
    unsigned long long mb = (unsigned long long)__double_as_longlong(vmax);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long other = __shfl_xor(mb, o, 64);
        mb = other > mb ? other : mb;
    }
    if ((tid & 63) == 0) sm.wmax[tid >> 6] = mb;
    __syncthreads();
    if (tid == 0) {
        unsigned long long m = sm.wmax[0];
        for (int k = 1; k < BLOCK / 64; ++k) m = sm.wmax[k] > m ? sm.wmax[k] : m;
        if (m) atomicMax(J.max_bits, m);
        sm.base = sm.n_local ? (uint32_t)atomicAdd(J.n_peaks, (int)sm.n_local) : 0u;
    }
    __syncthreads();
    for (int k = 0; k < my_n; ++k) {
        GfttPeak p;
        p.rbits = (unsigned long long)__double_as_longlong(my_r[k]);
        p.idx = (uint32_t)my_idx[k];
        p.pad = 0;
        J.peaks[sm.base + my_slot[k]] = p;
    }
}

// ---- selection --------------------------------------------------------------

constexpr int CAPW = kGfttWindow;             // window of peaks sorted in LDS
constexpr int CHUNK = BLOCK;                  // candidates decided together
constexpr int OCC_LDS = 1024;                 // occupied points cached in LDS

struct Key {
    unsigned long long hi;   // bits of R (R > 0, so the bits order like R)
    uint32_t lo;             // complemented raster index: larger = earlier
};

__device__ __forceinline__ bool key_less(Key a, Key b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

__device__ __forceinline__ uint32_t key_byte(Key k, int d)
{
    return d < 8 ? (uint32_t)(k.hi >> (56 - 8 * d)) & 0xFFu : (k.lo >> (24 - 8 * (d - 8))) & 0xFFu;
}

// Keys whose leading d bytes equal those of p.
__device__ __forceinline__ bool key_prefix_eq(Key k, Key p, int d)
{
    if (d == 0) return true;
    if (d <= 8) {
        const unsigned long long m = d == 8 ? ~0ull : ~((1ull << (64 - 8 * d)) - 1);
        return (k.hi & m) == (p.hi & m);
    }
    const uint32_t m = d == 12 ? ~0u : ~((1u << (32 - 8 * (d - 8))) - 1);
    return k.hi == p.hi && (k.lo & m) == (p.lo & m);
}

__device__ __forceinline__ Key key_set_byte(Key k, int d, uint32_t v)
{
    if (d < 8) {
        const int s = 56 - 8 * d;
        k.hi = (k.hi & ~(0xFFull << s)) | ((unsigned long long)v << s);
    } else {
        const int s = 24 - 8 * (d - 8);
        k.lo = (k.lo & ~(0xFFu << s)) | (v << s);
    }
    return k;
}

struct SelSmem {
    unsigned long long whi[CAPW];
    uint32_t wlo[CAPW];
    uint32_t taken[kGfttMaxCorners];          // x | y << 16
    float2 occ[OCC_LDS];
    int32_t cx[CHUNK], cy[CHUNK];
    uint32_t hist[256];
    unsigned long long sel[CHUNK / 64], und[CHUNK / 64];
    uint32_t wcount;
    Key bound;
    int32_t done_flag;
    uint32_t need;
};

__device__ __forceinline__ bool eligible(Key k, unsigned long long thr_bits, bool bounded, Key bound)
{
    return k.hi > thr_bits && (!bounded || key_less(k, bound));
}

__global__ __launch_bounds__(BLOCK) void k_gftt_select(const GfttJob *__restrict__ jobs, double quality,
                                                       int min_dist, int max_corners)
{
    __shared__ SelSmem sm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const GfttJob &J = jobs[blockIdx.x];
    const int W = J.w;
    const int np = *J.n_peaks;
    const double rmax = __longlong_as_double((long long)*J.max_bits);
    const double thr = quality * rmax;
    const unsigned long long thr_bits = (unsigned long long)__double_as_longlong(thr);
    const long long md2 = (long long)min_dist * min_dist;
    const double md2d = (double)md2;
    const GfttPeak *peaks = J.peaks;
    const int n_occ = J.n_occupied;

    for (int k = tid; k < n_occ && k < OCC_LDS; k += BLOCK) sm.occ[k] = make_float2(J.occupied[2 * k], J.occupied[2 * k + 1]);
    // eligible peaks in total
    if (tid == 0) sm.wcount = 0;
    __syncthreads();
    {
        uint32_t c = 0;
        for (int k = tid; k < np; k += BLOCK) c += peaks[k].rbits > thr_bits;
        if (c) atomicAdd(&sm.wcount, c);
    }
    __syncthreads();
    int remaining = (int)sm.wcount;
    int nt = 0;
    bool bounded = false;
    Key bound{0, 0};
    __syncthreads();

    while (nt < max_corners && remaining > 0) {
        // ---- the next window: the best min(CAPW, remaining) eligible peaks
        const int wn = remaining < CAPW ? remaining : CAPW;
        Key low{0, 0};                          // window = eligible keys >= low
        if (wn < remaining) {
            uint32_t need = (uint32_t)wn;
            Key prefix{0, 0};
            for (int d = 0; d < 12; ++d) {
                for (int k = tid; k < 256; k += BLOCK) sm.hist[k] = 0;
                __syncthreads();
                for (int k = tid; k < np; k += BLOCK) {
                    const Key key{peaks[k].rbits, ~peaks[k].idx};
                    if (eligible(key, thr_bits, bounded, bound) && key_prefix_eq(key, prefix, d))
                        atomicAdd(&sm.hist[key_byte(key, d)], 1u);
                }
                __syncthreads();
                if (tid == 0) {
                    uint32_t cum = 0;
                    int g = 255;
                    for (; g > 0; --g) {
                        if (cum + sm.hist[g] >= need) break;
                        cum += sm.hist[g];
                    }
                    sm.need = need - cum;
                    sm.done_flag = (sm.hist[g] == need - cum) ? 1 : 0;
                    sm.bound = key_set_byte(prefix, d, (uint32_t)g);
                }
                __syncthreads();
                need = sm.need;
                prefix = sm.bound;
                const bool whole = sm.done_flag != 0;
                __syncthreads();
                if (whole) break;
            }
            low = prefix;
        }
        // ---- gather the window and sort it (descending) in LDS
        if (tid == 0) sm.wcount = 0;
        __syncthreads();
        for (int k = tid; k < np; k += BLOCK) {
            const Key key{peaks[k].rbits, ~peaks[k].idx};
            if (eligible(key, thr_bits, bounded, bound) && !key_less(key, low)) {
                const uint32_t s = atomicAdd(&sm.wcount, 1u);
                if (s < (uint32_t)CAPW) {
                    sm.whi[s] = key.hi;
                    sm.wlo[s] = key.lo;
                }
            }
        }
        __syncthreads();
        int pw = 1;
        while (pw < wn) pw <<= 1;
        for (int k = wn + tid; k < pw; k += BLOCK) { sm.whi[k] = 0; sm.wlo[k] = 0; }
        __syncthreads();
        for (int size = 2; size <= pw; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = tid; k < pw / 2; k += BLOCK) {
                    const int lo = 2 * k - (k & (stride - 1));
                    const int hi = lo + stride;
                    const bool desc = (lo & size) == 0;
                    const Key a{sm.whi[lo], sm.wlo[lo]}, b{sm.whi[hi], sm.wlo[hi]};
                    if (key_less(a, b) == desc) {
                        sm.whi[lo] = b.hi; sm.wlo[lo] = b.lo;
                        sm.whi[hi] = a.hi; sm.wlo[hi] = a.lo;
                    }
                }
                __syncthreads();
            }
        }
        // ---- accept in rank order, CHUNK candidates at a time
        for (int c0 = 0; c0 < wn && nt < max_corners; c0 += CHUNK) {
            const int k = c0 + tid;
            const bool valid = k < wn;
            int x = 0, y = 0;
            bool blocked = !valid;
            if (valid) {
                const int idx = (int)~sm.wlo[k];
                y = idx / W;
                x = idx - y * W;
                for (int q = 0; q < nt && !blocked; ++q) {
                    const uint32_t p = sm.taken[q];
                    const long long dx = x - (int)(p & 0xFFFFu), dy = y - (int)(p >> 16);
                    if (dx * dx + dy * dy < md2) blocked = true;
                }
                for (int q = 0; q < n_occ && !blocked; ++q) {
                    const float2 o = q < OCC_LDS ? sm.occ[q] : make_float2(J.occupied[2 * q], J.occupied[2 * q + 1]);
                    double dx, dy, dd;
                    {
#pragma clang fp contract(off)
                        dx = (double)x - (double)o.x;
                        dy = (double)y - (double)o.y;
                        dd = dx * dx + dy * dy;
                    }
                    if (dd < md2d) blocked = true;
                }
            }
            sm.cx[tid] = x;
            sm.cy[tid] = y;
            __syncthreads();
            // conflicts with better candidates of this chunk
            unsigned long long m[CHUNK / 64];
#pragma unroll
            for (int w = 0; w < CHUNK / 64; ++w) m[w] = 0;
            if (!blocked) {
                for (int u = 0; u < tid; ++u) {
                    const long long dx = x - sm.cx[u], dy = y - sm.cy[u];
                    if (dx * dx + dy * dy < md2) m[u >> 6] |= 1ull << (u & 63);
                }
            }
            const unsigned long long und0 = __ballot(!blocked);
            if (lane == 0) { sm.und[wv] = und0; sm.sel[wv] = 0; }
            __syncthreads();
            // candidates not blocked by earlier corners: taken iff no better
            // taken candidate conflicts; decided in rounds
            while (true) {
                bool any = false;
#pragma unroll
                for (int w = 0; w < CHUNK / 64; ++w) any |= sm.und[w] != 0;
                if (!any) break;
                const bool mine = (sm.und[wv] >> lane) & 1ull;
                bool in = false, out = false;
                if (mine) {
                    bool hit = false, wait = false;
#pragma unroll
                    for (int w = 0; w < CHUNK / 64; ++w) {
                        hit |= (m[w] & sm.sel[w]) != 0;
                        wait |= (m[w] & sm.und[w]) != 0;
                    }
                    out = hit;
                    in = !hit && !wait;
                }
                const unsigned long long bin = __ballot(in), bout = __ballot(out);
                __syncthreads();
                if (lane == 0) {
                    sm.sel[wv] |= bin;
                    sm.und[wv] &= ~(bin | bout);
                }
                __syncthreads();
            }
            // the first (max_corners - nt) taken candidates are kept
            int before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < CHUNK / 64; ++w) {
                const unsigned long long s = sm.sel[w];
                total += __popcll(s);
                if (w < wv) before += __popcll(s);
                else if (w == wv) before += __popcll(s & ((1ull << lane) - 1));
            }
            const bool mine = (sm.sel[wv] >> lane) & 1ull;
            const int pos = nt + before;
            if (mine && pos < max_corners) {
                sm.taken[pos] = (uint32_t)x | ((uint32_t)y << 16);
                J.out_xy[2 * pos] = (float)x;
                J.out_xy[2 * pos + 1] = (float)y;
            }
            nt = min(nt + total, max_corners);
            __syncthreads();
        }
        remaining -= wn;
        bounded = true;
        bound = Key{sm.whi[wn - 1], sm.wlo[wn - 1]};
        __syncthreads();
    }
    if (tid == 0) *J.count = nt;
}

__global__ void k_gftt_reset(const GfttJob *__restrict__ jobs, int njobs)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < njobs) {
        *jobs[k].n_peaks = 0;
        *jobs[k].max_bits = 0ull;
    }
}

}  // namespace

hipError_t launch_gftt(const GfttJob *d_jobs, int njobs, int total_tiles, int radius, int border, double quality,
                       int min_dist, int max_corners, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    k_gftt_reset<<<(njobs + 255) / 256, 256, 0, s>>>(d_jobs, njobs);
    switch (radius) {
    case 0: k_gftt_peaks<0><<<total_tiles, BLOCK, 0, s>>>(d_jobs, njobs, border); break;
    case 1: k_gftt_peaks<1><<<total_tiles, BLOCK, 0, s>>>(d_jobs, njobs, border); break;
    case 2: k_gftt_peaks<2><<<total_tiles, BLOCK, 0, s>>>(d_jobs, njobs, border); break;
    default: k_gftt_peaks<3><<<total_tiles, BLOCK, 0, s>>>(d_jobs, njobs, border); break;
    }
    k_gftt_select<<<njobs, BLOCK, 0, s>>>(d_jobs, quality, min_dist, max_corners);
    return hipGetLastError();
}

}  // namespace lkmi
