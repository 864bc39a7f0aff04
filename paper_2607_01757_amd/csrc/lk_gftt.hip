// Shi-Tomasi corner detection ("good features to track") for gfx950: the
// detector that seeds and replenishes LK tracks in the paper's GFTT+LK
// front-end (Sec. IV, Sec. V-E).  The definition computed (integer Scharr
// structure tensor, binary64 smaller eigenvalue, 3x3 non-maximum suppression,
// quality threshold, greedy minimum-distance selection in rank order) is the
// one stated in lk.h; results are exact, not approximations of it.
//
// Four launches per call, all frames of the call at once:
//   k_gftt_reset   zero the per-frame peak counters and maxima (a fill kernel,
//                  safe under graph capture);
//   k_gftt_peaks   one 64x16 tile per workgroup: the frame window with a halo
//                  is staged in LDS, gradients, block sums and the response
//                  are formed there, every in-frame 3x3 local maximum with
//                  R > 0 is appended to the frame's peak list and the frame
//                  maximum is raised with one atomic per workgroup;
//   k_gftt_compact keeps the peaks above the quality threshold that no cached
//                  occupied point blocks;
//   k_gftt_select  one workgroup per frame: the quality threshold follows
//                  from the maximum; windows of the best remaining peaks are
//                  found by radix selection on the 96-bit rank key (R bits,
//                  then the complemented raster index), sorted in LDS, and
//                  accepted 512 at a time against the corners taken so far
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

template <int R>
struct alignas(16) PeakSmem {
    static constexpr int IH = TH + 4 + 2 * R, IW = 96;               // frame rows y0-2-R.., columns x0-16..
    static constexpr int GW = TW + 2 + 2 * R, GH = TH + 2 + 2 * R;   // gradients from (x0-1-R, y0-1-R)
    static constexpr int RW = TW + 2, RH = TH + 2;                   // responses from (x0-1, y0-1)
    uint8_t img[IH][IW];
    uint32_t g[GH][GW];            // gx | gy << 16, both int16
    double r[RH][RW];
    uint32_t n_local;
    uint32_t base;
    unsigned long long wmax[BLOCK / 64];
};

__device__ __forceinline__ int reflect1(int i, int n)       // one reflection; n >= 2, -n < i < 2n - 1
{
    i = i < 0 ? -i : i;
    return i >= n ? 2 * (n - 1) - i : i;
}

template <int R>
__global__ __launch_bounds__(BLOCK) void k_gftt_peaks(const GfttJob *__restrict__ jobs,
                                                      const int32_t *__restrict__ tile_job, int border)
{
    using S = PeakSmem<R>;
    __shared__ S sm;
    const int tid = threadIdx.x;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const GfttJob J = jobs[__builtin_amdgcn_readfirstlane(tile_job[tile])];
    const int t = tile - J.tile_begin;
    const int W = J.w, H = J.h;
    const int x0 = (t % J.tiles_x) * TW, y0 = (t / J.tiles_x) * TH;

    if (tid == 0) sm.n_local = 0;
    // 1. frame rows [y0-2-R, y0+TH+2+R) x columns [x0-16, x0+80) as bytes,
    //    16-byte loads; a sample outside the frame holds its reflect-101
    //    sample (only those at distance 1 are ever read)
    {
        const bool vec_ok = (J.pitch & 15) == 0 && (reinterpret_cast<uintptr_t>(J.img) & 15) == 0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(J.img), (short)0, J.pitch * H, 0x00020000);
        for (int e = tid; e < S::IH * (S::IW / 16); e += BLOCK) {
            const int j = e / (S::IW / 16), c = e - j * (S::IW / 16);
            const int Y = reflect1(min(max(y0 - 2 - R + j, -2), H + 1), H);
            const int X0 = x0 - 16 + 16 * c;
            if (vec_ok && X0 >= 0 && X0 + 16 <= W) {
                *reinterpret_cast<uint4 *>(&sm.img[j][16 * c]) =
                    __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, Y * J.pitch + X0, 0, 0));
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int X = reflect1(min(max(X0 + k, -2), W + 1), W);
                    sm.img[j][16 * c + k] = J.img[(size_t)Y * J.pitch + X];
                }
            }
        }
    }
    __syncthreads();
    // 2. gradients: slot (X, Y) holds the Scharr gradient at the reflect-101
    //    image (X, Y) of that position, so the block sums below read their
    //    taps without any reflection.  Only slots the sums can reach are
    //    formed: X in [-1-R, W+R), Y in [-1-R, H+R).
    for (int e = tid; e < S::GH * S::GW; e += BLOCK) {
        const int j = e / S::GW, i = e - j * S::GW;
        const int X = x0 - 1 - R + i, Y = y0 - 1 - R + j;
        uint32_t v = 0;
        if (X >= -1 - R && X < W + R && Y >= -1 - R && Y < H + R) {
            const int xc = reflect101(X, W) - (x0 - 16), yc = reflect101(Y, H) - (y0 - 2 - R);
            const int a00 = sm.img[yc - 1][xc - 1], a01 = sm.img[yc - 1][xc], a02 = sm.img[yc - 1][xc + 1];
            const int a10 = sm.img[yc][xc - 1], a12 = sm.img[yc][xc + 1];
            const int a20 = sm.img[yc + 1][xc - 1], a21 = sm.img[yc + 1][xc], a22 = sm.img[yc + 1][xc + 1];
            const int gx = 3 * (a02 - a00) + 10 * (a12 - a10) + 3 * (a22 - a20);
            const int gy = 3 * (a20 - a00) + 10 * (a21 - a01) + 3 * (a22 - a02);
            v = (uint32_t)(gx & 0xFFFF) | ((uint32_t)gy << 16);
        }
        sm.g[j][i] = v;
    }
    __syncthreads();
    // 3. block sums (exact integers) and the response on [x0-1, x0+TW+1) x
    //    [y0-1, y0+TH+1); positions outside the frame never win a comparison
    for (int e = tid; e < S::RH * S::RW; e += BLOCK) {
        const int j = e / S::RW, i = e - j * S::RW;
        const int X = x0 - 1 + i, Y = y0 - 1 + j;
        double v = -__builtin_inf();
        if (X >= 0 && X < W && Y >= 0 && Y < H) {
            int32_t a = 0, b = 0, c = 0;
#pragma unroll
            for (int dj = 0; dj <= 2 * R; ++dj)
#pragma unroll
                for (int di = 0; di <= 2 * R; ++di) {
                    const uint32_t q = sm.g[j + dj][i + di];
                    const int32_t gx = (int32_t)(int16_t)(q & 0xFFFF), gy = (int32_t)q >> 16;
                    a += gx * gx;
                    b += gx * gy;
                    c += gy * gy;
                }
            v = min_eig(a, b, c);
        }
        sm.r[j][i] = v;
    }
    __syncthreads();
    // 4. maximum, optional response map, peaks
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

// ---- threshold --------------------------------------------------------------
//
// The threshold needs the frame maximum, known only once every tile is done:
// this grid keeps the peaks above it (gridDim.x workgroups per frame, one
// atomic per wavefront).  Their order does not matter: selection orders
// candidates by the total rank key.
constexpr int kCompactBlocks = 32;

// ---- occupied points ----------------------------------------------------------
//
// The first OCC_LDS occupied points of a frame, grouped by the cells of a grid
// of cs x cs pixels with cs >= min_dist (at most OCC_GRID cells): a point
// closer than min_dist to an integer pixel lies in that pixel's cell or one of
// its 8 neighbours (points off the frame, or not finite, go to the nearest
// border cell, where they are still checked and never match), so a pixel
// checks only those 9 cells, with the binary64 distance rule of the selection.

constexpr int OCC_LDS = 1024;                 // occupied points cached in LDS
constexpr int OCC_GRID = 4096;                // cells of their grid

struct OccGridSmem {
    float2 occ[OCC_LDS];                       // the cached points, grouped by cell
    uint32_t end[OCC_GRID];                    // end of each cell's group in occ
    uint32_t wsum[16];
};

struct OccGrid {
    int cs, gx, gy, nl;
};

// Built by all NT threads of the workgroup; ends with a barrier.
template <int NT>
__device__ OccGrid occ_grid_build(const GfttJob &J, int n_occ, int min_dist, OccGridSmem &g)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    OccGrid G;
    G.nl = n_occ < OCC_LDS ? n_occ : OCC_LDS;
    G.cs = min_dist > 1 ? min_dist : 1;
    for (;;) {
        G.gx = (J.w + G.cs - 1) / G.cs;
        G.gy = (J.h + G.cs - 1) / G.cs;
        if (G.gx * G.gy <= OCC_GRID) break;
        G.cs += (G.cs >> 2) + 1;
    }
    const int ncell = G.gx * G.gy;
    auto cell_of = [&](float ox, float oy) {
        const float lim = (float)(2 * G.cs);
        const int ix = (int)floorf(fminf(fmaxf(ox, -lim), (float)J.w + lim));
        const int iy = (int)floorf(fminf(fmaxf(oy, -lim), (float)J.h + lim));
        const int cx = ix < 0 ? 0 : min(ix / G.cs, G.gx - 1), cy = iy < 0 ? 0 : min(iy / G.cs, G.gy - 1);
        return cy * G.gx + cx;
    };
    if (G.nl > 0) {
        for (int k = tid; k < ncell; k += NT) g.end[k] = 0;
        __syncthreads();
        for (int k = tid; k < G.nl; k += NT) atomicAdd(&g.end[cell_of(J.occupied[2 * k], J.occupied[2 * k + 1])], 1u);
        __syncthreads();
        // exclusive prefix sum over the cells, PER consecutive cells per thread
        constexpr int PER = OCC_GRID / NT;
        uint32_t v[PER], tsum = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid * PER + i;
            v[i] = c < ncell ? g.end[c] : 0u;
            tsum += v[i];
        }
        uint32_t incl = tsum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) g.wsum[wv] = incl;
        __syncthreads();
        uint32_t run = incl - tsum;
        for (int w = 0; w < wv; ++w) run += g.wsum[w];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int c = tid * PER + i;
            if (c < ncell) g.end[c] = run;
            run += v[i];
        }
        __syncthreads();
        // scatter: each cell's counter ends at the end of its group
        for (int k = tid; k < G.nl; k += NT) {
            const float ox = J.occupied[2 * k], oy = J.occupied[2 * k + 1];
            const uint32_t at = atomicAdd(&g.end[cell_of(ox, oy)], 1u);
            g.occ[at] = make_float2(ox, oy);
        }
    }
    __syncthreads();
    return G;
}

// Some cached occupied point lies at binary64 squared distance < md2d from
// the integer pixel (x, y).
__device__ __forceinline__ bool occ_grid_blocked(const OccGrid &G, const OccGridSmem &g, int x, int y, double md2d)
{
    bool blocked = false;
    const int ccx = x / G.cs, ccy = y / G.cs;
    for (int yy = max(ccy - 1, 0); yy <= min(ccy + 1, G.gy - 1) && !blocked; ++yy) {
        const int c0 = yy * G.gx + max(ccx - 1, 0), c1 = yy * G.gx + min(ccx + 1, G.gx - 1);
        // the three cells of a row are consecutive groups
        const int b = c0 == 0 ? 0 : (int)g.end[c0 - 1], e = (int)g.end[c1];
        for (int q = b; q < e && !blocked; ++q) {
            const float2 o = g.occ[q];
            double dd;
            {
#pragma clang fp contract(off)
                const double dx = (double)x - (double)o.x, dy = (double)y - (double)o.y;
                dd = dx * dx + dy * dy;
            }
            blocked |= dd < md2d;
        }
    }
    return blocked;
}

__global__ __launch_bounds__(BLOCK) void k_gftt_compact(const GfttJob *__restrict__ jobs, double quality,
                                                       int min_dist)
{
    __shared__ uint32_t s_cnt[BLOCK / 64], s_base;
    __shared__ uint32_t s_hist[256];
    __shared__ OccGridSmem s_grid;
    const GfttJob &J = jobs[blockIdx.y];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    static_assert(BLOCK == 256, "one histogram bin per thread");
    s_hist[threadIdx.x] = 0u;
    const int np = *J.n_peaks;
    // peaks that a cached occupied point blocks can never be selected: they
    // are dropped here (the selection still checks every occupied point)
    const int n_occ = __builtin_amdgcn_readfirstlane(J.n_occupied_dev ? *J.n_occupied_dev : J.n_occupied);
    const bool filter = n_occ > 0 && min_dist > 0;
    OccGrid G{1, 1, 1, 0};
    if (filter) G = occ_grid_build<BLOCK>(J, n_occ, min_dist, s_grid);
    const double md2d = (double)min_dist * (double)min_dist;
    const int W = J.w;
    auto kept = [&](const GfttPeak &p) {
        if (!filter) return true;
        const int y = (int)(p.idx / (uint32_t)W), x = (int)p.idx - y * W;
        return !occ_grid_blocked(G, s_grid, x, y, md2d);
    };
    const unsigned long long max_bits = *J.max_bits;
    const double thr = quality * __longlong_as_double((long long)max_bits);
    const unsigned long long thr_bits = (unsigned long long)__double_as_longlong(thr);
    // the candidates' R bits lie in (thr_bits, max_bits]: they share the
    // leading d0 bytes of those two, and byte d0 is histogrammed for the
    // selection's first radix pass
    const unsigned long long diff = max_bits ^ thr_bits;
    const int d0 = diff ? (__clzll((long long)diff) >> 3) : 8;
    const int hshift = d0 < 8 ? 56 - 8 * d0 : 0;
    __syncthreads();                           // s_hist is cleared (when no grid was built)
    // this workgroup's slice of the frame's peaks, in steps of BLOCK
    const int per = (np + gridDim.x - 1) / gridDim.x;
    const int k_lo = min(np, (int)blockIdx.x * per), k_hi = min(np, k_lo + per);
    uint32_t mine = 0;
    for (int k0 = k_lo; k0 < k_hi; k0 += BLOCK) {
        const int k = k0 + threadIdx.x;
        if (k < k_hi) {
            const GfttPeak p = J.peaks[k];
            if (p.rbits > thr_bits && kept(p)) {
                mine += 1u;
                if (d0 < 8) atomicAdd(&s_hist[(uint32_t)(p.rbits >> hshift) & 0xFFu], 1u);
            }
        }
    }
    __syncthreads();
    if (d0 < 8 && s_hist[threadIdx.x]) atomicAdd(&J.hist[threadIdx.x], s_hist[threadIdx.x]);
    // wavefront and workgroup totals, one global atomic
    uint32_t wsum = mine;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
    if (lane == 0) s_cnt[wv] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < BLOCK / 64; ++w) tot += s_cnt[w];
        s_base = tot ? (uint32_t)atomicAdd(J.n_cand, (int)tot) : 0u;
    }
    __syncthreads();
    // write in the same order: wavefronts in turn, lanes by their prefix
    uint32_t base = s_base;
    for (int k0 = k_lo; k0 < k_hi; k0 += BLOCK) {
        const int k = k0 + threadIdx.x;
        GfttPeak p{};
        bool keep = false;
        if (k < k_hi) {
            p = J.peaks[k];
            keep = p.rbits > thr_bits && kept(p);
        }
        const unsigned long long m = __ballot(keep);
        uint32_t wc = (uint32_t)__popcll(m);
        if (lane == 0) s_cnt[wv] = wc;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            const uint32_t c = s_cnt[w];
            before += w < wv ? c : 0u;
            all += c;
        }
        if (keep) J.cand[base + before + (uint32_t)__popcll(m & ((1ull << lane) - 1))] = p;
        base += all;
        __syncthreads();
    }
}

// ---- selection --------------------------------------------------------------

constexpr int CAPW = kGfttWindow;             // window of peaks sorted in LDS
constexpr int TG_CELLS = 2048;                // cells of the taken-corner grid, at most
constexpr int SBLOCK = 512;                   // threads of the selection workgroup
constexpr int CHUNK = SBLOCK;                 // candidates decided together
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

struct alignas(16) SelSmem {
    unsigned long long whi[CAPW];
    uint32_t wlo[CAPW];
    uint32_t taken[kGfttMaxCorners + 16];     // x | y << 16
    OccGridSmem grid;                          // the cached occupied points
    int32_t cx[CHUNK], cy[CHUNK];
    int32_t tg_head[TG_CELLS];                 // taken corners by grid cell: first index, -1 for none
    int32_t tg_next[kGfttMaxCorners + 16];     // the next index in the same cell
    uint32_t hist[SBLOCK / 64][256];           // one histogram per wavefront
    unsigned long long cmask[CHUNK][CHUNK / 64];   // conflicts with better candidates of the chunk
    unsigned long long sel[CHUNK / 64], und[CHUNK / 64];
    uint32_t wcount, bcount;
    Key bound;
    int32_t done_flag;
    uint32_t need;
};

__device__ __forceinline__ bool eligible(Key k, bool bounded, Key bound)
{
    return !bounded || key_less(k, bound);
}

// The corners taken so far, grouped by the cells of a grid of cs x cs
// pixels with cs >= min_dist (at most TG_CELLS cells), each cell a list
// threaded through tg_next: a corner closer than min_dist to a pixel lies in
// that pixel's cell or one of its 8 neighbours.
struct TakenGrid {
    int cs, gx, gy;
};

__device__ __forceinline__ TakenGrid taken_grid(int w, int h, int min_dist)
{
    TakenGrid T;
    T.cs = min_dist > 1 ? min_dist : 1;
    for (;;) {
        T.gx = (w + T.cs - 1) / T.cs;
        T.gy = (h + T.cs - 1) / T.cs;
        if (T.gx * T.gy <= TG_CELLS) break;
        T.cs += (T.cs >> 2) + 1;
    }
    return T;
}

// Some taken corner lies at squared distance < md2 from the in-frame pixel (x, y).
__device__ __forceinline__ bool taken_blocked(const TakenGrid &T, const int32_t *head, const int32_t *next,
                                              const uint32_t *taken, int x, int y, int md2)
{
    const int ccx = x / T.cs, ccy = y / T.cs;
    bool blocked = false;
    for (int yy = max(ccy - 1, 0); yy <= min(ccy + 1, T.gy - 1) && !blocked; ++yy)
        for (int xx = max(ccx - 1, 0); xx <= min(ccx + 1, T.gx - 1) && !blocked; ++xx)
            for (int q = head[yy * T.gx + xx]; q >= 0 && !blocked; q = next[q]) {
                const uint32_t p = taken[q];
                const int dx = x - (int)(p & 0xFFFFu), dy = y - (int)(p >> 16);
                blocked = dx * dx + dy * dy < md2;
            }
    return blocked;
}

// Slot of this lane among the lanes of its wavefront that set `take`, in an
// array whose fill counter is *ctr (one atomic per wavefront).
__device__ __forceinline__ uint32_t wave_append(bool take, uint32_t *ctr)
{
    const unsigned long long m = __ballot(take);
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        if (lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
        base = __shfl(base, leader, 64);
    }
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
}

__global__ __launch_bounds__(SBLOCK) void k_gftt_select(const GfttJob *__restrict__ jobs, double quality,
                                                       int min_dist, int max_corners)
{
    __shared__ SelSmem sm;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const GfttJob &J = jobs[blockIdx.x];
    const int W = J.w;
    const int np = *J.n_cand;                  // every candidate is above the threshold
    const int md2 = min_dist * min_dist;
    const double md2d = (double)md2;
    const bool spaced = min_dist >= 2;         // distinct pixels are always >= 1 apart
    const GfttPeak *cand = J.cand;
    const int n_occ = __builtin_amdgcn_readfirstlane(J.n_occupied_dev ? *J.n_occupied_dev : J.n_occupied);
    // every candidate's R bits lie in (thr_bits, max_bits] (the threshold is
    // formed as the compaction forms it)
    const unsigned long long max_bits = *J.max_bits;
    const unsigned long long thr_bits =
        (unsigned long long)__double_as_longlong(quality * __longlong_as_double((long long)max_bits));

    const TakenGrid T = taken_grid(W, J.h, min_dist);
    for (int c = tid; c < TG_CELLS; c += SBLOCK) sm.tg_head[c] = -1;
    const OccGrid G = occ_grid_build<SBLOCK>(J, n_occ, min_dist, sm.grid);   // ends with a barrier
    int remaining = np;
    int nt = 0;
    bool bounded = false;
    Key bound{0, 0};
    __syncthreads();

    while (nt < max_corners && remaining > 0) {
        // ---- the next window: the best min(CAPW, remaining) candidates
        const int wn = remaining < CAPW ? remaining : CAPW;
        Key low{0, 0};                          // window = eligible keys >= low
        // the list the passes read: the candidates, or, once few keys are at
        // or above the boundary bucket, a copy of just those keys (in the
        // frame's peak list, no longer needed after the compaction)
        const GfttPeak *src = cand;
        int nsrc = np;
        bool filtered = false;
        if (wn < remaining) {
            uint32_t need = (uint32_t)wn;
            // the eligible keys' R bits lie in (thr_bits, top]: their leading
            // bytes are those thr_bits and top share, so the passes start
            // after them
            const unsigned long long top = bounded ? bound.hi : max_bits;
            const unsigned long long diff = top ^ thr_bits;
            const int d0 = diff ? (__clzll((long long)diff) >> 3) : 8;
            Key prefix{d0 >= 8 ? top : (d0 == 0 ? 0ull : top & ~((1ull << (64 - 8 * d0)) - 1)), 0};
            for (int d = d0; d < 12; ++d) {
                for (int k = tid; k < (SBLOCK / 64) * 256; k += SBLOCK) (&sm.hist[0][0])[k] = 0;
                __syncthreads();
                // the first window's first digit: every candidate is eligible
                // and carries the prefix, so the compaction's histogram is
                // this pass's count
                const bool counted = d == d0 && !bounded && d0 < 8;
                if (counted && tid < 256) sm.hist[0][tid] = J.hist[tid];
                for (int k0 = 0; k0 < (counted ? 0 : nsrc); k0 += 8 * SBLOCK) {
                    Key key[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int k = k0 + i * SBLOCK + tid;
                        key[i] = k < nsrc ? Key{src[k].rbits, ~src[k].idx} : Key{0, 0};
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        if (key[i].hi != 0 && eligible(key[i], bounded, bound) && key_prefix_eq(key[i], prefix, d))
                            atomicAdd(&sm.hist[wv][key_byte(key[i], d)], 1u);
                }
                __syncthreads();
                if (wv == 0) {
                    // lane l holds digits 4l .. 4l+3; suffix sums from the top
                    uint32_t t[4], ls = 0;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        t[i] = 0;
#pragma unroll
                        for (int w = 0; w < SBLOCK / 64; ++w) t[i] += sm.hist[w][4 * lane + i];
                        ls += t[i];
                    }
                    uint32_t above = 0;              // sum over lanes > lane
                    uint32_t run = ls;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t v = __shfl_down(run, o, 64);
                        if (lane + o < 64) run += v;
                    }
                    above = run - ls;
                    uint32_t cum = above;
#pragma unroll
                    for (int i = 3; i >= 0; --i) {
                        if (cum < need && need <= cum + t[i]) {
                            sm.need = need - cum;
                            sm.done_flag = t[i] == need - cum ? 1 : 0;
                            sm.bound = key_set_byte(prefix, d, (uint32_t)(4 * lane + i));
                            sm.bcount = t[i];
                        }
                        cum += t[i];
                    }
                }
                __syncthreads();
                need = sm.need;
                prefix = sm.bound;
                const bool whole = sm.done_flag != 0;
                const int kept = (int)((uint32_t)wn - need + sm.bcount);   // keys >= the bucket's lower bound
                __syncthreads();
                if (whole) break;
                if (!filtered && 4 * kept <= nsrc) {
                    // copy the eligible keys >= prefix (its lower bytes are 0):
                    // the keys above the bucket and the bucket itself
                    if (tid == 0) sm.wcount = 0;
                    __syncthreads();
                    // (8 keys per thread in flight, as in the counting passes)
                    for (int k0 = 0; k0 < nsrc; k0 += 8 * SBLOCK) {
                        GfttPeak p[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int k = k0 + i * SBLOCK + tid;
                            p[i] = k < nsrc ? src[k] : GfttPeak{};
                        }
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int k = k0 + i * SBLOCK + tid;
                            const Key key{p[i].rbits, ~p[i].idx};
                            const bool take = k < nsrc && eligible(key, bounded, bound) && !key_less(key, prefix);
                            const uint32_t at = wave_append(take, &sm.wcount);
                            if (take) J.peaks[at] = p[i];
                        }
                    }
                    __syncthreads();             // the copy is visible to the whole workgroup
                    src = J.peaks;
                    nsrc = (int)sm.wcount;
                    filtered = true;
                    __syncthreads();
                }
            }
            low = prefix;
        }
        // ---- gather the window and sort it (descending) in LDS; keys a
        // taken corner already blocks can never be taken and stay out
        if (tid == 0) sm.wcount = 0;
        __syncthreads();
        const bool screen = spaced && nt > 0;
        for (int k0 = 0; k0 < nsrc; k0 += 8 * SBLOCK) {
            Key key[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int k = k0 + i * SBLOCK + tid;
                key[i] = k < nsrc ? Key{src[k].rbits, ~src[k].idx} : Key{0, 0};
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bool take = key[i].hi != 0 && eligible(key[i], bounded, bound) && !key_less(key[i], low);
                if (take && screen) {
                    const int idx = (int)~key[i].lo, yk = idx / W, xk = idx - yk * W;
                    take = !taken_blocked(T, sm.tg_head, sm.tg_next, sm.taken, xk, yk, md2);
                }
                const uint32_t s = wave_append(take, &sm.wcount);
                if (take && s < (uint32_t)CAPW) {
                    sm.whi[s] = key[i].hi;
                    sm.wlo[s] = key[i].lo;
                }
            }
        }
        __syncthreads();
        const int wu = min((int)sm.wcount, CAPW);   // the window's keys no taken corner blocks
        int pw = 1;
        while (pw < wu) pw <<= 1;
        for (int k = wu + tid; k < pw; k += SBLOCK) { sm.whi[k] = 0; sm.wlo[k] = 0; }
        __syncthreads();
        constexpr int PAIRS = CAPW / 2 / SBLOCK;
        for (int size = 2; size <= pw; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                int lo[PAIRS];
                Key a[PAIRS], b[PAIRS];
#pragma unroll
                for (int i = 0; i < PAIRS; ++i) {
                    const int k = tid + i * SBLOCK;
                    lo[i] = 2 * k - (k & (stride - 1));
                    if (k < pw / 2) {
                        a[i] = Key{sm.whi[lo[i]], sm.wlo[lo[i]]};
                        b[i] = Key{sm.whi[lo[i] + stride], sm.wlo[lo[i] + stride]};
                    }
                }
#pragma unroll
                for (int i = 0; i < PAIRS; ++i) {
                    const int k = tid + i * SBLOCK;
                    if (k < pw / 2 && key_less(a[i], b[i]) == ((lo[i] & size) == 0)) {
                        sm.whi[lo[i]] = b[i].hi; sm.wlo[lo[i]] = b[i].lo;
                        sm.whi[lo[i] + stride] = a[i].hi; sm.wlo[lo[i] + stride] = a[i].lo;
                    }
                }
                __syncthreads();
            }
        }
        // ---- accept in rank order, CHUNK candidates at a time
        for (int c0 = 0; c0 < wu && nt < max_corners; c0 += CHUNK) {
            const int k = c0 + tid;
            const bool valid = k < wu;
            int x = 0, y = 0;
            bool blocked = !valid;
            if (valid) {
                const int idx = (int)~sm.wlo[k];
                y = idx / W;
                x = idx - y * W;
            }
            // corners taken so far (those of earlier chunks: the window
            // holds none an earlier window's corners block)
            if (spaced && valid && nt > 0) blocked = taken_blocked(T, sm.tg_head, sm.tg_next, sm.taken, x, y, md2);
            // occupied points (binary64 distance): the grid, then any beyond the cache
            if (valid && n_occ > 0) {
                blocked = blocked || occ_grid_blocked(G, sm.grid, x, y, md2d);
                for (int q = OCC_LDS; q < n_occ && !blocked; ++q) {
                    double dd;
                    {
#pragma clang fp contract(off)
                        const double dx = (double)x - (double)J.occupied[2 * q], dy = (double)y - (double)J.occupied[2 * q + 1];
                        dd = dx * dx + dy * dy;
                    }
                    blocked |= dd < md2d;
                }
            }
            // the candidates no taken corner or occupied point blocks, packed
            // in rank order at cx / cy [0, mu)
            {
                const unsigned long long free_bits = __ballot(!blocked);
                if (lane == 0) sm.und[wv] = free_bits;
            }
            __syncthreads();
            int mu = 0, at = 0;
#pragma unroll
            for (int w = 0; w < CHUNK / 64; ++w) {
                const int c = __popcll(sm.und[w]);
                mu += c;
                at += w < wv ? c : 0;
            }
            at += __popcll(sm.und[wv] & ((1ull << lane) - 1));
            if (!blocked) {
                sm.cx[at] = x;
                sm.cy[at] = y;
            }
            __syncthreads();
            // packed candidate t = tid: its conflicts with the better packed
            // candidates u < t (squared distance < min_dist^2), one 64-bit
            // mask per group of 64, 8 tests per step
            const bool live = tid < mu;
            if (live && spaced) {
                const int xt = sm.cx[tid], yt = sm.cy[tid];
                const int4 *x4 = reinterpret_cast<const int4 *>(sm.cx), *y4 = reinterpret_cast<const int4 *>(sm.cy);
#pragma unroll
                for (int w = 0; w < CHUNK / 64; ++w) {
                    if (64 * w > tid) break;
                    unsigned long long mw = 0;
                    const int u_end = min(tid, 64 * w + 64);
                    for (int u0 = 64 * w; u0 < u_end; u0 += 8) {
                        const int4 xa = x4[u0 / 4], xb = x4[u0 / 4 + 1], ya = y4[u0 / 4], yb = y4[u0 / 4 + 1];
                        const int ux[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
                        const int uy[8] = {ya.x, ya.y, ya.z, ya.w, yb.x, yb.y, yb.z, yb.w};
                        unsigned long long bits = 0;
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int dx = xt - ux[i], dy = yt - uy[i];
                            bits |= (unsigned long long)((u0 + i < tid) && (dx * dx + dy * dy < md2)) << i;
                        }
                        mw |= bits << (u0 & 63);
                    }
                    sm.cmask[tid][w] = mw;
                }
            }
            __syncthreads();
            // wavefront 0 applies the greedy rule in rank order, a group of 64
            // packed candidates at a time: a candidate is taken iff no taken
            // better candidate conflicts with it.  Within a group the rule is
            // resolved in rounds: an undecided candidate with a taken better
            // conflict is rejected; one whose better conflicts are all decided
            // and rejected is taken (the best undecided one always is, so
            // every round decides at least one)
            if (wv == 0) {
                unsigned long long sel[CHUNK / 64];
#pragma unroll
                for (int g = 0; g < CHUNK / 64; ++g) {
                    sel[g] = 0;
                    if (64 * g >= mu) continue;
                    const int t = 64 * g + lane;
                    const bool tl = t < mu;
                    bool hit = false;
                    unsigned long long mg = 0;
                    if (tl && spaced) {
#pragma unroll
                        for (int w = 0; w < CHUNK / 64; ++w)
                            if (w < g) hit |= (sm.cmask[t][w] & sel[w]) != 0;
                        mg = sm.cmask[t][g];
                    }
                    unsigned long long und = __ballot(tl && !hit), taken = 0;
                    while (und) {
                        const bool me = (und >> lane) & 1ull;
                        const bool rej = me && (mg & taken) != 0;
                        const bool tak = me && !rej && (mg & und) == 0;
                        const unsigned long long bt = __ballot(tak), br = __ballot(rej);
                        taken |= bt;
                        und &= ~(bt | br);
                    }
                    sel[g] = taken;
                }
                if (lane == 0)
#pragma unroll
                    for (int g = 0; g < CHUNK / 64; ++g) sm.sel[g] = sel[g];
            }
            __syncthreads();
            // the first (max_corners - nt) taken candidates are kept
            int before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < CHUNK / 64; ++w) {
                const unsigned long long sw = sm.sel[w];
                total += __popcll(sw);
                if (w < wv) before += __popcll(sw);
                else if (w == wv) before += __popcll(sw & ((1ull << lane) - 1));
            }
            const bool mine = live && ((sm.sel[wv] >> lane) & 1ull);
            const int pos = nt + before;
            if (mine && pos < max_corners) {
                const int xm = sm.cx[tid], ym = sm.cy[tid];
                sm.taken[pos] = (uint32_t)xm | ((uint32_t)ym << 16);
                // into its grid cell's list (corners of one cell may arrive together)
                sm.tg_next[pos] = atomicExch(&sm.tg_head[(ym / T.cs) * T.gx + xm / T.cs], pos);
            }
            nt = min(nt + total, max_corners);
            __syncthreads();
        }
        remaining -= wn;
        bounded = true;
        bound = low;                 // the window was every eligible key >= low
        __syncthreads();
    }
    // corners in order, written once
    for (int q = tid; q < nt; q += SBLOCK) {
        const uint32_t p = sm.taken[q];
        J.out_xy[2 * q] = (float)(p & 0xFFFFu);
        J.out_xy[2 * q + 1] = (float)(p >> 16);
    }
    if (tid == 0) *J.count = nt;
}

// One workgroup of 256 threads per frame: counters, maximum, histogram.
__global__ void k_gftt_reset(const GfttJob *__restrict__ jobs)
{
    const GfttJob &J = jobs[blockIdx.x];
    J.hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        *J.n_peaks = 0;
        *J.n_cand = 0;
        *J.max_bits = 0ull;
    }
}

}  // namespace

hipError_t launch_gftt(const GfttJob *d_jobs, const int32_t *d_tile_job, int njobs, int total_tiles, int radius,
                       int border, double quality, int min_dist, int max_corners, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    k_gftt_reset<<<njobs, 256, 0, s>>>(d_jobs);
    switch (radius) {
    case 0: k_gftt_peaks<0><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    case 1: k_gftt_peaks<1><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    case 2: k_gftt_peaks<2><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    default: k_gftt_peaks<3><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    }
    k_gftt_compact<<<dim3(kCompactBlocks, njobs), BLOCK, 0, s>>>(d_jobs, quality, min_dist);
    k_gftt_select<<<njobs, SBLOCK, 0, s>>>(d_jobs, quality, min_dist, max_corners);
    return hipGetLastError();
}

}  // namespace lkmi
