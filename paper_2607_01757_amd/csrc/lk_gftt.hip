// Shi-Tomasi corner detection ("good features to track") for gfx950: the
// detector that seeds and replenishes LK tracks in the paper's GFTT+LK
// front-end (Sec. IV, Sec. V-E).  The definition computed (integer Scharr
// structure tensor, binary64 smaller eigenvalue, 3x3 non-maximum suppression,
// quality threshold, greedy minimum-distance selection in rank order) is the
// one stated in lk.h; results are exact, not approximations of it.
//
// Five launches per call, all frames of the call at once:
//   k_gftt_reset   zero the per-frame peak counters, maxima and bucket
//                  counters (a fill kernel, safe under graph capture);
//   k_gftt_peaks   the response, its 3x3 local maxima with R > 0 appended to
//                  the frame's peak list, the frame maximum raised with one
//                  atomic per workgroup: block radius 0 and 1 walk 60x32
//                  strips (60x64 in large calls) with one wavefront each
//                  (k_gftt_peaks_strip), radius 2 and 3 stage 64x16 tiles
//                  in LDS;
//   k_gftt_compact counts the peaks above the quality threshold that no
//                  cached occupied point blocks, in all and by bucket (the 8
//                  key bits after those the threshold and the maximum share),
//                  and marks them (one bit each) or, with occupied points,
//                  appends them to the candidate list;
//   k_gftt_bucket  writes them by bucket, best first;
//   k_gftt_select  one workgroup per frame: windows of the best remaining
//                  candidates are found from the bucket counts and, inside
//                  the last bucket a window reaches, by radix selection on the
//                  96-bit rank key (R bits, then the complemented raster
//                  index); they are sorted in LDS and accepted 512 at a time
//                  against the corners taken so far and the occupied points.
//                  The acceptance within a chunk resolves the greedy rule
//                  exactly (a candidate is taken iff no better candidate that
//                  is taken lies too close).
#include "lk_internal.h"
#include "lk_key.h"

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

// Correctly rounded square root of x, for x = 0 or x >= 1 (the discriminant
// below is a sum of squares of integers): the hardware reciprocal square root
// refined by Markstein's method (one Newton step on the pair (sqrt x,
// 1/(2 sqrt x)), then two corrections by the exact residual x - s^2, each one
// fused operation).  This is the compiler's own sequence for sqrt without its
// rescaling of tiny and huge arguments, which never applies here, so the
// results are its results, bit for bit.
__device__ __forceinline__ double sqrt_ge1(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-h, s, 0.5);
    s = __builtin_fma(s, r, s);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    d = __builtin_fma(-s, s, x);
    s = __builtin_fma(d, h, s);
    return x == 0.0 ? 0.0 : s;
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
    const double s = sqrt_ge1(disc);
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

// ---- responses and peaks, block radius 0 and 1: one wavefront per strip ------
//
// A strip is 60 output columns x SH output rows (32, or 64 in large calls);
// lane i owns frame column X = x0 - 2 + i and walks down the rows.  Per row
// it forms the Scharr gradient of its column from the staged frame bytes (at
// the reflect-101 position, as the tiled kernel does), the three products,
// their horizontal (2r+1)-sums over neighbouring lanes by wave-shift DPP, and
// their vertical sums over the last 2r+1 rows in registers; the response
// follows from the sums as in the tiled kernel.  Non-maximum suppression is separable: the
// maximum over a 3x3 block is the maximum of three row maxima, each the
// maximum of a lane and its two neighbours (again by wave shifts), and a
// response is a local maximum iff it equals that maximum (no response is
// NaN).  Lanes 0 and 63 hold no valid sums, lanes 1 and 62 no valid maxima:
// lanes 2 .. 61 produce the strip's 60 columns.  Same integers, same binary64
// operations, same comparisons as the tiled kernel: the same response map
// and peaks, bit for bit.

constexpr int kStripWaves = 1;                // strips per workgroup, one per wavefront

template <int R, int SH>
struct alignas(16) StripSmem {
    static constexpr int IH = SH + 2 * R + 4, IW = 80;            // frame rows y0-2-R.., columns sx0..
    static constexpr int NBUF = 128;
    uint8_t img[IH][IW];
    GfttPeak buf[NBUF];                                           // peaks waiting for a global slot
};

// Lane i's value from lane i - 1 (wave_shr:1) and from lane i + 1
// (wave_shl:1); the end lanes, which have no such neighbour, get 0.
__device__ __forceinline__ int32_t from_left(int32_t v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int32_t from_right(int32_t v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }

// a * b for |a|, |b| < 2^23 with a product that fits 32 bits (the gradients:
// |g| <= 4080): the full-rate 24-bit multiply, which the compiler does not
// pick by itself here
__device__ __forceinline__ int32_t mul_i24(int32_t a, int32_t b)
{
    int32_t p;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(p) : "v"(a), "v"(b));
    return p;
}

// a * b + c, same conditions
__device__ __forceinline__ int32_t mad_i24(int32_t a, int32_t b, int32_t c)
{
    int32_t p;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(p) : "v"(a), "v"(b), "v"(c));
    return p;
}

// max of two responses.  No response is NaN, so the quieting fmax asks of
// its operands is not needed: the plain instruction.
__device__ __forceinline__ double max_r(double a, double b)
{
    double m;
    asm("v_max_f64 %0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    return m;
}

// max of a lane's response and those of its two neighbours (0 at the end
// lanes, whose maxima are not used)
__device__ __forceinline__ double max3_lanes(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int32_t lo = (int32_t)(uint32_t)u, hi = (int32_t)(uint32_t)(u >> 32);
    const double l = __longlong_as_double((long long)(((unsigned long long)(uint32_t)from_left(hi) << 32) |
                                                       (uint32_t)from_left(lo)));
    const double r = __longlong_as_double((long long)(((unsigned long long)(uint32_t)from_right(hi) << 32) |
                                                       (uint32_t)from_right(lo)));
    return max_r(v, max_r(l, r));
}

template <int R, int SH>
__global__ __launch_bounds__(64 * kStripWaves) void k_gftt_peaks_strip(const GfttJob *__restrict__ jobs,
                                                                      const int32_t *__restrict__ tile_job,
                                                                      int n_tiles, int border)
{
    static_assert(R == 0 || R == 1, "block radius 0 or 1");
    using S = StripSmem<R, SH>;
    __shared__ S sms[kStripWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    S &sm = sms[wv];
    // strips of one workgroup are consecutive; a wavefront past the last one
    // stages the last one again and leaves after the barrier
    const int tile_w = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kStripWaves + wv);
    const bool has = tile_w < n_tiles;
    const int tile = has ? tile_w : n_tiles - 1;
    const GfttJob J = jobs[__builtin_amdgcn_readfirstlane(tile_job[tile])];
    const int t = tile - J.tile_begin;
    const int W = J.w, H = J.h;
    const int x0 = (t % J.tiles_x) * kGfttStripW, y0 = (t / J.tiles_x) * SH;
    const int sx0 = (x0 - 3) & ~7, sy0 = y0 - 2 - R;
    // 1. frame rows [sy0, sy0 + IH) x columns [sx0, sx0 + 80) as bytes (the
    //    walk reads columns x0 - 3 .. x0 + 62), 8-byte loads; a sample
    //    outside the frame holds its reflect-101 sample (only those at
    //    distance 1 are ever read)
    {
        const bool vec_ok = (J.pitch & 7) == 0 && (reinterpret_cast<uintptr_t>(J.img) & 7) == 0;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(J.img), (short)0, J.pitch * H, 0x00020000);
        for (int e = lane; e < S::IH * (S::IW / 8); e += 64) {
            const int j = e / (S::IW / 8), c = e - j * (S::IW / 8);
            const int Y = reflect1(min(max(sy0 + j, -2), H + 1), H);
            const int X0 = sx0 + 8 * c;
            if (vec_ok && X0 >= 0 && X0 + 8 <= W) {
                *reinterpret_cast<uint2 *>(&sm.img[j][8 * c]) =
                    __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, Y * J.pitch + X0, 0, 0));
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int X = reflect1(min(max(X0 + k, -2), W + 1), W);
                    sm.img[j][8 * c + k] = J.img[(size_t)Y * J.pitch + X];
                }
            }
        }
    }
    __syncthreads();
    if (!has) return;
    // 2. the walk.  Column X of this lane; its gradient slot is formed when
    //    the sums can reach it (X in [-1-R, W+R)), at the reflect-101 column.
    const int X = x0 - 2 + lane;
    const bool xslot = X >= -1 - R && X < W + R;
    const int xc = (xslot ? reflect101(X, W) : 0) - sx0;       // staged column of the gradient's centre
    const bool xout = lane >= 2 && lane < 62 && X < W;          // an output column of the strip
    const bool xin = X >= 0 && X < W;
    const int ye = min(y0 + SH, H);                             // output rows y0 .. ye-1
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    double vmax = 0.0;
    uint32_t nbuf = 0;                                          // peaks in sm.buf (wave-uniform)
    auto flush = [&]() {
        uint32_t base = 0;
        if (lane == 0) base = (uint32_t)atomicAdd(J.n_peaks, (int)nbuf);
        base = __shfl(base, 0, 64);
        __builtin_amdgcn_wave_barrier();                        // entries of the other lanes
        for (uint32_t k = lane; k < nbuf; k += 64) J.peaks[base + k] = sm.buf[k];
        __builtin_amdgcn_wave_barrier();
        nbuf = 0;
    };
    // The walk, in two forms.  Where every gradient row of the strip lies in
    // [0, H) (strips away from the top and bottom edges) the staged rows of
    // consecutive gradient rows are consecutive, and the separable form of the
    // Scharr gradient rolls: with d(j) = I(j, x+1) - I(j, x-1) and
    // s(j) = 3 I(j, x-1) + 10 I(j, x) + 3 I(j, x+1) on staged row j,
    // gx = 3 d(j-1) + 10 d(j) + 3 d(j+1) and gy = s(j+1) - s(j-1), and each
    // gradient row reads one new staged row.  Elsewhere each gradient row
    // reads its 3x3 taps at the reflect-101 row.
    auto walk = [&](auto roll_tag, auto inside_tag) {
        constexpr bool ROLL = decltype(roll_tag)::value;
        // INSIDE: every lane's column lies in the frame (strips away from the
        // left and right edges), so no lane needs a column test
        constexpr bool INSIDE = decltype(inside_tag)::value;
        const bool xs = INSIDE || xslot, xi = INSIDE || xin;
        const bool xo = INSIDE ? (lane >= 2 && lane < 62) : xout;
        int32_t hxx[3] = {0, 0, 0}, hxy[3] = {0, 0, 0}, hyy[3] = {0, 0, 0};   // products of gradient rows
        int32_t hd[3] = {0, 0, 0}, hs[3] = {0, 0, 0};          // d and s of three staged rows (ROLL)
        auto row_taps = [&](int j, int32_t &d, int32_t &sj) {
            const int l = sm.img[j][xc - 1], c = sm.img[j][xc], r = sm.img[j][xc + 1];
            d = r - l;
            sj = 3 * (l + r) + 10 * c;
        };
        // Gradient row Yg into product slot (O + 2) % 3 (slot 0 for R = 0).
        // Ring roles (ROLL): staged rows yc - 1, yc, yc + 1 in slots O, O + 1,
        // O + 2 (mod 3); calls with O = 0, 1, 2, 0, ... on consecutive rows.
        auto grad_row = [&](auto o_slot, int Yg) {
            constexpr int O = decltype(o_slot)::value, M = (O + 1) % 3, N = (O + 2) % 3;
            constexpr int P = R == 1 ? N : 0;
            int32_t pxx = 0, pxy = 0, pyy = 0;
            if constexpr (ROLL) {
                if (xs) {
                    row_taps(Yg - sy0 + 1, hd[N], hs[N]);
                    const int gx = mad_i24(3, hd[O] + hd[N], mul_i24(10, hd[M]));
                    const int gy = hs[N] - hs[O];
                    pxx = mul_i24(gx, gx);
                    pxy = mul_i24(gx, gy);
                    pyy = mul_i24(gy, gy);
                }
            } else {
                if (xs && Yg >= -1 - R && Yg < H + R) {
                    const int yc = reflect101(Yg, H) - sy0;
                    const int a00 = sm.img[yc - 1][xc - 1], a01 = sm.img[yc - 1][xc], a02 = sm.img[yc - 1][xc + 1];
                    const int a10 = sm.img[yc][xc - 1], a12 = sm.img[yc][xc + 1];
                    const int a20 = sm.img[yc + 1][xc - 1], a21 = sm.img[yc + 1][xc], a22 = sm.img[yc + 1][xc + 1];
                    const int gx = 3 * (a02 - a00) + 10 * (a12 - a10) + 3 * (a22 - a20);
                    const int gy = 3 * (a20 - a00) + 10 * (a21 - a01) + 3 * (a22 - a02);
                    pxx = mul_i24(gx, gx);
                    pxy = mul_i24(gx, gy);
                    pyy = mul_i24(gy, gy);
                }
            }
            if constexpr (R == 1) {
                pxx += from_left(pxx) + from_right(pxx);
                pxy += from_left(pxy) + from_right(pxy);
                pyy += from_left(pyy) + from_right(pyy);
            }
            hxx[P] = pxx;
            hxy[P] = pxy;
            hyy[P] = pyy;
        };
        // Rows are walked three at a time with every ring slot a fixed
        // register: step k (response row Yr = y0 - 1 + k) puts the horizontal
        // sums of gradient row Yr + R in slot (k + 2) % 3 (R = 1: slots 0 and 1
        // start with rows y0 - 2 and y0 - 1; R = 0 uses slot 0 alone), its
        // response and row maximum in slot k % 3, and reads the previous row's
        // response from slot (k + 2) % 3.  The block sum and the 3x3 maximum
        // are symmetric in the slots, so no register moves between rows.
        if constexpr (ROLL) {
            // the first gradient row (y0 - 1 - R, staged row 1) has ring slot
            // O = 1 (R = 1) or 0 (R = 0): its staged rows 0 and 1 first
            constexpr int O0 = R == 1 ? 1 : 0;
            if (xs) {
                row_taps(0, hd[O0], hs[O0]);
                row_taps(1, hd[(O0 + 1) % 3], hs[(O0 + 1) % 3]);
            }
        }
        if constexpr (R == 1) {
            grad_row(S1{}, y0 - 2);                             // into product slot 0
            grad_row(S2{}, y0 - 1);                             // slot 1
        }
        double rr[3] = {0.0, 0.0, 0.0}, mm[3] = {0.0, 0.0, 0.0};
        auto step = [&](auto w_slot, auto p_slot, int Yr, bool out) {
            constexpr int Ws = decltype(w_slot)::value, Ps = decltype(p_slot)::value;
            grad_row(w_slot, Yr + R);                           // product slot Ps (R = 1)
            double v = -__builtin_inf();
            if (xi && (ROLL || (Yr >= 0 && Yr < H))) {         // (every row of a rolling walk is in the frame)
                const int32_t a = R == 1 ? hxx[0] + hxx[1] + hxx[2] : hxx[0];
                const int32_t b = R == 1 ? hxy[0] + hxy[1] + hxy[2] : hxy[0];
                const int32_t c = R == 1 ? hyy[0] + hyy[1] + hyy[2] : hyy[0];
                v = min_eig(a, b, c);
            }
            mm[Ws] = max3_lanes(v);
            if (out) {
                // output row Yr - 1: the response of row Yr - 1 against the 3x3 maximum
                const int Yo = Yr - 1;
                const double r = rr[Ps];
                bool peak = false;
                if (xo) {
                    if (J.response) J.response[(size_t)Yo * W + X] = r;
                    vmax = max_r(vmax, r);                      // (never NaN, never -0)
                    const double mx = max_r(mm[0], max_r(mm[1], mm[2]));
                    peak = r > 0.0 && r == mx && X >= border && Yo >= border && X < W - border && Yo < H - border;
                }
                const unsigned long long bal = __ballot(peak);
                if (bal) {
                    if (peak) {
                        GfttPeak pk;
                        pk.rbits = (unsigned long long)__double_as_longlong(r);
                        pk.idx = (uint32_t)(Yo * W + X);
                        pk.pad = 0;
                        // the lane's rank among the row's peaks
                        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        sm.buf[nbuf + rank] = pk;
                    }
                    nbuf += (uint32_t)__popcll(bal);
                    if (nbuf > S::NBUF - 64) flush();           // a full row must still fit
                }
            }
            rr[Ws] = v;
        };
        step(S0{}, S2{}, y0 - 1, false);                        // rows y0 - 1 and y0: no output yet
        step(S1{}, S0{}, y0, false);
        for (int Yr = y0 + 1;; Yr += 3) {                       // ye >= y0 + 1
            step(S2{}, S1{}, Yr, true);
            if (Yr + 1 > ye) break;
            step(S0{}, S2{}, Yr + 1, true);
            if (Yr + 2 > ye) break;
            step(S1{}, S0{}, Yr + 2, true);
            if (Yr + 3 > ye) break;
        }
    };
    // gradient rows y0 - 1 - R .. ye + R; lane columns x0 - 2 .. x0 + 61
    const bool rolls = y0 - 1 - R >= 0 && ye + R <= H - 1;
    const bool inside = x0 - 2 >= 0 && x0 + 61 < W;
    if (rolls && inside)
        walk(std::true_type{}, std::true_type{});
    else if (rolls)
        walk(std::true_type{}, std::false_type{});
    else
        walk(std::false_type{}, std::false_type{});
    // the rest of the peaks, and the strip's maximum (one atomic each)
    {
        if (nbuf) flush();
        unsigned long long mb = (unsigned long long)__double_as_longlong(vmax);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long other = __shfl_xor(mb, o, 64);
            mb = other > mb ? other : mb;
        }
        if (lane == 0 && mb) atomicMax(J.max_bits, mb);
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

// The occupied points of a frame (read on the device where the count is),
// and whether the compaction filters by them; the same for every thread.
__device__ __forceinline__ int gftt_n_occupied(const GfttJob &J)
{
    return __builtin_amdgcn_readfirstlane(J.n_occupied_dev ? *J.n_occupied_dev : J.n_occupied);
}
__device__ __forceinline__ bool gftt_filtered(const GfttJob &J, int min_dist)
{
    return gftt_n_occupied(J) > 0 && min_dist > 0;
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
    const int n_occ = gftt_n_occupied(J);
    const bool filter = gftt_filtered(J, min_dist);
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
    // leading lz bits of those two (none exist when the two are equal), and
    // the 8 key bits after those, their bucket, are histogrammed
    const unsigned long long diff = max_bits ^ thr_bits;
    const int lz = diff ? __clzll((long long)diff) : 64;
    __syncthreads();                           // s_hist is cleared (when no grid was built)
    // this workgroup's slice of the frame's peaks (a multiple of 64 long),
    // CB per thread at a time: the kept ones counted by bucket.  Without
    // occupied points they are marked in the keep bits (a wavefront's 64
    // consecutive peaks are two words; the words of a slice are its
    // workgroup's alone) and counted in all; with them (most peaks blocked)
    // each batch's kept peaks get one range of the candidate list (one global
    // atomic), wavefronts in turn, lanes by their ballot prefix (the order
    // does not matter: the selection ranks by the total key)
    const int per = ((np + gridDim.x - 1) / gridDim.x + 63) & ~63;
    const int k_lo = min(np, (int)blockIdx.x * per), k_hi = min(np, k_lo + per);
    constexpr int CB = 8;
    uint32_t mine = 0;                         // the wavefront's kept peaks (keep-bit form)
    for (int k0 = k_lo; k0 < k_hi; k0 += CB * BLOCK) {
        GfttPeak p[CB];
        unsigned long long m[CB];
        uint32_t wc = 0;
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int k = k0 + i * BLOCK + (int)threadIdx.x;
            p[i] = k < k_hi ? J.peaks[k] : GfttPeak{};
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int k = k0 + i * BLOCK + (int)threadIdx.x;
            const bool keep = k < k_hi && p[i].rbits > thr_bits && kept(p[i]);
            if (keep && lz < 64) atomicAdd(&s_hist[key_digit(Key{p[i].rbits, ~p[i].idx}, lz)], 1u);
            m[i] = __ballot(keep);
            wc += (uint32_t)__popcll(m[i]);
            const int base = k0 + i * BLOCK + 64 * wv;           // the wavefront's first peak
            if (!filter && lane == 0 && base < k_hi) {
                J.keep[base >> 5] = (uint32_t)m[i];
                J.keep[(base >> 5) + 1] = (uint32_t)(m[i] >> 32);
            }
        }
        if (!filter) {
            mine += wc;
            continue;
        }
        if (lane == 0) s_cnt[wv] = wc;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            const uint32_t c = s_cnt[w];
            before += w < wv ? c : 0u;
            all += c;
        }
        if (threadIdx.x == 0) s_base = all ? (uint32_t)atomicAdd(J.n_cand, (int)all) : 0u;
        __syncthreads();
        uint32_t at = s_base + before;
        const unsigned long long lt = (1ull << lane) - 1;
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            if ((m[i] >> lane) & 1ull) J.cand[at + (uint32_t)__popcll(m[i] & lt)] = p[i];
            at += (uint32_t)__popcll(m[i]);
        }
        __syncthreads();                       // s_cnt and s_base are reused
    }
    if (!filter) {
        // workgroup total of the keep-bit form, one global atomic
        if (lane == 0) s_cnt[wv] = mine;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < BLOCK / 64; ++w) tot += s_cnt[w];
            if (tot) atomicAdd(J.n_cand, (int)tot);
        }
    }
    if (lz < 64 && s_hist[threadIdx.x]) atomicAdd(&J.hist[threadIdx.x], s_hist[threadIdx.x]);
}

// ---- candidates by bucket -----------------------------------------------------
//
// A candidate's bucket is the 8 bits of its rank key that the compaction
// histogrammed.  This grid (gridDim.x workgroups per frame) writes the
// candidates by bucket, larger buckets first (in any order within a bucket),
// to the list the selection reads: every bucket, and every run of buckets, is
// then one contiguous range, and the selection reads only the buckets a
// window can reach instead of every candidate.  Without occupied points the
// candidates are the peaks the keep bits mark and go to the candidate list;
// with them they are the appended candidate list and go to the peak list.
__global__ __launch_bounds__(BLOCK) void k_gftt_bucket(const GfttJob *__restrict__ jobs, double quality,
                                                      int min_dist)
{
    __shared__ uint32_t s_pos[256], s_cnt[256], s_wsum[BLOCK / 64];
    const GfttJob &J = jobs[blockIdx.y];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nc = *J.n_cand;
    if (nc == 0) return;                       // (then the bucket bits may not exist)
    const bool filter = gftt_filtered(J, min_dist);
    const GfttPeak *src = filter ? J.cand : J.peaks;
    GfttPeak *dst = filter ? J.peaks : J.cand;
    const int np = filter ? nc : *J.n_peaks;
    const unsigned long long max_bits = *J.max_bits;
    const unsigned long long thr_bits =
        (unsigned long long)__double_as_longlong(quality * __longlong_as_double((long long)max_bits));
    // candidates exist, so thr_bits < max_bits
    const int lz = __clzll((long long)(max_bits ^ thr_bits));
    // start of bucket b = the candidates in buckets above b: thread t scans
    // bucket 255 - t
    const uint32_t h = J.hist[255 - tid];
    uint32_t incl = h;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) s_wsum[wv] = incl;
    s_cnt[tid] = 0u;
    __syncthreads();
    uint32_t start = incl - h;
    for (int w = 0; w < wv; ++w) start += s_wsum[w];
    // this workgroup's slice of the peaks, read once, CB per thread at a
    // time: the kept ones counted by bucket, a range of each bucket reserved
    // (one global atomic per bucket the batch holds), then written
    const int per = ((np + gridDim.x - 1) / gridDim.x + 63) & ~63;
    const int k_lo = min(np, (int)blockIdx.x * per), k_hi = min(np, k_lo + per);
    constexpr int CB = 8;
    for (int k0 = k_lo; k0 < k_hi; k0 += CB * BLOCK) {
        GfttPeak p[CB];
        uint32_t d[CB];
        bool keep[CB];
        // the keep bits first: only the kept peaks are read
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int k = k0 + i * BLOCK + tid;
            keep[i] = k < k_hi && (filter || ((J.keep[k >> 5] >> (k & 31)) & 1u));
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            const int k = k0 + i * BLOCK + tid;
            p[i] = keep[i] ? src[k] : GfttPeak{};
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            d[i] = key_digit(Key{p[i].rbits, ~p[i].idx}, lz);
            if (keep[i]) atomicAdd(&s_cnt[d[i]], 1u);
        }
        __syncthreads();
        {
            const int b = 255 - tid;
            const uint32_t c = s_cnt[b];
            s_pos[b] = c ? start + (uint32_t)atomicAdd(&J.cursor[b], c) : 0u;
        }
        __syncthreads();
        s_cnt[tid] = 0u;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CB; ++i)
            if (keep[i]) dst[s_pos[d[i]] + atomicAdd(&s_cnt[d[i]], 1u)] = p[i];
        __syncthreads();
        s_cnt[tid] = 0u;                       // (read by no thread before the next barrier)
        __syncthreads();
    }
}

// ---- selection --------------------------------------------------------------

constexpr int CAPW = kGfttWindow;             // window of peaks sorted in LDS
constexpr int TG_CELLS = 2048;                // cells of the taken-corner grid, at most
constexpr int SBLOCK = 1024;                  // threads of the selection workgroup
constexpr int CHUNK = 512;                    // candidates decided together (the first CHUNK threads)
constexpr int KPT = 4;                        // keys per thread in flight in the list passes
typedef short s16x2 __attribute__((ext_vector_type(2)));

struct alignas(16) SelSmem {
    unsigned long long whi[CAPW];
    uint32_t wlo[CAPW];
    uint32_t taken[kGfttMaxCorners + 16];     // x | y << 16
    OccGridSmem grid;                          // the cached occupied points
    uint32_t cxy[CHUNK];                       // packed candidates: x | y << 16
    int32_t tg_head[TG_CELLS];                 // taken corners by grid cell: first index, -1 for none
    int32_t tg_next[kGfttMaxCorners + 16];     // the next index in the same cell
    uint32_t hist[SBLOCK / 64][256];           // one histogram per wavefront
    unsigned long long cmask[CHUNK][CHUNK / 64];   // conflicts with better candidates of the chunk
    unsigned long long sel[CHUNK / 64], und[CHUNK / 64];
    uint32_t bstart[256], bcnt[256];           // the list range of each bucket
    uint32_t bwsum[4];
    int32_t bb, be;
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
    // the candidates by bucket (the bucket layout's list), and the other
    // list, free now, for short copies
    const bool occ_filtered = gftt_filtered(J, min_dist);
    const GfttPeak *list = occ_filtered ? J.peaks : J.cand;
    GfttPeak *spare = occ_filtered ? J.cand : J.peaks;
    const int n_occ = gftt_n_occupied(J);
    // every candidate's R bits lie in (thr_bits, max_bits] (the threshold is
    // formed as the compaction forms it)
    const unsigned long long max_bits = *J.max_bits;
    const unsigned long long thr_bits =
        (unsigned long long)__double_as_longlong(quality * __longlong_as_double((long long)max_bits));
    // they share the leading lz bits of those two (when the two are equal
    // there are none); the 8 key bits after those are their bucket, and
    // bucket b holds list positions [bstart[b], bstart[b] + bcnt[b]), larger
    // buckets first
    const unsigned long long diff0 = max_bits ^ thr_bits;
    const int lz = diff0 ? __clzll((long long)diff0) : 63;
    const Key shared{max_bits, 0};              // (its leading lz bits)
    {
        uint32_t h = 0, incl = 0;              // thread t < 256 scans bucket 255 - t
        if (tid < 256) {
            h = J.hist[255 - tid];
            incl = h;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            if (lane == 63) sm.bwsum[wv] = incl;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t start = incl - h;
            for (int w = 0; w < wv; ++w) start += sm.bwsum[w];
            sm.bstart[255 - tid] = start;
            sm.bcnt[255 - tid] = h;
        }
    }

    const TakenGrid T = taken_grid(W, J.h, min_dist);
    for (int c = tid; c < TG_CELLS; c += SBLOCK) sm.tg_head[c] = -1;
    const OccGrid G = occ_grid_build<SBLOCK>(J, n_occ, min_dist, sm.grid);   // ends with a barrier
    int remaining = np;
    int nt = 0;
    bool bounded = false;
    Key bound{0, 0};
    __syncthreads();

    while (nt < max_corners && remaining > 0) {
        // ---- the next window: the best min(CAPW, remaining) candidates,
        // ranks [consumed, consumed + wn) of the descending order
        const int consumed = np - remaining;
        const int wn = remaining < CAPW ? remaining : CAPW;
        if (tid < 256) {
            const int b0 = (int)sm.bstart[tid], b1 = b0 + (int)sm.bcnt[tid];
            if (b0 <= consumed && consumed < b1) sm.bb = tid;
            if (b0 <= consumed + wn - 1 && consumed + wn - 1 < b1) sm.be = tid;
        }
        __syncthreads();
        const int bb = sm.bb & 255, be = sm.be & 255;   // buckets of the first and the last rank, bb >= be
        // the window's keys: every eligible key of buckets bb .. be + 1 (list
        // range A) and those of bucket be (range B) that are >= low
        const int a_lo = (int)sm.bstart[bb], a_hi = (int)sm.bstart[be];
        const GfttPeak *srcB = list + sm.bstart[be];
        int nB = (int)sm.bcnt[be];
        const Key bucket_low = key_with_digit(shared, lz, (uint32_t)be);
        Key low = wn < remaining ? bucket_low : Key{0, 0};
        if (wn < remaining && consumed + wn < (int)(sm.bstart[be] + sm.bcnt[be])) {
            // the window ends inside bucket be: radix selection of its best
            // `need` eligible keys, by the digits after the bucket's
            const uint32_t need_be = (uint32_t)(consumed + wn - max(consumed, (int)sm.bstart[be]));
            uint32_t need = need_be;
            Key prefix = bucket_low;
            bool filtered = false;
            for (int d = lz + 8; d < 96; d += 8) {
                for (int k = tid; k < (SBLOCK / 64) * 256; k += SBLOCK) (&sm.hist[0][0])[k] = 0;
                __syncthreads();
                for (int k0 = 0; k0 < nB; k0 += KPT * SBLOCK) {
                    Key key[KPT];
#pragma unroll
                    for (int i = 0; i < KPT; ++i) {
                        const int k = k0 + i * SBLOCK + tid;
                        key[i] = k < nB ? Key{srcB[k].rbits, ~srcB[k].idx} : Key{0, 0};
                    }
#pragma unroll
                    for (int i = 0; i < KPT; ++i)
                        if (key[i].hi != 0 && eligible(key[i], bounded, bound) && key_prefix_eq(key[i], prefix, d))
                            atomicAdd(&sm.hist[wv][key_digit(key[i], d)], 1u);
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
                    uint32_t run = ls;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t v = __shfl_down(run, o, 64);
                        if (lane + o < 64) run += v;
                    }
                    uint32_t cum = run - ls;             // sum over lanes > lane
#pragma unroll
                    for (int i = 3; i >= 0; --i) {
                        if (cum < need && need <= cum + t[i]) {
                            sm.need = need - cum;
                            sm.done_flag = t[i] == need - cum ? 1 : 0;
                            sm.bound = key_with_digit(prefix, d, (uint32_t)(4 * lane + i));
                            sm.bcount = t[i];
                        }
                        cum += t[i];
                    }
                }
                __syncthreads();
                need = sm.need;
                prefix = sm.bound;
                const bool whole = sm.done_flag != 0;
                const int kept = (int)(need_be - need + sm.bcount);   // bucket keys >= the new prefix
                __syncthreads();
                if (whole) break;
                if (!filtered && 4 * kept <= nB) {
                    // copy bucket be's eligible keys >= prefix (its lower bytes
                    // are 0) to the spare list, KPT keys per thread in flight
                    if (tid == 0) sm.wcount = 0;
                    __syncthreads();
                    for (int k0 = 0; k0 < nB; k0 += KPT * SBLOCK) {
                        GfttPeak pk[KPT];
#pragma unroll
                        for (int i = 0; i < KPT; ++i) {
                            const int k = k0 + i * SBLOCK + tid;
                            pk[i] = k < nB ? srcB[k] : GfttPeak{};
                        }
#pragma unroll
                        for (int i = 0; i < KPT; ++i) {
                            const int k = k0 + i * SBLOCK + tid;
                            const Key key{pk[i].rbits, ~pk[i].idx};
                            const bool take = k < nB && eligible(key, bounded, bound) && !key_less(key, prefix);
                            const uint32_t at = wave_append(take, &sm.wcount);
                            if (take) spare[at] = pk[i];
                        }
                    }
                    __syncthreads();             // the copy is visible to the whole workgroup
                    srcB = spare;
                    nB = (int)sm.wcount;
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
        const int nA = a_hi - a_lo, ngat = nA + nB;
        for (int k0 = 0; k0 < ngat; k0 += KPT * SBLOCK) {
            Key key[KPT];
#pragma unroll
            for (int i = 0; i < KPT; ++i) {
                const int k = k0 + i * SBLOCK + tid;
                const GfttPeak *q = k < nA ? list + a_lo + k : srcB + (k - nA);
                key[i] = k < ngat ? Key{q->rbits, ~q->idx} : Key{0, 0};
            }
#pragma unroll
            for (int i = 0; i < KPT; ++i) {
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
        // Bitonic sort, descending, of pw slots (keys past wu are 0, below
        // every key): thread tid holds elements E tid .. E tid + E - 1 in
        // registers; the compare-exchanges of stride below E stay inside a
        // thread, those of stride E .. 32 E go to lane tid ^ (stride / E) of
        // the same wavefront, and only those of stride 64 E and more pass
        // through LDS (6 barrier pairs for 2048 keys instead of a barrier per
        // stage).
        constexpr int E = CAPW / SBLOCK;
        static_assert(E == 2 || E == 4, "two or four window keys per thread");
        Key kk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = E * tid + e;
            kk[e] = i < wu ? Key{sm.whi[i], sm.wlo[i]} : Key{0, 0};
        }
        // element i keeps the larger key of (i, i ^ stride) iff i is the lower
        // one of a descending block ((i & size) == 0) or the upper one of an
        // ascending block
        auto keep = [&](int e, Key o, int stride, int size) {
            const int i = E * tid + e;
            const bool keep_max = ((i & size) == 0) == ((i & stride) == 0);
            const bool o_less = key_less(o, kk[e]);
            if (keep_max != o_less) kk[e] = o;
        };
        for (int size = 2; size <= pw; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                if (stride >= 64 * E) {
                    __syncthreads();                     // the last stage's reads are done
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        sm.whi[E * tid + e] = kk[e].hi;
                        sm.wlo[E * tid + e] = kk[e].lo;
                    }
                    __syncthreads();
                    Key o[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int j = (E * tid + e) ^ stride;
                        o[e] = Key{sm.whi[j], sm.wlo[j]};
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) keep(e, o[e], stride, size);
                } else if (stride >= E) {
                    // all exchanges in flight before the first use
                    const int m = stride / E;
                    Key o[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        o[e].hi = __shfl_xor(kk[e].hi, m, 64);
                        o[e].lo = __shfl_xor(kk[e].lo, m, 64);
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) keep(e, o[e], stride, size);
                } else {
                    // inside the thread (the elements of a pair share (i & size))
                    auto cex = [&](Key &a, Key &b, int i) {
                        if (key_less(a, b) == ((i & size) == 0)) {
                            const Key t = a;
                            a = b;
                            b = t;
                        }
                    };
                    if constexpr (E == 2) {
                        cex(kk[0], kk[1], 2 * tid);
                    } else {
                        if (stride == 2) {
                            cex(kk[0], kk[2], 4 * tid);
                            cex(kk[1], kk[3], 4 * tid + 1);
                        } else {
                            cex(kk[0], kk[1], 4 * tid);
                            cex(kk[2], kk[3], 4 * tid + 2);
                        }
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            sm.whi[E * tid + e] = kk[e].hi;
            sm.wlo[E * tid + e] = kk[e].lo;
        }
        __syncthreads();
        // ---- accept in rank order, CHUNK candidates at a time
        for (int c0 = 0; c0 < wu && nt < max_corners; c0 += CHUNK) {
            const int k = c0 + tid;
            const bool valid = tid < CHUNK && k < wu;   // the first CHUNK threads hold the chunk
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
                if (lane == 0 && wv < CHUNK / 64) sm.und[wv] = free_bits;
            }
            __syncthreads();
            int mu = 0, at = 0;
#pragma unroll
            for (int w = 0; w < CHUNK / 64; ++w) {
                const int c = __popcll(sm.und[w]);
                mu += c;
                at += w < wv ? c : 0;
            }
            if (!blocked) {
                at += __popcll(sm.und[wv] & ((1ull << lane) - 1));
                sm.cxy[at] = (uint32_t)x | ((uint32_t)y << 16);
            }
            __syncthreads();
            // conflicts of packed candidate t with the better packed ones
            // u < t (squared distance < min_dist^2), one 64-bit mask per group
            // of 64: the triangle's 64 x 64 blocks (row group g, column group
            // h <= g) are dealt to the wavefronts in turn, a lane per row.
            // Positions are int16 pairs (coordinates < 32768): one packed
            // subtract and one 16-bit dot product give dx^2 + dy^2 exactly
            // (at most 2 * 32767^2 < 2^31).
            if (spaced) {
                const int ng = (mu + 63) >> 6;
                const int nblk = ng * (ng + 1) / 2;
                const uint4 *p4 = reinterpret_cast<const uint4 *>(sm.cxy);
                for (int blk = wv; blk < nblk; blk += SBLOCK / 64) {
                    int g = 0;
                    while ((g + 1) * (g + 2) / 2 <= blk) ++g;
                    const int h = blk - g * (g + 1) / 2;
                    const int t = 64 * g + lane;
                    if (t < mu) {
                        const s16x2 pt = __builtin_bit_cast(s16x2, sm.cxy[t]);
                        const int u_end = h < g ? 64 : lane;    // columns 64 h + [0, u_end)
                        unsigned long long mw = 0;
                        for (int i0 = 0; i0 < u_end; i0 += 8) {
                            const uint4 a = p4[(64 * h + i0) / 4], b = p4[(64 * h + i0) / 4 + 1];
                            const uint32_t pu[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
                            uint32_t bits = 0;
#pragma unroll
                            for (int i = 0; i < 8; ++i) {
                                const s16x2 d = pt - __builtin_bit_cast(s16x2, pu[i]);
                                const int dd = __builtin_amdgcn_sdot2(d, d, 0, false);
                                bits |= (uint32_t)(dd < md2 && i0 + i < u_end) << i;
                            }
                            mw |= (unsigned long long)bits << i0;
                        }
                        sm.cmask[t][h] = mw;
                    }
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
            const bool mine = tid < mu && ((sm.sel[wv] >> lane) & 1ull);
            const int pos = nt + before;
            if (mine && pos < max_corners) {
                const uint32_t pm = sm.cxy[tid];
                const int xm = (int)(pm & 0xFFFFu), ym = (int)(pm >> 16);
                sm.taken[pos] = pm;
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
    J.cursor[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        *J.n_peaks = 0;
        *J.n_cand = 0;
        *J.max_bits = 0ull;
    }
}

}  // namespace

hipError_t launch_gftt(const GfttJob *d_jobs, const int32_t *d_tile_job, int njobs, int total_tiles, int tile_h,
                       int radius, int border, double quality, int min_dist, int max_corners, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    k_gftt_reset<<<njobs, 256, 0, s>>>(d_jobs);
    // the tile shape of each radius is the host's (gftt_tile_shape)
    switch (radius) {
    case 0:
    case 1: {
        const dim3 grid((total_tiles + kStripWaves - 1) / kStripWaves), block(64 * kStripWaves);
        const bool tall = tile_h == kGfttStripHTall;
        if (radius == 0 && tall) k_gftt_peaks_strip<0, kGfttStripHTall><<<grid, block, 0, s>>>(d_jobs, d_tile_job, total_tiles, border);
        else if (radius == 0) k_gftt_peaks_strip<0, kGfttStripH><<<grid, block, 0, s>>>(d_jobs, d_tile_job, total_tiles, border);
        else if (tall) k_gftt_peaks_strip<1, kGfttStripHTall><<<grid, block, 0, s>>>(d_jobs, d_tile_job, total_tiles, border);
        else k_gftt_peaks_strip<1, kGfttStripH><<<grid, block, 0, s>>>(d_jobs, d_tile_job, total_tiles, border);
        break;
    }
    case 2: k_gftt_peaks<2><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    default: k_gftt_peaks<3><<<total_tiles, BLOCK, 0, s>>>(d_jobs, d_tile_job, border); break;
    }
    k_gftt_compact<<<dim3(kCompactBlocks, njobs), BLOCK, 0, s>>>(d_jobs, quality, min_dist);
    k_gftt_bucket<<<dim3(kCompactBlocks, njobs), BLOCK, 0, s>>>(d_jobs, quality, min_dist);
    k_gftt_select<<<njobs, SBLOCK, 0, s>>>(d_jobs, quality, min_dist, max_corners);
    return hipGetLastError();
}

}  // namespace lkmi
