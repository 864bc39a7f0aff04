// HIP kernels of liblkmi for CDNA4 (gfx950): Gaussian pyramid, binary16
// gradient planes, and the per-keypoint pyramidal Lucas-Kanade tracker.
//
// Pyramid (the binomial blur-and-decimate step) and gradient planes are
// HBM-streaming stencils: one workgroup per output tile, the input tile plus
// halo staged in LDS with reflect-101 borders, separable passes in LDS.
//
// Tracker: one wavefront (64 lanes) per keypoint.  The win x win window is cut
// into vertical strips: lane (column group cg, row segment sg) owns CW
// columns x R rows of window pixels, so consecutive lanes read consecutive
// pixels of a row (coalesced) and each lane reuses bilinear taps between its
// vertically adjacent pixels.  Because the window offsets are integers, every
// pixel of the window shares one set of bilinear weights, so a lane holds the
// taps of the target frame in registers (as left tap and right-minus-left
// difference in the one-column layouts) and only reloads them when the
// integer part of the estimate moves.  Sums over the window (the 2x2 normal
// matrix and the mismatch vector) are reduced with DPP adds and one lane read
// in a fixed order: every lane obtains the same bits, control flow stays
// wave-uniform, and a point's result does not depend on what else is in the
// launch.  No MFMA: nothing here is a dense
// contraction.
#include "lk_internal.h"

#include <type_traits>

namespace lkmi {
namespace {

constexpr int kThreads = 256;            // 4 wavefronts per workgroup
constexpr int kWave = 64;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int reflect101(int i, int n)
{
    // single reflection about the end samples; callers keep -n < i < 2n - 1
    i = i < 0 ? -i : i;
    return i >= n ? 2 * (n - 1) - i : i;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float uniform_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the 64 lanes of a wavefront, in one fixed order: pairs, quads,
// 8-lane halves and 16-lane rows by DPP, then row 0 + row 1 into row 1 and
// row 2 + row 3 into row 3 (row broadcast of lane 15), then rows 0-1 into
// rows 2-3 (row broadcast of lane 31); lane 63 then holds the total, which is
// read into a scalar register, so every lane gets the same bits.
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x141>(v);   // row_half_mirror: quad <-> quad within 8 lanes
    v += dpp_move<0x140>(v);   // row_mirror: half-row <-> half-row within 16 lanes
    // the row broadcasts write every row (a row without a source adds 0), so
    // each is one DPP add; only lane 63's sum is read
    v += dpp_move<0x142>(v);
    v += dpp_move<0x143>(v);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Pixel loads by element kind.
enum Kind { K_U8 = 0, K_F32 = 1, K_F16 = 2 };

template <int KIND>
__device__ __forceinline__ float ldpx(const void *p, int idx)
{
    if constexpr (KIND == K_U8) return (float)static_cast<const uint8_t *>(p)[idx];
    else if constexpr (KIND == K_F32) return static_cast<const float *>(p)[idx];
    else return __half2float(static_cast<const __half *>(p)[idx]);
}

// =================================================================== pyramid

// The [1 4 6 4 1] / 16 tap sum, one rounding per operation in this order
// (the same in every pyramid kernel, so fused and per-level builds agree bit
// for bit; on 8-bit data and their first two levels every step is exact).
__device__ __forceinline__ float binom5(float q0, float q1, float q2, float q3, float q4)
{
#pragma clang fp contract(off)
    return ((q0 + q4) + 4.0f * (q1 + q3) + 6.0f * q2) * 0.0625f;
}

constexpr int kInW = 2 * kDownTileW + 3;   // input tile columns incl. halo
constexpr int kInH = 2 * kDownTileH + 3;
constexpr int kBufWord3 = 0x00020000;      // buffer resource word 3, gfx9 family: raw 32-bit access

// Interior tiles stage their input with 16-byte loads starting CHUNK pixels
// before the tile so that every load is aligned; border tiles take the
// reflect-101 path one pixel at a time.
template <int SK> struct Chunk { static constexpr int PX = SK == K_U8 ? 16 : (SK == K_F16 ? 8 : 4); };
template <int SK> struct InRow {
    static constexpr int PX = Chunk<SK>::PX;
    static constexpr int N = (PX + 2 * kDownTileW + 1 + PX - 1) / PX;   // chunks per input row
    static constexpr int W = N * PX;                                     // staged columns
};
constexpr int kInWMax = InRow<K_U8>::W > kInW ? InRow<K_U8>::W : kInW;

struct DownSmem {
    float in[kInH][kInWMax + 1];
    float h[kInH][kDownTileW + 4];
};

template <int SK>
__device__ __forceinline__ void unpack_chunk(uint4 v, float *dst)
{
    if constexpr (SK == K_U8) {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) dst[k] = (float)((w[k >> 2] >> (8 * (k & 3))) & 0xFFu);
    } else if constexpr (SK == K_F16) {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float2 f = __half22float2(__builtin_bit_cast(__half2, w[k]));
            dst[2 * k] = f.x;
            dst[2 * k + 1] = f.y;
        }
    } else {
        dst[0] = __builtin_bit_cast(float, v.x); dst[1] = __builtin_bit_cast(float, v.y);
        dst[2] = __builtin_bit_cast(float, v.z); dst[3] = __builtin_bit_cast(float, v.w);
    }
}

template <int SK, bool F16>
__device__ void downsample_tile(const DownJob &j, int tile, DownSmem &sm)
{
    constexpr int es = SK == K_U8 ? 1 : (SK == K_F16 ? 2 : 4);
    const int tx = tile % j.tiles_x, ty = tile / j.tiles_x;
    const int ox0 = tx * kDownTileW, oy0 = ty * kDownTileH;
    const int sx0 = 2 * ox0 - 2, sy0 = 2 * oy0 - 2;
    constexpr int PX = Chunk<SK>::PX;
    // staged columns cover input x in [a0, a0 + InRow::W); a0 is 16-byte aligned
    const int a0 = sx0 + 2 - PX;
    const bool vec_ok = ((j.spitch * es) & 15) == 0 && (reinterpret_cast<uintptr_t>(j.src) & 15) == 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(j.src), (short)0, j.spitch * j.sh * es, kBufWord3);
    for (int i = threadIdx.x; i < kInH * InRow<SK>::N; i += kThreads) {
        const int r = i / InRow<SK>::N, c = i - r * InRow<SK>::N;
        const int gy = reflect101(min(sy0 + r, j.sh + 1), j.sh);
        const int x0 = a0 + c * PX;
        float *dst = &sm.in[r][c * PX];
        if (vec_ok && x0 >= 0 && x0 + PX <= j.sw) {
            const uint4 v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (gy * j.spitch + x0) * es, 0, 0));
            unpack_chunk<SK>(v, dst);
        } else {
            // chunk crosses a frame edge: reflect-101 per pixel (never more
            // than one reflection: x stays within [-PX, sw + PX))
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int gx = reflect101(clampi(x0 + k, -2, j.sw + 1), j.sw);
                dst[k] = ldpx<SK>(j.src, gy * j.spitch + gx);
            }
        }
    }
    const int off = PX - 2;                          // staged column of input x = sx0
    __syncthreads();
    // horizontal [1 4 6 4 1] at even columns; exact for short dyadic values
    for (int i = threadIdx.x; i < kInH * kDownTileW; i += kThreads) {
        const int r = i / kDownTileW, c = i - r * kDownTileW;
        const float *q = &sm.in[r][2 * c + off];
        sm.h[r][c] = binom5(q[0], q[1], q[2], q[3], q[4]);
    }
    __syncthreads();
    // vertical: each thread makes 4 consecutive outputs of one row
    {
        const int r = threadIdx.x >> 4, c = (threadIdx.x & 15) * 4;
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = binom5(sm.h[2 * r][c + k], sm.h[2 * r + 1][c + k], sm.h[2 * r + 2][c + k], sm.h[2 * r + 3][c + k],
                          sm.h[2 * r + 4][c + k]);
        const int ox = ox0 + c, oy = oy0 + r;
        if (oy < j.dh) {
            if (ox + 3 < j.dw) {
                if constexpr (F16) {
                    const __half2 a = __floats2half2_rn(v[0], v[1]), b = __floats2half2_rn(v[2], v[3]);
                    uint2 u;
                    u.x = __builtin_bit_cast(uint32_t, a);
                    u.y = __builtin_bit_cast(uint32_t, b);
                    *reinterpret_cast<uint2 *>(static_cast<__half *>(j.dst) + oy * j.dpitch + ox) = u;
                } else {
                    *reinterpret_cast<float4 *>(static_cast<float *>(j.dst) + oy * j.dpitch + ox) =
                        make_float4(v[0], v[1], v[2], v[3]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (ox + k < j.dw) {
                        if constexpr (F16) static_cast<__half *>(j.dst)[oy * j.dpitch + ox + k] = __float2half_rn(v[k]);
                        else static_cast<float *>(j.dst)[oy * j.dpitch + ox + k] = v[k];
                    }
            }
        }
    }
}

__device__ void downsample_dispatch(const DownJob &j, int tile)
{
    __shared__ DownSmem sm;   // one LDS block shared by all instantiations
    if (j.src_u8) {
        if (j.dst_f16) downsample_tile<K_U8, true>(j, tile, sm);
        else downsample_tile<K_U8, false>(j, tile, sm);
    } else if (j.dst_f16) {
        downsample_tile<K_F16, true>(j, tile, sm);
    } else {
        downsample_tile<K_F32, false>(j, tile, sm);
    }
}

__global__ __launch_bounds__(kThreads) void k_downsample(DownJob j)
{
    downsample_dispatch(j, xcd_block(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(kThreads) void k_downsample_batched(const DownJob *jobs, const int32_t *tile_job)
{
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const DownJob j = jobs[uniform_i(tile_job[tile])];
    downsample_dispatch(j, tile - j.tile_begin);
}

// ------------------------------------------------ levels 1 and 2 in one pass
//
// Workgroup = one 32 x 16 tile of level 2 at (ox2, oy2).  Binary16 storage
// also writes the gradient plane of level 1 for the 64 x 32 tile under it,
// from the level-1 region (exact before the binary16 rounding, so it carries
// the bits of the gradient-plane kernel); level 0 has no stored plane (the
// tracker forms its binary16 gradients from the 8-bit frame).  Level 1 is formed
// on the region x1 in [2 ox2 - 2, 2 ox2 + 65), y1 in [2 oy2 - 2, 2 oy2 + 33)
// (the 64 x 32 tile under the level-2 tile plus the two-pixel halo the
// level-2 filter needs) from level 0 staged as bytes; the level-1 tile is
// written, and level 2 is filtered from the region in LDS.  Region entries
// outside level 1 are never read: the level-2 taps are reflected (reflect-101)
// into level 1 first, and the reflected positions lie inside the region
// whenever the level-2 tile is not empty.  Level 1 is rounded to its storage
// type before level 2 is formed from it, as a per-level build does.

constexpr int kP1W = 2 * kP12TileW + 3, kP1H = 2 * kP12TileH + 3;     // level-1 region 67 x 35
constexpr int kP0H = 2 * kP1H + 3;                                      // level-0 rows 73
constexpr int kP0Chunks = 10;                                           // 16-byte chunks per level-0 row
constexpr int kP0W = 16 * kP0Chunks;                                    // staged level-0 columns 160

struct alignas(16) P12Smem {
    union {                                   // the staged bytes are dead once level 1 is formed
        uint8_t in[kP0H][kP0W];
        float h2[kP1H][kP12TileW + 1];
    };
    float l1[kP1H][kP1W + 1];
};

// Two 16-bit unsigned integers in one register (packed 16-bit adds).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }

__device__ __forceinline__ float to_storage(float v, bool f16)
{
    return f16 ? __half2float(__float2half_rn(v)) : v;
}

template <bool F16>
__device__ void pyr12_tile(const Pyr12Job &j, int tile, P12Smem &sm)
{
    const int ox2 = (tile % j.tiles_x) * kP12TileW, oy2 = (tile / j.tiles_x) * kP12TileH;
    const int rx1 = 2 * ox2 - 2, ry1 = 2 * oy2 - 2;          // level-1 region origin
    const int a0 = 4 * ox2 - 16, sy0 = 2 * ry1 - 2;          // level-0 staging origin (16-byte aligned x)
    constexpr bool f16 = F16;
    // 1. level 0 rows [sy0, sy0 + 73) x columns [a0, a0 + 160) as bytes;
    //    samples outside the frame hold the reflect-101 sample
    const bool vec_ok = (j.spitch & 15) == 0 && (reinterpret_cast<uintptr_t>(j.src) & 15) == 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t *>(j.src), (short)0, j.spitch * j.sh, kBufWord3);
    //    every 16-byte load of a thread is issued before the first is
    //    stored, so a thread waits for memory once, not once per chunk
    constexpr int NCH = kP0H * kP0Chunks, PER = (NCH + kThreads - 1) / kThreads;
    uint4 v[PER];
    bool vec[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * kThreads;
        const int r = i / kP0Chunks, c = i - r * kP0Chunks;
        const int gy = reflect101(clampi(sy0 + r, -2, j.sh + 1), j.sh);
        const int x0 = a0 + 16 * c;
        vec[q] = i < NCH && vec_ok && x0 >= 0 && x0 + 16 <= j.sw;
        if (vec[q]) v[q] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, gy * j.spitch + x0, 0, 0));
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * kThreads;
        if (i >= NCH) continue;
        const int r = i / kP0Chunks, c = i - r * kP0Chunks;
        if (vec[q]) {
            *reinterpret_cast<uint4 *>(&sm.in[r][16 * c]) = v[q];
        } else {
            const int gy = reflect101(clampi(sy0 + r, -2, j.sh + 1), j.sh);
            const int x0 = a0 + 16 * c;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int gx = reflect101(clampi(x0 + k, -2, j.sw + 1), j.sw);
                sm.in[r][16 * c + k] = j.src[gy * j.spitch + gx];
            }
        }
    }
    __syncthreads();
    // 2. level-1 region by column walk: thread = (pair of columns, group of
    //    rows); the horizontal sums of level-0 rows slide down with the
    //    outputs.  The 7 taps of a column pair come from 3 aligned dwords.
    {
        constexpr int NP = (kP1W + 1) / 2;                       // 34 column pairs (column 67 is padding)
        constexpr int G = kThreads / NP;                         // 7 row groups
        constexpr int RPG = (kP1H + G - 1) / G;                  // 5 rows each
        const int pr = threadIdx.x % NP, g = threadIdx.x / NP;
        if (g < G) {
            const int c = 2 * pr;
            const int r_lo = g * RPG, r_hi = min(kP1H, r_lo + RPG);
            // level-1 x1 = rx1 + c has its centre tap at staged column 2 c + 12:
            // taps of columns c and c + 1 are staged bytes 2c+10 .. 2c+16, inside
            // the dwords at bytes [2c+8, 2c+20) (4-byte aligned: c is even)
            const uint32_t *col = reinterpret_cast<const uint32_t *>(&sm.in[0][2 * c + 8]);
            // On 8-bit data the binomial filter is exact in float (see
            // binom5), so it is formed here in integers: the horizontal sums
            // (weights 1 4 6 4 1, at most 255 x 16) and the vertical sum of
            // five of them (at most 255 x 256 = 65280), then one conversion
            // and the scaling by 1 / 256, both exact: the same bits as binom5
            // twice.  Both columns of the pair go through the sums at once, as
            // the two 16-bit halves of one register (packed 16-bit integer
            // adds; every sum fits 16 bits): the byte permutes place tap k of
            // column c and tap k + 2 of column c + 1 side by side.
            auto hsum2 = [&](int row) {
                const uint32_t *q = col + row * (kP0W / 4);
                const uint32_t w0 = q[0], w1 = q[1], w2 = q[2];
                const u16x2 p0 = as_u16x2(__builtin_amdgcn_perm(w1, w0, 0x0c040c02u));   // t2 | t4
                const u16x2 p1 = as_u16x2(__builtin_amdgcn_perm(w1, w0, 0x0c050c03u));   // t3 | t5
                const u16x2 p2 = as_u16x2(__builtin_amdgcn_perm(w1, w0, 0x0c060c04u));   // t4 | t6
                const u16x2 p3 = as_u16x2(__builtin_amdgcn_perm(w1, w0, 0x0c070c05u));   // t5 | t7
                const u16x2 p4 = as_u16x2(__builtin_amdgcn_perm(w2, w1, 0x0c040c02u));   // t6 | t8
                return (p0 + p4) + (u16x2)4 * (p1 + p3) + (u16x2)6 * p2;
            };
            auto vsum = [](u16x2 s0, u16x2 s1, u16x2 s2, u16x2 s3, u16x2 s4) {
                const uint32_t v = __builtin_bit_cast(uint32_t, (s0 + s4) + (u16x2)4 * (s1 + s3) + (u16x2)6 * s2);
                return make_float2((float)(v & 0xFFFFu) * (1.0f / 256.0f), (float)(v >> 16) * (1.0f / 256.0f));
            };
            // output row r uses level-0 staged rows 2 r .. 2 r + 4
            u16x2 h0 = hsum2(2 * r_lo), h1 = hsum2(2 * r_lo + 1), h2 = hsum2(2 * r_lo + 2);
            for (int r = r_lo; r < r_hi; ++r) {
                const u16x2 h3 = hsum2(2 * r + 3), h4 = hsum2(2 * r + 4);
                const float2 v = vsum(h0, h1, h2, h3, h4);
                sm.l1[r][c] = to_storage(v.x, f16);
                sm.l1[r][c + 1] = to_storage(v.y, f16);
                h0 = h2; h1 = h3; h2 = h4;
            }
        }
    }
    __syncthreads();
    // 3. write the level-1 tile (region rows/columns 2 .. 33 / 2 .. 65): each
    //    thread stores 8 consecutive pixels of one row
    {
        const int r = threadIdx.x >> 3, c = (threadIdx.x & 7) * 8;
        const int y1 = ry1 + 2 + r, x1 = rx1 + 2 + c;
        if (y1 < j.h1) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = sm.l1[r + 2][c + 2 + k];
            if (x1 + 7 < j.w1) {
                if constexpr (f16) {
                    uint4 u;
                    u.x = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[0], v[1]));
                    u.y = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[2], v[3]));
                    u.z = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[4], v[5]));
                    u.w = __builtin_bit_cast(uint32_t, __floats2half2_rn(v[6], v[7]));
                    *reinterpret_cast<uint4 *>(static_cast<__half *>(j.dst1) + (size_t)y1 * j.pitch1 + x1) = u;
                } else {
                    float *d = static_cast<float *>(j.dst1) + (size_t)y1 * j.pitch1 + x1;
                    *reinterpret_cast<float4 *>(d) = make_float4(v[0], v[1], v[2], v[3]);
                    *reinterpret_cast<float4 *>(d + 4) = make_float4(v[4], v[5], v[6], v[7]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (x1 + k < j.w1) {
                        if constexpr (f16) static_cast<__half *>(j.dst1)[(size_t)y1 * j.pitch1 + x1 + k] = __float2half_rn(v[k]);
                        else static_cast<float *>(j.dst1)[(size_t)y1 * j.pitch1 + x1 + k] = v[k];
                    }
            }
        }
    }
    const bool x_inside = rx1 >= 0 && rx1 + kP1W <= j.w1;
    if constexpr (F16) {
        // 3b. level-1 gradient plane of the 64 x 32 tile: thread = 4 columns x
        //     2 rows; neighbours reflected into level 1 (reflect-101) where the
        //     region reaches past it
        const int c = 4 * (threadIdx.x & 15), r = 2 * (threadIdx.x >> 4);
        const int x1 = rx1 + 2 + c, y1 = ry1 + 2 + r;
        const bool y_in = ry1 >= 0 && ry1 + kP1H <= j.h1;
        int cols[6], rows[4];
#pragma unroll
        for (int m = 0; m < 6; ++m)
            cols[m] = x_inside ? c + 1 + m : reflect101(clampi(x1 - 1 + m, -1, j.w1), j.w1) - rx1;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            rows[m] = y_in ? r + 1 + m : reflect101(clampi(y1 - 1 + m, -1, j.h1), j.h1) - ry1;
        float t[4][6];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int m = 0; m < 6; ++m) t[a][m] = sm.l1[rows[a]][cols[m]];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (y1 + k >= j.h1 || x1 >= j.w1) continue;
            __half2 g[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float gx = (3.0f * (t[k][m + 2] - t[k][m]) + 10.0f * (t[k + 1][m + 2] - t[k + 1][m])
                                  + 3.0f * (t[k + 2][m + 2] - t[k + 2][m])) * 0.03125f;
                const float gy = (3.0f * (t[k + 2][m] - t[k][m]) + 10.0f * (t[k + 2][m + 1] - t[k][m + 1])
                                  + 3.0f * (t[k + 2][m + 2] - t[k][m + 2])) * 0.03125f;
                g[m] = __floats2half2_rn(gx, gy);
            }
            __half2 *dst = j.g1 + (size_t)(y1 + k) * j.gpitch1 + x1;
            if (x1 + 3 < j.w1) {
                uint4 u;
                u.x = __builtin_bit_cast(uint32_t, g[0]);
                u.y = __builtin_bit_cast(uint32_t, g[1]);
                u.z = __builtin_bit_cast(uint32_t, g[2]);
                u.w = __builtin_bit_cast(uint32_t, g[3]);
                *reinterpret_cast<uint4 *>(dst) = u;
            } else {
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    if (x1 + m < j.w1) dst[m] = g[m];
            }
        }
    }
    // 4. level-2 horizontal pass at the level-1 rows of the region; taps
    //    reflected into level 1 (identity away from its left and right edges)
    for (int i = threadIdx.x; i < kP1H * kP12TileW; i += kThreads) {
        const int r = i / kP12TileW, c = i - r * kP12TileW;
        float v = 0.0f;
        if (ox2 + c < j.w2) {           // columns past level 2 are never used
            float q[5];
            if (x_inside) {
#pragma unroll
                for (int k = 0; k < 5; ++k) q[k] = sm.l1[r][2 * c + k];
            } else {
#pragma unroll
                for (int k = 0; k < 5; ++k) q[k] = sm.l1[r][reflect101(rx1 + 2 * c + k, j.w1) - rx1];
            }
            v = binom5(q[0], q[1], q[2], q[3], q[4]);
        }
        sm.h2[r][c] = v;
    }
    __syncthreads();
    // 5. level-2 vertical pass (taps reflected into level 1) and store: each
    //    thread makes 2 consecutive pixels of one row
    {
        const int r = threadIdx.x >> 4, c = (threadIdx.x & 15) * 2;
        const int y2 = oy2 + r, x2 = ox2 + c;
        if (y2 < j.h2) {
            // region row of level-1 row 2 y2 - 2 + k: 2 r + k when the region
            // lies inside level 1, else that row reflected into level 1
            const bool y_inside = ry1 >= 0 && ry1 + kP1H <= j.h1;
            float v[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                float q[5];
                if (y_inside) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) q[k] = sm.h2[2 * r + k][c + m];
                } else {
#pragma unroll
                    for (int k = 0; k < 5; ++k) q[k] = sm.h2[reflect101(2 * y2 - 2 + k, j.h1) - ry1][c + m];
                }
                v[m] = binom5(q[0], q[1], q[2], q[3], q[4]);
            }
            if constexpr (f16) {
                __half *d = static_cast<__half *>(j.dst2) + (size_t)y2 * j.pitch2 + x2;
                if (x2 + 1 < j.w2) *reinterpret_cast<__half2 *>(d) = __floats2half2_rn(v[0], v[1]);
                else if (x2 < j.w2) d[0] = __float2half_rn(v[0]);
            } else {
                float *d = static_cast<float *>(j.dst2) + (size_t)y2 * j.pitch2 + x2;
                if (x2 + 1 < j.w2) *reinterpret_cast<float2 *>(d) = make_float2(v[0], v[1]);
                else if (x2 < j.w2) d[0] = v[0];
            }
        }
    }
}

// ddst (nullable): the pyramid's device descriptor, written with desc by one
// thread of workgroup 0 (only launches after this one read it), which saves
// the descriptor-write launch of a build.
__global__ __launch_bounds__(kThreads) void k_pyr12(Pyr12Job j, PyrDesc *ddst, PyrDesc desc)
{
    __shared__ P12Smem sm;
    if (ddst && blockIdx.x == 0 && threadIdx.x == 0) *ddst = desc;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    if (j.f16) pyr12_tile<true>(j, tile, sm);
    else pyr12_tile<false>(j, tile, sm);
}

__global__ __launch_bounds__(kThreads) void k_pyr12_batched(const Pyr12Job *jobs, const int32_t *tile_job,
                                                            const PyrDescWrite *descs, int n_descs)
{
    __shared__ P12Smem sm;
    // the device descriptors of the pyramids being built, one per workgroup of
    // the first n_descs (only launches after this one read them); this saves
    // the descriptor-write launch of a build
    if ((int)blockIdx.x < n_descs) {
        static_assert(sizeof(PyrDesc) % 4 == 0, "descriptor copied as words");
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&descs[blockIdx.x].desc);
        uint32_t *dst = reinterpret_cast<uint32_t *>(descs[blockIdx.x].dst);
        for (int i = threadIdx.x; i < (int)(sizeof(PyrDesc) / 4); i += kThreads) dst[i] = src[i];
    }
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const Pyr12Job j = jobs[uniform_i(tile_job[tile])];
    if (j.f16) pyr12_tile<true>(j, tile - j.tile_begin, sm);
    else pyr12_tile<false>(j, tile - j.tile_begin, sm);
}

// ------------------------------------------------------ binary16 gradient planes

// Staged window of a gradient tile: rows y0-1 .. y0+TH, columns from x0-16
// (16-byte aligned for both 8-bit and binary16 sources), as floats.
constexpr int kGradSW = kGradTileW + 32;

struct alignas(16) GradSmem {
    float s[kGradTileH + 2][kGradSW];
};

template <int SK>
__device__ void grad_tile(const GradJob &j, int tile, GradSmem &sm)
{
    constexpr int es = SK == K_U8 ? 1 : 2;
    constexpr int PX = 16 / es;                          // pixels per 16-byte chunk
    constexpr int NCH = kGradSW / PX;                     // chunks per staged row
    auto &s = sm.s;
    const int tx = tile % j.tiles_x, ty = tile / j.tiles_x;
    const int x0 = tx * kGradTileW, y0 = ty * kGradTileH;
    const int a0 = x0 - 16;                               // staged column 0
    const bool vec_ok = ((j.spitch * es) & 15) == 0 && (reinterpret_cast<uintptr_t>(j.src) & 15) == 0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(j.src), (short)0, j.spitch * j.h * es, kBufWord3);
    // 1. rows y0-1 .. y0+TH (reflect-101 into the level), columns a0 .. a0+SW;
    //    16-byte loads for chunks inside the level, per pixel (reflected) at its edges
    for (int i = threadIdx.x; i < (kGradTileH + 2) * NCH; i += kThreads) {
        const int r = i / NCH, c = i - r * NCH;
        const int gy = reflect101(min(y0 - 1 + r, j.h), j.h);
        const int xs = a0 + c * PX;
        float *dst = &s[r][c * PX];
        if (vec_ok && xs >= 0 && xs + PX <= j.w) {
            const uint4 v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (gy * j.spitch + xs) * es, 0, 0));
            unpack_chunk<SK>(v, dst);
        } else {
#pragma unroll
            for (int k = 0; k < PX; ++k) {
                const int gx = reflect101(clampi(xs + k, -1, j.w), j.w);
                dst[k] = ldpx<SK>(j.src, gy * j.spitch + gx);
            }
        }
    }
    __syncthreads();
    // 2. each thread: 4 consecutive pixels of one row (staged columns
    //    16 + c - 1 .. 16 + c + 4 of rows r .. r + 2)
    {
        const int r = threadIdx.x >> 4, c = (threadIdx.x & 15) * 4;
        const int x = x0 + c, y = y0 + r;
        if (y < j.h) {
            float t[3][6];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int k = 0; k < 6; ++k) t[a][k] = s[r + a][15 + c + k];
            __half2 g[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float gx = (3.0f * (t[0][k + 2] - t[0][k]) + 10.0f * (t[1][k + 2] - t[1][k])
                                  + 3.0f * (t[2][k + 2] - t[2][k])) * 0.03125f;
                const float gy = (3.0f * (t[2][k] - t[0][k]) + 10.0f * (t[2][k + 1] - t[0][k + 1])
                                  + 3.0f * (t[2][k + 2] - t[0][k + 2])) * 0.03125f;
                g[k] = __floats2half2_rn(gx, gy);
            }
            if (x + 3 < j.w) {
                uint4 u;
                u.x = __builtin_bit_cast(uint32_t, g[0]);
                u.y = __builtin_bit_cast(uint32_t, g[1]);
                u.z = __builtin_bit_cast(uint32_t, g[2]);
                u.w = __builtin_bit_cast(uint32_t, g[3]);
                *reinterpret_cast<uint4 *>(j.dst + (size_t)y * j.dpitch + x) = u;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (x + k < j.w) j.dst[(size_t)y * j.dpitch + x + k] = g[k];
            }
        }
    }
}

__device__ void grad_dispatch(const GradJob &j, int tile)
{
    __shared__ GradSmem sm;
    if (j.src_u8) grad_tile<K_U8>(j, tile, sm);
    else grad_tile<K_F16>(j, tile, sm);
}

__global__ __launch_bounds__(kThreads) void k_grad(GradJob j) { grad_dispatch(j, xcd_block(blockIdx.x, gridDim.x)); }

__global__ __launch_bounds__(kThreads) void k_grad_batched(const GradJob *jobs, const int32_t *tile_job)
{
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const GradJob j = jobs[uniform_i(tile_job[tile])];
    grad_dispatch(j, tile - j.tile_begin);
}

// =================================================================== tracker

// Buffer resource of one pyramid level: 32-bit offsets, and every access
// beyond the level's bytes returns zero instead of faulting.

struct Plane {
    __amdgpu_buffer_rsrc_t rs;
    int pitch, w, h;
};

// A pointer every lane holds the same copy of, moved to scalar registers.
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// Level descriptor read from memory, made provably wave-uniform (the
// descriptor is the same for the whole wavefront), so that buffer resources
// built from it live in scalar registers.
// Descriptors and batch tables are written before a kernel that reads them
// starts and never while it runs, at wave-uniform addresses: they are read
// through the constant address space, i.e. with scalar loads.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_constant(const T *p)
{
    return (const __attribute__((address_space(4))) T *)(uintptr_t)p;
}

__device__ __forceinline__ BatchItem load_item(const BatchItem *items, int i)
{
    const auto *q = as_constant(items) + i;
    BatchItem it;
    it.prev = q->prev;
    it.next = q->next;
    it.pt_offset = q->pt_offset;
    it.n = q->n;
    it.first_wave = q->first_wave;
    it.limit = q->limit;
    return it;
}

__device__ __forceinline__ LevelDesc uniform_level(const LevelDesc &d)
{
    const auto *q = as_constant(&d);
    LevelDesc u;
    u.img = q->img;
    u.grad = q->grad;
    u.pitch = q->pitch;
    u.gpitch = q->gpitch;
    u.w = q->w;
    u.h = q->h;
    return u;
}

template <int KIND>
__device__ __forceinline__ Plane make_plane(const void *base, int pitch, int w, int h)
{
    constexpr int es = KIND == K_U8 ? 1 : (KIND == K_F16 ? 2 : 4);
    Plane p;
    p.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, pitch * h * es, kBufWord3);
    p.pitch = pitch; p.w = w; p.h = h;
    return p;
}

template <int KIND>
__device__ __forceinline__ float bload(const Plane &p, int idx)
{
    if constexpr (KIND == K_U8) return (float)__builtin_amdgcn_raw_buffer_load_b8(p.rs, idx, 0, 0);
    else if constexpr (KIND == K_F16)
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(p.rs, idx * 2, 0, 0)));
    else return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(p.rs, idx * 4, 0, 0));
}

// One element of a plane at byte offset voff + soff (soff: a wave-uniform
// offset that the load takes from a scalar register).
template <int KIND>
__device__ __forceinline__ float bload_at(const Plane &p, int voff, int soff)
{
    if constexpr (KIND == K_U8) return (float)__builtin_amdgcn_raw_buffer_load_b8(p.rs, voff, soff, 0);
    else if constexpr (KIND == K_F16)
        return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(p.rs, voff, soff, 0)));
    else return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(p.rs, voff, soff, 0));
}

__device__ __forceinline__ float2 bload_h2(const __amdgpu_buffer_rsrc_t &rs, int idx)
{
    return __half22float2(__builtin_bit_cast(__half2, __builtin_amdgcn_raw_buffer_load_b32(rs, idx * 4, 0, 0)));
}

// Taps x and x+1 of one row of an 8-bit or binary16 plane (boff: byte offset
// of x) with one 8-byte load from the 4-byte-aligned offset at or below it,
// which holds both: one memory instruction instead of two.  The caller keeps
// the 8 bytes inside the plane (the bytes past x+1 are read and dropped).
template <int KIND>
__device__ __forceinline__ float2 bload_pair(const Plane &p, int boff, int soff)
{
    static_assert(KIND == K_U8 || KIND == K_F16, "8-bit or binary16 elements");
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(p.rs, boff & ~3, soff, 0);
    const uint32_t lo = v[0], hi = v[1];    // (copied out: see fast_template_planes)
    const uint32_t w = __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(boff & 3) * 8u);
    if constexpr (KIND == K_U8) return make_float2((float)(w & 0xFFu), (float)((w >> 8) & 0xFFu));
    else return __half22float2(__builtin_bit_cast(__half2, w));
}

// LDS writes of a wavefront become visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane layout of the window: lane (cg, sg) owns CW columns x R rows of
// window pixels starting at (c0, r0).  WMAX is the largest window of the
// layout; it fixes the staged regions.
template <int CW_, int R_, int WMAX_, int WPB_, int OCC_, bool EXACT_ = false>
struct Geo {
    static constexpr int CW = CW_, R = R_, WMAX = WMAX_, WPB = WPB_;
    // EXACT: a build for win = WMAX only, where the strips tile the window
    // exactly (every row of an active lane is valid)
    static constexpr bool EXACT = EXACT_;
    static constexpr int OCC = OCC_;                           // wavefronts per SIMD the registers must allow
    static constexpr int EXX = ((WMAX + CW - 1) / CW) * CW;   // window columns covered by lanes
    static constexpr int EXY = ((WMAX + R - 1) / R) * R;
    static constexpr int TW = EXX + 1, TH = EXY + 1;           // bilinear taps
    static constexpr int SW = TW + 2, SH = TH + 2;             // taps plus the Scharr halo
    // column walk of the gradient build: lanes are tap columns, GROUPS row
    // groups side by side, RPG tap rows each
    static constexpr int TBW = EXX + 2, TBH = EXY + 2;         // interpolated template incl. a one-pixel halo
    // LDS row stride of the interpolated template, chosen so that the lane
    // segments of a wavefront (rows r0 = 0, R, 2R) fall on disjoint banks:
    // the LDS serves a wavefront as two halves of 32 lanes over 32 banks,
    // and 7 x 35 = 21, 14 x 35 = 10 (mod 32) put the 21-lane segments of the
    // 1x7 layout on banks 0-20 and 21-31 (first half), 0-9 and 10-30 (second
    // half); 16 x 34 = 0 (mod 32) with 31-lane segments gives one segment per
    // half for the 1x16 layout
    static constexpr int TBS = CW == 1 && R == 7 ? 35 : (CW == 1 && R == 16 ? 34 : (TBW | 1));
    // first of four zero columns past the template in rows 0 .. R+1 (1x7
    // layout): with the lane segments above, the active lanes of the second
    // half leave bank 31 + 3 a free at row a, so an idle lane reading there
    // adds no conflict; -1: not used
    static constexpr int ZC = CW == 1 && R == 7 ? 31 : -1;
    static_assert(ZC < 0 || (ZC >= TBW && ZC + 4 <= TBS), "zero block inside the template rows");
    static_assert(!EXACT || (EXX == WMAX && EXY == WMAX && ZC >= 0), "exact build of a layout that tiles the window");
    static constexpr int LDS_OLD = SW * SH + 2 * TW * TH;      // staged level + two gradient planes
    static constexpr int LDS_FAST = SW * SH + TBS * TBH;       // staged level + interpolated template
    static constexpr int LDS = LDS_OLD > LDS_FAST ? LDS_OLD : LDS_FAST;   // floats per wave
    static constexpr int CPASS = (TW + 63) / 64;
    static constexpr int GROUPS = TW <= 64 ? 64 / TW : 1;
    static constexpr int RPG = (TH + GROUPS - 1) / GROUPS;
};

// Inactive lanes mirror lane 0's geometry (every address they form is
// valid) and contribute nothing.
struct LaneCfg {
    int c0, r0;
    bool active;
    bool lane0;
};

template <class G>
__device__ __forceinline__ LaneCfg lane_cfg(int win, int lane)
{
    if constexpr (G::EXACT) win = G::WMAX;
    const int ncg = (win + G::CW - 1) / G::CW, nsg = (win + G::R - 1) / G::R;
    LaneCfg c;
    c.active = lane < ncg * nsg;
    // an inactive lane takes the geometry of an active lane of its own
    // 32-lane half where there is one (same LDS addresses: no bank conflict)
    const int src = c.active ? lane : ((lane & 31) < ncg * nsg ? (lane & 31) : 0);
    const int cg = src % ncg, sg = src / ncg;
    c.c0 = cg * G::CW;
    c.r0 = sg * G::R;
    c.lane0 = lane == 0;
    return c;
}

__device__ __forceinline__ bool c_valid(const LaneCfg &c, int win, int i, int j)
{
    return c.active && (c.r0 + i < win) && (c.c0 + j < win);
}

// c_valid for layout G (in an exact build every pixel of an active lane is
// in the window)
template <class G>
__device__ __forceinline__ bool g_valid(const LaneCfg &c, int win, int i, int j)
{
    if constexpr (G::EXACT) return c.active;
    else return c_valid(c, win, i, j);
}

struct Weights {
    float w00, w10, w01, w11;
};

__device__ __forceinline__ Weights bilinear_weights(float ax, float ay)
{
    Weights w;
    w.w00 = (1.0f - ax) * (1.0f - ay);
    w.w10 = ax * (1.0f - ay);
    w.w01 = (1.0f - ax) * ay;
    w.w11 = ax * ay;
    return w;
}

// One bilinear sample from its four taps, in one fixed order of fused
// multiply-adds: template and target samples round identically, so equal
// frames give an exactly zero mismatch.
__device__ __forceinline__ float bilerp(const Weights &w, float a, float b, float c, float d)
{
    return fmaf(w.w11, d, fmaf(w.w01, c, fmaf(w.w10, b, w.w00 * a)));
}

// The one-column layouts sample in lerp form instead: along each tap row
// (left tap plus ax times the right-minus-left difference), then down the
// column.  Template and target samples take the same operations on the same
// taps, so equal frames still give an exactly zero mismatch; a row's
// interpolation serves the two samples above and below it, and the target
// taps are kept as (left, difference) pairs, so an iteration spends two
// fused multiply-adds and one subtraction per sample.
__device__ __forceinline__ float lerp_row(float ax, float left, float diff) { return fmaf(ax, diff, left); }
__device__ __forceinline__ float lerp_col(float ay, float top, float bottom) { return fmaf(ay, bottom - top, top); }

// Binary16 rounding of a float (round to nearest even), returned as float.
__device__ __forceinline__ float round_f16(float v) { return __half2float(__float2half_rn(v)); }

// Template data of level l in LDS.  E (SW x SH): the level region from
// (tx_lo, ty_lo) with a one-pixel halo around the tap positions; GX, GY
// (TW x TH): Scharr gradients at tap positions (tx_lo + 1 + tc, ty_lo + 1 +
// tr).  Entries at positions outside the level hold values that are never
// read: lanes read taps at positions clamped to the level (bilinear taps
// replicate the edges), and the gradient at a clamped position only uses the
// level with reflect-101 borders.
//
// Float levels: E is staged with coalesced loads (reflect-101 applied to the
// addresses near an edge), then each lane walks one tap column down E with a
// three-row window and writes the gradients (R16: rounded to binary16, the
// level-0 gradients of binary16 storage, which are formed here, exactly on
// the 8-bit frame, instead of stored).  Binary16 levels >= 1: the value and
// the stored gradients are read at the clamped tap positions.
template <class G, int KIND, bool PLANES, bool R16 = false>
__device__ __forceinline__ void stage_taps(const LevelDesc &L, int tx_lo, int ty_lo, int lane, float *lds)
{
    float *E = lds, *TX = lds + G::SW * G::SH, *TY = TX + G::TW * G::TH;
    const Plane P = make_plane<KIND>(L.img, L.pitch, L.w, L.h);
    // this path serves windows near a level edge only: an opaque copy of the
    // lane index keeps its per-lane index arithmetic here instead of letting
    // the compiler hoist it into every pass (registers and instructions the
    // common path would pay for)
    asm volatile("" : "+v"(lane));
    lane &= kWave - 1;
    if constexpr (!PLANES) {
        // region inside the level (the common case): no reflection needed
        const bool inside = tx_lo >= 0 && ty_lo >= 0 && tx_lo + G::SW <= L.w && ty_lo + G::SH <= L.h;
        if (inside) {
            const int base = ty_lo * L.pitch + tx_lo;
#pragma unroll
            for (int k = 0; k < (G::SW * G::SH + kWave - 1) / kWave; ++k) {
                const int idx = lane + k * kWave;
                if (idx < G::SW * G::SH) {
                    const int r = idx / G::SW, c = idx - r * G::SW;
                    E[idx] = bload<KIND>(P, base + r * L.pitch + c);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < (G::SW * G::SH + kWave - 1) / kWave; ++k) {
                const int idx = lane + k * kWave;
                if (idx < G::SW * G::SH) {
                    const int r = idx / G::SW, c = idx - r * G::SW;
                    const int y = reflect101(clampi(ty_lo + r, -1, L.h), L.h);
                    const int x = reflect101(clampi(tx_lo + c, -1, L.w), L.w);
                    E[idx] = bload<KIND>(P, y * L.pitch + x);
                }
            }
        }
        wave_lds_sync();
        const int grp = lane / G::TW < G::GROUPS ? lane / G::TW : G::GROUPS;   // GROUPS: idle lane
#pragma unroll
        for (int cp = 0; cp < G::CPASS; ++cp) {
            const int tc = cp * 64 + (G::CPASS > 1 ? lane : lane - grp * G::TW);
            const bool col_ok = grp < G::GROUPS && tc < G::TW;
            const int tcs = col_ok ? tc : 0;                      // idle lanes read a valid column
            const int tr0 = (grp < G::GROUPS ? grp : 0) * G::RPG;
            // rows tr, tr+1, tr+2 of E around tap row tr: D = right - left,
            // S = 3 left + 10 centre + 3 right
            const float *e = E + tr0 * G::SW + tcs;
            float d0 = e[2] - e[0], s0 = fmaf(3.0f, e[0] + e[2], 10.0f * e[1]);
            e += G::SW;
            float d1 = e[2] - e[0], s1 = fmaf(3.0f, e[0] + e[2], 10.0f * e[1]);
#pragma unroll
            for (int t = 0; t < G::RPG; ++t) {
                e += G::SW;
                const int tr = tr0 + t;
                const bool ok = col_ok && tr < G::TH;
                const float a = ok ? e[0] : 0.0f, b = ok ? e[1] : 0.0f, c = ok ? e[2] : 0.0f;
                const float d2 = c - a, s2 = fmaf(3.0f, a + c, 10.0f * b);
                if (ok) {
                    const float gx = (3.0f * d0 + 10.0f * d1 + 3.0f * d2) * 0.03125f, gy = (s2 - s0) * 0.03125f;
                    TX[tr * G::TW + tc] = R16 ? round_f16(gx) : gx;
                    TY[tr * G::TW + tc] = R16 ? round_f16(gy) : gy;
                }
                d0 = d1; d1 = d2; s0 = s1; s1 = s2;
            }
        }
    } else {
        const __amdgpu_buffer_rsrc_t grs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<__half2 *>(L.grad), (short)0, L.gpitch * L.h * 4, kBufWord3);
#pragma unroll
        for (int k = 0; k < (G::TW * G::TH + kWave - 1) / kWave; ++k) {
            const int idx = lane + k * kWave;
            if (idx < G::TW * G::TH) {
                const int tr = idx / G::TW, tc = idx - tr * G::TW;
                const int x = clampi(tx_lo + 1 + tc, 0, L.w - 1);
                const int y = clampi(ty_lo + 1 + tr, 0, L.h - 1);
                E[(tr + 1) * G::SW + tc + 1] = bload<KIND>(P, y * L.pitch + x);
                const float2 g = bload_h2(grs, y * L.gpitch + x);
                TX[idx] = g.x;
                TY[idx] = g.y;
            }
        }
    }
    wave_lds_sync();
}

// Template T, Gx, Gy of this lane's pixels from the tap planes, reading
// every tap at its position clamped to the level.  (cx0, cy0): level
// position of tap plane entry (0, 0).
template <class G>
__device__ __forceinline__ void lane_template(const float *lds, const LaneCfg &lc, int win, const Weights &w,
                                              float ax, float ay, int tx0, int ty0, int cx0, int cy0, int lw, int lh,
                                              float (&T)[G::R][G::CW], float (&GX)[G::R][G::CW],
                                              float (&GY)[G::R][G::CW])
{
    const float *E = lds, *TX = lds + G::SW * G::SH, *TY = TX + G::TW * G::TH;
    int cc[G::CW + 1], cr[G::R + 1], er[G::R + 1];
#pragma unroll
    for (int j = 0; j <= G::CW; ++j) cc[j] = clampi(tx0 + j, 0, lw - 1) - cx0;
#pragma unroll
    for (int i = 0; i <= G::R; ++i) {
        const int r = clampi(ty0 + i, 0, lh - 1) - cy0;
        cr[i] = r * G::TW;
        er[i] = (r + 1) * G::SW + 1;
    }
#pragma unroll
    for (int i = 0; i < G::R; ++i)
#pragma unroll
        for (int j = 0; j < G::CW; ++j) {
            const int t00 = cr[i] + cc[j], t10 = cr[i] + cc[j + 1], t01 = cr[i + 1] + cc[j], t11 = cr[i + 1] + cc[j + 1];
            const int e00 = er[i] + cc[j], e10 = er[i] + cc[j + 1], e01 = er[i + 1] + cc[j], e11 = er[i + 1] + cc[j + 1];
            const bool ok = g_valid<G>(lc, win, i, j);
            const float v = G::CW == 1 ? lerp_col(ay, lerp_row(ax, E[e00], E[e10] - E[e00]),
                                                  lerp_row(ax, E[e01], E[e11] - E[e01]))
                                       : bilerp(w, E[e00], E[e10], E[e01], E[e11]);
            const float u = bilerp(w, TX[t00], TX[t10], TX[t01], TX[t11]);
            const float q = bilerp(w, TY[t00], TY[t10], TY[t01], TY[t11]);
            T[i][j] = ok ? v : 0.0f;
            GX[i][j] = ok ? u : 0.0f;
            GY[i][j] = ok ? q : 0.0f;
        }
}

// Raw taps of the target level with this lane's first tap at (bx, by);
// indices clamped to the level (bilinear taps replicate the edges).
// `inside`: the taps of every lane lie inside the level (decided for the
// whole wavefront by the caller), so no index needs clamping.
template <class G, int KIND, bool PAIR = false>
__device__ __forceinline__ void load_taps(const Plane &P, int bx, int by, bool inside,
                                          float (&t)[G::R + 1][G::CW + 1])
{
    if (inside) {
        if constexpr (PAIR) {
            // one 8-byte load per row (bload_pair; the caller keeps the taps
            // off the level's last row); scalar row offsets only while they
            // keep the loads 4-byte aligned
            static_assert(G::CW == 1, "one window column per lane");
            constexpr int es = KIND == K_U8 ? 1 : 2;
            const int voff = (by * P.pitch + bx) * es;
            auto rows = [&](auto scalar_rows) {
                constexpr bool SR = decltype(scalar_rows)::value;
#pragma unroll
                for (int i = 0; i <= G::R; ++i) {
                    const float2 ab = bload_pair<KIND>(P, SR ? voff : voff + i * P.pitch * es,
                                                       SR ? i * P.pitch * es : 0);
                    t[i][0] = ab.x;
                    t[i][1] = ab.y;
                }
            };
            if (G::R <= 7 && ((P.pitch * es) & 3) == 0) rows(std::true_type{});
            else rows(std::false_type{});
        } else if constexpr (G::R <= 7) {
            // one vector offset for the lane's first tap; the row offsets are
            // wave-uniform and go in the scalar offset of each load (taller
            // strips keep per-row vector offsets: their scalar registers are
            // short)
            constexpr int es = KIND == K_U8 ? 1 : (KIND == K_F16 ? 2 : 4);
            const int voff = (by * P.pitch + bx) * es;
#pragma unroll
            for (int i = 0; i <= G::R; ++i)
#pragma unroll
                for (int j = 0; j <= G::CW; ++j) t[i][j] = bload_at<KIND>(P, voff + j * es, i * P.pitch * es);
        } else {
            const int base = by * P.pitch + bx;
#pragma unroll
            for (int i = 0; i <= G::R; ++i)
#pragma unroll
                for (int j = 0; j <= G::CW; ++j) t[i][j] = bload<KIND>(P, base + i * P.pitch + j);
        }
        return;
    }
    int xs[G::CW + 1];
#pragma unroll
    for (int j = 0; j <= G::CW; ++j) xs[j] = clampi(bx + j, 0, P.w - 1);
#pragma unroll
    for (int i = 0; i <= G::R; ++i) {
        const int row = clampi(by + i, 0, P.h - 1) * P.pitch;
#pragma unroll
        for (int j = 0; j <= G::CW; ++j) t[i][j] = bload<KIND>(P, row + xs[j]);
    }
}

// Target taps of a lane (load_taps); the one-column layouts keep each tap
// row as (left, right - left) for lerp_row.
template <class G, int KIND, bool PAIR = false>
__device__ __forceinline__ void load_lane_taps(const Plane &P, int bx, int by, bool inside,
                                               float (&t)[G::R + 1][G::CW + 1])
{
    load_taps<G, KIND, PAIR>(P, bx, by, inside, t);
    if constexpr (G::CW == 1)
#pragma unroll
        for (int i = 0; i <= G::R; ++i) t[i][1] = t[i][1] - t[i][0];
}

// Row group g and column c of a lane when NG groups of RW lanes lie side by
// side.  The LDS serves a wavefront as two halves of 32 lanes over 32 banks;
// an idle lane (past the groups) repeats an active lane of its own half, so
// its accesses hit the same addresses (a broadcast) and add no conflicts.
template <int RW, int NG>
__device__ __forceinline__ void group_lane(int lane, int &g, int &c)
{
    constexpr int ACT = NG * RW;
    int l = lane;
    if (lane >= ACT) l = ACT > 32 ? 32 + (lane - ACT) % (ACT - 32) : lane % ACT;
    g = l / RW;
    c = l - g * RW;
}

// The rectangle [x0, x0 + RW) x [y0, y0 + RH) of a level into wave-private
// LDS, dense with row stride RW.  Lanes are (row group, column): each load
// instruction fills rows of the rectangle, its row offset a scalar.  Lanes
// beyond the groups and rows beyond the rectangle repeat an element another
// lane writes (same address, same value), so no load is predicated and the
// loads of a lane issue back to back.  With `inside` (wave-uniform) every
// position is in the level; otherwise positions are clamped to it (bilinear
// taps replicate the edges).
template <int KIND, int RW, int RH, int DS = RW>
__device__ __forceinline__ void load_rect(const Plane &P, int x0, int y0, bool inside, int lane, float *dst)
{
    constexpr int es = KIND == K_U8 ? 1 : (KIND == K_F16 ? 2 : 4);
    constexpr int NG = RW <= 64 ? 64 / RW : 1;          // row groups side by side
    constexpr int CP = RW <= 64 ? 1 : (RW + 63) / 64;   // column passes
    constexpr int KS = (RH + NG - 1) / NG;
    constexpr bool RAGGED = KS * NG != RH;                // the last step has rows past the end
#pragma unroll
    for (int cp = 0; cp < CP; ++cp) {
        int g, c;
        if constexpr (RW <= 64) {
            group_lane<RW, NG>(lane, g, c);
        } else {
            g = 0;
            c = min(lane + 64 * cp, RW - 1);              // the last pass repeats the last column
        }
        // steps of KB rows per group, unrolled within a step (bounds the
        // registers the loads in flight take on large windows)
        constexpr int KB = KS <= 12 ? KS : 8;
        if (inside) {
            const int voff = ((y0 + g) * P.pitch + x0 + c) * es;
#pragma unroll 1
            for (int k0 = 0; k0 < KS; k0 += KB) {
                float *d = dst + (g + NG * k0) * DS + c;
                const int so = k0 * NG * P.pitch * es;
#pragma unroll
                for (int kk = 0; kk < KB; ++kk) {
                    const int k = k0 + kk;
                    if (k >= KS) break;
                    if (RAGGED && k == KS - 1) {
                        const int r = min(g + NG * k, RH - 1);
                        dst[r * DS + c] = bload_at<KIND>(P, ((y0 + r) * P.pitch + x0 + c) * es, 0);
                    } else {
                        d[kk * NG * DS] = bload_at<KIND>(P, voff, so + kk * NG * P.pitch * es);
                    }
                }
            }
        } else {
            const int xs = clampi(x0 + c, 0, P.w - 1);
#pragma unroll 1
            for (int k0 = 0; k0 < KS; k0 += KB) {
#pragma unroll
                for (int kk = 0; kk < KB; ++kk) {
                    const int k = k0 + kk;
                    if (k >= KS) break;
                    const int r = RAGGED && k == KS - 1 ? min(g + NG * k, RH - 1) : g + NG * k;
                    const int ys = clampi(y0 + r, 0, P.h - 1);
                    dst[r * DS + c] = bload_at<KIND>(P, (ys * P.pitch + xs) * es, 0);
                }
            }
        }
    }
}

// Template of a window whose staged region lies inside the level (one
// column per lane).  The level region E is staged, the template is sampled
// bilinearly once on the (win+2)^2 grid of window positions plus a one-pixel
// halo (Tb), and each lane takes T and the Scharr gradients of its strip
// from Tb.  In exact arithmetic this equals sampling the Scharr planes of
// the level bilinearly (both are linear filters with the same weights at
// every window position); only the rounding order differs.
template <class G, int KIND>
__device__ __forceinline__ void fast_template(const Plane &P, int tx_lo, int ty_lo, float ax, float ay,
                                              const LaneCfg &lc, int win, int lane, float *lds,
                                              float (&T)[G::R][G::CW], float (&GX)[G::R][G::CW],
                                              float (&GY)[G::R][G::CW])
{
    static_assert(G::CW == 1, "one window column per lane");
    constexpr int R = G::R, SW = G::SW, SH = G::SH, TBW = G::TBW, TBH = G::TBH, TBS = G::TBS;
    float *E = lds, *Tb = lds + SW * SH;
    load_rect<KIND, SW, SH>(P, tx_lo, ty_lo, true, lane, E);
    wave_lds_sync();
    {
        // lanes are Tb columns, NG groups of RPG consecutive rows side by side
        // (the last group starts RPG rows before the end, so an overlapped row
        // is computed twice from the same data and written with the same
        // bits); lanes beyond the groups repeat a lane of their half
        constexpr int NG = 64 / TBW, RPG = (TBH + NG - 1) / NG;
        int g, b;
        group_lane<TBW, NG>(lane, g, b);
        const int g0 = min(g * RPG, TBH - RPG);
        const float *e = E + g0 * SW + b;
        float *t = Tb + g0 * TBS + b;
        float h0 = lerp_row(ax, e[0], e[1] - e[0]);
        constexpr int KB = RPG <= 12 ? RPG : 8;
#pragma unroll 1
        for (int k0 = 0; k0 < RPG; k0 += KB) {
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                const int k = k0 + kk;
                if (k >= RPG) break;
                const float *q = e + (k + 1) * SW;
                const float h1 = lerp_row(ax, q[0], q[1] - q[0]);
                t[k * TBS] = lerp_col(ay, h0, h1);
                h0 = h1;
            }
        }
    }
    // In an exact build every row of an active lane is valid, and the one
    // idle lane reads the zero block, so its T, GX and GY come out zero: no
    // row needs a select
    if constexpr (G::EXACT)
        if (lane < 4 * (R + 2)) Tb[(lane >> 2) * TBS + G::ZC + (lane & 3)] = 0.0f;
    wave_lds_sync();
    // the lane's strip: rows a = 0 .. R+1 of Tb around its column, with a
    // three-row sliding window of D = right - left and S = (3 l + 10 c + 3 r) / 32
    auto strip = [&](const float *tb, auto masked) {
        constexpr bool MASKED = decltype(masked)::value;
        float d0 = 0.0f, d1 = 0.0f, s0 = 0.0f, s1 = 0.0f, c1 = 0.0f;
#pragma unroll
        for (int a = 0; a < R + 2; ++a) {
            const float l = tb[a * TBS], c = tb[a * TBS + 1], r = tb[a * TBS + 2];
            const float d2 = r - l, s2 = fmaf(0.09375f, l + r, 0.3125f * c);
            if (a >= 2) {
                const int i = a - 2;
                const bool ok = !MASKED || c_valid(lc, win, i, 0);
                T[i][0] = c1;              // invalid pixels have GX = GY = 0: they add nothing
                GX[i][0] = ok ? fmaf(0.3125f, d1, 0.09375f * (d0 + d2)) : 0.0f;
                GY[i][0] = ok ? s2 - s0 : 0.0f;
            }
            d0 = d1; d1 = d2; s0 = s1; s1 = s2; c1 = c;
        }
    };
    if constexpr (G::EXACT)
        strip(lc.active ? Tb + lc.r0 * TBS + lc.c0 : Tb + G::ZC, std::false_type{});
    else
        strip(Tb + lc.r0 * TBS + lc.c0, std::true_type{});
}

// Template of a window whose taps lie inside the level, binary16 storage
// (one column per lane): each lane loads the taps of its strip straight into
// registers -- R+1 rows of left and right taps of the stored level (8-bit at
// level 0) and of the stored (Gx, Gy) plane, one 8-byte load per row of each
// -- and samples T, Gx and Gy in the lerp form the target samples use.
// No LDS.  (bx, by): the lane's first tap; the caller keeps the taps off the
// level's last row (the level's 8-byte loads read up to 3 elements past the
// right tap, which stays inside the level's buffer on every other row).  An
// idle lane of an exact build reads beyond the buffers (zeros), so its T,
// Gx and Gy are zero.
template <class G, int KIND>
__device__ __forceinline__ void fast_template_planes(const Plane &P, const LevelDesc &L, int bx, int by, float ax,
                                                     float ay, const LaneCfg &lc, int win, float (&T)[G::R][G::CW],
                                                     float (&GX)[G::R][G::CW], float (&GY)[G::R][G::CW])
{
    static_assert(G::CW == 1, "one window column per lane");
    constexpr int R = G::R;
    constexpr int es = KIND == K_U8 ? 1 : 2;
    constexpr int kFar = 0x40000000;       // beyond every level and gradient plane
    const __amdgpu_buffer_rsrc_t grs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<__half2 *>(L.grad), (short)0, L.gpitch * L.h * 4, kBufWord3);
    const bool live = !G::EXACT || lc.active;
    const int voff = live ? (by * P.pitch + bx) * es : kFar;
    const int goff = live ? (by * L.gpitch + bx) * 4 : kFar;
    float el[R + 1], ed[R + 1], xl[R + 1], xd[R + 1], yl[R + 1], yd[R + 1];
    // row offsets in scalar registers for short strips whose row pitch keeps
    // the 8-byte loads aligned; otherwise in the vector offset (taller strips:
    // their scalar registers are short)
    auto rows = [&](auto scalar_rows) {
        constexpr bool SR = decltype(scalar_rows)::value;
#pragma unroll
        for (int i = 0; i <= R; ++i) {
            const int vi = SR ? voff : voff + i * P.pitch * es;
            const int si = SR ? i * P.pitch * es : 0;
            const int gvi = SR ? goff : goff + i * L.gpitch * 4;
            const int gsi = SR ? i * L.gpitch * 4 : 0;
            const float2 ab = bload_pair<KIND>(P, vi, si);
            const auto g = __builtin_amdgcn_raw_buffer_load_b64(grs, gvi, gsi, 0);
            // elements copied to scalars first: a bit cast of a vector element
            // itself reads element 0 whatever the index (clang codegen)
            const uint32_t g0 = g[0], g1 = g[1];
            const float2 gl = __half22float2(__builtin_bit_cast(__half2, g0));
            const float2 gr = __half22float2(__builtin_bit_cast(__half2, g1));
            el[i] = ab.x; ed[i] = ab.y - ab.x;
            xl[i] = gl.x; xd[i] = gr.x - gl.x;
            yl[i] = gl.y; yd[i] = gr.y - gl.y;
        }
    };
    if (R <= 7 && ((P.pitch * es) & 3) == 0) rows(std::true_type{});
    else rows(std::false_type{});
    float e0 = lerp_row(ax, el[0], ed[0]), x0 = lerp_row(ax, xl[0], xd[0]), y0 = lerp_row(ax, yl[0], yd[0]);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const float e1 = lerp_row(ax, el[i + 1], ed[i + 1]);
        const float x1 = lerp_row(ax, xl[i + 1], xd[i + 1]);
        const float y1 = lerp_row(ax, yl[i + 1], yd[i + 1]);
        const bool ok = g_valid<G>(lc, win, i, 0);
        T[i][0] = lerp_col(ay, e0, e1);      // invalid pixels have GX = GY = 0: they add nothing
        GX[i][0] = ok ? lerp_col(ay, x0, x1) : 0.0f;
        GY[i][0] = ok ? lerp_col(ay, y0, y1) : 0.0f;
        e0 = e1; x0 = x1; y0 = y1;
    }
}

// Template of a level-0 window whose taps lie inside the frame, binary16
// storage (one column per lane): the binary16 (Gx, Gy) of level 0 are not
// stored; each lane forms those of its taps from the 8-bit frame instead.
// Per frame row by-1 .. by+R+1 it loads the four bytes at columns bx-1 ..
// bx+2 (one 8-byte load from the 4-byte-aligned offset at or below them),
// forms the central differences and [3 10 3] sums of its two tap columns,
// and per tap row the Scharr gradients, exact on 8-bit data, then rounds
// them to binary16: the values a stored plane would hold.  T, Gx and Gy are
// sampled in the lerp form the target samples use.  (bx, by): the lane's
// first tap; the caller keeps rows by-1 .. by+R+1 and columns bx-1 .. bx+2
// inside the frame and off its last row (the 8-byte loads read up to 4
// bytes past column bx+2).  An idle lane of an exact build reads beyond the
// buffer (zeros), so its T, Gx and Gy are zero.
template <class G>
__device__ __forceinline__ void fast_template_u8_r16(const Plane &P, int bx, int by, float ax, float ay,
                                                     const LaneCfg &lc, int win, float (&T)[G::R][G::CW],
                                                     float (&GX)[G::R][G::CW], float (&GY)[G::R][G::CW])
{
    static_assert(G::CW == 1, "one window column per lane");
    constexpr int R = G::R;
    constexpr int kFar = 0x40000000;       // beyond every frame
    const bool live = !G::EXACT || lc.active;
    const int voff = live ? (by - 1) * P.pitch + bx - 1 : kFar;
    // every row's load first (one wait), then the rows in order with a
    // three-row window of differences and sums
    uint32_t lo[R + 3], hi[R + 3];
#pragma unroll
    for (int k = 0; k < R + 3; ++k) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(P.rs, (voff + k * P.pitch) & ~3, 0, 0);
        lo[k] = v[0]; hi[k] = v[1];    // (copied out: see fast_template_planes)
    }
    float dl0 = 0.0f, dr0 = 0.0f, sl0 = 0.0f, sr0 = 0.0f, dl1 = 0.0f, dr1 = 0.0f, sl1 = 0.0f, sr1 = 0.0f;
    float tl1 = 0.0f, tr1 = 0.0f, e0 = 0.0f, x0 = 0.0f, y0 = 0.0f;
#pragma unroll
    for (int k = 0; k < R + 3; ++k) {
        const uint32_t w = __builtin_amdgcn_alignbit(hi[k], lo[k], (uint32_t)((voff + k * P.pitch) & 3) * 8u);
        const float q0 = (float)(w & 0xFFu), q1 = (float)((w >> 8) & 0xFFu);
        const float q2 = (float)((w >> 16) & 0xFFu), q3 = (float)(w >> 24);
        const float dl2 = q2 - q0, dr2 = q3 - q1;
        const float sl2 = fmaf(3.0f, q0 + q2, 10.0f * q1), sr2 = fmaf(3.0f, q1 + q3, 10.0f * q2);
        if (k >= 2) {
            // tap row i = k - 2 (frame row by + i, the middle of the window)
            const int i = k - 2;
            const float gxl = round_f16(fmaf(3.0f, dl0 + dl2, 10.0f * dl1) * 0.03125f);
            const float gxr = round_f16(fmaf(3.0f, dr0 + dr2, 10.0f * dr1) * 0.03125f);
            const float gyl = round_f16((sl2 - sl0) * 0.03125f);
            const float gyr = round_f16((sr2 - sr0) * 0.03125f);
            const float e1 = lerp_row(ax, tl1, tr1 - tl1);
            const float x1 = lerp_row(ax, gxl, gxr - gxl);
            const float y1 = lerp_row(ax, gyl, gyr - gyl);
            if (i >= 1) {
                const bool ok = g_valid<G>(lc, win, i - 1, 0);
                T[i - 1][0] = lerp_col(ay, e0, e1);      // invalid pixels have GX = GY = 0: they add nothing
                GX[i - 1][0] = ok ? lerp_col(ay, x0, x1) : 0.0f;
                GY[i - 1][0] = ok ? lerp_col(ay, y0, y1) : 0.0f;
            }
            e0 = e1; x0 = x1; y0 = y1;
        }
        dl0 = dl1; dr0 = dr1; sl0 = sl1; sr0 = sr1;
        dl1 = dl2; dr1 = dr2; sl1 = sl2; sr1 = sr2;
        tl1 = q1; tr1 = q2;
    }
}

struct PassResult {
    int status;
    float ox, oy;      // end point, level-0 pixels
    float fx, fy;      // end point minus start point (level-0 flow)
    float res;         // mean |T - J| over the level-0 window
};

// The end of a pass at level 0: end point q = p + g + d (u = q - c in level
// coordinates, fu = its floor as clamped for the tap base), the mean
// |T - J(q + x)| over the window and the final in-frame check.
template <class G>
__device__ __forceinline__ void finish_level0(const LaneCfg &lc, int win, float nw, const float (&T)[G::R][G::CW],
                                              const float (&jt)[G::R + 1][G::CW + 1], float ux, float uy, float fux,
                                              float fuy, int cix, int ciy, float cfx, float cfy, const LevelDesc &LJ,
                                              PassResult &pr)
{
    pr.ox = (float)cix + ux;
    pr.oy = (float)ciy + uy;
    pr.fx = ux - cfx;
    pr.fy = uy - cfy;
    float acc = 0.0f;
    if constexpr (G::CW == 1) {
        const float ax = ux - fux, ay = uy - fuy;
        float h0 = lerp_row(ax, jt[0][0], jt[0][1]);
#pragma unroll
        for (int i = 0; i < G::R; ++i) {
            const float h1 = lerp_row(ax, jt[i + 1][0], jt[i + 1][1]);
            acc += g_valid<G>(lc, win, i, 0) ? fabsf(T[i][0] - lerp_col(ay, h0, h1)) : 0.0f;
            h0 = h1;
        }
    } else {
        const Weights w = bilinear_weights(ux - fux, uy - fuy);
#pragma unroll
        for (int i = 0; i < G::R; ++i)
#pragma unroll
            for (int j = 0; j < G::CW; ++j) {
                const float jv = bilerp(w, jt[i][j], jt[i][j + 1], jt[i + 1][j], jt[i + 1][j + 1]);
                acc += c_valid(lc, win, i, j) ? fabsf(T[i][j] - jv) : 0.0f;
            }
    }
    pr.res = uniform_f(wave_sum(acc)) / nw;
    if (!(ux >= (float)(-cix) && ux <= (float)(LJ.w - 1 - cix) && uy >= (float)(-ciy) && uy <= (float)(LJ.h - 1 - ciy)))
        pr.status = LK_LOST_OOB;
}

// One coarse-to-fine pass of pyramid I (template) into pyramid J (target).
template <int ST, class G>
__device__ PassResult run_pass(const PyrDesc &I, const PyrDesc &J, float px, float py, float gx, float gy,
                               const TrackArgs &a, const LaneCfg &lc, int lane, float *lds, int32_t *iters)
{
    constexpr int R = G::R, CW = G::CW;
    const int win = G::EXACT ? G::WMAX : a.win, h = (win - 1) >> 1, L = a.levels;
    const float nw = (float)(win * win);
    PassResult pr;
    pr.status = LK_OK;
    pr.ox = px; pr.oy = py; pr.fx = 0.0f; pr.fy = 0.0f; pr.res = 0.0f;
    const LevelDesc L0 = uniform_level(I.lv[0]);
    const int w0 = L0.w, h0 = L0.h;
    if (!(px >= 0.0f && px <= (float)(w0 - 1) && py >= 0.0f && py <= (float)(h0 - 1))) {
        pr.status = LK_LOST_OOB;
        return pr;
    }
    float T[R][CW], GX[R][CW], GY[R][CW];
    float dx = 0.0f, dy = 0.0f;
    float cfx = 0.0f, cfy = 0.0f;
    int cix = 0, ciy = 0;
    for (int l = L - 1; l >= 0; --l) {
        const LevelDesc LI = uniform_level(I.lv[l]);
        const LevelDesc LJ = uniform_level(J.lv[l]);
        const float cxs = ldexpf(px, -l), cys = ldexpf(py, -l);   // exact scaling
        const float flx = floorf(cxs), fly = floorf(cys);
        cix = uniform_i((int)flx); ciy = uniform_i((int)fly);
        cfx = cxs - flx; cfy = cys - fly;                         // exact
        // ---- template T, Gx, Gy on the window around c = p / 2^l
        {
            const int tx_lo = cix - h - 1, ty_lo = ciy - h - 1;
            wave_lds_sync();          // the previous level's reads of this LDS are done
            bool fast = false;
            if constexpr (ST == LK_STORAGE_F32 && G::CW == 1)
                fast = tx_lo >= 0 && ty_lo >= 0 && tx_lo + G::SW <= LI.w && ty_lo + G::SH <= LI.h;
            if constexpr (ST == LK_STORAGE_F16 && G::CW == 1) {
                // every lane's taps (columns cix - h .. cix - h + EXX, rows
                // likewise) inside the level and off its last row; at level 0
                // also the one-pixel ring its gradients are formed from
                if (l == 0)
                    fast = cix - h - 1 >= 0 && ciy - h - 1 >= 0 && cix - h + G::EXX + 1 < LI.w &&
                           ciy - h + G::EXY + 1 < LI.h - 1;
                else
                    fast = cix - h >= 0 && ciy - h >= 0 && cix - h + G::EXX < LI.w && ciy - h + G::EXY < LI.h - 1;
            }
            if (fast) {
                if constexpr (ST == LK_STORAGE_F16 && G::CW == 1) {
                    const int bx = cix - h + lc.c0, by = ciy - h + lc.r0;
                    if (l == 0)
                        fast_template_u8_r16<G>(make_plane<K_U8>(LI.img, LI.pitch, LI.w, LI.h), bx, by, cfx, cfy, lc,
                                                win, T, GX, GY);
                    else
                        fast_template_planes<G, K_F16>(make_plane<K_F16>(LI.img, LI.pitch, LI.w, LI.h), LI, bx, by,
                                                       cfx, cfy, lc, win, T, GX, GY);
                }
                if constexpr (ST == LK_STORAGE_F32 && G::CW == 1) {
                    if (l == 0)
                        fast_template<G, K_U8>(make_plane<K_U8>(LI.img, LI.pitch, LI.w, LI.h), tx_lo, ty_lo, cfx, cfy,
                                               lc, win, lane, lds, T, GX, GY);
                    else
                        fast_template<G, K_F32>(make_plane<K_F32>(LI.img, LI.pitch, LI.w, LI.h), tx_lo, ty_lo, cfx,
                                                cfy, lc, win, lane, lds, T, GX, GY);
                }
            } else {
                if (l == 0) stage_taps<G, K_U8, false, ST == LK_STORAGE_F16>(LI, tx_lo, ty_lo, lane, lds);
                else if constexpr (ST == LK_STORAGE_F16) stage_taps<G, K_F16, true>(LI, tx_lo, ty_lo, lane, lds);
                else stage_taps<G, K_F32, false>(LI, tx_lo, ty_lo, lane, lds);
                lane_template<G>(lds, lc, win, bilinear_weights(cfx, cfy), cfx, cfy, cix - h + lc.c0, ciy - h + lc.r0,
                                 cix - h, ciy - h, LI.w, LI.h, T, GX, GY);
            }
        }
        float sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                sxx = fmaf(GX[i][j], GX[i][j], sxx);
                sxy = fmaf(GX[i][j], GY[i][j], sxy);
                syy = fmaf(GY[i][j], GY[i][j], syy);
            }
        const float Gxx = uniform_f(wave_sum(sxx)), Gxy = uniform_f(wave_sum(sxy)), Gyy = uniform_f(wave_sum(syy));
        // Eigenvalue test: lambda_min = det / lambda_max, with the determinant
        // formed exactly in double (products of floats are exact there) and
        // lambda_max, which has no cancellation, in float.
        const double ddet = (double)Gxx * (double)Gyy - (double)Gxy * (double)Gxy;
        const float det = (float)ddet;
        {
            // lambda_min / (N_w 255^2) >= min_eig, as det >= min_eig N_w 255^2
            // lambda_max with lambda_max > 0 (a flat window, lambda_max = 0, and
            // NaN fail); the uniform scalar work runs on the vector ALU, so the
            // hardware square root (1 ulp) replaces the refined one and no
            // division is needed
            const float lmax =
                0.5f * ((Gxx + Gyy) + __builtin_amdgcn_sqrtf((Gxx - Gyy) * (Gxx - Gyy) + 4.0f * Gxy * Gxy));
            if (!(lmax > 0.0f && det >= a.min_eig * (nw * 65025.0f) * lmax)) {
                pr.status = LK_LOST_EIG;
                pr.ox = ldexpf((float)cix + (cfx + gx), l);
                pr.oy = ldexpf((float)ciy + (cfy + gy), l);
                return pr;
            }
        }
        const float rdet = __builtin_amdgcn_rcpf(det);      // 1 ulp
        const float lox = (float)(-h - cix), hix = (float)(LJ.w - 1 + h - cix);
        const float loy = (float)(-h - ciy), hiy = (float)(LJ.h - 1 + h - ciy);
        const float eps2 = a.eps * a.eps;
        const Plane PJ = l == 0 ? make_plane<K_U8>(LJ.img, LJ.pitch, LJ.w, LJ.h)
                                : (ST == LK_STORAGE_F16 ? make_plane<K_F16>(LJ.img, LJ.pitch, LJ.w, LJ.h)
                                                        : make_plane<K_F32>(LJ.img, LJ.pitch, LJ.w, LJ.h));
        // target taps of this level, whose first tap sits at (bx - h, by - h)
        float jt[R + 1][CW + 1];
        // binary16 kernels load a row's two taps with one 8-byte load (memory
        // instructions, not arithmetic, bound them), which must not start on
        // the level's last row
        constexpr bool PAIR = ST == LK_STORAGE_F16 && G::CW == 1;
        auto load_target = [&](int bx, int by) {
            const bool inside = bx - h >= 0 && by - h >= 0 && bx - h + G::EXX < PJ.w &&
                                by - h + G::EXY < PJ.h - (PAIR ? 1 : 0);
            if (l == 0) load_lane_taps<G, K_U8, PAIR>(PJ, bx - h + lc.c0, by - h + lc.r0, inside, jt);
            else if constexpr (ST == LK_STORAGE_F16)
                load_lane_taps<G, K_F16, PAIR>(PJ, bx - h + lc.c0, by - h + lc.r0, inside, jt);
            else load_lane_taps<G, K_F32>(PJ, bx - h + lc.c0, by - h + lc.r0, inside, jt);
        };
        // The taps of the first estimate are loaded before the iterations
        // (its integer part clamped to the level's range: an estimate outside
        // ends the pass before any tap is read, and the clamped loads stay in
        // the level), then again whenever the integer part moves.  Loading
        // here, rather than at the first iteration, also keeps the previous
        // level's taps from flowing into this level (which costs a register
        // copy of every tap per level).
        int jbx = uniform_i(cix + (int)fminf(fmaxf(floorf(cfx + gx), lox), hix));
        int jby = uniform_i(ciy + (int)fminf(fmaxf(floorf(cfy + gy), loy), hiy));
        load_target(jbx, jby);
        // The cell [fbx, fbx + 1) x [fby, fby + 1) of the loaded taps (level
        // coordinates relative to c, exact small integers).  While an estimate
        // stays in it, its integer part is the loaded one, and when the cell
        // lies inside the in-bounds box the estimate is in bounds: four
        // compares stand in for the bounds test, the floors, the conversions
        // and the base comparison (the clamped first base holds no estimate
        // outside the box, so the first iteration takes the full test then).
        float fbx = (float)(jbx - cix), fby = (float)(jby - ciy);
        float fbx1 = fbx + 1.0f, fby1 = fby + 1.0f;
        bool cell_in = fbx1 <= hix && fby1 <= hiy;         // fbx >= lox, fby >= loy by the clamp
        dx = 0.0f; dy = 0.0f;
        int k = 0;
        bool oob = false;
        while (k < a.max_iters) {
            ++k;
            const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
            if (!(cell_in && ux >= fbx && ux < fbx1 && uy >= fby && uy < fby1)) {
                if (!(ux >= lox && ux <= hix && uy >= loy && uy <= hiy)) {
                    oob = true;          // the window left the level before this step
                    break;
                }
                const float fux = floorf(ux), fuy = floorf(uy);
                const int bx = uniform_i(cix + (int)fux), by = uniform_i(ciy + (int)fuy);
                if (bx != jbx || by != jby) {
                    load_target(bx, by);
                    jbx = bx; jby = by;
                }
                fbx = fux; fby = fuy;
                fbx1 = fbx + 1.0f; fby1 = fby + 1.0f;
                cell_in = fbx >= lox && fbx1 <= hix && fby >= loy && fby1 <= hiy;
            }
            float bxs = 0.0f, bys = 0.0f;
            if constexpr (CW == 1) {
                const float ax = ux - fbx, ay = uy - fby;
                float h0 = lerp_row(ax, jt[0][0], jt[0][1]);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    const float h1 = lerp_row(ax, jt[i + 1][0], jt[i + 1][1]);
                    const float e = T[i][0] - lerp_col(ay, h0, h1);
                    bxs = fmaf(e, GX[i][0], bxs);
                    bys = fmaf(e, GY[i][0], bys);
                    h0 = h1;
                }
            } else {
                const Weights w = bilinear_weights(ux - fbx, uy - fby);
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < CW; ++j) {
                        const float e = T[i][j] - bilerp(w, jt[i][j], jt[i][j + 1], jt[i + 1][j], jt[i + 1][j + 1]);
                        bxs = fmaf(e, GX[i][j], bxs);
                        bys = fmaf(e, GY[i][j], bys);
                    }
            }
            const float bx_ = uniform_f(wave_sum(bxs)), by_ = uniform_f(wave_sum(bys));
            const float ex = (Gyy * bx_ - Gxy * by_) * rdet;
            const float ey = (Gxx * by_ - Gxy * bx_) * rdet;
            dx += ex;
            dy += ey;
            if (ex * ex + ey * ey < eps2) break;
        }
        if (oob) {
            const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
            pr.status = LK_LOST_OOB;
            pr.ox = ldexpf((float)cix + ux, l);
            pr.oy = ldexpf((float)ciy + uy, l);
            if (iters && lc.lane0) iters[l] = k - 1;
            return pr;
        }
        if (iters && lc.lane0) iters[l] = k;
        if (l > 0) {
            gx = 2.0f * (gx + dx);
            gy = 2.0f * (gy + dy);
            continue;
        }
        if constexpr (G::R <= 7 && ST == LK_STORAGE_F32) {
            // level 0 of the 1x7 float32 kernel: the end point and the residual here,
            // where the last iteration's taps serve unless the tap base moved
            // (the other layouts and storages keep fewer registers live by
            // reloading after the loop)
            const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
            const float fux = fminf(fmaxf(floorf(ux), (float)(-cix - h - 2)), (float)(LJ.w + h + 2 - cix));
            const float fuy = fminf(fmaxf(floorf(uy), (float)(-ciy - h - 2)), (float)(LJ.h + h + 2 - ciy));
            const int bx = uniform_i(cix + (int)fux), by = uniform_i(ciy + (int)fuy);
            if (bx != jbx || by != jby) load_target(bx, by);
            finish_level0<G>(lc, win, nw, T, jt, ux, uy, fux, fuy, cix, ciy, cfx, cfy, LJ, pr);
        }
    }
    if constexpr (!(G::R <= 7 && ST == LK_STORAGE_F32)) {
        const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
        const LevelDesc LJ = uniform_level(J.lv[0]);
        const Plane PJ = make_plane<K_U8>(LJ.img, LJ.pitch, LJ.w, LJ.h);
        const float fux = fminf(fmaxf(floorf(ux), (float)(-cix - h - 2)), (float)(LJ.w + h + 2 - cix));
        const float fuy = fminf(fmaxf(floorf(uy), (float)(-ciy - h - 2)), (float)(LJ.h + h + 2 - ciy));
        const int bx = uniform_i(cix + (int)fux), by = uniform_i(ciy + (int)fuy);
        const bool inside = bx - h >= 0 && by - h >= 0 && bx - h + G::EXX < PJ.w && by - h + G::EXY < PJ.h;
        float jt[R + 1][CW + 1];
        load_lane_taps<G, K_U8>(PJ, bx - h + lc.c0, by - h + lc.r0, inside, jt);
        finish_level0<G>(lc, win, nw, T, jt, ux, uy, fux, fuy, cix, ciy, cfx, cfy, LJ, pr);
    }
    return pr;
}

template <int ST, class G>
__device__ void track_point(const PyrDesc &prev, const PyrDesc &next, const TrackArgs &a, int idx, int lane,
                            float *lds)
{
    const LaneCfg lc = lane_cfg<G>(a.win, lane);
    const int L = a.levels;
    const float px = uniform_f(a.pts[2 * idx]), py = uniform_f(a.pts[2 * idx + 1]);
    float gx = 0.0f, gy = 0.0f;
    if (a.use_guess) {
        gx = ldexpf(uniform_f(a.guess[2 * idx]) - px, -(L - 1));
        gy = ldexpf(uniform_f(a.guess[2 * idx + 1]) - py, -(L - 1));
    }
    int32_t *itp = a.iters ? a.iters + (size_t)idx * 2 * L : nullptr;
    if (itp && lc.lane0)
        for (int l = 0; l < 2 * L; ++l) itp[l] = 0;
    // the one-column layouts inline both passes (their LDS accesses stay
    // local-data-share instructions); the wide layout is left to the compiler
    PassResult f, b;
    if constexpr (G::CW == 1) {
        [[clang::always_inline]] f = run_pass<ST, G>(prev, next, px, py, gx, gy, a, lc, lane, lds, itp);
    } else {
        f = run_pass<ST, G>(prev, next, px, py, gx, gy, a, lc, lane, lds, itp);
    }
    int status = f.status;
    if (status == LK_OK && a.fb_thresh > 0.0f) {
        int32_t *itb = itp ? itp + L : nullptr;
        if constexpr (G::CW == 1) {
            [[clang::always_inline]] b = run_pass<ST, G>(next, prev, f.ox, f.oy, 0.0f, 0.0f, a, lc, lane, lds, itb);
        } else {
            b = run_pass<ST, G>(next, prev, f.ox, f.oy, 0.0f, 0.0f, a, lc, lane, lds, itb);
        }
        if (b.status != LK_OK) {
            status = LK_LOST_FB;
        } else {
            // p' - p = (q - p) + backward flow; q - p is exact for nearby floats
            const float vx = (f.ox - px) + b.fx, vy = (f.oy - py) + b.fy;
            if (sqrtf(vx * vx + vy * vy) > a.fb_thresh) status = LK_LOST_FB;
        }
    }
    if (lane == 0) {
        a.out_pts[2 * idx] = f.ox;
        a.out_pts[2 * idx + 1] = f.oy;
        a.status[idx] = (uint8_t)status;
        a.residual[idx] = f.res;
    }
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
// XCD works on one contiguous range of points (and of frames), which keeps
// the pyramids it reads in its own L2.

template <int ST, class G>
__global__ __launch_bounds__(G::WPB * 64) __attribute__((amdgpu_waves_per_eu(G::OCC)))
void k_track(const PyrDesc *prev, const PyrDesc *next, TrackArgs a)
{
    __shared__ float s_lds[G::WPB * G::LDS];
    const int wib = threadIdx.x >> 6;
    const int wave = uniform_i(xcd_block(blockIdx.x, gridDim.x) * G::WPB + wib);
    if (wave >= a.n) return;
    if constexpr (G::CW == 1) {
        [[clang::always_inline]] track_point<ST, G>(*prev, *next, a, wave, threadIdx.x & (kWave - 1), s_lds + wib * G::LDS);
    } else {
        track_point<ST, G>(*prev, *next, a, wave, threadIdx.x & (kWave - 1), s_lds + wib * G::LDS);
    }
}

template <int ST, class G>
__global__ __launch_bounds__(G::WPB * 64) __attribute__((amdgpu_waves_per_eu(G::OCC)))
void k_track_batched(const BatchItem *items, int n_items, TrackArgs a)
{
    __shared__ float s_lds[G::WPB * G::LDS];
    const int wib = threadIdx.x >> 6;
    const int wave = uniform_i(xcd_block(blockIdx.x, gridDim.x) * G::WPB + wib);
    if (wave >= a.n) return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (as_constant(items)[mid].first_wave <= wave) lo = mid; else hi = mid - 1;
    }
    lo = uniform_i(lo);
    const BatchItem it = load_item(items, lo);
    if (it.limit && wave - it.first_wave >= *as_constant(it.limit)) return;   // past the item's live count
    const int idx = (int)(it.pt_offset + (wave - it.first_wave));
    if constexpr (G::CW == 1) {
        [[clang::always_inline]] track_point<ST, G>(*it.prev, *it.next, a, idx, threadIdx.x & (kWave - 1), s_lds + wib * G::LDS);
    } else {
        track_point<ST, G>(*it.prev, *it.next, a, idx, threadIdx.x & (kWave - 1), s_lds + wib * G::LDS);
    }
}

// Persistent form: a fixed grid whose wavefronts take chunks of `chunk`
// consecutive keypoints from work counters, one per XCD, each in a 256-byte
// slot of its own (XCD x first drains keypoints [x n/8, (x+1) n/8), then
// helps the others).  Every wavefront leaves after one failed fetch per
// counter, so the grid always drains.  The counters are zeroed by
// k_reset_counters before each launch.
template <int ST, class G>
__global__ __launch_bounds__(G::WPB * 64) __attribute__((amdgpu_waves_per_eu(G::OCC)))
void k_track_persist(const BatchItem *items, int n_items, TrackArgs a, int *counters, int chunk)
{
    __shared__ float s_lds[G::WPB * G::LDS];
    const int wib = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int xcd = blockIdx.x & 7;
    for (int probe = 0; probe < 8; ++probe) {
        const int owner = (xcd + probe) & 7;
        const int first = (int)((long)a.n * owner / 8), end = (int)((long)a.n * (owner + 1) / 8);
        for (;;) {
            // every lane takes part in the fetch (lane 0 adds the chunk, the
            // others 0) so the index is never defined in a divergent branch;
            // lane 0's old value starts this wavefront's chunk
            const int w = __builtin_amdgcn_readfirstlane(
                atomicAdd(&counters[owner * kCounterStride], lane == 0 ? chunk : 0));
            const int w0 = first + w;
            if (w0 >= end) break;
            const int w1 = min(w0 + chunk, end);
            int lo = 0;
            for (int wave = w0; wave < w1; ++wave) {
                // items are ordered by first_wave: continue the search from
                // the previous keypoint's item
                int hi = n_items - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (as_constant(items)[mid].first_wave <= wave) lo = mid; else hi = mid - 1;
                }
                lo = uniform_i(lo);
                const BatchItem it = load_item(items, lo);
                if (it.limit && wave - it.first_wave >= *as_constant(it.limit)) continue;
                const int idx = (int)(it.pt_offset + (wave - it.first_wave));
                if constexpr (G::CW == 1) {
                    [[clang::always_inline]] track_point<ST, G>(*it.prev, *it.next, a, idx, lane,
                                                                s_lds + wib * G::LDS);
                } else {
                    track_point<ST, G>(*it.prev, *it.next, a, idx, lane, s_lds + wib * G::LDS);
                }
            }
        }
    }
}

__global__ void k_reset_counters(int *c)
{
    if (threadIdx.x < 8) c[threadIdx.x * kCounterStride] = 0;
}

// Layouts: (CW, R) = (1, 7) for windows up to 21, (1, 16) up to 31; each
// keeps ceil(win/CW) * ceil(win/R) <= 64 lanes.
// The 21x21 layouts run one wavefront per workgroup: keypoints take different
// numbers of iterations, and a workgroup's LDS is released only when its last
// wavefront ends, so larger workgroups hold idle LDS (measured on the 64-stream
// step: 0.224 ms with 1 wavefront per workgroup, 0.230 with 2, 0.233 with 4,
// 0.243 with 8).
using GeoW21 = Geo<1, 7, 21, 1, 4>;
using GeoW21X = Geo<1, 7, 21, 1, 6, true>;     // win = 21 exactly: 80 registers, 6 wavefronts per SIMD
using GeoW21X2 = Geo<1, 7, 21, 2, 6, true>;    // the same, 2 and 4 wavefronts per workgroup (tuner shapes)
using GeoW21X4 = Geo<1, 7, 21, 4, 6, true>;
using GeoW21XP = Geo<1, 7, 21, 1, 5, true>;    // persistent grid (its loop needs more registers than 6 waves allow)
using GeoW31 = Geo<1, 16, 31, 4, 2>;

// Copies pyramid descriptors into device memory, in stream order.
__global__ void k_write_desc(PyrDesc *dst, PyrDesc src) { if (threadIdx.x == 0) *dst = src; }

__global__ void k_write_descs(const PyrDescWrite *w, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *w[i].dst = w[i].desc;
}

// One level (and its gradient plane) as float, for diagnostics; kind: the
// element type of the level (level 0 is 8-bit).
// grad_u8: the binary16 gradients of an 8-bit level (binary16 storage, level
// 0, which has no stored plane), formed as the tracker forms them.
__global__ __launch_bounds__(kThreads) void k_read_level(LevelDesc lv, int kind, int grad_u8, float *dst,
                                                         float *dgrad)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= lv.w * lv.h) return;
    const int y = i / lv.w, x = i - y * lv.w;
    dst[i] = kind == K_U8    ? ldpx<K_U8>(lv.img, y * lv.pitch + x)
             : kind == K_F16 ? ldpx<K_F16>(lv.img, y * lv.pitch + x)
                             : ldpx<K_F32>(lv.img, y * lv.pitch + x);
    if (dgrad && grad_u8) {
        // Scharr on the frame with reflect-101 borders, exact, then rounded
        auto px = [&](int yy, int xx) {
            return ldpx<K_U8>(lv.img, reflect101(yy, lv.h) * lv.pitch + reflect101(xx, lv.w));
        };
        const float dA = px(y - 1, x + 1) - px(y - 1, x - 1), dB = px(y, x + 1) - px(y, x - 1);
        const float dC = px(y + 1, x + 1) - px(y + 1, x - 1);
        const float sA = fmaf(3.0f, px(y - 1, x - 1) + px(y - 1, x + 1), 10.0f * px(y - 1, x));
        const float sC = fmaf(3.0f, px(y + 1, x - 1) + px(y + 1, x + 1), 10.0f * px(y + 1, x));
        dgrad[2 * i] = round_f16(fmaf(3.0f, dA + dC, 10.0f * dB) * 0.03125f);
        dgrad[2 * i + 1] = round_f16((sC - sA) * 0.03125f);
    } else if (dgrad && lv.grad) {
        const float2 g = __half22float2(lv.grad[y * lv.gpitch + x]);
        dgrad[2 * i] = g.x;
        dgrad[2 * i + 1] = g.y;
    }
}

template <class G>
inline unsigned blocks_for(long waves) { return (unsigned)((waves + G::WPB - 1) / G::WPB); }

template <int ST, class G>
hipError_t launch_track_g(const PyrDesc *prev, const PyrDesc *next, const TrackArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_track<ST, G>), dim3(blocks_for<G>(a.n)), dim3(G::WPB * 64), 0, s, prev, next, a);
    return hipGetLastError();
}

template <int ST>
hipError_t launch_track_st(const PyrDesc *prev, const PyrDesc *next, const TrackArgs &a, hipStream_t s)
{
    switch (choose_layout(a.win)) {
    case LAYOUT_W21:
        return a.win == GeoW21X::WMAX ? launch_track_g<ST, GeoW21X>(prev, next, a, s)
                                      : launch_track_g<ST, GeoW21>(prev, next, a, s);
    case LAYOUT_W31: return launch_track_g<ST, GeoW31>(prev, next, a, s);
    default: return hipErrorInvalidValue;      // no layout for this window
    }
}

template <int ST, class G>
hipError_t launch_track_batched_g(const BatchItem *items, int n_items, const TrackArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_track_batched<ST, G>), dim3(blocks_for<G>(a.n)), dim3(G::WPB * 64), 0, s, items, n_items, a);
    return hipGetLastError();
}

template <int ST>
hipError_t launch_track_batched_st(const BatchItem *items, int n_items, const TrackArgs &a, hipStream_t s, int wpg)
{
    switch (choose_layout(a.win)) {
    case LAYOUT_W21:
        if (a.win != GeoW21X::WMAX) return wpg <= 1 ? launch_track_batched_g<ST, GeoW21>(items, n_items, a, s)
                                                     : hipErrorInvalidValue;
        if (wpg == 2) return launch_track_batched_g<ST, GeoW21X2>(items, n_items, a, s);
        if (wpg == 4) return launch_track_batched_g<ST, GeoW21X4>(items, n_items, a, s);
        return wpg <= 1 ? launch_track_batched_g<ST, GeoW21X>(items, n_items, a, s) : hipErrorInvalidValue;
    case LAYOUT_W31:
        return wpg == 0 || wpg == GeoW31::WPB ? launch_track_batched_g<ST, GeoW31>(items, n_items, a, s)
                                               : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Window side -> lane layout: (CW, R) = (1, 7) up to 21, (1, 16) up to 31;
// LAYOUT_NONE above (the host rejects such windows before any launch).
int choose_layout(int win)
{
    if (win <= 21) return LAYOUT_W21;
    if (win <= LK_MAX_WIN) return LAYOUT_W31;
    return LAYOUT_NONE;
}

// Wavefronts per workgroup a batched tracker launch can take for `win`
// (0: the layout's default): 1, 2 or 4 for the exact 21 x 21 build.
bool track_waves_supported(int win, int wpg)
{
    if (wpg == 0) return choose_layout(win) != LAYOUT_NONE;
    if (win == GeoW21X::WMAX) return wpg == 1 || wpg == 2 || wpg == 4;
    if (choose_layout(win) == LAYOUT_W21) return wpg == 1;
    if (choose_layout(win) == LAYOUT_W31) return wpg == GeoW31::WPB;
    return false;
}

hipError_t launch_downsample(const DownJob &job, hipStream_t stream)
{
    const int tiles = job.tiles_x * ((job.dh + kDownTileH - 1) / kDownTileH);
    hipLaunchKernelGGL(k_downsample, dim3(tiles), dim3(kThreads), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_downsample_batched(const DownJob *d_jobs, const int32_t *d_tile_job, int total_tiles,
                                     hipStream_t stream)
{
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_downsample_batched, dim3(total_tiles), dim3(kThreads), 0, stream, d_jobs, d_tile_job);
    return hipGetLastError();
}

hipError_t launch_pyr12(const Pyr12Job &job, PyrDesc *ddst, const PyrDesc &desc, hipStream_t stream)
{
    const int tiles = job.tiles_x * ((job.h2 + kP12TileH - 1) / kP12TileH);
    hipLaunchKernelGGL(k_pyr12, dim3(tiles), dim3(kThreads), 0, stream, job, ddst, desc);
    return hipGetLastError();
}

hipError_t launch_pyr12_batched(const Pyr12Job *d_jobs, const int32_t *d_tile_job, int total_tiles,
                                const PyrDescWrite *d_descs, int n_descs, hipStream_t stream)
{
    if (total_tiles <= 0) return hipSuccess;
    if (n_descs > total_tiles) return hipErrorInvalidValue;      // one descriptor per workgroup at most
    hipLaunchKernelGGL(k_pyr12_batched, dim3(total_tiles), dim3(kThreads), 0, stream, d_jobs, d_tile_job, d_descs,
                       n_descs);
    return hipGetLastError();
}

hipError_t launch_grad(const GradJob &job, hipStream_t stream)
{
    const int tiles = job.tiles_x * ((job.h + kGradTileH - 1) / kGradTileH);
    hipLaunchKernelGGL(k_grad, dim3(tiles), dim3(kThreads), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_grad_batched(const GradJob *d_jobs, const int32_t *d_tile_job, int total_tiles,
                               hipStream_t stream)
{
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_batched, dim3(total_tiles), dim3(kThreads), 0, stream, d_jobs, d_tile_job);
    return hipGetLastError();
}

hipError_t launch_track(const PyrDesc *prev, const PyrDesc *next, int storage, const TrackArgs &a,
                        hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    return storage == LK_STORAGE_F16 ? launch_track_st<LK_STORAGE_F16>(prev, next, a, stream)
                                     : launch_track_st<LK_STORAGE_F32>(prev, next, a, stream);
}

hipError_t launch_write_desc(PyrDesc *dst, const PyrDesc &src, hipStream_t stream)
{
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, stream, dst, src);
    return hipGetLastError();
}

hipError_t launch_write_descs(const PyrDescWrite *d_w, int n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_write_descs, dim3((n + 63) / 64), dim3(64), 0, stream, d_w, n);
    return hipGetLastError();
}

template <int ST, class G>
hipError_t launch_track_persist_g(const BatchItem *items, int n_items, const TrackArgs &a, int *counters,
                                  int grid, int chunk, hipStream_t s)
{
    const int need = (a.n + G::WPB - 1) / G::WPB;
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters);
    hipLaunchKernelGGL((k_track_persist<ST, G>), dim3(grid < need ? grid : need), dim3(G::WPB * 64), 0, s, items,
                       n_items, a, counters, chunk);
    return hipGetLastError();
}

template <int ST>
hipError_t launch_track_persist_st(const BatchItem *items, int n_items, const TrackArgs &a, int *counters,
                                   int blocks_per_cu, int num_cus, int chunk, hipStream_t s)
{
    const int grid = blocks_per_cu * num_cus;
    switch (choose_layout(a.win)) {
    case LAYOUT_W21:
        return a.win == GeoW21X::WMAX
                   ? launch_track_persist_g<ST, GeoW21XP>(items, n_items, a, counters, grid, chunk, s)
                   : launch_track_persist_g<ST, GeoW21>(items, n_items, a, counters, grid, chunk, s);
    case LAYOUT_W31:
        return launch_track_persist_g<ST, GeoW31>(items, n_items, a, counters, grid, chunk, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_track_persistent(const BatchItem *d_items, int n_items, int total_points, const TrackArgs &a,
                                   int storage, int *d_counters, int blocks_per_cu, int num_cus, int chunk,
                                   hipStream_t stream)
{
    if (total_points <= 0) return hipSuccess;
    if (chunk < 1) return hipErrorInvalidValue;
    TrackArgs b = a;
    b.n = total_points;
    return storage == LK_STORAGE_F16
               ? launch_track_persist_st<LK_STORAGE_F16>(d_items, n_items, b, d_counters, blocks_per_cu, num_cus,
                                                         chunk, stream)
               : launch_track_persist_st<LK_STORAGE_F32>(d_items, n_items, b, d_counters, blocks_per_cu, num_cus,
                                                         chunk, stream);
}

hipError_t launch_track_batched(const BatchItem *d_items, int n_items, int total_points, const TrackArgs &a,
                                int storage, hipStream_t stream, int waves_per_group)
{
    if (total_points <= 0) return hipSuccess;
    TrackArgs b = a;
    b.n = total_points;
    return storage == LK_STORAGE_F16
               ? launch_track_batched_st<LK_STORAGE_F16>(d_items, n_items, b, stream, waves_per_group)
               : launch_track_batched_st<LK_STORAGE_F32>(d_items, n_items, b, stream, waves_per_group);
}

hipError_t launch_read_level(const LevelDesc &lv, int level, int storage, float *dst, float *dgrad,
                             hipStream_t stream)
{
    const int kind = level == 0 ? K_U8 : (storage == LK_STORAGE_F16 ? K_F16 : K_F32);
    const long n = (long)lv.w * lv.h;
    const int grad_u8 = level == 0 && storage == LK_STORAGE_F16;
    hipLaunchKernelGGL(k_read_level, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, stream,
                       lv, kind, grad_u8, dst, dgrad);
    return hipGetLastError();
}

}  // namespace lkmi
