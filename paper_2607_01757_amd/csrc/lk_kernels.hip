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
// raw taps of the target frame in registers and only reloads them when the
// integer part of the estimate moves.  Sums over the window (the 2x2 normal
// matrix and the mismatch vector) are reduced with DPP row operations, one
// swizzle and two lane reads, in a fixed order: every lane obtains the same
// bits, control flow stays wave-uniform, and a point's result does not depend
// on what else is in the launch.  No MFMA: nothing here is a dense
// contraction.
#include "lk_internal.h"

#include <climits>

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

// Sum over the 64 lanes of a wavefront.  Every lane returns the same value:
// each step adds a lane's value to its partner's with the operands swapped,
// and float addition is commutative.
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x141>(v);   // row_half_mirror: quad <-> quad within 8 lanes
    v += dpp_move<0x140>(v);   // row_mirror: half-row <-> half-row within 16 lanes
    v += __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));  // lane ^ 16
    float lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    return lo + hi;
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

constexpr int kInW = 2 * kDownTileW + 3;   // input tile columns incl. halo
constexpr int kInH = 2 * kDownTileH + 3;

struct DownSmem {
    float in[kInH][kInW + 1];
    float h[kInH][kDownTileW + 1];
};

template <int SK, bool F16>
__device__ void downsample_tile(const DownJob &j, int tile, DownSmem &sm)
{
    auto &s_in = sm.in;
    auto &s_h = sm.h;
    const int tx = tile % j.tiles_x, ty = tile / j.tiles_x;
    const int ox0 = tx * kDownTileW, oy0 = ty * kDownTileH;
    const int sx0 = 2 * ox0 - 2, sy0 = 2 * oy0 - 2;
    for (int i = threadIdx.x; i < kInH * kInW; i += kThreads) {
        const int r = i / kInW, c = i - r * kInW;
        const int gy = reflect101(min(sy0 + r, j.sh + 1), j.sh);
        const int gx = reflect101(min(sx0 + c, j.sw + 1), j.sw);
        s_in[r][c] = ldpx<SK>(j.src, gy * j.spitch + gx);
    }
    __syncthreads();
    // horizontal [1 4 6 4 1] at even columns; exact for short dyadic values
    for (int i = threadIdx.x; i < kInH * kDownTileW; i += kThreads) {
        const int r = i / kDownTileW, c = i - r * kDownTileW;
        const float *q = &s_in[r][2 * c];
        s_h[r][c] = ((q[0] + q[4]) + 4.0f * (q[1] + q[3]) + 6.0f * q[2]) * 0.0625f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kDownTileH * kDownTileW; i += kThreads) {
        const int r = i / kDownTileW, c = i - r * kDownTileW;
        const int ox = ox0 + c, oy = oy0 + r;
        if (ox < j.dw && oy < j.dh) {
            const float v = ((s_h[2 * r][c] + s_h[2 * r + 4][c]) + 4.0f * (s_h[2 * r + 1][c] + s_h[2 * r + 3][c])
                             + 6.0f * s_h[2 * r + 2][c]) * 0.0625f;
            if constexpr (F16) static_cast<__half *>(j.dst)[oy * j.dpitch + ox] = __float2half_rn(v);
            else static_cast<float *>(j.dst)[oy * j.dpitch + ox] = v;
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

__global__ __launch_bounds__(kThreads) void k_downsample(DownJob j) { downsample_dispatch(j, blockIdx.x); }

__device__ __forceinline__ int find_job_u(const int32_t *first_tile_of, int stride_bytes, int n, int tile)
{
    // last job whose tile_begin <= tile (jobs are sorted by tile_begin)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int tb = *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(first_tile_of)
                                                           + (size_t)mid * stride_bytes);
        if (tb <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_downsample_batched(const DownJob *jobs, int njobs)
{
    const int tile = blockIdx.x;
    const int jid = uniform_i(find_job_u(&jobs[0].tile_begin, sizeof(DownJob), njobs, tile));
    const DownJob j = jobs[jid];
    downsample_dispatch(j, tile - j.tile_begin);
}

// ------------------------------------------------------ binary16 gradient planes

struct GradSmem {
    float s[kGradTileH + 2][kGradTileW + 3];
};

template <int SK>
__device__ void grad_tile(const GradJob &j, int tile, GradSmem &sm)
{
    auto &s = sm.s;
    const int tx = tile % j.tiles_x, ty = tile / j.tiles_x;
    const int x0 = tx * kGradTileW, y0 = ty * kGradTileH;
    for (int i = threadIdx.x; i < (kGradTileH + 2) * (kGradTileW + 2); i += kThreads) {
        const int r = i / (kGradTileW + 2), c = i - r * (kGradTileW + 2);
        const int gy = reflect101(min(y0 - 1 + r, j.h), j.h);
        const int gx = reflect101(min(x0 - 1 + c, j.w), j.w);
        s[r][c] = ldpx<SK>(j.src, gy * j.spitch + gx);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kGradTileH * kGradTileW; i += kThreads) {
        const int r = i / kGradTileW, c = i - r * kGradTileW;
        const int x = x0 + c, y = y0 + r;
        if (x < j.w && y < j.h) {
            const float gx = (3.0f * (s[r][c + 2] - s[r][c]) + 10.0f * (s[r + 1][c + 2] - s[r + 1][c])
                              + 3.0f * (s[r + 2][c + 2] - s[r + 2][c])) * 0.03125f;
            const float gy = (3.0f * (s[r + 2][c] - s[r][c]) + 10.0f * (s[r + 2][c + 1] - s[r][c + 1])
                              + 3.0f * (s[r + 2][c + 2] - s[r][c + 2])) * 0.03125f;
            j.dst[y * j.dpitch + x] = __floats2half2_rn(gx, gy);
        }
    }
}

__device__ void grad_dispatch(const GradJob &j, int tile)
{
    __shared__ GradSmem sm;
    if (j.src_u8) grad_tile<K_U8>(j, tile, sm);
    else grad_tile<K_F16>(j, tile, sm);
}

__global__ __launch_bounds__(kThreads) void k_grad(GradJob j) { grad_dispatch(j, blockIdx.x); }

__global__ __launch_bounds__(kThreads) void k_grad_batched(const GradJob *jobs, int njobs)
{
    const int tile = blockIdx.x;
    const int jid = uniform_i(find_job_u(&jobs[0].tile_begin, sizeof(GradJob), njobs, tile));
    const GradJob j = jobs[jid];
    grad_dispatch(j, tile - j.tile_begin);
}

// =================================================================== tracker

// Where a lane sits in the window.  Inactive lanes mirror lane 0's geometry
// (so every address they form is valid) and contribute nothing.
struct LaneCfg {
    int c0, r0;          // first window column / row of this lane
    int ext_x, ext_y;    // columns / rows spanned by all lanes' pixels
    bool active;
    bool lane0;          // writes per-point diagnostics
};

template <int CW, int R>
__device__ __forceinline__ LaneCfg lane_cfg(int win, int lane)
{
    const int ncg = (win + CW - 1) / CW, nsg = (win + R - 1) / R;
    LaneCfg c;
    c.active = lane < ncg * nsg;
    const int cg = c.active ? lane % ncg : 0, sg = c.active ? lane / ncg : 0;
    c.c0 = cg * CW;
    c.r0 = sg * R;
    c.ext_x = ncg * CW;
    c.ext_y = nsg * R;
    c.lane0 = lane == 0;
    return c;
}

__device__ __forceinline__ bool c_valid(const LaneCfg &c, int win, int i, int j)
{
    return c.active && (c.r0 + i < win) && (c.c0 + j < win);
}

// Raw taps of the target level around integer base (bx, by) = this lane's
// first tap; indices clamped to the level (bilinear taps replicate edges).
template <int KIND, int CW, int R>
__device__ __forceinline__ void load_taps(const LevelDesc &L, int bx, int by, float (&t)[R + 1][CW + 1])
{
    int xs[CW + 1];
#pragma unroll
    for (int j = 0; j <= CW; ++j) xs[j] = clampi(bx + j, 0, L.w - 1);
#pragma unroll
    for (int i = 0; i <= R; ++i) {
        const int row = clampi(by + i, 0, L.h - 1) * L.pitch;
#pragma unroll
        for (int j = 0; j <= CW; ++j) t[i][j] = ldpx<KIND>(L.img, row + xs[j]);
    }
}

template <int CW, int R>
__device__ __forceinline__ void load_taps_any(const LevelDesc &L, int level, int storage, int bx, int by,
                                              float (&t)[R + 1][CW + 1])
{
    if (level == 0) load_taps<K_U8, CW, R>(L, bx, by, t);
    else if (storage == LK_STORAGE_F16) load_taps<K_F16, CW, R>(L, bx, by, t);
    else load_taps<K_F32, CW, R>(L, bx, by, t);
}

// Template of this lane: T, Gx, Gy at its window pixels, bilinear with the
// shared weights w from the taps at positions (tx0 + j, ty0 + i), i <= R,
// j <= CW.  Taps are clamped to the level; the Scharr stencil of a tap is
// reflected about the level edges (reflect-101).  Tap rows are produced one
// at a time and folded into the pixel rows they feed, which keeps few
// registers live.

template <int KIND, int CW>
__device__ __forceinline__ void tap_row_scharr(const LevelDesc &L, int tx0, int y, bool interior,
                                               float (&v)[CW + 1], float (&gx)[CW + 1], float (&gy)[CW + 1])
{
    if (interior) {
        float e0[CW + 3], e1[CW + 3], e2[CW + 3];
        const int r0 = (y - 1) * L.pitch + tx0 - 1, r1 = r0 + L.pitch, r2 = r1 + L.pitch;
#pragma unroll
        for (int k = 0; k < CW + 3; ++k) {
            e0[k] = ldpx<KIND>(L.img, r0 + k);
            e1[k] = ldpx<KIND>(L.img, r1 + k);
            e2[k] = ldpx<KIND>(L.img, r2 + k);
        }
#pragma unroll
        for (int j = 0; j <= CW; ++j) {
            v[j] = e1[j + 1];
            gx[j] = (3.0f * (e0[j + 2] - e0[j]) + 10.0f * (e1[j + 2] - e1[j]) + 3.0f * (e2[j + 2] - e2[j])) * 0.03125f;
            gy[j] = (3.0f * (e2[j] - e0[j]) + 10.0f * (e2[j + 1] - e0[j + 1]) + 3.0f * (e2[j + 2] - e0[j + 2])) * 0.03125f;
        }
    } else {
        const int yc = clampi(y, 0, L.h - 1);
        const int ym = reflect101(yc - 1, L.h) * L.pitch, yp = reflect101(yc + 1, L.h) * L.pitch;
        const int yr = yc * L.pitch;
#pragma unroll
        for (int j = 0; j <= CW; ++j) {
            const int x = clampi(tx0 + j, 0, L.w - 1);
            const int xm = reflect101(x - 1, L.w), xp = reflect101(x + 1, L.w);
            const float a00 = ldpx<KIND>(L.img, ym + xm), a01 = ldpx<KIND>(L.img, ym + x), a02 = ldpx<KIND>(L.img, ym + xp);
            const float a10 = ldpx<KIND>(L.img, yr + xm), a11 = ldpx<KIND>(L.img, yr + x), a12 = ldpx<KIND>(L.img, yr + xp);
            const float a20 = ldpx<KIND>(L.img, yp + xm), a21 = ldpx<KIND>(L.img, yp + x), a22 = ldpx<KIND>(L.img, yp + xp);
            v[j] = a11;
            gx[j] = (3.0f * (a02 - a00) + 10.0f * (a12 - a10) + 3.0f * (a22 - a20)) * 0.03125f;
            gy[j] = (3.0f * (a20 - a00) + 10.0f * (a21 - a01) + 3.0f * (a22 - a02)) * 0.03125f;
        }
    }
}

template <int KIND, int CW>
__device__ __forceinline__ void tap_row_planes(const LevelDesc &L, int tx0, int y, float (&v)[CW + 1],
                                               float (&gx)[CW + 1], float (&gy)[CW + 1])
{
    const int yc = clampi(y, 0, L.h - 1);
#pragma unroll
    for (int j = 0; j <= CW; ++j) {
        const int x = clampi(tx0 + j, 0, L.w - 1);
        v[j] = ldpx<KIND>(L.img, yc * L.pitch + x);
        const float2 g = __half22float2(L.grad[yc * L.gpitch + x]);
        gx[j] = g.x;
        gy[j] = g.y;
    }
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

// PLANES: read stored gradient planes instead of computing Scharr.
template <int KIND, bool PLANES, int CW, int R>
__device__ __forceinline__ void build_template(const LevelDesc &L, int tx0, int ty0, bool interior, const Weights &w,
                                               const LaneCfg &lc, int win, float (&T)[R][CW], float (&GX)[R][CW],
                                               float (&GY)[R][CW])
{
    float pv[CW + 1], pgx[CW + 1], pgy[CW + 1];   // previous tap row
#pragma unroll
    for (int i = 0; i <= R; ++i) {
        float v[CW + 1], gx[CW + 1], gy[CW + 1];
        if constexpr (PLANES) tap_row_planes<KIND, CW>(L, tx0, ty0 + i, v, gx, gy);
        else tap_row_scharr<KIND, CW>(L, tx0, ty0 + i, interior, v, gx, gy);
        if (i > 0) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const bool ok = c_valid(lc, win, i - 1, j);
                const float t = bilerp(w, pv[j], pv[j + 1], v[j], v[j + 1]);
                const float u = bilerp(w, pgx[j], pgx[j + 1], gx[j], gx[j + 1]);
                const float q = bilerp(w, pgy[j], pgy[j + 1], gy[j], gy[j + 1]);
                T[i - 1][j] = ok ? t : 0.0f;
                GX[i - 1][j] = ok ? u : 0.0f;
                GY[i - 1][j] = ok ? q : 0.0f;
            }
        }
#pragma unroll
        for (int j = 0; j <= CW; ++j) { pv[j] = v[j]; pgx[j] = gx[j]; pgy[j] = gy[j]; }
    }
}

struct PassResult {
    int status;
    float ox, oy;      // end point, level-0 pixels
    float fx, fy;      // end point minus start point (level-0 flow)
    float res;         // mean |T - J| over the level-0 window
};

// One coarse-to-fine pass of pyramid I (template) into pyramid J (target).
template <int ST, int CW, int R>
__device__ PassResult run_pass(const PyrDesc &I, const PyrDesc &J, float px, float py, float gx, float gy,
                               const TrackArgs &a, const LaneCfg &lc, int32_t *iters)
{
    const int win = a.win, h = (win - 1) >> 1, L = a.levels;
    const float nw = (float)(win * win);
    PassResult pr;
    pr.status = LK_OK;
    pr.ox = px; pr.oy = py; pr.fx = 0.0f; pr.fy = 0.0f; pr.res = 0.0f;
    if (!(px >= 0.0f && px <= (float)(I.lv[0].w - 1) && py >= 0.0f && py <= (float)(I.lv[0].h - 1))) {
        pr.status = LK_LOST_OOB;
        return pr;
    }
    float T[R][CW], GX[R][CW], GY[R][CW];
    float jt[R + 1][CW + 1];
    float dx = 0.0f, dy = 0.0f;
    float cfx = 0.0f, cfy = 0.0f;
    int cix = 0, ciy = 0;
    for (int l = L - 1; l >= 0; --l) {
        const LevelDesc &LI = I.lv[l];
        const LevelDesc &LJ = J.lv[l];
        const float cxs = ldexpf(px, -l), cys = ldexpf(py, -l);   // exact scaling
        const float flx = floorf(cxs), fly = floorf(cys);
        cix = (int)flx; ciy = (int)fly;
        cfx = cxs - flx; cfy = cys - fly;                         // exact
        // ---- template T, Gx, Gy on the window around c = p / 2^l
        {
            const int tx0 = cix - h + lc.c0, ty0 = ciy - h + lc.r0;
            const Weights w = bilinear_weights(cfx, cfy);
            const bool interior = (cix - h - 1 >= 0) && (cix - h + lc.ext_x + 1 <= LI.w - 1)
                                  && (ciy - h - 1 >= 0) && (ciy - h + lc.ext_y + 1 <= LI.h - 1);
            if constexpr (ST == LK_STORAGE_F16) {
                if (l == 0) build_template<K_U8, true, CW, R>(LI, tx0, ty0, interior, w, lc, win, T, GX, GY);
                else build_template<K_F16, true, CW, R>(LI, tx0, ty0, interior, w, lc, win, T, GX, GY);
            } else {
                if (l == 0) build_template<K_U8, false, CW, R>(LI, tx0, ty0, interior, w, lc, win, T, GX, GY);
                else build_template<K_F32, false, CW, R>(LI, tx0, ty0, interior, w, lc, win, T, GX, GY);
            }
        }
        float sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                sxx += GX[i][j] * GX[i][j];
                sxy += GX[i][j] * GY[i][j];
                syy += GY[i][j] * GY[i][j];
            }
        const float Gxx = uniform_f(wave_sum(sxx)), Gxy = uniform_f(wave_sum(sxy)), Gyy = uniform_f(wave_sum(syy));
        // eigenvalue test in double from the float sums (no cancellation from squaring)
        {
            const double dxx = Gxx, dxy = Gxy, dyy = Gyy;
            const double lam = 0.5 * (dxx + dyy - sqrt((dxx - dyy) * (dxx - dyy) + 4.0 * dxy * dxy));
            const double meig = lam / ((double)nw * 65025.0);
            if (!(meig >= (double)a.min_eig)) {
                pr.status = LK_LOST_EIG;
                pr.ox = ldexpf((float)cix + (cfx + gx), l);
                pr.oy = ldexpf((float)ciy + (cfy + gy), l);
                return pr;
            }
        }
        const float det = Gxx * Gyy - Gxy * Gxy;
        const float lox = (float)(-h - cix), hix = (float)(LJ.w - 1 + h - cix);
        const float loy = (float)(-h - ciy), hiy = (float)(LJ.h - 1 + h - ciy);
        const float eps2 = a.eps * a.eps;
        int jbx = INT_MIN, jby = INT_MIN;
        dx = 0.0f; dy = 0.0f;
        int k = 0;
        while (k < a.max_iters) {
            ++k;
            const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
            if (!(ux >= lox && ux <= hix && uy >= loy && uy <= hiy)) {
                pr.status = LK_LOST_OOB;
                pr.ox = ldexpf((float)cix + ux, l);
                pr.oy = ldexpf((float)ciy + uy, l);
                if (iters && lc.lane0) iters[l] = k - 1;
                return pr;
            }
            const float fux = floorf(ux), fuy = floorf(uy);
            const int bx = cix + (int)fux, by = ciy + (int)fuy;
            if (bx != jbx || by != jby) {
                load_taps_any<CW, R>(LJ, l, ST, bx - h + lc.c0, by - h + lc.r0, jt);
                jbx = bx; jby = by;
            }
            const Weights w = bilinear_weights(ux - fux, uy - fuy);
            float bxs = 0.0f, bys = 0.0f;
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < CW; ++j) {
                    const float jv = bilerp(w, jt[i][j], jt[i][j + 1], jt[i + 1][j], jt[i + 1][j + 1]);
                    const float e = T[i][j] - jv;
                    bxs += e * GX[i][j];
                    bys += e * GY[i][j];
                }
            const float bx_ = uniform_f(wave_sum(bxs)), by_ = uniform_f(wave_sum(bys));
            const float ex = (Gyy * bx_ - Gxy * by_) / det;
            const float ey = (Gxx * by_ - Gxy * bx_) / det;
            dx += ex;
            dy += ey;
            if (ex * ex + ey * ey < eps2) break;
        }
        if (iters && lc.lane0) iters[l] = k;
        if (l > 0) {
            gx = 2.0f * (gx + dx);
            gy = 2.0f * (gy + dy);
        }
    }
    // level 0: c = p; end point q = p + g + d
    const float ux = (cfx + gx) + dx, uy = (cfy + gy) + dy;
    pr.ox = (float)cix + ux;
    pr.oy = (float)ciy + uy;
    pr.fx = ux - cfx;
    pr.fy = uy - cfy;
    {
        const LevelDesc &LJ = J.lv[0];
        // the last update is not range-checked: keep the tap base finite and
        // near the frame before converting (taps are clamped anyway)
        const float fux = fminf(fmaxf(floorf(ux), (float)(-cix - h - 2)), (float)(LJ.w + h + 2 - cix));
        const float fuy = fminf(fmaxf(floorf(uy), (float)(-ciy - h - 2)), (float)(LJ.h + h + 2 - ciy));
        load_taps<K_U8, CW, R>(LJ, cix + (int)fux - h + lc.c0, ciy + (int)fuy - h + lc.r0, jt);
        const Weights w = bilinear_weights(ux - fux, uy - fuy);
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const float jv = bilerp(w, jt[i][j], jt[i][j + 1], jt[i + 1][j], jt[i + 1][j + 1]);
                acc += c_valid(lc, win, i, j) ? fabsf(T[i][j] - jv) : 0.0f;
            }
        pr.res = uniform_f(wave_sum(acc)) / nw;
        if (!(ux >= (float)(-cix) && ux <= (float)(LJ.w - 1 - cix) && uy >= (float)(-ciy)
              && uy <= (float)(LJ.h - 1 - ciy)))
            pr.status = LK_LOST_OOB;
    }
    return pr;
}

template <int ST, int CW, int R>
__device__ void track_point(const PyrDesc &prev, const PyrDesc &next, const TrackArgs &a, int idx, int lane)
{
    const LaneCfg lc = lane_cfg<CW, R>(a.win, lane);
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
    PassResult f = run_pass<ST, CW, R>(prev, next, px, py, gx, gy, a, lc, itp);
    int status = f.status;
    if (status == LK_OK && a.fb_thresh > 0.0f) {
        PassResult b = run_pass<ST, CW, R>(next, prev, f.ox, f.oy, 0.0f, 0.0f, a, lc, itp ? itp + L : nullptr);
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

template <int ST, int CW, int R>
__global__ __launch_bounds__(kThreads) void k_track(const PyrDesc *prev, const PyrDesc *next, TrackArgs a)
{
    const int wave = uniform_i((int)((blockIdx.x * kThreads + threadIdx.x) / kWave));
    if (wave >= a.n) return;
    track_point<ST, CW, R>(*prev, *next, a, wave, threadIdx.x & (kWave - 1));
}

template <int ST, int CW, int R>
__global__ __launch_bounds__(kThreads) void k_track_batched(const BatchItem *items, int n_items, TrackArgs a)
{
    const int wave = uniform_i((int)((blockIdx.x * kThreads + threadIdx.x) / kWave));
    if (wave >= a.n) return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_wave <= wave) lo = mid; else hi = mid - 1;
    }
    lo = uniform_i(lo);
    const BatchItem &it = items[lo];
    const int idx = (int)(it.pt_offset + (wave - it.first_wave));
    track_point<ST, CW, R>(*it.prev, *it.next, a, idx, threadIdx.x & (kWave - 1));
}

// Copies pyramid descriptors into device memory, in stream order.
__global__ void k_write_desc(PyrDesc *dst, PyrDesc src) { if (threadIdx.x == 0) *dst = src; }

__global__ void k_write_descs(const PyrDescWrite *w, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *w[i].dst = w[i].desc;
}

// Level l >= 1 (and its gradient plane) as float, for diagnostics.
__global__ __launch_bounds__(kThreads) void k_read_level(LevelDesc lv, int storage, float *dst, float *dgrad)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= lv.w * lv.h) return;
    const int y = i / lv.w, x = i - y * lv.w;
    dst[i] = storage == LK_STORAGE_F16 ? ldpx<K_F16>(lv.img, y * lv.pitch + x) : ldpx<K_F32>(lv.img, y * lv.pitch + x);
    if (dgrad && lv.grad) {
        const float2 g = __half22float2(lv.grad[y * lv.gpitch + x]);
        dgrad[2 * i] = g.x;
        dgrad[2 * i + 1] = g.y;
    }
}

inline unsigned blocks_for(long waves) { return (unsigned)((waves * kWave + kThreads - 1) / kThreads); }

template <int ST>
hipError_t launch_track_st(const PyrDesc *prev, const PyrDesc *next, const TrackArgs &a, hipStream_t s)
{
    const unsigned grid = blocks_for(a.n);
    switch (choose_layout(a.win)) {
    case LAYOUT_W21: hipLaunchKernelGGL((k_track<ST, 1, 7>), dim3(grid), dim3(kThreads), 0, s, prev, next, a); break;
    case LAYOUT_W31: hipLaunchKernelGGL((k_track<ST, 1, 16>), dim3(grid), dim3(kThreads), 0, s, prev, next, a); break;
    default: hipLaunchKernelGGL((k_track<ST, 4, 16>), dim3(grid), dim3(kThreads), 0, s, prev, next, a); break;
    }
    return hipGetLastError();
}

template <int ST>
hipError_t launch_track_batched_st(const BatchItem *items, int n_items, const TrackArgs &a, hipStream_t s)
{
    const unsigned grid = blocks_for(a.n);
    switch (choose_layout(a.win)) {
    case LAYOUT_W21: hipLaunchKernelGGL((k_track_batched<ST, 1, 7>), dim3(grid), dim3(kThreads), 0, s, items, n_items, a); break;
    case LAYOUT_W31: hipLaunchKernelGGL((k_track_batched<ST, 1, 16>), dim3(grid), dim3(kThreads), 0, s, items, n_items, a); break;
    default: hipLaunchKernelGGL((k_track_batched<ST, 4, 16>), dim3(grid), dim3(kThreads), 0, s, items, n_items, a); break;
    }
    return hipGetLastError();
}

}  // namespace

// Window side -> lane layout: (CW, R) = (1, 7) up to 21, (1, 16) up to 31,
// (4, 16) up to 63; each keeps ceil(win/CW) * ceil(win/R) <= 64 lanes.
int choose_layout(int win)
{
    if (win <= 21) return LAYOUT_W21;
    if (win <= 31) return LAYOUT_W31;
    return LAYOUT_W63;
}

hipError_t launch_downsample(const DownJob &job, hipStream_t stream)
{
    const int tiles = job.tiles_x * ((job.dh + kDownTileH - 1) / kDownTileH);
    hipLaunchKernelGGL(k_downsample, dim3(tiles), dim3(kThreads), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_downsample_batched(const DownJob *d_jobs, int njobs, int total_tiles, hipStream_t stream)
{
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_downsample_batched, dim3(total_tiles), dim3(kThreads), 0, stream, d_jobs, njobs);
    return hipGetLastError();
}

hipError_t launch_grad(const GradJob &job, hipStream_t stream)
{
    const int tiles = job.tiles_x * ((job.h + kGradTileH - 1) / kGradTileH);
    hipLaunchKernelGGL(k_grad, dim3(tiles), dim3(kThreads), 0, stream, job);
    return hipGetLastError();
}

hipError_t launch_grad_batched(const GradJob *d_jobs, int njobs, int total_tiles, hipStream_t stream)
{
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_batched, dim3(total_tiles), dim3(kThreads), 0, stream, d_jobs, njobs);
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

hipError_t launch_track_batched(const BatchItem *d_items, int n_items, int total_points, const TrackArgs &a,
                                int storage, hipStream_t stream)
{
    if (total_points <= 0) return hipSuccess;
    TrackArgs b = a;
    b.n = total_points;
    return storage == LK_STORAGE_F16 ? launch_track_batched_st<LK_STORAGE_F16>(d_items, n_items, b, stream)
                                     : launch_track_batched_st<LK_STORAGE_F32>(d_items, n_items, b, stream);
}

hipError_t launch_read_level(const LevelDesc &lv, int storage, float *dst, float *dgrad, hipStream_t stream)
{
    const long n = (long)lv.w * lv.h;
    hipLaunchKernelGGL(k_read_level, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, stream,
                       lv, storage, dst, dgrad);
    return hipGetLastError();
}

}  // namespace lkmi
