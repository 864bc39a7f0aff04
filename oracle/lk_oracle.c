/*
 * lk_oracle.c -- plain FP64 reference of pyramidal Lucas-Kanade tracking.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library.  The product library never
 * links, loads or calls it, and the two share no code, header or table.
 *
 * What is computed.  The paper tracks keypoints frame to frame and from the
 * left to the right camera with pyramidal LK optical flow (Sec. III, inherited
 * from VINS-Fusion; Sec. IV lists it as the LK baseline; Sec. V-A uses the
 * cross-camera flow as a stereo gate) but defines none of its internals.  The
 * definition written out here is the classical one: Lucas and Kanade's
 * template registration in Bouguet's pyramidal form (template gradients, a
 * 2x2 normal matrix fixed per level, additive updates, coarse-to-fine flow
 * propagation), a binomial Gaussian pyramid, Scharr derivatives and the
 * forward-backward check of Kalal et al.  All arithmetic is double; there is
 * no blocking, fusion or reordering beyond the plain definition.
 *
 * Conventions (each a reading of a point the paper leaves open):
 *   - pixel centres at integers, (0,0) the top-left pixel, x right, y down;
 *     level l coordinates are level-0 coordinates times 2^-l exactly;
 *   - pyramid: separable [1 4 6 4 1]/16 blur with reflect-101 borders, then
 *     every second sample; level sizes (n+1)/2; no rounding of levels unless
 *     binary16 storage is requested (then every stored level >= 1 and every
 *     gradient plane is rounded to nearest-even binary16 and the next level
 *     is built from the stored one);
 *   - gradients: Scharr [3 10 3] x [-1 0 1] / 32 on the level grid,
 *     reflect-101 borders;
 *   - bilinear sampling with floor() base, taps clamped to the image;
 *   - status: OK, LOST_EIG (normalised minimum eigenvalue of the 2x2 normal
 *     matrix below min_eig, checked at every level), LOST_OOB (window left the
 *     level, or the final point left the image), LOST_FB.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define LKO_MAX_LEVELS 8

enum { LKO_OK = 0, LKO_LOST_EIG = 1, LKO_LOST_OOB = 2, LKO_LOST_FB = 3 };

typedef struct {
    int32_t win;          /* odd window side, 3..63 */
    int32_t levels;       /* 1..8 */
    int32_t max_iters;    /* per level, >= 1 */
    int32_t use_guess;    /* 0/1 */
    int32_t f16_storage;  /* 0/1: round stored levels >= 1 and gradients to binary16 */
    int32_t nthreads;     /* worker threads over keypoints, >= 1 */
    double eps;           /* stop when |eta| < eps (level px) */
    double min_eig;       /* LOST_EIG threshold on lambda_min / (win^2 * 255^2) */
    double fb_thresh;     /* > 0 enables the forward-backward check (level-0 px) */
} lko_params;

/* ---------------------------------------------------------------- basics */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* reflect-101: -1 -> 1, -2 -> 2, n -> n-2, n+1 -> n-3 (single reflection) */
static int reflect101(int i, int n)
{
    if (n == 1) return 0;
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

int lko_level_dims(int w, int h, int levels, int32_t *ws, int32_t *hs)
{
    if (levels < 1 || levels > LKO_MAX_LEVELS || w < 1 || h < 1) return -1;
    ws[0] = w; hs[0] = h;
    for (int l = 1; l < levels; ++l) {
        ws[l] = (ws[l - 1] + 1) / 2;
        hs[l] = (hs[l - 1] + 1) / 2;
    }
    return (ws[levels - 1] >= 4 && hs[levels - 1] >= 4) ? 0 : -1;
}

/* Round to the nearest binary16 value, ties to even, returned as a double.
 * Values whose magnitude rounds past the largest finite half become inf. */
double lko_round_f16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                     /* |x| = m 2^e, m in [0.5, 1) */
    int lead = e - 1;                 /* exponent of the leading bit */
    if (lead < -14) lead = -14;       /* subnormal range: fixed quantum 2^-24 */
    double q = ldexp(1.0, lead - 10);
    double r = nearbyint(x / q) * q;  /* default rounding mode: half to even */
    if (fabs(r) > 65504.0) return copysign(INFINITY, x);
    return r;
}

/* One pyramid step: blur with [1 4 6 4 1]/16 both ways (reflect-101), keep
 * even samples.  dst is ((sw+1)/2) x ((sh+1)/2). */
void lko_downsample(const double *src, int sw, int sh, double *dst)
{
    static const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    int dw = (sw + 1) / 2, dh = (sh + 1) / 2;
    for (int y = 0; y < dh; ++y)
        for (int x = 0; x < dw; ++x) {
            double acc = 0.0;
            for (int j = 0; j < 5; ++j) {
                int sy = reflect101(2 * y + j - 2, sh);
                for (int i = 0; i < 5; ++i) {
                    int sx = reflect101(2 * x + i - 2, sw);
                    acc += k[j] * k[i] * src[(size_t)sy * sw + sx];
                }
            }
            dst[(size_t)y * dw + x] = acc;
        }
}

/* Scharr derivatives divided by 32, reflect-101 borders. */
void lko_scharr(const double *src, int w, int h, double *gx, double *gy)
{
    for (int y = 0; y < h; ++y) {
        int ym = reflect101(y - 1, h), yp = reflect101(y + 1, h);
        for (int x = 0; x < w; ++x) {
            int xm = reflect101(x - 1, w), xp = reflect101(x + 1, w);
#define P(yy, xx) src[(size_t)(yy) * w + (xx)]
            gx[(size_t)y * w + x] = (3.0 * (P(ym, xp) - P(ym, xm)) + 10.0 * (P(y, xp) - P(y, xm))
                                     + 3.0 * (P(yp, xp) - P(yp, xm))) / 32.0;
            gy[(size_t)y * w + x] = (3.0 * (P(yp, xm) - P(ym, xm)) + 10.0 * (P(yp, x) - P(ym, x))
                                     + 3.0 * (P(yp, xp) - P(ym, xp))) / 32.0;
#undef P
        }
    }
}

/* Bilinear sample at (u, v): floor base, taps clamped to the image. */
double lko_sample(const double *img, int w, int h, double u, double v)
{
    double fu = floor(u), fv = floor(v);
    double a = u - fu, b = v - fv;
    int x0 = (int)fu, y0 = (int)fv;
    int xa = clampi(x0, 0, w - 1), xb = clampi(x0 + 1, 0, w - 1);
    int ya = clampi(y0, 0, h - 1), yb = clampi(y0 + 1, 0, h - 1);
    return (1.0 - a) * (1.0 - b) * img[(size_t)ya * w + xa] + a * (1.0 - b) * img[(size_t)ya * w + xb]
         + (1.0 - a) * b * img[(size_t)yb * w + xa] + a * b * img[(size_t)yb * w + xb];
}

/* ---------------------------------------------------------------- pyramid */

typedef struct {
    int L;
    int w[LKO_MAX_LEVELS], h[LKO_MAX_LEVELS];
    double *img[LKO_MAX_LEVELS], *gx[LKO_MAX_LEVELS], *gy[LKO_MAX_LEVELS];
} pyr_t;

static void pyr_free(pyr_t *P)
{
    for (int l = 0; l < P->L; ++l) { free(P->img[l]); free(P->gx[l]); free(P->gy[l]); }
    P->L = 0;
}

static int pyr_build(pyr_t *P, const double *level0, int w, int h, int L, int f16)
{
    int32_t ws[LKO_MAX_LEVELS], hs[LKO_MAX_LEVELS];
    memset(P, 0, sizeof *P);
    if (lko_level_dims(w, h, L, ws, hs) != 0) return -1;
    P->L = L;
    for (int l = 0; l < L; ++l) {
        size_t n = (size_t)ws[l] * hs[l];
        P->w[l] = ws[l]; P->h[l] = hs[l];
        P->img[l] = malloc(n * sizeof(double));
        P->gx[l] = malloc(n * sizeof(double));
        P->gy[l] = malloc(n * sizeof(double));
        if (!P->img[l] || !P->gx[l] || !P->gy[l]) { pyr_free(P); return -2; }
        if (l == 0) memcpy(P->img[0], level0, n * sizeof(double));
        else {
            lko_downsample(P->img[l - 1], ws[l - 1], hs[l - 1], P->img[l]);
            if (f16) for (size_t i = 0; i < n; ++i) P->img[l][i] = lko_round_f16(P->img[l][i]);
        }
        lko_scharr(P->img[l], ws[l], hs[l], P->gx[l], P->gy[l]);
        if (f16)
            for (size_t i = 0; i < n; ++i) {
                P->gx[l][i] = lko_round_f16(P->gx[l][i]);
                P->gy[l][i] = lko_round_f16(P->gy[l][i]);
            }
    }
    return 0;
}

/* Levels (and optionally gradients) of one image, concatenated level-major,
 * each level compact (row length = level width). */
int lko_build_pyramid(const double *level0, int w, int h, int L, int f16,
                      double *out_img, double *out_gx, double *out_gy)
{
    pyr_t P;
    int rc = pyr_build(&P, level0, w, h, L, f16);
    if (rc) return rc;
    size_t off = 0;
    for (int l = 0; l < L; ++l) {
        size_t n = (size_t)P.w[l] * P.h[l];
        if (out_img) memcpy(out_img + off, P.img[l], n * sizeof(double));
        if (out_gx) memcpy(out_gx + off, P.gx[l], n * sizeof(double));
        if (out_gy) memcpy(out_gy + off, P.gy[l], n * sizeof(double));
        off += n;
    }
    pyr_free(&P);
    return 0;
}

/* ---------------------------------------------------------------- tracker */

typedef struct { double eig, oob, conv, fb; } margins_t;

typedef struct {
    double *T, *Gx, *Gy;   /* win*win template and its gradients */
} scratch_t;

/* Distance of (x, y) inside the box [lo, hx] x [lo, hy]; negative (or NaN)
 * outside.  The box is closed. */
static double box_dist(double x, double y, double lo, double hx, double hy)
{
    double d = x - lo;
    if (hx - x < d) d = hx - x;
    if (y - lo < d) d = y - lo;
    if (hy - y < d) d = hy - y;
    return d;
}

/* One coarse-to-fine pass from template pyramid I to target pyramid J.
 * (px, py): level-0 point in I.  (g0x, g0y): initial flow at level L-1.
 * Returns the status; writes the level-0 end point and residual. */
static int track_pass(const pyr_t *I, const pyr_t *J, double px, double py,
                      double g0x, double g0y, const lko_params *prm, scratch_t *s,
                      double *ox, double *oy, double *res, int32_t *iters, margins_t *m)
{
    const int L = prm->levels, win = prm->win, h = (win - 1) / 2, nw = win * win;
    double gx = g0x, gy = g0y, dx = 0.0, dy = 0.0;
    *ox = px; *oy = py; *res = 0.0;
    {
        double d0 = box_dist(px, py, 0.0, I->w[0] - 1.0, I->h[0] - 1.0);
        if (!(d0 >= 0.0)) return LKO_LOST_OOB;
    }
    for (int l = L - 1; l >= 0; --l) {
        const int W = I->w[l], H = I->h[l];
        const double sc = ldexp(1.0, -l);
        const double cx = px * sc, cy = py * sc;
        double Gxx = 0.0, Gxy = 0.0, Gyy = 0.0;
        for (int i = 0; i < win; ++i)
            for (int j = 0; j < win; ++j) {
                double u = cx + (j - h), v = cy + (i - h);
                double t = lko_sample(I->img[l], W, H, u, v);
                double ax = lko_sample(I->gx[l], W, H, u, v);
                double ay = lko_sample(I->gy[l], W, H, u, v);
                s->T[i * win + j] = t; s->Gx[i * win + j] = ax; s->Gy[i * win + j] = ay;
                Gxx += ax * ax; Gxy += ax * ay; Gyy += ay * ay;
            }
        dx = 0.0; dy = 0.0;
        double lam = 0.5 * (Gxx + Gyy - sqrt((Gxx - Gyy) * (Gxx - Gyy) + 4.0 * Gxy * Gxy));
        double meig = lam / ((double)nw * 255.0 * 255.0);
        double me = fabs(meig / prm->min_eig - 1.0);
        if (me < m->eig) m->eig = me;
        if (meig < prm->min_eig) {
            *ox = px + (gx + dx) / sc; *oy = py + (gy + dy) / sc;
            return LKO_LOST_EIG;
        }
        double det = Gxx * Gyy - Gxy * Gxy;
        for (int k = 1; k <= prm->max_iters; ++k) {
            double qx = cx + gx + dx, qy = cy + gy + dy;
            double bd = box_dist(qx, qy, -h, W - 1.0 + h, H - 1.0 + h);
            if (fabs(bd) < m->oob) m->oob = fabs(bd);
            if (!(bd >= 0.0)) {
                *ox = qx / sc; *oy = qy / sc;
                return LKO_LOST_OOB;
            }
            double bx = 0.0, by = 0.0;
            for (int i = 0; i < win; ++i)
                for (int j = 0; j < win; ++j) {
                    double e = s->T[i * win + j]
                             - lko_sample(J->img[l], W, H, qx + (j - h), qy + (i - h));
                    bx += e * s->Gx[i * win + j];
                    by += e * s->Gy[i * win + j];
                }
            double ex = (Gyy * bx - Gxy * by) / det;
            double ey = (Gxx * by - Gxy * bx) / det;
            dx += ex; dy += ey;
            if (iters) iters[l] = k;
            double nrm = sqrt(ex * ex + ey * ey);
            double mc = fabs(nrm / prm->eps - 1.0);
            if (mc < m->conv) m->conv = mc;
            if (nrm < prm->eps) break;
        }
        if (l > 0) { gx = 2.0 * (gx + dx); gy = 2.0 * (gy + dy); }
    }
    /* level 0: c = p */
    double qx = px + gx + dx, qy = py + gy + dy;
    *ox = qx; *oy = qy;
    double bd = box_dist(qx, qy, 0.0, J->w[0] - 1.0, J->h[0] - 1.0);
    if (fabs(bd) < m->oob) m->oob = fabs(bd);
    double acc = 0.0;
    for (int i = 0; i < win; ++i)
        for (int j = 0; j < win; ++j)
            acc += fabs(s->T[i * win + j]
                        - lko_sample(J->img[0], J->w[0], J->h[0], qx + (j - h), qy + (i - h)));
    *res = acc / nw;
    if (!(bd >= 0.0)) return LKO_LOST_OOB;
    return LKO_OK;
}

typedef struct {
    const pyr_t *I, *J;
    const double *pts, *guess;
    const lko_params *prm;
    int begin, end;
    double *out_pts, *residual, *margins;
    uint8_t *status;
    int32_t *iters;
    int rc;
} job_t;

static void *run_job(void *arg)
{
    job_t *jb = (job_t *)arg;
    const lko_params *prm = jb->prm;
    const int L = prm->levels, nw = prm->win * prm->win;
    scratch_t s;
    s.T = malloc(3 * (size_t)nw * sizeof(double));
    if (!s.T) { jb->rc = -2; return NULL; }
    s.Gx = s.T + nw; s.Gy = s.T + 2 * nw;
    for (int n = jb->begin; n < jb->end; ++n) {
        double px = jb->pts[2 * n], py = jb->pts[2 * n + 1];
        double g0x = 0.0, g0y = 0.0;
        if (prm->use_guess && jb->guess) {
            double sc = ldexp(1.0, -(L - 1));
            g0x = (jb->guess[2 * n] - px) * sc;
            g0y = (jb->guess[2 * n + 1] - py) * sc;
        }
        margins_t m = {DBL_MAX, DBL_MAX, DBL_MAX, DBL_MAX};
        int32_t *it = jb->iters ? jb->iters + (size_t)n * 2 * L : NULL;
        if (it) memset(it, 0, 2 * (size_t)L * sizeof(int32_t));
        double qx, qy, res;
        int st = track_pass(jb->I, jb->J, px, py, g0x, g0y, prm, &s, &qx, &qy, &res, it, &m);
        if (st == LKO_OK && prm->fb_thresh > 0.0) {
            double bx, by, bres;
            int bst = track_pass(jb->J, jb->I, qx, qy, 0.0, 0.0, prm, &s, &bx, &by, &bres,
                                 it ? it + L : NULL, &m);
            if (bst != LKO_OK) st = LKO_LOST_FB;
            else {
                double fbd = sqrt((bx - px) * (bx - px) + (by - py) * (by - py));
                m.fb = fabs(fbd - prm->fb_thresh);
                if (fbd > prm->fb_thresh) st = LKO_LOST_FB;
            }
        }
        jb->out_pts[2 * n] = qx; jb->out_pts[2 * n + 1] = qy;
        jb->status[n] = (uint8_t)st;
        jb->residual[n] = res;
        if (jb->margins) {
            jb->margins[4 * n + 0] = m.eig; jb->margins[4 * n + 1] = m.oob;
            jb->margins[4 * n + 2] = m.conv; jb->margins[4 * n + 3] = m.fb;
        }
    }
    free(s.T);
    return NULL;
}

static int check_params(int w, int h, const lko_params *p)
{
    int32_t ws[LKO_MAX_LEVELS], hs[LKO_MAX_LEVELS];
    if (!p) return -1;
    if (p->win < 3 || p->win > 63 || (p->win & 1) == 0) return -1;
    if (p->max_iters < 1 || !(p->eps > 0.0) || !(p->min_eig >= 0.0)) return -1;
    if (p->nthreads < 1) return -1;
    return lko_level_dims(w, h, p->levels, ws, hs);
}

static int track_pyrs(const pyr_t *I, const pyr_t *J, const double *pts, const double *guess,
                      int n, const lko_params *prm, double *out_pts, uint8_t *status,
                      double *residual, int32_t *iters, double *margins)
{
    int T = prm->nthreads;
    if (T > n) T = n > 0 ? n : 1;
    job_t jobs[256];
    pthread_t th[256];
    if (T > 256) T = 256;
    int rc = 0;
    for (int t = 0; t < T; ++t) {
        jobs[t] = (job_t){I, J, pts, guess, prm, (int)((long)n * t / T), (int)((long)n * (t + 1) / T),
                          out_pts, residual, margins, status, iters, 0};
    }
    if (T == 1) run_job(&jobs[0]);
    else {
        for (int t = 0; t < T; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
        for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
    }
    for (int t = 0; t < T; ++t) if (jobs[t].rc) rc = jobs[t].rc;
    return rc;
}

/* Track n points from image prev to image next (both w x h, row-major,
 * double).  pts/guess/out_pts are n x 2 (x, y).  iters (n x 2L: forward
 * levels 0..L-1, then backward) and margins (n x 4: eig, oob, conv, fb) may
 * be NULL.  Returns 0, -1 for invalid arguments, -2 for out of memory. */
int lko_track_f64(const double *prev, const double *next, int w, int h,
                  const double *pts, const double *guess, int n, const lko_params *prm,
                  double *out_pts, uint8_t *status, double *residual,
                  int32_t *iters, double *margins)
{
    if (check_params(w, h, prm) != 0 || n < 0 || !prev || !next) return -1;
    if (n == 0) return 0;
    pyr_t I, J;
    int rc = pyr_build(&I, prev, w, h, prm->levels, prm->f16_storage);
    if (rc) return rc;
    rc = pyr_build(&J, next, w, h, prm->levels, prm->f16_storage);
    if (rc) { pyr_free(&I); return rc; }
    rc = track_pyrs(&I, &J, pts, guess, n, prm, out_pts, status, residual, iters, margins);
    pyr_free(&I); pyr_free(&J);
    return rc;
}

/* Same for 8-bit images with a row pitch in bytes. */
int lko_track_u8(const uint8_t *prev, const uint8_t *next, int w, int h, int pitch,
                 const double *pts, const double *guess, int n, const lko_params *prm,
                 double *out_pts, uint8_t *status, double *residual,
                 int32_t *iters, double *margins)
{
    if (check_params(w, h, prm) != 0 || n < 0 || !prev || !next || pitch < w) return -1;
    double *a = malloc((size_t)w * h * sizeof(double));
    double *b = malloc((size_t)w * h * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            a[(size_t)y * w + x] = prev[(size_t)y * pitch + x];
            b[(size_t)y * w + x] = next[(size_t)y * pitch + x];
        }
    int rc = lko_track_f64(a, b, w, h, pts, guess, n, prm, out_pts, status, residual, iters, margins);
    free(a); free(b);
    return rc;
}

/* ------------------------------------------------------------------ GFTT
 * Shi-Tomasi corner detection ("good features to track"), the detector the
 * paper's GFTT+LK baseline uses to seed and replenish tracks (Sec. IV,
 * Sec. V-E).  The paper does not define it; the classical definition is
 * written out here:
 *   1. raw Scharr gradients (the [3 10 3] x [-1 0 1] stencil without the
 *      1/32 scale, so they are integers), reflect-101 borders;
 *   2. structure tensor a = sum gx^2, b = sum gx gy, c = sum gy^2 over the
 *      (2r+1)^2 block around each pixel, reflect-101 borders, exact integers;
 *   3. response R = lambda_min = ((a + c) - sqrt((a - c)^2 + 4 b^2)) / 2,
 *      evaluated in double in exactly this order (no fused operations);
 *   4. candidates: R > quality * max R and R >= each of its 8 neighbours
 *      (pixels within `border` of the edge are never candidates);
 *   5. candidates ordered by R descending, ties by raster index ascending;
 *      taken greedily while no taken or occupied point lies at squared
 *      distance < min_dist^2, until max_corners are taken.
 * Writes the corners (x, y) and returns their count, or -1 on bad input. */
static long long sq_ll(long long v) { return v * v; }

int lko_gftt_response(const uint8_t *img, int w, int h, int pitch, int r, double *resp)
{
    if (!img || !resp || w < 3 || h < 3 || r < 0 || r > 3 || pitch < w) return -1;
    int *gx = malloc((size_t)w * h * sizeof(int)), *gy = malloc((size_t)w * h * sizeof(int));
    if (!gx || !gy) { free(gx); free(gy); return -2; }
    for (int y = 0; y < h; ++y) {
        int ym = reflect101(y - 1, h), yp = reflect101(y + 1, h);
        for (int x = 0; x < w; ++x) {
            int xm = reflect101(x - 1, w), xp = reflect101(x + 1, w);
#define Q(yy, xx) ((int)img[(size_t)(yy) * pitch + (xx)])
            gx[(size_t)y * w + x] = 3 * (Q(ym, xp) - Q(ym, xm)) + 10 * (Q(y, xp) - Q(y, xm)) + 3 * (Q(yp, xp) - Q(yp, xm));
            gy[(size_t)y * w + x] = 3 * (Q(yp, xm) - Q(ym, xm)) + 10 * (Q(yp, x) - Q(ym, x)) + 3 * (Q(yp, xp) - Q(ym, xp));
#undef Q
        }
    }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            long long a = 0, b = 0, c = 0;
            for (int j = -r; j <= r; ++j)
                for (int i = -r; i <= r; ++i) {
                    size_t o = (size_t)reflect101(y + j, h) * w + reflect101(x + i, w);
                    a += sq_ll(gx[o]);
                    b += (long long)gx[o] * gy[o];
                    c += sq_ll(gy[o]);
                }
            volatile double t = (double)(a - c);
            volatile double u = (double)b;
            volatile double d1 = t * t;
            volatile double d2 = 4.0 * u * u;
            volatile double disc = d1 + d2;
            volatile double s = sqrt(disc);
            volatile double tr = (double)(a + c);
            resp[(size_t)y * w + x] = (tr - s) * 0.5;
        }
    free(gx); free(gy);
    return 0;
}

typedef struct { double r; int idx; } cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = pa, *b = pb;
    if (a->r > b->r) return -1;
    if (a->r < b->r) return 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx);
}

int lko_gftt(const uint8_t *img, int w, int h, int pitch, int r, double quality, int min_dist, int max_corners,
             int border, const float *occupied, int n_occupied, float *out_xy)
{
    if (!img || w < 3 || h < 3 || !(quality >= 0.0) || min_dist < 0 || max_corners < 0 || border < 0) return -1;
    if (n_occupied > 0 && !occupied) return -1;
    double *R = malloc((size_t)w * h * sizeof(double));
    cand_t *cand = malloc((size_t)w * h * sizeof(cand_t));
    int *taken = malloc(((size_t)max_corners + 1) * 2 * sizeof(int));
    if (!R || !cand || !taken) { free(R); free(cand); free(taken); return -2; }
    int rc = lko_gftt_response(img, w, h, pitch, r, R);
    if (rc) { free(R); free(cand); free(taken); return rc; }
    double rmax = 0.0;
    for (size_t i = 0; i < (size_t)w * h; ++i) if (R[i] > rmax) rmax = R[i];
    double thr = quality * rmax;
    int nc = 0;
    for (int y = border; y < h - border; ++y)
        for (int x = border; x < w - border; ++x) {
            double v = R[(size_t)y * w + x];
            if (!(v > thr) || !(v > 0.0)) continue;
            int peak = 1;
            for (int j = -1; j <= 1 && peak; ++j)
                for (int i = -1; i <= 1; ++i) {
                    int yy = y + j, xx = x + i;
                    if ((i || j) && yy >= 0 && yy < h && xx >= 0 && xx < w && R[(size_t)yy * w + xx] > v) { peak = 0; break; }
                }
            if (peak) { cand[nc].r = v; cand[nc].idx = y * w + x; ++nc; }
        }
    qsort(cand, nc, sizeof(cand_t), cand_cmp);
    long long md2 = (long long)min_dist * min_dist;
    int nt = 0;
    for (int k = 0; k < nc && nt < max_corners; ++k) {
        int x = cand[k].idx % w, y = cand[k].idx / w, ok = 1;
        for (int t = 0; t < nt && ok; ++t)
            if (sq_ll(x - taken[2 * t]) + sq_ll(y - taken[2 * t + 1]) < md2) ok = 0;
        for (int t = 0; t < n_occupied && ok; ++t) {
            double dx = (double)x - (double)occupied[2 * t], dy = (double)y - (double)occupied[2 * t + 1];
            if (dx * dx + dy * dy < (double)md2) ok = 0;
        }
        if (!ok) continue;
        taken[2 * nt] = x; taken[2 * nt + 1] = y; ++nt;
    }
    if (out_xy)
        for (int t = 0; t < nt; ++t) { out_xy[2 * t] = (float)taken[2 * t]; out_xy[2 * t + 1] = (float)taken[2 * t + 1]; }
    free(R); free(cand); free(taken);
    return nt;
}
