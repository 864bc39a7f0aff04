/* Exercises the FP64 oracle (oracle/lk_oracle.c, compiled into this program)
 * under host sanitizers: tracking on 8-bit frames of several sizes and row
 * pitches, every window size and level count the oracle accepts, binary16
 * storage, the forward-backward check, guesses, one and several threads,
 * points on and outside the borders and not finite, the corner detector
 * with occupied points, and invalid arguments.  Prints a checksum and exits
 * 0; a sanitizer report makes the run fail.  Test infrastructure. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lk_oracle.c"

static unsigned long long g_state = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

/* smooth texture plus noise, shifted by (dx, dy) for the second frame */
static void frame(uint8_t *img, int w, int h, int pitch, double dx, double dy)
{
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < pitch; ++x) {
            double v = 0.0;
            if (x < w) {
                const double u = x - dx, t = y - dy;
                v = 128.0 + 60.0 * sin(0.21 * u + 0.05 * t) + 40.0 * cos(0.17 * t - 0.11 * u)
                    + 20.0 * sin(0.5 * u) * cos(0.43 * t) + 4.0 * (urand() - 0.5);
            }
            img[(size_t)y * pitch + x] = (uint8_t)(v < 0.0 ? 0.0 : (v > 255.0 ? 255.0 : v));
        }
}

static double g_sum = 0.0;

static void track_case(int w, int h, int pitch, int win, int levels, int f16, int fb, int threads, int guess)
{
    uint8_t *a = malloc((size_t)pitch * h), *b = malloc((size_t)pitch * h);
    frame(a, w, h, pitch, 0.0, 0.0);
    frame(b, w, h, pitch, 1.3, -0.7);
    enum { N = 40 };
    double pts[2 * N], gs[2 * N], out[2 * N], res[N], mar[4 * N];
    uint8_t st[N];
    int32_t it[N * 2 * LKO_MAX_LEVELS];
    for (int i = 0; i < N; ++i) {
        pts[2 * i] = urand() * (w - 1);
        pts[2 * i + 1] = urand() * (h - 1);
        gs[2 * i] = pts[2 * i] + 1.0;
        gs[2 * i + 1] = pts[2 * i + 1] - 0.5;
    }
    pts[0] = 0.0; pts[1] = 0.0;                       /* corners and edges */
    pts[2] = w - 1; pts[3] = h - 1;
    pts[4] = -0.5; pts[5] = 3.0;                      /* outside */
    pts[6] = NAN; pts[7] = 1.0;                       /* not finite */
    pts[8] = 1e30; pts[9] = -1e30;
    gs[10] = 1e9; gs[11] = 2.0;                       /* a guess far off the frame */
    lko_params p;
    memset(&p, 0, sizeof p);
    p.win = win; p.levels = levels; p.max_iters = 30; p.use_guess = guess; p.f16_storage = f16;
    p.nthreads = threads; p.eps = 0.01; p.min_eig = 1e-6; p.fb_thresh = fb ? 1.0 : 0.0;
    const int rc = lko_track_u8(a, b, w, h, pitch, pts, guess ? gs : NULL, N, &p, out, st, res, it, mar);
    if (rc != 0) { fprintf(stderr, "track rc %d (w %d h %d win %d L %d)\n", rc, w, h, win, levels); exit(2); }
    for (int i = 0; i < N; ++i) {
        g_sum += st[i];
        if (st[i] == 0) g_sum += out[2 * i] + out[2 * i + 1] + res[i];
    }
    free(a); free(b);
}

int main(void)
{
    static const int sizes[][3] = {{64, 48, 64}, {33, 17, 40}, {160, 120, 163}, {8, 8, 8}};
    static const int wins[] = {3, 9, 21, 31, 63};
    for (int s = 0; s < 4; ++s)
        for (int wi = 0; wi < 5; ++wi)
            for (int levels = 1; levels <= 4; ++levels) {
                const int w = sizes[s][0], h = sizes[s][1], pitch = sizes[s][2];
                int32_t ws[LKO_MAX_LEVELS], hs[LKO_MAX_LEVELS];
                if (lko_level_dims(w, h, levels, ws, hs) != 0) continue;   /* coarsest level below 4 x 4 */
                for (int f16 = 0; f16 <= 1; ++f16)
                    track_case(w, h, pitch, wins[wi], levels, f16, (wi + levels) & 1, (s & 1) ? 4 : 1,
                               (levels + f16) & 1);
            }
    /* invalid arguments are rejected */
    {
        uint8_t img[64];
        double p2[2] = {1.0, 1.0}, o2[2], r1;
        uint8_t s1;
        lko_params p;
        memset(&p, 0, sizeof p);
        p.win = 4; p.levels = 1; p.max_iters = 5; p.nthreads = 1; p.eps = 0.01;
        if (lko_track_u8(img, img, 8, 8, 8, p2, NULL, 1, &p, o2, &s1, &r1, NULL, NULL) != -1) return 3;
        p.win = 3; p.levels = 9;
        if (lko_track_u8(img, img, 8, 8, 8, p2, NULL, 1, &p, o2, &s1, &r1, NULL, NULL) != -1) return 4;
        p.levels = 1;
        if (lko_track_u8(img, img, 8, 8, 4, p2, NULL, 1, &p, o2, &s1, &r1, NULL, NULL) != -1) return 5;
    }
    /* corner detection with occupied points, several radii and borders */
    for (int s = 0; s < 3; ++s) {
        const int w = sizes[s][0], h = sizes[s][1], pitch = sizes[s][2];
        uint8_t *img = malloc((size_t)pitch * h);
        frame(img, w, h, pitch, 0.0, 0.0);
        float occ[6] = {5.0f, 5.0f, (float)(w / 2), (float)(h / 2), -3.0f, NAN};
        float xy[2 * 64];
        for (int r = 0; r <= 3; ++r) {
            const int n = lko_gftt(img, w, h, pitch, r, 0.01, 4, 64, r, occ, 3, xy);
            if (n < 0) { fprintf(stderr, "gftt rc %d\n", n); return 6; }
            for (int i = 0; i < n; ++i) g_sum += xy[2 * i] + xy[2 * i + 1];
        }
        free(img);
    }
    printf("oracle sanitizer run ok, checksum %.6f\n", g_sum);
    return 0;
}
