"""A second, independent FP64 implementation of pyramidal Lucas-Kanade
tracking, for tiny inputs -- TEST INFRASTRUCTURE.

It exists to pin ``lk_oracle.c`` against something other than itself: the
two are written separately and share nothing but the definition of the
method.  Here every stage is a library routine or a whole-array numpy
expression instead of the C oracle's explicit loops:

* pyramid step: ``scipy.ndimage.correlate1d`` with the binomial kernel
  [1 4 6 4 1] / 16 along each axis, mode 'mirror' (reflect-101), then every
  second sample (blur then decimate, the Burt-Adelson reduce step);
* gradients: ``scipy.ndimage.correlate`` with the Scharr kernel / 32, mode
  'mirror';
* bilinear sampling: ``scipy.ndimage.map_coordinates`` (order 1, mode
  'nearest': the taps replicate the edge, as clamping the tap indices does);
* the eigenvalue test: ``numpy.linalg.eigvalsh`` of the 2x2 normal matrix;
* the Gauss-Newton step: ``numpy.linalg.solve``.

The method (Bouguet's pyramidal form of Lucas-Kanade): per level, coarse to
fine, the template and its gradients are sampled on the window around
p / 2^l; the point is lost if the smallest eigenvalue of the normal matrix,
divided by win^2 255^2, is below min_eig; then Gauss-Newton steps with the
normal matrix fixed, each preceded by the check that the window still
overlaps the level, stopping after the first step shorter than eps; the
flow guess doubles from level to level.  The end point must lie in the
image; the residual is the mean absolute mismatch over the level-0 window;
the forward-backward check runs the same pass from the end point back.
Binary16 storage rounds every stored level >= 1 and every gradient plane to
binary16 (numpy's float16 conversion, round to nearest even).

Only small frames and few points: the per-iteration work is a few numpy
calls per point.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

OK, LOST_EIG, LOST_OOB, LOST_FB = 0, 1, 2, 3

BINOMIAL = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
SCHARR_X = np.array([[-3.0, 0.0, 3.0], [-10.0, 0.0, 10.0], [-3.0, 0.0, 3.0]]) / 32.0


def _f16(a: np.ndarray) -> np.ndarray:
    return a.astype(np.float16).astype(np.float64)


def build(img: np.ndarray, levels: int, f16: bool = False):
    """Levels and (gx, gy) gradient planes, each a list of 2-D float64 arrays."""
    lv = [np.asarray(img, dtype=np.float64)]
    for _ in range(1, levels):
        b = ndimage.correlate1d(lv[-1], BINOMIAL, axis=0, mode="mirror")
        b = ndimage.correlate1d(b, BINOMIAL, axis=1, mode="mirror")
        nxt = b[::2, ::2].copy()
        lv.append(_f16(nxt) if f16 else nxt)
    gx = [ndimage.correlate(a, SCHARR_X, mode="mirror") for a in lv]
    gy = [ndimage.correlate(a, SCHARR_X.T, mode="mirror") for a in lv]
    if f16:
        gx = [_f16(a) for a in gx]
        gy = [_f16(a) for a in gy]
    return lv, gx, gy


def _sample(a: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    return ndimage.map_coordinates(a, [ys, xs], order=1, mode="nearest", prefilter=False)


def _inside(x, y, lo_x, lo_y, hi_x, hi_y) -> bool:
    return bool(lo_x <= x <= hi_x and lo_y <= y <= hi_y)


def _pass(I, J, p, g, win, L, max_iters, eps, min_eig, iters):
    """One coarse-to-fine pass; returns (status, end point, residual)."""
    h = (win - 1) // 2
    off = np.arange(-h, h + 1, dtype=np.float64)
    ox, oy = np.meshgrid(off, off)
    ox, oy = ox.ravel(), oy.ravel()
    Il, Gxl, Gyl = I
    Jl = J[0]
    W0, H0 = Il[0].shape[1], Il[0].shape[0]
    if not _inside(p[0], p[1], 0.0, 0.0, W0 - 1.0, H0 - 1.0):
        return LOST_OOB, p.copy(), 0.0
    g = g.copy()
    d = np.zeros(2)
    T0 = None
    for l in range(L - 1, -1, -1):
        Hl, Wl = Il[l].shape
        c = p / 2.0 ** l
        xs, ys = c[0] + ox, c[1] + oy
        T = _sample(Il[l], xs, ys)
        gx = _sample(Gxl[l], xs, ys)
        gy = _sample(Gyl[l], xs, ys)
        G = np.array([[gx @ gx, gx @ gy], [gx @ gy, gy @ gy]])
        d = np.zeros(2)
        if np.linalg.eigvalsh(G)[0] / (win * win * 255.0 ** 2) < min_eig:
            return LOST_EIG, (c + g) * 2.0 ** l, 0.0
        for k in range(1, max_iters + 1):
            q = c + g + d
            if not _inside(q[0], q[1], -h, -h, Wl - 1.0 + h, Hl - 1.0 + h):
                return LOST_OOB, q * 2.0 ** l, 0.0
            e = T - _sample(Jl[l], q[0] + ox, q[1] + oy)
            eta = np.linalg.solve(G, np.array([e @ gx, e @ gy]))
            d = d + eta
            iters[l] = k
            if np.hypot(eta[0], eta[1]) < eps:
                break
        if l > 0:
            g = 2.0 * (g + d)
        else:
            T0 = T
    q = p + g + d
    res = float(np.mean(np.abs(T0 - _sample(Jl[0], q[0] + ox, q[1] + oy))))
    if not _inside(q[0], q[1], 0.0, 0.0, W0 - 1.0, H0 - 1.0):
        return LOST_OOB, q, res
    return OK, q, res


def track(prev, nxt, pts, guess=None, *, win=21, levels=3, max_iters=30, eps=0.01, min_eig=1e-4,
          fb_thresh=0.0, f16=False):
    """Same contract as ``oracle.track`` (points, status, residual, iteration
    counts N x 2 x L); no margins."""
    I = build(prev, levels, f16)
    J = build(nxt, levels, f16)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    n = len(pts)
    out = np.zeros((n, 2))
    st = np.zeros(n, np.uint8)
    res = np.zeros(n)
    it = np.zeros((n, 2, levels), np.int32)
    for i in range(n):
        p = pts[i]
        g = np.zeros(2) if guess is None else (np.asarray(guess[i], np.float64) - p) / 2.0 ** (levels - 1)
        s, q, r = _pass(I, J, p, g, win, levels, max_iters, eps, min_eig, it[i, 0])
        if s == OK and fb_thresh > 0.0:
            sb, pb, _ = _pass(J, I, q, np.zeros(2), win, levels, max_iters, eps, min_eig, it[i, 1])
            if sb != OK or np.hypot(*(pb - p)) > fb_thresh:
                s = LOST_FB
        out[i], st[i], res[i] = q, s, r
    return out, st, res, it
