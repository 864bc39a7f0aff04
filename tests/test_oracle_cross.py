"""Cross-implementation pin: the C oracle against the independent numpy/scipy
implementation in ``oracle/mini_lk.py`` on tiny inputs.

Both compute the same definition in FP64 by different routes (explicit loops
and the closed-form eigenvalue and 2x2 solve in C; scipy filters, scipy
sampling, eigvalsh and linalg.solve in numpy), so they may differ only by
rounding: end points within 1e-9 px, identical status and iteration counts,
residuals within 1e-9 gray.  A decision whose deciding quantity lies within
1e-7 (relative, or px) of its threshold could flip on rounding alone; such
points are counted and must be rare.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import mini_lk


def smooth(w, h, seed, dx=0.0, dy=0.0):
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    xs, ys = xs - dx, ys - dy
    out = np.full((h, w), 110.0)
    for _ in range(14):
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        s, a = rng.uniform(2.5, 7.0), rng.uniform(-60, 60)
        out += a * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * s * s))
    return out


def texture_pair(w, h, seed, shift):
    pad = 16
    canvas = synth.texture_canvas(h + 2 * pad, w + 2 * pad, seed)
    from scipy import ndimage
    moved = ndimage.shift(canvas, (shift[1], shift[0]), order=1, mode="nearest", prefilter=False)
    a = synth.quantize_u8(canvas[pad:pad + h, pad:pad + w])
    b = synth.quantize_u8(moved[pad:pad + h, pad:pad + w] + np.random.default_rng(seed).normal(0, 2.0, (h, w)))
    return a, b


def check(prev, nxt, pts, guess=None, **kw):
    r = oracle.track(prev, nxt, pts, guess, **kw)
    m_pts, m_st, m_res, m_it = mini_lk.track(prev, nxt, pts, guess, **kw)
    eps = kw.get("eps", 0.01)
    # decisions within 1e-7 of a threshold may flip on rounding (conv margin in px)
    close = (r.margins[:, 0] <= 1e-7) | (r.margins[:, 1] <= 1e-7) | (r.margins[:, 2] <= 1e-7 * eps) \
        | (r.margins[:, 3] <= 1e-7)
    keep = ~close
    assert close.sum() <= max(1, len(pts) // 20)
    assert np.array_equal(r.status[keep], m_st[keep])
    assert np.array_equal(r.iters[keep], m_it[keep])
    both = keep & (r.status == 0)
    np.testing.assert_allclose(r.pts[both], m_pts[both], atol=1e-9, rtol=0)
    np.testing.assert_allclose(r.residual[both], m_res[both], atol=1e-9, rtol=0)
    # lost points: the same last estimate (they carry no contract, but both follow the same steps)
    lost = keep & (r.status != 0) & np.isfinite(r.pts).all(axis=1)
    np.testing.assert_allclose(r.pts[lost], m_pts[lost], atol=1e-9, rtol=0)
    return r


@pytest.mark.parametrize("win,levels", [(5, 1), (7, 2), (9, 3), (7, 3)])
def test_smooth_float_frames(win, levels):
    w, h = 72, 56
    I = smooth(w, h, 1)
    J = smooth(w, h, 1, 1.3, -0.8)
    pts = synth.uniform_points(np.random.default_rng(win), 24, w, h, border=6).astype(np.float64)
    r = check(I, J, pts, win=win, levels=levels, max_iters=40, eps=1e-3, min_eig=1e-7)
    assert (r.status == 0).sum() >= 12


@pytest.mark.parametrize("f16", [False, True])
def test_textured_8bit_frames_with_fb(f16):
    w, h = 96, 80
    a, b = texture_pair(w, h, 5, (2.4, -1.7))
    pts = synth.uniform_points(np.random.default_rng(3), 30, w, h, border=4)
    r = check(a, b, pts, win=9, levels=3, max_iters=30, eps=0.01, min_eig=1e-6, fb_thresh=0.5, f16=f16)
    assert (r.status == 0).sum() >= 15
    assert (r.status == oracle.LOST_FB).sum() + (r.status == 0).sum() >= 20


def test_guesses_borders_and_lost_points():
    w, h = 64, 48
    a, b = texture_pair(w, h, 9, (-3.2, 2.1))
    pts = np.array([[0.0, 0.0], [63.0, 47.0], [1.5, 23.0], [62.2, 2.5], [30.0, 24.0], [-0.5, 10.0],
                    [20.0, 48.0], [40.25, 11.75], [10.0, 40.0], [55.5, 30.5]])
    guess = pts + np.array([-3.0, 2.0])
    guess[4] = [-40.0, 24.0]                 # puts the coarse window off the level
    r = check(a, b, pts, guess, win=7, levels=2, max_iters=20, eps=0.01, min_eig=1e-6, fb_thresh=1.0)
    assert r.status[5] == oracle.LOST_OOB and r.status[6] == oracle.LOST_OOB and r.status[4] == oracle.LOST_OOB


def test_flat_and_striped_frames():
    w, h = 48, 40
    flat = np.full((h, w), 70.0)
    xs = np.arange(w, dtype=np.float64)
    stripes = np.tile(90 + 50 * np.sin(xs / 3.0), (h, 1))
    pts = np.array([[20.0, 20.0], [10.5, 30.25]])
    for img in (flat, stripes):
        r = check(img, img, pts, win=7, levels=2, min_eig=1e-9)
        assert np.all(r.status == oracle.LOST_EIG)
