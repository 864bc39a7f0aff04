"""Pins of the whole FP64 tracker against what the method fixes exactly.

* exact sub-pixel recovery on a bilinear-polynomial image (every stage --
  binomial pyramid, Scharr, bilinear sampling -- is exact on span{1,x,y,xy});
* the first Gauss-Newton step on that image in closed form (analytic G and
  sum of gradients, numpy.linalg.solve) -- pins the normal matrix, the 2x2
  solve and the sign of the update;
* the eigenvalue test against numpy.linalg.eigvalsh of the analytic G;
* identical frames -> exactly zero flow, one iteration per level;
* constant and one-dimensional textures -> LOST_EIG (aperture problem);
* integer shifts of an 8-bit texture -> exact recovery, zero residual;
* brute-force SSD search on tiny inputs (scipy bilinear sampling);
* equivariance: scene shifts, swapping the frames, one level vs three;
* out-of-bounds and forward-backward status rules, guesses, threading.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth

A, B, CC, E, X0, Y0 = 0.02, 1.1, -0.6, 120.0, 97.3, 71.9


def poly_img(w, h, dx=0.0, dy=0.0, a=A):
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    xs = xs - dx
    ys = ys - dy
    return a * (xs - X0) * (ys - Y0) + B * xs + CC * ys + E


def analytic_grad(x, y, a=A):
    return a * (y - Y0) + B, a * (x - X0) + CC


@pytest.mark.parametrize("levels", [1, 3])
def test_exact_subpixel_recovery_on_polynomial(levels):
    rng = np.random.default_rng(100 + levels)
    w, h = 220, 180
    I = poly_img(w, h)
    for trial in range(4):
        d = rng.uniform(-3.0, 3.0, 2) if levels == 1 else rng.uniform(-8.0, 8.0, 2)
        J = poly_img(w, h, d[0], d[1])
        margin = (10 + 4) * 2 ** (levels - 1) + 9
        pts = rng.uniform([margin, margin], [w - 1 - margin, h - 1 - margin], (12, 2))
        r = oracle.track(I, J, pts, win=21, levels=levels, max_iters=100, eps=1e-12, min_eig=1e-9)
        assert np.all(r.status == oracle.OK)
        np.testing.assert_allclose(r.pts, pts + d, atol=1e-9, rtol=0)


def test_first_gauss_newton_step_closed_form():
    # One level, one iteration, zero initial flow.  For J(x) = I(x - d) on a
    # bilinear polynomial the error image is exactly
    #   e = I(c+x) - I(c+x-d) = grad I(c+x) . d - a dx dy,
    # so the step is eta = G^-1 sum(e grad) = d - a dx dy G^-1 sum(grad).
    w, h = 160, 140
    I = poly_img(w, h)
    rng = np.random.default_rng(7)
    win, hw = 15, 7
    for _ in range(5):
        d = rng.uniform(-2.0, 2.0, 2)
        J = poly_img(w, h, d[0], d[1])
        p = rng.uniform(40, 100, 2)
        r = oracle.track(I, J, p[None], win=win, levels=1, max_iters=1, eps=1e-12, min_eig=0.0)
        offs = np.arange(-hw, hw + 1, dtype=np.float64)
        X, Y = np.meshgrid(p[0] + offs, p[1] + offs)
        gx, gy = analytic_grad(X.ravel(), Y.ravel())
        G = np.array([[gx @ gx, gx @ gy], [gx @ gy, gy @ gy]])
        S = np.array([gx.sum(), gy.sum()])
        eta = d - A * d[0] * d[1] * np.linalg.solve(G, S)
        np.testing.assert_allclose(r.pts[0], p + eta, atol=1e-9, rtol=0)
        assert r.iters[0, 0, 0] == 1 and r.status[0] == oracle.OK


def test_min_eigenvalue_threshold_matches_eigvalsh():
    w, h = 120, 120
    I = poly_img(w, h)
    win, hw = 21, 10
    p = np.array([[60.25, 55.5]])
    offs = np.arange(-hw, hw + 1, dtype=np.float64)
    X, Y = np.meshgrid(p[0, 0] + offs, p[0, 1] + offs)
    gx, gy = analytic_grad(X.ravel(), Y.ravel())
    G = np.array([[gx @ gx, gx @ gy], [gx @ gy, gy @ gy]])
    m = np.linalg.eigvalsh(G)[0] / (win * win * 255.0 ** 2)
    lo = oracle.track(I, I, p, win=win, levels=1, min_eig=m * (1 - 1e-7))
    hi = oracle.track(I, I, p, win=win, levels=1, min_eig=m * (1 + 1e-7))
    assert lo.status[0] == oracle.OK and hi.status[0] == oracle.LOST_EIG
    np.testing.assert_allclose(lo.margins[0, 0], 1e-7 / (1 - 1e-7), rtol=1e-4)


def texture(h, w, seed):
    return synth.quantize_u8(synth.texture_canvas(h, w, seed))


def test_identical_frames_zero_flow():
    img = texture(240, 320, 1)
    rng = np.random.default_rng(1)
    pts = synth.uniform_points(rng, 200, 320, 240)
    r = oracle.track(img, img, pts, win=21, levels=3, min_eig=1e-6)
    ok = r.status == oracle.OK
    assert ok.mean() > 0.9
    assert np.array_equal(r.pts[ok], pts[ok].astype(np.float64))
    assert np.all(r.iters[ok, 0, :] == 1)
    assert np.all(r.residual[ok] == 0.0)


def test_constant_and_one_dimensional_patches_lost_eig():
    pts = np.array([[40.0, 30.0], [20.5, 50.25], [64.7, 33.3]])
    const = np.full((80, 100), 77, dtype=np.uint8)
    r = oracle.track(const, const, pts, min_eig=1e-12)
    assert np.all(r.status == oracle.LOST_EIG)
    xs = np.arange(100, dtype=np.float64)
    stripes = np.tile(100 + 60 * np.sin(xs / 4.0), (80, 1))          # I = f(x)
    r = oracle.track(stripes, stripes, pts, min_eig=1e-12)
    assert np.all(r.status == oracle.LOST_EIG)


def shifted_pair(h, w, dx, dy, seed, pad=24):
    canvas = texture(h + 2 * pad, w + 2 * pad, seed)
    prev = canvas[pad:pad + h, pad:pad + w]
    nxt = canvas[pad - dy:pad - dy + h, pad - dx:pad - dx + w]       # nxt(x) = prev(x - d)
    return np.ascontiguousarray(prev), np.ascontiguousarray(nxt)


@pytest.mark.parametrize("d", [(3, -2), (-7, 5), (12, 9), (0, 1)])
def test_integer_shift_exact(d):
    prev, nxt = shifted_pair(200, 260, d[0], d[1], seed=abs(d[0]) + 3)
    rng = np.random.default_rng(d[0] + 20)
    pts = synth.uniform_points(rng, 120, 260, 200, border=40)
    r = oracle.track(prev, nxt, pts, win=21, levels=3, max_iters=100, eps=1e-9, min_eig=1e-6)
    ok = r.status == oracle.OK
    assert ok.mean() > 0.8
    np.testing.assert_allclose(r.pts[ok], pts[ok] + np.array(d, float), atol=1e-6, rtol=0)
    assert np.all(r.residual[ok] < 1e-5)
    # with the default eps the end point is within the last step of the truth
    r2 = oracle.track(prev, nxt, pts, win=21, levels=3, min_eig=1e-6)
    ok2 = r2.status == oracle.OK
    assert np.abs(r2.pts[ok2] - (pts[ok2] + np.array(d, float))).max() < 0.02


def test_residual_is_mean_absolute_level0_mismatch():
    # J = integer shift of I plus a +-3 checkerboard: at the true alignment
    # every |T - J| is exactly 3, and the checkerboard is orthogonal to the
    # smooth texture's gradients, so LK stays at the true shift.
    d = (4, -3)
    pad = 24
    canvas = (60 + 0.5 * synth.texture_canvas(200 + 2 * pad, 260 + 2 * pad, 31)).round()
    prev = canvas[pad:pad + 200, pad:pad + 260]
    nxt = canvas[pad - d[1]:pad - d[1] + 200, pad - d[0]:pad - d[0] + 260].copy()
    ys, xs = np.mgrid[0:200, 0:260]
    nxt += 3.0 * np.where((xs + ys) % 2 == 0, 1.0, -1.0)
    # integer keypoints: the bilinear weights are (0, 0), so the sampled
    # checkerboard keeps its full +-3 amplitude at the true alignment
    pts = np.round(synth.uniform_points(np.random.default_rng(8), 150, 260, 200, border=40)).astype(np.float32)
    r = oracle.track(prev, nxt, pts, win=21, levels=1, max_iters=1, eps=1e-9, min_eig=0.0,
                     guess=pts + np.array(d, np.float32))
    step = np.abs(r.pts - (pts + np.array(d, float))).max(axis=1)
    near = step < 0.005                     # the single step stayed at the alignment
    assert near.sum() >= 25
    # there every |T - J| is 3 up to the blur of the sub-pixel step (< 6 step + texture mismatch)
    np.testing.assert_allclose(r.residual[near], 3.0, atol=0.1)


def smooth_img(w, h, dx=0.0, dy=0.0):
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    xs, ys = xs - dx, ys - dy
    out = 100.0 + 0 * xs
    for (cx, cy, s, a) in [(10.0, 12.0, 5.0, 70.0), (21.0, 18.0, 4.0, -60.0), (15.0, 25.0, 6.0, 40.0),
                           (24.0, 8.0, 3.5, 50.0)]:
        out += a * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * s * s))
    return out


def test_brute_force_ssd_on_tiny_inputs():
    rng = np.random.default_rng(42)
    w = h = 32
    win, hw = 7, 3
    offs = np.arange(-hw, hw + 1, dtype=np.float64)
    for _ in range(6):
        d = rng.uniform(-1.5, 1.5, 2)
        I = smooth_img(w, h)
        J = smooth_img(w, h, d[0], d[1])
        p = rng.uniform(12.0, 19.0, 2)
        r = oracle.track(I, J, p[None], win=win, levels=1, max_iters=200, eps=1e-10, min_eig=0.0)
        assert r.status[0] == oracle.OK
        X, Y = np.meshgrid(p[0] + offs, p[1] + offs)
        T = ndimage.map_coordinates(I, [Y.ravel(), X.ravel()], order=1, mode="nearest")

        def ssd(cands):
            out = np.empty(len(cands))
            for k, (ux, uy) in enumerate(cands):
                Js = ndimage.map_coordinates(J, [Y.ravel() + uy, X.ravel() + ux], order=1, mode="nearest")
                out[k] = np.sum((T - Js) ** 2)
            return out
        # coarse grid (1/16 px over +-2 px), then 1/128 px around the best
        g = np.arange(-32, 33) / 16.0
        cands = np.array([(a, b) for a in g for b in g])
        best = cands[np.argmin(ssd(cands))]
        f = np.arange(-8, 9) / 128.0
        cands = np.array([(best[0] + a, best[1] + b) for a in f for b in f])
        best = cands[np.argmin(ssd(cands))]
        assert np.abs((r.pts[0] - p) - best).max() <= 1.0 / 64.0


def test_scene_shift_equivariance():
    prev, nxt = shifted_pair(200, 260, 5, -3, seed=8, pad=40)
    big_prev, big_nxt = shifted_pair(200 + 8, 260 + 8, 5, -3, seed=8, pad=36)
    # big frames are the same scene moved by (+4, +4) (a multiple of 2^(L-1))
    assert np.array_equal(big_prev[4:204, 4:264], prev)
    rng = np.random.default_rng(3)
    # windows stay (h + 4) 2^(L-1) px clear of the borders, where reflect-101
    # padding differs between the two frame sizes
    pts = synth.uniform_points(rng, 80, 260, 200, border=60)
    r1 = oracle.track(prev, nxt, pts, win=21, levels=3, min_eig=1e-6)
    r2 = oracle.track(big_prev, big_nxt, pts + 4.0, win=21, levels=3, min_eig=1e-6)
    assert np.array_equal(r1.status, r2.status)
    np.testing.assert_allclose(r2.pts - 4.0, r1.pts, atol=1e-9)


def test_swapping_frames_inverts_the_flow():
    d = np.array([6.0, -4.0])
    prev, nxt = shifted_pair(200, 260, 6, -4, seed=12)
    rng = np.random.default_rng(5)
    pts = synth.uniform_points(rng, 80, 260, 200, border=40).astype(np.float64)
    r = oracle.track(nxt, prev, pts + d, win=21, levels=3, max_iters=100, eps=1e-9, min_eig=1e-6)
    ok = r.status == oracle.OK
    np.testing.assert_allclose(r.pts[ok], pts[ok], atol=1e-6)


def test_one_level_and_three_levels_agree_for_subpixel_motion():
    w, h = 64, 64
    I = smooth_img(w, h) + smooth_img(w, h, 30.0, 28.0) - 100.0
    J = smooth_img(w, h, 0.6, -0.4) + smooth_img(w, h, 30.6, 27.6) - 100.0
    pts = np.array([[20.0, 18.5], [40.2, 44.7], [30.5, 30.5]])
    r1 = oracle.track(I, J, pts, win=9, levels=1, max_iters=200, eps=1e-11, min_eig=0.0)
    r3 = oracle.track(I, J, pts, win=9, levels=3, max_iters=200, eps=1e-11, min_eig=0.0)
    assert np.all(r1.status == 0) and np.all(r3.status == 0)
    np.testing.assert_allclose(r1.pts, r3.pts, atol=1e-7)


def test_out_of_bounds_rules():
    # Polynomial frames, motion along x only, so one Gauss-Newton step is the
    # exact motion (no a*dx*dy term): the end point is known in closed form.
    w, h = 160, 120
    I = poly_img(w, h)
    p = np.array([[12.0, 60.0]])
    kw = dict(win=7, levels=1, max_iters=1, eps=1e-12, min_eig=0.0)
    inside = oracle.track(I, poly_img(w, h, -11.0, 0.0), p, **kw)
    assert inside.status[0] == oracle.OK
    np.testing.assert_allclose(inside.pts[0], [1.0, 60.0], atol=1e-9)
    # the step ends at x = -1: inside the level box [-h, W-1+h] but outside
    # the image, so the final check marks it lost
    out = oracle.track(I, poly_img(w, h, -13.0, 0.0), p, **kw)
    assert out.status[0] == oracle.LOST_OOB
    np.testing.assert_allclose(out.pts[0], [-1.0, 60.0], atol=1e-9)
    # a guess that puts the window off the level fails before any sampling
    g = oracle.track(I, I, p, np.array([[-3.0 - 1e-9, 60.0]]), **kw)
    assert g.status[0] == oracle.LOST_OOB and g.iters[0, 0, 0] == 0
    g = oracle.track(I, I, p, np.array([[-3.0, 60.0]]), **kw)      # closed box: on the edge is in
    assert g.iters[0, 0, 0] == 1
    # points outside the image, or not numbers, are lost at entry
    bad = np.array([[-0.5, 60.0], [40.0, 119.5], [np.nan, 50.0], [30.0, np.inf]])
    r = oracle.track(I, I, bad, win=7, levels=2, min_eig=0.0)
    assert np.all(r.status == oracle.LOST_OOB)
    nan_guess = oracle.track(I, I, p, np.array([[np.nan, 60.0]]), **kw)
    assert nan_guess.status[0] == oracle.LOST_OOB


def test_forward_backward_rule():
    p = synth.pair(3)
    fwd = oracle.track(p.prev, p.next, p.pts, win=21, levels=3, min_eig=1e-6)
    ok = fwd.status == oracle.OK
    back = oracle.track(p.next, p.prev, fwd.pts[ok], win=21, levels=3, min_eig=1e-6)
    fbd = np.linalg.norm(back.pts - p.pts[ok].astype(np.float64), axis=1)
    thr = float(np.median(fbd[back.status == 0]))
    r = oracle.track(p.prev, p.next, p.pts, win=21, levels=3, min_eig=1e-6, fb_thresh=thr)
    want = np.where((back.status != 0) | (fbd > thr), oracle.LOST_FB, oracle.OK)
    assert np.array_equal(r.status[ok], want)
    assert np.array_equal(r.pts, fwd.pts)
    # the backward pass contributes its own iteration counts
    assert np.all(r.iters[ok, 1, 0] >= 1)


def test_iteration_cap_is_not_a_failure():
    prev, nxt = shifted_pair(120, 160, 4, 3, seed=6)
    pts = synth.uniform_points(np.random.default_rng(0), 40, 160, 120, border=30)
    r = oracle.track(prev, nxt, pts, win=15, levels=2, max_iters=1, min_eig=1e-6)
    assert np.all(r.iters[r.status == 0, 0, :] == 1)
    assert (r.status == oracle.OK).mean() > 0.8


def test_initial_guess_extends_capture_range():
    d = np.array([44.0, -36.0])
    prev, nxt = shifted_pair(240, 320, 44, -36, seed=21, pad=48)
    pts = synth.uniform_points(np.random.default_rng(9), 60, 320, 240, border=60).astype(np.float64)
    guess = pts + d + np.array([0.7, -0.4])
    r = oracle.track(prev, nxt, pts, guess, win=21, levels=3, max_iters=100, eps=1e-9, min_eig=1e-6)
    ok = r.status == oracle.OK
    assert ok.mean() > 0.9
    np.testing.assert_allclose(r.pts[ok], pts[ok] + d, atol=1e-6)
    # without the guess a 56 px motion is beyond a 3-level, 21x21 capture range
    r0 = oracle.track(prev, nxt, pts, win=21, levels=3, max_iters=100, eps=1e-9, min_eig=1e-6)
    good = (r0.status == 0) & (np.abs(r0.pts - (pts + d)).max(axis=1) < 1e-3)
    assert good.mean() < 0.5


def test_threads_do_not_change_results():
    p = synth.pair(4)
    r1 = oracle.track(p.prev, p.next, p.pts, fb_thresh=1.0, min_eig=1e-6, nthreads=1)
    r8 = oracle.track(p.prev, p.next, p.pts, fb_thresh=1.0, min_eig=1e-6, nthreads=8)
    for a, b in [(r1.pts, r8.pts), (r1.status, r8.status), (r1.residual, r8.residual),
                 (r1.iters, r8.iters), (r1.margins, r8.margins)]:
        assert np.array_equal(a, b)


def test_invalid_arguments_rejected():
    img = np.zeros((40, 40), np.uint8)
    pts = np.zeros((1, 2))
    for kw in [dict(win=4), dict(win=1), dict(win=65), dict(levels=0), dict(levels=9),
               dict(max_iters=0), dict(eps=0.0), dict(levels=5)]:
        with pytest.raises(ValueError):
            oracle.track(img, img, pts, **kw)
