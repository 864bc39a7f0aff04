"""Pins of the oracle's decision margins (the distances of every decision to
its threshold, which decide which points the GPU parity rule may treat as
near a threshold).  Each margin is checked against a value fixed in closed
form, not against the oracle's own formula:

* convergence, | |eta_k| - eps | in level px, minimised over all steps: on
  a bilinear-polynomial frame pair J(x) = I(x - d) every Gauss-Newton step
  is known exactly (the error image is grad I . r - a r_x r_y for the
  remaining motion r, so eta = r - a r_x r_y G^-1 sum(grad I));
* out of bounds, the distance of an estimate to the box it must stay in, in
  the level's own px: motion along x only makes one step exact, so the end
  point lands on a chosen x; identical frames keep a point exactly in place;
  a guess puts the coarse window a chosen distance off its level;
* forward-backward, | fb - fb_thresh | in px: identical frames and integer
  shifts bring the backward pass back onto p (fb = 0);
* eigenvalue: pinned in test_oracle_tracker (relative to min_eig).
"""
import numpy as np

import oracle
import synth

A, B, CC, E, X0, Y0 = 0.02, 1.1, -0.6, 120.0, 97.3, 71.9
BIG = np.finfo(np.float64).max


def poly_img(w, h, dx=0.0, dy=0.0):
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    xs, ys = xs - dx, ys - dy
    return A * (xs - X0) * (ys - Y0) + B * xs + CC * ys + E


def analytic_grad(x, y):
    return A * (y - Y0) + B, A * (x - X0) + CC


def closed_form_steps(p, d, win, n):
    """The first n Gauss-Newton steps (level 0, one level, zero start) on the
    polynomial pair J(x) = I(x - d)."""
    hw = (win - 1) // 2
    offs = np.arange(-hw, hw + 1, dtype=np.float64)
    X, Y = np.meshgrid(p[0] + offs, p[1] + offs)
    gx, gy = analytic_grad(X.ravel(), Y.ravel())
    G = np.array([[gx @ gx, gx @ gy], [gx @ gy, gy @ gy]])
    GS = np.linalg.solve(G, np.array([gx.sum(), gy.sum()]))
    acc = np.zeros(2)
    steps = []
    for _ in range(n):
        r = d - acc
        eta = r - A * r[0] * r[1] * GS
        steps.append(eta)
        acc = acc + eta
    return np.array(steps)


def test_convergence_margin_is_the_closest_step_in_px():
    w, h = 200, 160
    I = poly_img(w, h)
    rng = np.random.default_rng(11)
    win = 15
    for _ in range(4):
        d = rng.uniform(1.0, 3.0, 2) * rng.choice([-1, 1], 2)
        J = poly_img(w, h, d[0], d[1])
        p = rng.uniform(60, 130, 2)
        steps = closed_form_steps(p, d, win, 6)
        norms = np.linalg.norm(steps, axis=1)
        assert norms[1] > 10 * norms[2] and norms[1] < 0.3 * norms[0]     # contraction
        # eps just below |eta_2|: step 2 does not converge, step 3 does
        eps = 0.9 * norms[1]
        r = oracle.track(I, J, p[None], win=win, levels=1, max_iters=10, eps=eps, min_eig=0.0)
        assert r.status[0] == oracle.OK and r.iters[0, 0, 0] == 3
        want = min(abs(norms[k] - eps) for k in range(3))
        assert abs(want - 0.1 * norms[1]) < 1e-12          # the minimum is at step 2, not the last step
        np.testing.assert_allclose(r.margins[0, 2], want, rtol=1e-7)
        np.testing.assert_allclose(r.pts[0], p + steps[:3].sum(axis=0), atol=1e-9)
        # one step allowed: the iteration cap ends the level after step 1
        r1 = oracle.track(I, J, p[None], win=win, levels=1, max_iters=1, eps=0.5 * norms[0], min_eig=0.0)
        assert r1.iters[0, 0, 0] == 1
        np.testing.assert_allclose(r1.margins[0, 2], 0.5 * norms[0], rtol=1e-7)


def test_out_of_bounds_margin_final_check_in_px():
    # motion along x only: the single step is exact and ends at x = +1 or -1;
    # the closest decision is the final in-image check, 1 px from x = 0
    w, h = 160, 120
    I = poly_img(w, h)
    p = np.array([[12.0, 60.0]])
    kw = dict(win=7, levels=1, max_iters=1, eps=1e-12, min_eig=0.0)
    for shift, x_end, st in [(-11.0, 1.0, oracle.OK), (-13.0, -1.0, oracle.LOST_OOB)]:
        r = oracle.track(I, poly_img(w, h, shift, 0.0), p, **kw)
        assert r.status[0] == st
        np.testing.assert_allclose(r.pts[0], [x_end, 60.0], atol=1e-9)
        np.testing.assert_allclose(r.margins[0, 1], 1.0, atol=1e-9)


def test_out_of_bounds_margin_identical_frames():
    # identical frames: the point stays exactly in place at every level, so
    # the closest decision is the final check: its distance to the image edge
    img = synth.quantize_u8(synth.texture_canvas(120, 160, 4))
    for p, want in [((160 - 1 - 0.375, 60.5), 0.375), ((40.0, 2.25), 2.25), ((80.5, 119 - 1.5), 1.5)]:
        r = oracle.track(img, img, np.array([p]), win=9, levels=3, min_eig=1e-9)
        assert r.status[0] == oracle.OK
        np.testing.assert_array_equal(r.pts[0], p)
        assert r.margins[0, 1] == want


def test_out_of_bounds_margin_on_a_coarse_level_is_in_that_levels_px():
    # two levels, 7x7 window (h = 3): a guess g puts the level-1 estimate at
    # g / 2; at x = -3.25 the window is 0.25 level-1 px off its level (lost
    # before any step), at x = -2.75 it is 0.25 px inside
    w, h = 160, 120
    I = poly_img(w, h)
    p = np.array([[40.0, 60.0]])
    kw = dict(win=7, levels=2, max_iters=1, eps=1e-12, min_eig=0.0)
    r = oracle.track(I, I, p, np.array([[-6.5, 60.0]]), **kw)
    assert r.status[0] == oracle.LOST_OOB and r.iters[0, 0, 1] == 0
    np.testing.assert_allclose(r.margins[0, 1], 0.25, atol=1e-12)
    np.testing.assert_allclose(r.pts[0], [-6.5, 60.0], atol=1e-12)


def test_forward_backward_margin():
    img = synth.quantize_u8(synth.texture_canvas(160, 200, 6))
    pts = synth.uniform_points(np.random.default_rng(6), 40, 200, 160, border=30)
    # identical frames: both passes stay in place, fb = 0 exactly
    r = oracle.track(img, img, pts, win=11, levels=3, min_eig=1e-6, fb_thresh=0.7)
    ok = r.status == oracle.OK
    assert ok.mean() > 0.9
    assert np.all(r.margins[ok, 3] == 0.7)
    # an integer shift (no noise): forward lands on p + d, backward on p
    pad = 24
    canvas = synth.quantize_u8(synth.texture_canvas(160 + 2 * pad, 200 + 2 * pad, 7))
    d = (3, -2)
    prev = np.ascontiguousarray(canvas[pad:pad + 160, pad:pad + 200])
    nxt = np.ascontiguousarray(canvas[pad - d[1]:pad - d[1] + 160, pad - d[0]:pad - d[0] + 200])
    r = oracle.track(prev, nxt, pts, win=11, levels=3, max_iters=100, eps=1e-9, min_eig=1e-6, fb_thresh=0.7)
    ok = r.status == oracle.OK
    assert ok.mean() > 0.8
    np.testing.assert_allclose(r.pts[ok], pts[ok] + np.array(d, float), atol=1e-6)
    np.testing.assert_allclose(r.margins[ok, 3], 0.7, atol=1e-5)
    # a threshold below the tiny fb distance: every such point is lost, margin fb - thresh
    r2 = oracle.track(img, img, pts, win=11, levels=3, min_eig=1e-6, fb_thresh=1e-30)
    assert np.all(r2.margins[r2.status != oracle.LOST_EIG, 3] == 1e-30)


def test_margins_not_reached_stay_unset():
    img = synth.quantize_u8(synth.texture_canvas(120, 160, 8))
    pts = np.array([[60.0, 60.0], [-1.0, 50.0]])
    r = oracle.track(img, img, pts, win=9, levels=2, min_eig=1e-6)
    # no forward-backward check: no fb margin; a point lost at entry takes no decision at all
    assert np.all(r.margins[:, 3] == BIG)
    assert r.status[1] == oracle.LOST_OOB and np.all(r.margins[1] == [BIG, BIG, BIG * 0.01, BIG])
    # a flat frame: lost at the eigenvalue test before any step or check
    flat = np.full((120, 160), 50, np.uint8)
    r = oracle.track(flat, flat, pts[:1], win=9, levels=2, min_eig=1e-6)
    assert r.status[0] == oracle.LOST_EIG
    assert r.margins[0, 0] == 1.0 and r.margins[0, 1] == BIG and r.margins[0, 3] == BIG
