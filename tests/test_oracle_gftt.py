"""Pins of the oracle's Shi-Tomasi (GFTT) detector.

* response vs scipy (raw Scharr via ndimage.correlate, block sums via
  ndimage.correlate with ones, mode='mirror' = reflect-101) and the smaller
  eigenvalue from numpy.linalg.eigvalsh;
* selection properties that fix the greedy rule without re-typing it:
  every corner is a 3x3 local maximum above quality * max, corners are at
  least min_dist apart, the first is the global maximum, and every
  candidate left out lies within min_dist of a corner of higher rank;
* equivariance under mirroring and transposing the frame;
* occupied points, empty and degenerate inputs.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth

SCHARR = np.array([[-3, 0, 3], [-10, 0, 10], [-3, 0, 3]], dtype=np.float64)


def ref_response(img, r):
    f = img.astype(np.float64)
    gx = ndimage.correlate(f, SCHARR, mode="mirror")
    gy = ndimage.correlate(f, SCHARR.T, mode="mirror")
    k = np.ones((2 * r + 1, 2 * r + 1))
    a = ndimage.correlate(gx * gx, k, mode="mirror")
    b = ndimage.correlate(gx * gy, k, mode="mirror")
    c = ndimage.correlate(gy * gy, k, mode="mirror")
    m = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    return np.linalg.eigvalsh(m)[..., 0]


@pytest.mark.parametrize("r", [0, 1, 2])
def test_response_matches_scipy_and_eigvalsh(r):
    img = synth.quantize_u8(synth.texture_canvas(61, 83, 5 + r))
    got = oracle.gftt_response(img, r)
    want = ref_response(img, r)
    # eigvalsh carries rounding of the order of the larger eigenvalue
    scale = ndimage.correlate(img.astype(np.float64), SCHARR, mode="mirror") ** 2
    scale = scale.max() * (2 * r + 1) ** 2
    np.testing.assert_allclose(got, want, atol=1e-9 * scale)


def rank_key(R, w, pts):
    return [(-R[int(y), int(x)], int(y) * w + int(x)) for x, y in pts]


@pytest.mark.parametrize("seed,min_dist,cap", [(0, 16, 200), (1, 8, 60), (2, 30, 500), (3, 1, 100)])
def test_selection_properties(seed, min_dist, cap):
    img = synth.quantize_u8(synth.texture_canvas(120, 160, seed))
    q = 0.02
    c = oracle.gftt(img, quality=q, min_dist=min_dist, max_corners=cap)
    R = oracle.gftt_response(img, 1)
    h, w = R.shape
    thr = q * R.max()
    assert 0 < len(c) <= cap
    keys = rank_key(R, w, c)
    assert keys == sorted(keys)                                  # selection order = rank order
    # candidates: 3x3 local maxima above the threshold
    peak = R >= ndimage.maximum_filter(R, size=3, mode="constant", cval=-np.inf)
    cand = np.argwhere(peak & (R > thr) & (R > 0))[:, ::-1]        # (x, y)
    cset = {(int(x), int(y)) for x, y in cand}
    for x, y in c:
        assert (int(x), int(y)) in cset
    first = min(rank_key(R, w, cand))
    assert keys[0] == first                                      # the global maximum comes first
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    assert d2.min() >= min_dist ** 2
    if len(c) < cap:
        # greedy maximality: a left-out candidate is close to a better corner
        sel = {(int(x), int(y)) for x, y in c}
        for (x, y) in cset - sel:
            k = (-R[y, x], y * w + x)
            near = [(cx, cy) for cx, cy in c if (cx - x) ** 2 + (cy - y) ** 2 < min_dist ** 2
                    and rank_key(R, w, [(cx, cy)])[0] < k]
            assert near, (x, y)


def test_mirror_and_transpose_equivariance():
    img = synth.quantize_u8(synth.texture_canvas(96, 128, 9))
    base = {tuple(p) for p in oracle.gftt(img, min_dist=5, max_corners=1000).astype(int).tolist()}
    w, h = 128, 96
    mir = {(w - 1 - x, y) for x, y in oracle.gftt(img[:, ::-1].copy(), min_dist=5, max_corners=1000).astype(int).tolist()}
    tr = {(y, x) for x, y in oracle.gftt(img.T.copy(), min_dist=5, max_corners=1000).astype(int).tolist()}
    # ties between equal responses may resolve differently after mirroring;
    # the sets of strong corners agree
    assert len(base ^ mir) <= 0.05 * len(base)
    assert len(base ^ tr) <= 0.05 * len(base)


def test_isolated_square_gives_its_four_corners():
    img = np.full((64, 64), 30, np.uint8)
    img[20:40, 24:44] = 220
    c = oracle.gftt(img, min_dist=4, max_corners=4)
    assert len(c) == 4
    xs, ys = sorted(set(c[:, 0])), sorted(set(c[:, 1]))
    assert len(xs) == 2 and len(ys) == 2
    # symmetric about the square's centre (33.5, 29.5)
    assert xs[0] + xs[1] == 24 + 43 and ys[0] + ys[1] == 20 + 39
    assert abs(xs[0] - 24) <= 1 and abs(ys[0] - 20) <= 1


def test_occupied_points_block_their_neighbourhood():
    img = synth.quantize_u8(synth.texture_canvas(120, 160, 4))
    free = oracle.gftt(img, min_dist=12, max_corners=50)
    occ = free[:10]
    c = oracle.gftt(img, min_dist=12, max_corners=50, occupied=occ)
    d2 = ((c[:, None, :] - occ[None, :, :]) ** 2).sum(-1)
    assert d2.min() >= 144
    assert not ({tuple(p) for p in c.tolist()} & {tuple(p) for p in occ.tolist()})


def test_degenerate_inputs():
    flat = np.full((40, 50), 77, np.uint8)
    assert len(oracle.gftt(flat)) == 0
    img = synth.quantize_u8(synth.texture_canvas(40, 50, 1))
    assert len(oracle.gftt(img, max_corners=0)) == 0
    c = oracle.gftt(img, border=10, min_dist=1, max_corners=1000)
    assert len(c) > 0
    assert np.all((c[:, 0] >= 10) & (c[:, 1] >= 10) & (c[:, 0] < 40) & (c[:, 1] < 30))
    with pytest.raises(ValueError):
        oracle.gftt(img, quality=-1.0)
