"""Pins of the oracle's building blocks against library routines and closed
forms (nothing here re-types the oracle's own formulas).

* pyramid step  -> scipy.ndimage.correlate1d(mode='mirror') + decimation
                   ('mirror' is reflect-101), and exactness on bilinear
                   polynomials;
* Scharr        -> scipy.ndimage.correlate(mode='mirror') and the exact
                   derivative of a bilinear polynomial;
* bilinear      -> scipy.ndimage.map_coordinates(order=1, mode='nearest');
* binary16      -> numpy's float16 conversion (round to nearest even);
* level sizes   -> ceil(n / 2) per level, coarsest level >= 4 px.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle

BINOM = np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16.0


def scipy_downsample(img):
    t = ndimage.correlate1d(img, BINOM, axis=1, mode="mirror")
    t = ndimage.correlate1d(t, BINOM, axis=0, mode="mirror")
    return t[::2, ::2]


@pytest.mark.parametrize("shape", [(7, 9), (8, 8), (33, 50), (61, 47), (480, 752)])
def test_downsample_matches_scipy(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.uniform(0, 255, size=shape)
    got = oracle.downsample(img)
    want = scipy_downsample(img)
    assert got.shape == ((shape[0] + 1) // 2, (shape[1] + 1) // 2)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)


def test_downsample_uint8_levels_exact():
    # an 8-bit image blurred by the binomial kernel is a dyadic rational: exact
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(40, 58)).astype(np.float64)
    assert np.array_equal(oracle.downsample(img), scipy_downsample(img))


def poly(a, b, c, e, x0, y0, xs, ys):
    return a * (xs - x0) * (ys - y0) + b * xs + c * ys + e


def test_downsample_exact_on_bilinear_polynomial():
    # binomial blur preserves span{1, x, y, xy}; the next level is the same
    # polynomial at (2x, 2y).  Reflect-101 contaminates 2 samples at each edge.
    h, w = 40, 56
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    img = poly(0.03, 1.7, -0.8, 90.0, 11.3, 7.9, xs, ys)
    got = oracle.downsample(img)
    ys2, xs2 = np.mgrid[0:got.shape[0], 0:got.shape[1]].astype(np.float64)
    want = poly(0.03, 1.7, -0.8, 90.0, 11.3, 7.9, 2 * xs2, 2 * ys2)
    np.testing.assert_allclose(got[1:-1, 1:-1], want[1:-1, 1:-1], atol=1e-10)


SCHARR_X = np.array([[-3, 0, 3], [-10, 0, 10], [-3, 0, 3]], dtype=np.float64) / 32.0


@pytest.mark.parametrize("shape", [(5, 6), (31, 17), (64, 80)])
def test_scharr_matches_scipy(shape):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    img = rng.uniform(0, 255, size=shape)
    gx, gy = oracle.scharr(img)
    np.testing.assert_allclose(gx, ndimage.correlate(img, SCHARR_X, mode="mirror"), atol=1e-11)
    np.testing.assert_allclose(gy, ndimage.correlate(img, SCHARR_X.T, mode="mirror"), atol=1e-11)


def test_scharr_exact_derivative_of_bilinear_polynomial():
    h, w = 30, 45
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    a, b, c = 0.05, 1.3, -2.1
    img = poly(a, b, c, 100.0, 4.0, 9.0, xs, ys)
    gx, gy = oracle.scharr(img)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(gx[inner], (a * (ys - 9.0) + b)[inner], atol=1e-11)
    np.testing.assert_allclose(gy[inner], (a * (xs - 4.0) + c)[inner], atol=1e-11)


def test_bilinear_matches_map_coordinates():
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 255, size=(13, 19))
    us = np.concatenate([rng.uniform(-3, 21, 300), [0.0, 18.0, -0.5, 18.5, 7.0]])
    vs = np.concatenate([rng.uniform(-3, 15, 300), [0.0, 12.0, 12.5, -0.25, 3.0]])
    want = ndimage.map_coordinates(img, [vs, us], order=1, mode="nearest")
    got = np.array([oracle.sample(img, u, v) for u, v in zip(us, vs)])
    np.testing.assert_allclose(got, want, atol=1e-10)


def test_bilinear_reproduces_bilinear_polynomial():
    ys, xs = np.mgrid[0:20, 0:20].astype(np.float64)
    img = poly(0.2, -1.0, 3.0, 5.0, 2.0, 1.0, xs, ys)
    rng = np.random.default_rng(3)
    for _ in range(50):
        u, v = rng.uniform(0, 19, 2)
        assert abs(oracle.sample(img, u, v) - poly(0.2, -1.0, 3.0, 5.0, 2.0, 1.0, u, v)) < 1e-11


def test_round_f16_matches_numpy():
    rng = np.random.default_rng(2)
    vals = np.concatenate([
        rng.uniform(-300, 300, 20000),
        rng.uniform(-1e-4, 1e-4, 2000),                    # subnormal range of binary16
        np.arange(0, 256) + 0.5 * 2.0 ** -3,               # exact ties in [128, 256)
        np.arange(0, 128) + 0.5 * 2.0 ** -4,               # exact ties in [64, 128)
        [0.0, -0.0, 65504.0, 65519.0, 2.0 ** -24, 3 * 2.0 ** -25, 2.0 ** -25],
    ])
    got = np.array([oracle.round_f16(v) for v in vals])
    want = vals.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, want)


def test_level_dims():
    rc, dims = oracle.level_dims(752, 480, 4)
    assert rc == 0 and dims == [(752, 480), (376, 240), (188, 120), (94, 60)]
    rc, dims = oracle.level_dims(1921, 1081, 3)
    assert rc == 0 and dims == [(1921, 1081), (961, 541), (481, 271)]
    assert oracle.level_dims(30, 30, 4)[0] == 0      # coarsest 4x4
    assert oracle.level_dims(30, 30, 5)[0] != 0      # coarsest 2x2 rejected
    assert oracle.level_dims(640, 480, 9)[0] != 0    # more than 8 levels rejected


def test_pyramid_f16_storage_matches_numpy_rounding():
    # stored levels >= 1 are binary16 and each level is built from the stored
    # previous one; gradients are computed from stored levels and rounded.
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, size=(48, 70)).astype(np.float64)
    lv, gx, gy = oracle.pyramid(img, 3, f16=True)
    ref = [img]
    for _ in range(2):
        ref.append(scipy_downsample(ref[-1]).astype(np.float16).astype(np.float64))
    for l in range(3):
        assert np.array_equal(lv[l], ref[l])
        rx = ndimage.correlate(ref[l], SCHARR_X, mode="mirror").astype(np.float16).astype(np.float64)
        ry = ndimage.correlate(ref[l], SCHARR_X.T, mode="mirror").astype(np.float16).astype(np.float64)
        assert np.array_equal(gx[l], rx)
        assert np.array_equal(gy[l], ry)


def test_pyramid_f32_levels_match_scipy_chain():
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, size=(64, 90)).astype(np.float64)
    lv, gx, gy = oracle.pyramid(img, 4)
    ref = img
    for l in range(1, 4):
        ref = scipy_downsample(ref)
        np.testing.assert_allclose(lv[l], ref, atol=1e-11)
    np.testing.assert_allclose(gx[3], ndimage.correlate(ref, SCHARR_X, mode="mirror"), atol=1e-11)
