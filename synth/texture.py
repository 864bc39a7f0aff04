"""Seeded procedural textures standing in for the camera images of the paper's
datasets (EuRoC 752x480, Botanic Garden 960x600, SubT-MRS 640x480; Table III).

A texture is 128 + a sum of Gaussian blobs + two octaves of value noise.  The
blob density is 400 blobs per 752x480 frame, kept constant on larger canvases.

This module draws images only.  It holds none of the tracker's arithmetic:
no pyramid, no gradient operator, no bilinear sampling.  Resampling for
synthetic motion is done with scipy.ndimage (see ``workloads``).
"""
from __future__ import annotations

import numpy as np

BLOBS_PER_PX = 400.0 / (752 * 480)
SIGMA_RANGE = (3.0, 20.0)
AMP_RANGE = (-80.0, 80.0)
# value-noise octaves: (lattice spacing px, amplitude gray levels)
NOISE_OCTAVES = ((32, 16.0), (16, 8.0))


def make_rng(*seed_parts: int) -> np.random.Generator:
    """PCG64 generator from a tuple of non-negative integers."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed_parts))))


def _smoothstep(t: np.ndarray) -> np.ndarray:
    return t * t * (3.0 - 2.0 * t)


def value_noise(height: int, width: int, spacing: int, rng: np.random.Generator) -> np.ndarray:
    """Lattice noise: U[-1,1] values every ``spacing`` px, smoothstep blend."""
    ny = height // spacing + 2
    nx = width // spacing + 2
    lat = rng.uniform(-1.0, 1.0, size=(ny, nx))
    ys = np.arange(height, dtype=np.float64) / spacing
    xs = np.arange(width, dtype=np.float64) / spacing
    iy = np.floor(ys).astype(np.int64)
    ix = np.floor(xs).astype(np.int64)
    ty = _smoothstep(ys - iy)[:, None]
    tx = _smoothstep(xs - ix)[None, :]
    v00 = lat[iy][:, ix]
    v10 = lat[iy][:, ix + 1]
    v01 = lat[iy + 1][:, ix]
    v11 = lat[iy + 1][:, ix + 1]
    top = v00 + (v10 - v00) * tx
    bot = v01 + (v11 - v01) * tx
    return top + (bot - top) * ty


def texture_canvas(height: int, width: int, seed: int) -> np.ndarray:
    """Float64 texture of shape (height, width), values roughly in [0, 255]."""
    rng = make_rng(0x7E47, seed)
    img = np.full((height, width), 128.0)
    n_blobs = max(1, int(round(BLOBS_PER_PX * height * width)))
    cx = rng.uniform(0, width, n_blobs)
    cy = rng.uniform(0, height, n_blobs)
    sig = rng.uniform(*SIGMA_RANGE, n_blobs)
    amp = rng.uniform(*AMP_RANGE, n_blobs)
    for k in range(n_blobs):
        r = int(np.ceil(4.0 * sig[k]))
        x0, x1 = max(0, int(cx[k]) - r), min(width, int(cx[k]) + r + 1)
        y0, y1 = max(0, int(cy[k]) - r), min(height, int(cy[k]) + r + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        s2 = 2.0 * sig[k] * sig[k]
        gx = np.exp(-((np.arange(x0, x1) - cx[k]) ** 2) / s2)
        gy = np.exp(-((np.arange(y0, y1) - cy[k]) ** 2) / s2)
        img[y0:y1, x0:x1] += amp[k] * np.outer(gy, gx)
    for spacing, a in NOISE_OCTAVES:
        img += a * value_noise(height, width, spacing, rng)
    return img


def quantize_u8(img: np.ndarray) -> np.ndarray:
    """Round half to even, clip to [0, 255], uint8."""
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)
