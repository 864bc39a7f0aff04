"""Seeded synthetic workloads shaped like the paper's camera streams.

The paper's datasets (Table III: EuRoC 752x480 at 20 Hz, NTU-VIRAL 752x480 at
10 Hz, Botanic Garden 960x600, SubT-MRS 640x480) and its keypoint caps (256,
160 on SubT-MRS; Sec. IV) fix the shapes.  No dataset is present, so these
generators stand in for them:

* ``pair``        -- one frame pair: texture, sub-pixel shift, noise, keypoints
                     (the 752x480, 150-keypoint single-pair workload);
* ``StereoSequence`` -- a left/right camera pair flying over a texture canvas
                     with smooth homography motion and per-frame gain;
* ``batch_streams`` -- many independent streams of mixed resolution and
                     keypoint count (the batched workload);
* ``ServingTrace`` -- Poisson arrivals of many streams (the serving workload).

Motion is rendered with ``scipy.ndimage`` resampling, not with any of the
tracker's own arithmetic.  Everything is a pure function of the seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

from .texture import make_rng, quantize_u8, texture_canvas

RESOLUTIONS = ((640, 480), (752, 480), (960, 600), (1280, 720), (1920, 1080))
PAD = 32          # canvas margin so that shifted sampling never reads outside
BORDER = 16       # keypoints are drawn this far inside the frame


@dataclass
class Pair:
    prev: np.ndarray                  # (H, W) uint8
    next: np.ndarray                  # (H, W) uint8
    pts: np.ndarray                   # (N, 2) float32, (x, y)
    gt: np.ndarray | None = None      # (N, 2) float64 true positions in ``next``
    guess: np.ndarray | None = None   # (N, 2) float32 or None
    shift: tuple | None = None

    @property
    def width(self) -> int:
        return int(self.prev.shape[1])

    @property
    def height(self) -> int:
        return int(self.prev.shape[0])


def uniform_points(rng: np.random.Generator, n: int, width: int, height: int,
                   border: int = BORDER) -> np.ndarray:
    lo = np.array([border, border], dtype=np.float64)
    hi = np.array([width - 1 - border, height - 1 - border], dtype=np.float64)
    return rng.uniform(lo, hi, size=(n, 2)).astype(np.float32)


def pair(seed: int, width: int = 752, height: int = 480, n_kp: int = 150,
         max_shift: float = 8.0, noise_sigma: float = 2.0) -> Pair:
    """Texture frame and a copy shifted by d ~ U[-max_shift, max_shift]^2 with
    bilinear resampling plus Gaussian noise on the second frame only."""
    canvas = texture_canvas(height + 2 * PAD, width + 2 * PAD, seed)
    rng = make_rng(0xC1, seed)
    d = rng.uniform(-max_shift, max_shift, size=2)
    pts = uniform_points(rng, n_kp, width, height)
    noise = rng.normal(0.0, noise_sigma, size=(height, width)) if noise_sigma > 0 else 0.0
    # scipy's shift: out(x) = in(x - shift); arrays are (row, col) = (y, x)
    moved = ndimage.shift(canvas, (d[1], d[0]), order=1, mode="nearest", prefilter=False)
    prev = quantize_u8(canvas[PAD:PAD + height, PAD:PAD + width])
    nxt = quantize_u8(moved[PAD:PAD + height, PAD:PAD + width] + noise)
    gt = pts.astype(np.float64) + d[None, :]
    return Pair(prev, nxt, pts, gt, None, (float(d[0]), float(d[1])))


def batch_streams(seed: int, n_streams: int = 64, kp_range=(150, 1500),
                  resolutions=RESOLUTIONS) -> list[Pair]:
    """Independent streams: resolution uniform over ``resolutions``,
    keypoints U[kp_range] (inclusive), single-pair motion per stream."""
    rng = make_rng(0xC3, seed)
    res_idx = rng.integers(0, len(resolutions), size=n_streams)
    kps = rng.integers(kp_range[0], kp_range[1] + 1, size=n_streams)
    out = []
    for s in range(n_streams):
        w, h = resolutions[int(res_idx[s])]
        out.append(pair(seed * 1000 + s, w, h, int(kps[s])))
    return out


# --------------------------------------------------------------------------
# Stereo sequence over a canvas with smooth homography motion
# --------------------------------------------------------------------------

def _sinusoid_path(rng, amplitude, max_rate, n_terms=3, periods=(60.0, 240.0)):
    """Sum of random-phase sinusoids with total amplitude <= ``amplitude`` and
    per-frame rate <= ``max_rate``; returns a callable of the frame index."""
    a = rng.uniform(0.3, 1.0, n_terms)
    a = a / a.sum() * amplitude
    w = 2.0 * np.pi / rng.uniform(*periods, n_terms)
    ph = rng.uniform(0.0, 2.0 * np.pi, n_terms)
    rate = float(np.sum(a * w))
    if rate > max_rate:
        a = a * (max_rate / rate)

    def f(t):
        return float(np.sum(a * np.sin(w * t + ph)))
    return f


@dataclass
class StereoSequence:
    """Left/right cameras over one texture canvas (about 4x the frame area).

    Frame-to-canvas map of the left camera at frame t is the homography
    H_t = [[R(th), c + tr], [p1, p2, 1]] applied to centred frame coordinates;
    the right camera sees the same canvas shifted by a per-sequence disparity.
    Rotation changes by at most ``max_rot_deg`` and translation by at most
    ``max_trans`` px per frame; perspective terms stay below 1e-5.
    """
    seed: int
    width: int = 752
    height: int = 480
    n_frames: int = 1000
    max_rot_deg: float = 3.0
    max_trans: float = 12.0
    gain_range: tuple = (0.9, 1.1)
    gain_mode: str = "smooth"     # "smooth": slowly varying exposure; "iid": independent per frame
    _canvas: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        cw, ch = 2 * self.width, 2 * self.height
        self._canvas = texture_canvas(ch, cw, self.seed)
        rng = make_rng(0xC2, self.seed)
        self.disparity = float(rng.uniform(8.0, 40.0))
        rad = np.deg2rad(self.max_rot_deg) * 0.95
        self._th = _sinusoid_path(rng, np.deg2rad(8.0), rad)
        self._tx = _sinusoid_path(rng, 0.28 * self.width, self.max_trans * 0.9)
        self._ty = _sinusoid_path(rng, 0.22 * self.height, self.max_trans * 0.9)
        self._p1 = _sinusoid_path(rng, 5e-6, 1e-6)
        self._p2 = _sinusoid_path(rng, 5e-6, 1e-6)
        lo, hi = self.gain_range
        if self.gain_mode == "iid":
            self._gains = rng.uniform(lo, hi, size=(self.n_frames, 2))
        else:
            # exposure drifts smoothly inside [lo, hi] (at most ~1% per frame);
            # the right camera follows the left one with a fixed offset
            drift = _sinusoid_path(rng, 1.0, 0.06)
            t = np.arange(self.n_frames)
            s = np.array([drift(k) for k in t])
            left = 0.5 * (lo + hi) + 0.5 * (hi - lo) * s
            right = np.clip(left * rng.uniform(0.98, 1.02), lo, hi)
            self._gains = np.stack([left, right], axis=1)
        self._centre = np.array([cw / 2.0, ch / 2.0])

    def homography(self, t: int, camera: int = 0) -> np.ndarray:
        """3x3 map from frame pixel coordinates (x, y, 1) to canvas (x, y, w)."""
        th = self._th(t)
        c, s = np.cos(th), np.sin(th)
        tx = self._centre[0] + self._tx(t)
        ty = self._centre[1] + self._ty(t)
        h = np.array([[c, -s, tx], [s, c, ty], [self._p1(t), self._p2(t), 1.0]])
        off = self.disparity if camera == 1 else 0.0
        centre = np.array([[1.0, 0.0, off - self.width / 2.0],
                           [0.0, 1.0, -self.height / 2.0],
                           [0.0, 0.0, 1.0]])
        return h @ centre

    @staticmethod
    def _apply(hm: np.ndarray, pts: np.ndarray) -> np.ndarray:
        p = np.concatenate([pts.astype(np.float64), np.ones((len(pts), 1))], axis=1) @ hm.T
        return p[:, :2] / p[:, 2:3]

    def frame(self, t: int, camera: int = 0) -> np.ndarray:
        ys, xs = np.mgrid[0:self.height, 0:self.width].astype(np.float64)
        hm = self.homography(t, camera)
        den = hm[2, 0] * xs + hm[2, 1] * ys + hm[2, 2]
        cx = (hm[0, 0] * xs + hm[0, 1] * ys + hm[0, 2]) / den
        cy = (hm[1, 0] * xs + hm[1, 1] * ys + hm[1, 2]) / den
        img = ndimage.map_coordinates(self._canvas, [cy, cx], order=1, mode="nearest",
                                      prefilter=False)
        return quantize_u8(img * self._gains[t % self.n_frames, camera])

    def temporal_gt(self, t: int, pts: np.ndarray) -> np.ndarray:
        """True positions in left frame t of left-frame t-1 points."""
        return self._apply(np.linalg.inv(self.homography(t, 0)) @ self.homography(t - 1, 0), pts)

    def stereo_gt(self, t: int, pts: np.ndarray) -> np.ndarray:
        """True positions in right frame t of left-frame t points."""
        return self._apply(np.linalg.inv(self.homography(t, 1)) @ self.homography(t, 0), pts)

    def points(self, t: int, n: int) -> np.ndarray:
        return uniform_points(make_rng(0xC2, self.seed, t), n, self.width, self.height)


# --------------------------------------------------------------------------
# Serving: Poisson arrivals from many streams
# --------------------------------------------------------------------------

@dataclass
class StreamSpec:
    stream: int
    width: int
    height: int
    n_kp: int
    rate_hz: float


@dataclass
class ServingTrace:
    """``n_streams`` cameras, each issuing frames as a Poisson process with
    rate U[20, 30] Hz; resolution fixed per stream from ``resolutions``;
    keypoints per frame U[150, 1500]."""
    seed: int
    n_streams: int = 256
    duration_s: float = 12.0
    rate_range: tuple = (20.0, 30.0)
    kp_range: tuple = (150, 1500)
    resolutions: tuple = RESOLUTIONS

    def __post_init__(self):
        rng = make_rng(0xC5, self.seed)
        res = rng.integers(0, len(self.resolutions), size=self.n_streams)
        kps = rng.integers(self.kp_range[0], self.kp_range[1] + 1, size=self.n_streams)
        rates = rng.uniform(*self.rate_range, size=self.n_streams)
        self.streams = [StreamSpec(s, *self.resolutions[int(res[s])], int(kps[s]), float(rates[s]))
                        for s in range(self.n_streams)]
        events = []
        for sp in self.streams:
            t = rng.exponential(1.0 / sp.rate_hz)
            k = 0
            while t < self.duration_s:
                events.append((t, sp.stream, k))
                t += rng.exponential(1.0 / sp.rate_hz)
                k += 1
        events.sort()
        self.events = events          # (time s, stream, frame index)


class FramePool:
    """A few pre-rendered frames per resolution, so that a long trace can be
    replayed without rendering every frame.  Frame k of a stream is pool
    entry (stream + k) mod size of its resolution: consecutive frames of a
    stream differ by a sub-pixel shift of up to 2 * max_shift px."""

    def __init__(self, seed: int, resolutions=RESOLUTIONS, per_res: int = 4,
                 max_shift: float = 8.0, noise_sigma: float = 2.0):
        self.frames: dict[tuple, list[np.ndarray]] = {}
        for ri, (w, h) in enumerate(resolutions):
            canvas = texture_canvas(h + 2 * PAD, w + 2 * PAD, seed * 100 + ri)
            rng = make_rng(0xC50, seed, ri)
            lst = []
            for _ in range(per_res):
                d = rng.uniform(-max_shift, max_shift, size=2)
                moved = ndimage.shift(canvas, (d[1], d[0]), order=1, mode="nearest", prefilter=False)
                noise = rng.normal(0.0, noise_sigma, size=(h, w))
                lst.append(quantize_u8(moved[PAD:PAD + h, PAD:PAD + w] + noise))
            self.frames[(w, h)] = lst

    def frame(self, width: int, height: int, stream: int, k: int) -> np.ndarray:
        lst = self.frames[(width, height)]
        return lst[(stream + k) % len(lst)]


# --------------------------------------------------------------------------
# Two-view correspondences for the epipolar check
# --------------------------------------------------------------------------

@dataclass
class TwoView:
    p: np.ndarray          # (n, 2) float32, earlier frame (pixels)
    q: np.ndarray          # (n, 2) float32, later frame
    intr: tuple            # (fx, fy, cx, cy)
    outlier: np.ndarray    # (n,) bool: q replaced by a point off its epipolar line


def _rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    return (np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]]) @ np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
            @ np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]]))


def two_view(seed: int, n: int, width: int = 752, height: int = 480, outlier_frac: float = 0.2,
             noise_px: float = 0.3, forward: bool = False) -> TwoView:
    """Points of a 3D scene (depth 4..20 units, in front of both cameras)
    seen by a camera and by the same camera after a small rotation and a
    translation (sideways, or along the axis with `forward`), projected with
    pinhole intrinsics, Gaussian pixel noise on both views; a fraction of the
    later positions is replaced by uniform random pixels (outliers)."""
    rng = make_rng(0xE9, seed)
    f = 0.6 * width
    intr = (f, f * rng.uniform(0.98, 1.02), width / 2.0 + rng.uniform(-8, 8), height / 2.0 + rng.uniform(-8, 8))
    K = np.array([[intr[0], 0, intr[2]], [0, intr[1], intr[3]], [0, 0, 1.0]])
    R = _rot(*rng.uniform(-0.03, 0.03, 3))
    t = np.array([0.0, 0.0, 1.0]) if forward else np.concatenate([rng.uniform(-0.5, 0.5, 2), rng.uniform(-0.1, 0.1, 1)])
    # pixels of the earlier view with random depths, lifted to 3D
    u = np.column_stack([rng.uniform(0, width - 1, n), rng.uniform(0, height - 1, n), np.ones(n)])
    X = (np.linalg.inv(K) @ u.T).T * rng.uniform(4.0, 20.0, (n, 1))
    X2 = (R @ X.T).T + t
    x2 = (K @ X2.T).T
    p = u[:, :2] + rng.normal(0.0, noise_px, (n, 2))
    q = x2[:, :2] / x2[:, 2:] + rng.normal(0.0, noise_px, (n, 2))
    out = rng.random(n) < outlier_frac
    q[out] = np.column_stack([rng.uniform(0, width - 1, out.sum()), rng.uniform(0, height - 1, out.sum())])
    return TwoView(p.astype(np.float32), q.astype(np.float32), tuple(float(v) for v in intr), out)


def ransac_samples(seed: int, n: int, h: int, k: int = 8) -> np.ndarray:
    """h draws of k distinct indices in [0, n) (int32, h x k)."""
    rng = make_rng(0xE8, seed)
    if n < k:
        return np.zeros((h, k), np.int32)
    return np.stack([rng.choice(n, k, replace=False) for _ in range(h)]).astype(np.int32).reshape(h, k)
