"""FP64 CPU oracle for pyramidal Lucas-Kanade tracking -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library does not, and the
oracle shares no code with it.  ``lk_oracle.c`` holds the definition (plain C,
double precision); this module compiles it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lk_oracle.c")
# LKO_LIB loads another build of the oracle (the mutation tests point it at
# deliberately broken copies to show that the pins catch them)
LIB = os.environ.get("LKO_LIB") or os.path.join(HERE, "liblkoracle.so")

OK, LOST_EIG, LOST_OOB, LOST_FB = 0, 1, 2, 3


class Params(C.Structure):
    _fields_ = [("win", C.c_int32), ("levels", C.c_int32), ("max_iters", C.c_int32),
                ("use_guess", C.c_int32), ("f16_storage", C.c_int32), ("nthreads", C.c_int32),
                ("eps", C.c_double), ("min_eig", C.c_double), ("fb_thresh", C.c_double)]


def build(force: bool = True) -> str:
    """Compile lk_oracle.c into liblkoracle.so (gcc, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-Wall", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("LKO_LIB") and (not os.path.exists(LIB)
                                              or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.lko_round_f16.restype = C.c_double
        L.lko_round_f16.argtypes = [C.c_double]
        L.lko_sample.restype = C.c_double
        L.lko_sample.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_double]
        L.lko_downsample.argtypes = [dp, C.c_int, C.c_int, dp]
        L.lko_scharr.argtypes = [dp, C.c_int, C.c_int, dp, dp]
        L.lko_level_dims.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.lko_build_pyramid.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp]
        trk = [C.c_void_p, C.c_void_p, C.c_int, C.c_int]
        tail = [dp, dp, C.c_int, C.POINTER(Params), dp, C.POINTER(C.c_uint8), dp,
                C.POINTER(C.c_int32), dp]
        L.lko_gftt_response.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.lko_gftt.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                               C.c_int, C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_float)]
        L.lko_track_f64.argtypes = trk + tail
        L.lko_track_u8.argtypes = trk + [C.c_int] + tail
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


# ------------------------------------------------------------- primitives

def round_f16(x: float) -> float:
    return lib().lko_round_f16(float(x))


def level_dims(w: int, h: int, levels: int):
    ws = (C.c_int32 * 8)()
    hs = (C.c_int32 * 8)()
    rc = lib().lko_level_dims(w, h, levels, ws, hs)
    return rc, [(ws[i], hs[i]) for i in range(levels)] if rc == 0 else None


def downsample(img: np.ndarray) -> np.ndarray:
    src = np.ascontiguousarray(img, dtype=np.float64)
    h, w = src.shape
    dst = np.empty(((h + 1) // 2, (w + 1) // 2))
    lib().lko_downsample(_p(src), w, h, _p(dst))
    return dst


def scharr(img: np.ndarray):
    src = np.ascontiguousarray(img, dtype=np.float64)
    h, w = src.shape
    gx = np.empty_like(src)
    gy = np.empty_like(src)
    lib().lko_scharr(_p(src), w, h, _p(gx), _p(gy))
    return gx, gy


def sample(img: np.ndarray, u: float, v: float) -> float:
    src = np.ascontiguousarray(img, dtype=np.float64)
    return lib().lko_sample(_p(src), src.shape[1], src.shape[0], float(u), float(v))


def pyramid(img: np.ndarray, levels: int, f16: bool = False):
    """Levels and gradient planes as lists of 2-D float64 arrays."""
    src = np.ascontiguousarray(img, dtype=np.float64)
    h, w = src.shape
    rc, dims = level_dims(w, h, levels)
    if rc != 0:
        raise ValueError("invalid pyramid shape")
    tot = sum(a * b for a, b in dims)
    im, gx, gy = np.empty(tot), np.empty(tot), np.empty(tot)
    rc = lib().lko_build_pyramid(_p(src), w, h, levels, int(f16), _p(im), _p(gx), _p(gy))
    if rc != 0:
        raise RuntimeError("lko_build_pyramid failed: %d" % rc)
    out_i, out_x, out_y, off = [], [], [], 0
    for (lw, lh) in dims:
        n = lw * lh
        out_i.append(im[off:off + n].reshape(lh, lw))
        out_x.append(gx[off:off + n].reshape(lh, lw))
        out_y.append(gy[off:off + n].reshape(lh, lw))
        off += n
    return out_i, out_x, out_y


# ------------------------------------------------------------- tracker

@dataclass
class Result:
    pts: np.ndarray        # (N, 2) float64
    status: np.ndarray     # (N,) uint8
    residual: np.ndarray   # (N,) float64
    iters: np.ndarray      # (N, 2, L) int32: forward / backward iterations per level
    margins: np.ndarray    # (N, 4) float64: eig (relative), oob (px), conv (px), fb (px)

    @property
    def conv_px(self):
        """Convergence margin in px: | |eta| - eps | for the closest step."""
        return self.margins[:, 2]


def track(prev, nxt, pts, guess=None, *, win=21, levels=3, max_iters=30, eps=0.01,
          min_eig=1e-4, fb_thresh=0.0, f16=False, nthreads=1) -> Result:
    """Track ``pts`` (N x 2, x/y) from ``prev`` to ``nxt``.  uint8 images go
    through the 8-bit entry, anything else through the float64 entry."""
    prev = np.ascontiguousarray(prev)
    nxt = np.ascontiguousarray(nxt)
    if prev.shape != nxt.shape or prev.ndim != 2:
        raise ValueError("frames must be equal 2-D arrays")
    h, w = prev.shape
    p64 = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = p64.shape[0]
    g64 = None if guess is None else np.ascontiguousarray(guess, dtype=np.float64).reshape(-1, 2)
    prm = Params(win, levels, max_iters, int(g64 is not None), int(f16), max(1, int(nthreads)),
                 eps, min_eig, fb_thresh)
    out = np.zeros((n, 2))
    st = np.zeros(n, dtype=np.uint8)
    res = np.zeros(n)
    it = np.zeros((n, 2, levels), dtype=np.int32)
    mg = np.zeros((n, 4))
    L = lib()
    args = (_p(p64), _p(g64), n, C.byref(prm), _p(out), _p(st, C.c_uint8), _p(res),
            _p(it, C.c_int32), _p(mg))
    if prev.dtype == np.uint8:
        rc = L.lko_track_u8(prev.ctypes.data, nxt.ctypes.data, w, h, w, *args)
    else:
        a = np.ascontiguousarray(prev, dtype=np.float64)
        b = np.ascontiguousarray(nxt, dtype=np.float64)
        rc = L.lko_track_f64(a.ctypes.data, b.ctypes.data, w, h, *args)
    if rc == -1:
        raise ValueError("invalid tracker arguments")
    if rc != 0:
        raise RuntimeError("oracle failed: %d" % rc)
    # conv margin is stored relative to eps; expose it in px as well
    mg[:, 2] = mg[:, 2] * eps
    return Result(out, st, res, it, mg)


# ------------------------------------------------------------- GFTT

def gftt_response(img, r=1):
    """Shi-Tomasi response (lambda_min of the raw-Scharr structure tensor)."""
    a = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = a.shape
    out = np.empty((h, w))
    rc = lib().lko_gftt_response(a.ctypes.data, w, h, w, r, _p(out))
    if rc != 0:
        raise ValueError("bad gftt arguments")
    return out


def gftt(img, *, r=1, quality=0.01, min_dist=16, max_corners=200, border=0, occupied=None):
    """Corners (N x 2 float32, integer pixel positions) in selection order."""
    a = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = a.shape
    occ = None if occupied is None or len(occupied) == 0 else np.ascontiguousarray(occupied, dtype=np.float32)
    out = np.zeros((max(max_corners, 1), 2), np.float32)
    n = lib().lko_gftt(a.ctypes.data, w, h, w, r, quality, min_dist, max_corners, border,
                       _p(occ, C.c_float), 0 if occ is None else len(occ), _p(out, C.c_float))
    if n < 0:
        raise ValueError("bad gftt arguments")
    return out[:n]
