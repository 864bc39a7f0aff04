"""ctypes binding of liblkmi (include/lk.h) -- argument marshalling only.

Every function named ``lk_*`` here calls the C entry point of the same name;
device arrays are torch tensors on the GPU (their ``data_ptr()`` is passed),
streams are torch streams (their ``cuda_stream`` handle is passed).  All
arithmetic runs in the HIP kernels of liblkmi.so; if the library is missing,
importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# LKMI_LIB: another build of the library (e.g. one with host-side sanitizers)
LIB_PATH = os.environ.get("LKMI_LIB") or os.path.join(PKG, "liblkmi.so")

LK_SUCCESS, LK_ERR_INVALID_ARG, LK_ERR_OUT_OF_MEMORY, LK_ERR_DEVICE = 0, 1, 2, 3
LK_ERR_BUSY, LK_ERR_NOT_READY, LK_ERR_NOT_FOUND, LK_ERR_NOT_IMPLEMENTED = 4, 5, 6, 7
LK_STORAGE_F32, LK_STORAGE_F16 = 0, 1
LK_OK, LK_LOST_EIG, LK_LOST_OOB, LK_LOST_FB = 0, 1, 2, 3
LK_MAX_LEVELS = 8
LK_MAX_WIN = 31
LK_NOALLOC_MAX_PAIRS = 4096

# Every symbol include/lk.h declares (checked by the CPU tests).
ABI_SYMBOLS = (
    "lk_params_default", "lk_params_check", "lk_last_error", "lk_context_create", "lk_context_destroy",
    "lk_context_bytes_in_use", "lk_pyramid_create", "lk_pyramid_destroy", "lk_pyramid_info",
    "lk_build_pyramid", "lk_build_pyramids", "lk_pyramid_read_level", "lk_track", "lk_track_batched",
    "lk_track_batched_noalloc",
    "lk_batch_create", "lk_batch_run", "lk_batch_tune", "lk_batch_config", "lk_batch_destroy",
    "lk_exec_buckets", "lk_exec_table_lookup",
    "lk_server_create", "lk_server_open_stream", "lk_server_submit", "lk_server_poll", "lk_server_close_stream",
    "lk_server_get_stats", "lk_server_fail_next_launches", "lk_server_destroy",
    "lk_detector_create", "lk_detect_corners", "lk_detector_destroy",
    "lk_pool_create", "lk_pool_step", "lk_pool_reset", "lk_pool_destroy",
    "lk_epipolar_check",
)
LK_GFTT_MAX_CORNERS = 4096


class lk_params(C.Structure):
    _fields_ = [("win", C.c_int32), ("levels", C.c_int32), ("max_iters", C.c_int32),
                ("use_guess", C.c_int32), ("eps", C.c_float), ("min_eig", C.c_float),
                ("fb_thresh", C.c_float), ("reserved", C.c_int32)]


class lk_pair(C.Structure):
    _fields_ = [("prev", C.c_void_p), ("next", C.c_void_p), ("pt_offset", C.c_int64),
                ("n", C.c_int32), ("reserved", C.c_int32)]


class lk_batch_desc(C.Structure):
    _fields_ = [("n_builds", C.c_int32), ("build_pyrs", C.POINTER(C.c_void_p)),
                ("build_imgs", C.POINTER(C.c_void_p)), ("build_pitches", C.POINTER(C.c_int32)),
                ("n_pairs", C.c_int32), ("pairs", C.POINTER(lk_pair)), ("d_pts", C.c_void_p),
                ("d_guess", C.c_void_p), ("params", lk_params), ("d_out_pts", C.c_void_p),
                ("d_status", C.c_void_p), ("d_residual", C.c_void_p), ("d_iters", C.c_void_p)]


class lk_exec_config(C.Structure):
    _fields_ = [("persistent", C.c_int32), ("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32),
                ("chunk", C.c_int32), ("waves_per_group", C.c_int32), ("reserved", C.c_int32)]


class lk_server_config(C.Structure):
    _fields_ = [("max_streams", C.c_int32), ("max_points", C.c_int32), ("levels", C.c_int32),
                ("storage", C.c_int32), ("params", lk_params), ("max_batch", C.c_int32),
                ("inflight", C.c_int32), ("queue_depth", C.c_int32), ("reserved", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64)]


class lk_timing(C.Structure):
    _fields_ = [("submit_ns", C.c_uint64), ("launch_ns", C.c_uint64), ("done_ns", C.c_uint64)]


class lk_server_stats(C.Structure):
    _fields_ = [("frames", C.c_uint64), ("batches", C.c_uint64), ("points", C.c_uint64),
                ("resident_bytes", C.c_uint64), ("open_streams", C.c_int32), ("reserved", C.c_int32)]


class lk_gftt_params(C.Structure):
    _fields_ = [("radius", C.c_int32), ("min_dist", C.c_int32), ("max_corners", C.c_int32),
                ("border", C.c_int32), ("quality", C.c_double)]


class lk_gftt_frame(C.Structure):
    _fields_ = [("img", C.c_void_p), ("w", C.c_int32), ("h", C.c_int32), ("pitch", C.c_int32),
                ("n_occupied", C.c_int32), ("occupied", C.c_void_p), ("out_xy", C.c_void_p),
                ("count", C.c_void_p), ("response", C.c_void_p)]


class lk_pool_state(C.Structure):
    _fields_ = [("pts", C.c_void_p), ("ids", C.c_void_p), ("right", C.c_void_p), ("count", C.c_void_p),
                ("next_id", C.c_void_p), ("stats", C.c_void_p)]


class lk_pool_scratch(C.Structure):
    _fields_ = [("t_pts", C.c_void_p), ("t_status", C.c_void_p), ("c_pts", C.c_void_p), ("c_ids", C.c_void_p),
                ("c_count", C.c_void_p), ("s_pts", C.c_void_p), ("s_status", C.c_void_p)]


class lk_pool_frame(C.Structure):
    _fields_ = [("stream", C.c_int32), ("reserved", C.c_int32), ("prev", C.c_void_p), ("next", C.c_void_p),
                ("right", C.c_void_p)]


class lk_epi_set(C.Structure):
    _fields_ = [("p", C.c_void_p), ("q", C.c_void_p), ("n", C.c_int32), ("h", C.c_int32), ("samples", C.c_void_p),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("counts", C.c_void_p),
                ("inliers", C.c_void_p), ("best", C.c_void_p), ("model", C.c_void_p)]


class LKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("lk error %d: %s" % (code, msg))
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblkmi.so is not built (run: python -m paper_2607_01757_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
    res = C.c_int
    sig = {
        "lk_params_default": (lk_params, []),
        "lk_params_check": (res, [C.POINTER(lk_params), i32]),
        "lk_last_error": (C.c_char_p, []),
        "lk_context_create": (res, [i32, u64, C.POINTER(vp)]),
        "lk_context_destroy": (None, [vp]),
        "lk_context_bytes_in_use": (u64, [vp]),
        "lk_pyramid_create": (res, [vp, i32, i32, i32, i32, C.POINTER(vp)]),
        "lk_pyramid_destroy": (res, [vp]),
        "lk_pyramid_info": (res, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "lk_build_pyramid": (res, [vp, vp, vp, i32, vp]),
        "lk_build_pyramids": (res, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(i32), i32, vp]),
        "lk_pyramid_read_level": (res, [vp, vp, i32, vp, vp, vp]),
        "lk_track": (res, [vp, vp, vp, vp, vp, i32, C.POINTER(lk_params), vp, vp, vp, vp, vp]),
        "lk_track_batched": (res, [vp, C.POINTER(lk_pair), i32, vp, vp, C.POINTER(lk_params), vp, vp, vp,
                                   vp, vp]),
        "lk_track_batched_noalloc": (res, [vp, C.POINTER(lk_pair), i32, vp, vp, C.POINTER(lk_params), vp, vp,
                                           vp, vp, vp]),
        "lk_batch_create": (res, [vp, C.POINTER(lk_batch_desc), C.POINTER(lk_exec_config), C.POINTER(vp)]),
        "lk_batch_run": (res, [vp, vp]),
        "lk_batch_tune": (res, [vp, vp, i32, C.POINTER(lk_exec_config), C.POINTER(C.c_float)]),
        "lk_batch_config": (res, [vp, C.POINTER(lk_exec_config)]),
        "lk_batch_destroy": (res, [vp]),
        "lk_exec_buckets": (res, [C.c_int64, i32, C.POINTER(i32), C.POINTER(i32)]),
        "lk_exec_table_lookup": (res, [vp, C.POINTER(lk_batch_desc), C.POINTER(lk_exec_config), C.POINTER(i32)]),
        "lk_server_create": (res, [vp, C.POINTER(lk_server_config), C.POINTER(vp)]),
        "lk_server_open_stream": (res, [vp, i32, i32, C.POINTER(C.c_uint32)]),
        "lk_server_submit": (res, [vp, C.c_uint32, vp, i32, vp, vp, i32, C.POINTER(C.c_uint64)]),
        "lk_server_poll": (res, [vp, C.c_uint64, vp, vp, vp, C.POINTER(i32), C.POINTER(lk_timing)]),
        "lk_server_close_stream": (res, [vp, C.c_uint32]),
        "lk_server_get_stats": (res, [vp, C.POINTER(lk_server_stats)]),
        "lk_server_fail_next_launches": (res, [vp, i32]),
        "lk_server_destroy": (None, [vp]),
        "lk_detector_create": (res, [vp, i32, C.c_int64, C.POINTER(vp)]),
        "lk_detect_corners": (res, [vp, C.POINTER(lk_gftt_frame), i32, C.POINTER(lk_gftt_params), vp]),
        "lk_detector_destroy": (res, [vp]),
        "lk_pool_create": (res, [vp, i32, i32, C.c_int64, C.POINTER(lk_pool_state), C.POINTER(lk_pool_scratch),
                                 C.POINTER(vp)]),
        "lk_pool_step": (res, [vp, C.POINTER(lk_pool_frame), i32, C.POINTER(lk_params), C.POINTER(lk_params),
                               C.POINTER(lk_gftt_params), vp]),
        "lk_pool_reset": (res, [vp, vp]),
        "lk_pool_destroy": (res, [vp]),
        "lk_epipolar_check": (res, [vp, C.POINTER(lk_epi_set), i32, C.c_double, vp]),
    }
    for name, (rt, at) in sig.items():
        f = getattr(lib, name)
        f.restype = rt
        f.argtypes = at
    return lib


lib = _load()


def _check(rc: int):
    if rc != LK_SUCCESS:
        raise LKError(rc, lib.lk_last_error().decode())


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------- C names

def lk_params_default() -> lk_params:
    return lib.lk_params_default()


def lk_params_check(params: lk_params, pyr_levels: int):
    _check(lib.lk_params_check(C.byref(params), pyr_levels))


def lk_last_error() -> str:
    return lib.lk_last_error().decode()


def lk_context_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    _check(lib.lk_context_create(device, hbm_budget_bytes, C.byref(h)))
    return h


def lk_context_destroy(ctx):
    lib.lk_context_destroy(ctx)


def lk_context_bytes_in_use(ctx) -> int:
    return lib.lk_context_bytes_in_use(ctx)


def lk_pyramid_create(ctx, w: int, h: int, levels: int, storage: int = LK_STORAGE_F32):
    p = C.c_void_p()
    _check(lib.lk_pyramid_create(ctx, w, h, levels, storage, C.byref(p)))
    return p


def lk_pyramid_destroy(pyr):
    _check(lib.lk_pyramid_destroy(pyr))


def lk_pyramid_info(pyr):
    v = [C.c_int32() for _ in range(4)]
    _check(lib.lk_pyramid_info(pyr, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def lk_build_pyramid(ctx, pyr, img, pitch: int | None = None, stream=None):
    """img: 2-D uint8 CUDA tensor (rows may be padded: pass the row pitch)."""
    if pitch is None:
        pitch = img.stride(0)
    _check(lib.lk_build_pyramid(ctx, pyr, _ptr(img), pitch, _stream(stream)))


def lk_build_pyramids(ctx, pyrs, imgs, pitches=None, stream=None):
    n = len(pyrs)
    if pitches is None:
        pitches = [im.stride(0) for im in imgs]
    P = (C.c_void_p * n)(*[p.value if isinstance(p, C.c_void_p) else p for p in pyrs])
    I = (C.c_void_p * n)(*[_ptr(im) for im in imgs])
    S = (C.c_int32 * n)(*pitches)
    _check(lib.lk_build_pyramids(ctx, P, I, S, n, _stream(stream)))


def lk_pyramid_read_level(ctx, pyr, level: int, dst, grad=None, stream=None):
    _check(lib.lk_pyramid_read_level(ctx, pyr, level, _ptr(dst), _ptr(grad), _stream(stream)))


def lk_track(ctx, prev, next, pts, guess, n: int, params: lk_params, out_pts, status, residual,
             iters=None, stream=None):
    _check(lib.lk_track(ctx, prev, next, _ptr(pts), _ptr(guess), n, C.byref(params), _ptr(out_pts),
                        _ptr(status), _ptr(residual), _ptr(iters), _stream(stream)))


def lk_track_batched(ctx, pairs, pts, guess, params: lk_params, out_pts, status, residual, iters=None,
                     stream=None):
    """pairs: sequence of (prev, next, pt_offset, n)."""
    arr = (lk_pair * len(pairs))()
    for i, (a, b, off, n) in enumerate(pairs):
        arr[i].prev = a.value if isinstance(a, C.c_void_p) else a
        arr[i].next = b.value if isinstance(b, C.c_void_p) else b
        arr[i].pt_offset = off
        arr[i].n = n
        arr[i].reserved = 0
    _check(lib.lk_track_batched(ctx, arr, len(pairs), _ptr(pts), _ptr(guess), C.byref(params),
                                _ptr(out_pts), _ptr(status), _ptr(residual), _ptr(iters), _stream(stream)))


def lk_track_batched_noalloc(ctx, pairs, pts, guess, params: lk_params, out_pts, status, residual, iters=None,
                             stream=None):
    """lk_track_batched with the batch table in the library's fixed device array."""
    arr = (lk_pair * max(len(pairs), 1))()
    for i, (a, b, off, n) in enumerate(pairs):
        arr[i].prev = a.value if isinstance(a, C.c_void_p) else a
        arr[i].next = b.value if isinstance(b, C.c_void_p) else b
        arr[i].pt_offset = off
        arr[i].n = n
        arr[i].reserved = 0
    _check(lib.lk_track_batched_noalloc(ctx, arr, len(pairs), _ptr(pts), _ptr(guess), C.byref(params),
                                        _ptr(out_pts), _ptr(status), _ptr(residual), _ptr(iters),
                                        _stream(stream)))


def _hv(p):
    return p.value if isinstance(p, C.c_void_p) else p


def lk_batch_create(ctx, build_pyrs, build_imgs, pairs, pts, guess, params: lk_params, out_pts, status,
                    residual, iters=None, config: lk_exec_config | None = None, build_pitches=None):
    """build_pyrs / build_imgs: pyramids rebuilt each run and their uint8
    CUDA frames; pairs: sequence of (prev, next, pt_offset, n)."""
    nb = len(build_pyrs)
    P = (C.c_void_p * max(nb, 1))(*[_hv(p) for p in build_pyrs])
    I = (C.c_void_p * max(nb, 1))(*[_ptr(im) for im in build_imgs])
    pitches = build_pitches if build_pitches is not None else [im.stride(0) for im in build_imgs]
    S = (C.c_int32 * max(nb, 1))(*pitches)
    arr = (lk_pair * max(len(pairs), 1))()
    for i, (a, b, off, n) in enumerate(pairs):
        arr[i].prev, arr[i].next, arr[i].pt_offset, arr[i].n, arr[i].reserved = _hv(a), _hv(b), off, n, 0
    d = lk_batch_desc(nb, P, I, S, len(pairs), arr, _ptr(pts), _ptr(guess), params, _ptr(out_pts), _ptr(status),
                      _ptr(residual), _ptr(iters))
    h = C.c_void_p()
    _check(lib.lk_batch_create(ctx, C.byref(d), C.byref(config) if config is not None else None, C.byref(h)))
    return h


def lk_exec_buckets(mean_pixels: int, mean_points: int):
    rb, kb = C.c_int32(), C.c_int32()
    _check(lib.lk_exec_buckets(int(mean_pixels), int(mean_points), C.byref(rb), C.byref(kb)))
    return rb.value, kb.value


def lk_exec_table_lookup(ctx, pairs, params: lk_params):
    """The tuned shape lk_batch_create(config=None) would take for these
    pairs: (lk_exec_config, found)."""
    arr = (lk_pair * max(len(pairs), 1))()
    for i, (a, b, off, n) in enumerate(pairs):
        arr[i].prev, arr[i].next, arr[i].pt_offset, arr[i].n, arr[i].reserved = _hv(a), _hv(b), off, n, 0
    d = lk_batch_desc(0, None, None, None, len(pairs), arr, None, None, params, None, None, None, None)
    cfg, found = lk_exec_config(), C.c_int32()
    _check(lib.lk_exec_table_lookup(ctx, C.byref(d), C.byref(cfg), C.byref(found)))
    return cfg, bool(found.value)


def lk_batch_run(batch, stream=None):
    _check(lib.lk_batch_run(batch, _stream(stream)))


def lk_batch_tune(batch, reps: int = 5, stream=None):
    cfg = lk_exec_config()
    ms = C.c_float()
    _check(lib.lk_batch_tune(batch, _stream(stream), reps, C.byref(cfg), C.byref(ms)))
    return cfg, ms.value


def lk_batch_config(batch) -> lk_exec_config:
    cfg = lk_exec_config()
    _check(lib.lk_batch_config(batch, C.byref(cfg)))
    return cfg


def lk_batch_destroy(batch):
    _check(lib.lk_batch_destroy(batch))


def lk_server_create(ctx, cfg: lk_server_config):
    h = C.c_void_p()
    _check(lib.lk_server_create(ctx, C.byref(cfg), C.byref(h)))
    return h


def lk_server_open_stream(srv, w: int, h: int) -> int:
    sid = C.c_uint32()
    _check(lib.lk_server_open_stream(srv, w, h, C.byref(sid)))
    return sid.value


def lk_server_submit(srv, sid: int, frame, pts, guess=None) -> int:
    """frame: 2-D uint8 numpy array; pts/guess: float32 numpy arrays N x 2."""
    import numpy as np
    frame = np.ascontiguousarray(frame, dtype=np.uint8)
    p = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 2)
    g = None if guess is None else np.ascontiguousarray(guess, dtype=np.float32).reshape(-1, 2)
    t = C.c_uint64()
    _check(lib.lk_server_submit(srv, sid, frame.ctypes.data, frame.shape[1], p.ctypes.data if len(p) else None,
                                None if g is None else g.ctypes.data, len(p), C.byref(t)))
    return t.value


def lk_server_poll(srv, ticket: int, max_points: int):
    """Returns None while not ready, else (pts, status, residual, timing)."""
    import numpy as np
    out = np.zeros((max_points, 2), np.float32)
    st = np.zeros(max_points, np.uint8)
    res = np.zeros(max_points, np.float32)
    n = C.c_int32()
    tm = lk_timing()
    rc = lib.lk_server_poll(srv, ticket, out.ctypes.data, st.ctypes.data, res.ctypes.data, C.byref(n), C.byref(tm))
    if rc == LK_ERR_NOT_READY:
        return None
    _check(rc)
    k = n.value
    return out[:k], st[:k], res[:k], (tm.submit_ns, tm.launch_ns, tm.done_ns)


def lk_server_close_stream(srv, sid: int):
    _check(lib.lk_server_close_stream(srv, sid))


def lk_server_get_stats(srv) -> lk_server_stats:
    st = lk_server_stats()
    _check(lib.lk_server_get_stats(srv, C.byref(st)))
    return st


def lk_server_fail_next_launches(srv, n: int):
    _check(lib.lk_server_fail_next_launches(srv, n))


def lk_server_destroy(srv):
    lib.lk_server_destroy(srv)


def lk_detector_create(ctx, max_frames: int, max_pixels: int):
    out = C.c_void_p()
    _check(lib.lk_detector_create(ctx, max_frames, max_pixels, C.byref(out)))
    return out


def lk_detect_corners(det, frames, params: lk_gftt_params, stream=None):
    """frames: sequence of dicts with img (2-D uint8 CUDA tensor), out_xy
    (float32 CUDA tensor, max_corners x 2), count (int32 CUDA tensor, 1) and
    optionally occupied (float32 CUDA tensor, n x 2), response (float64 CUDA
    tensor, h x w) and pitch."""
    n = len(frames)
    F = (lk_gftt_frame * max(n, 1))()
    for i, f in enumerate(frames):
        img = f["img"]
        occ = f.get("occupied")
        F[i] = lk_gftt_frame(_ptr(img), img.shape[1], img.shape[0], f.get("pitch", img.stride(0)),
                             0 if occ is None else occ.shape[0], _ptr(occ), _ptr(f["out_xy"]), _ptr(f["count"]),
                             _ptr(f.get("response")))
    _check(lib.lk_detect_corners(det, F, n, C.byref(params), _stream(stream)))


def lk_detector_destroy(det):
    _check(lib.lk_detector_destroy(det))


def lk_pool_create(ctx, n_streams: int, cap: int, max_pixels: int, state: dict, scratch: dict | None = None):
    """state / scratch: dicts of CUDA tensors named like the fields of
    lk_pool_state / lk_pool_scratch (see pool_state, pool_scratch)."""
    st = lk_pool_state(*[_ptr(state.get(k)) for k, _ in lk_pool_state._fields_])
    sc = None if scratch is None else lk_pool_scratch(*[_ptr(scratch[k]) for k, _ in lk_pool_scratch._fields_])
    out = C.c_void_p()
    _check(lib.lk_pool_create(ctx, n_streams, cap, max_pixels, C.byref(st), C.byref(sc) if sc is not None else None,
                              C.byref(out)))
    return out


def lk_pool_step(pool, frames, temporal: lk_params | None, stereo: lk_params | None, detect: lk_gftt_params,
                 stream=None):
    """frames: sequence of (stream index, prev pyramid or None, next pyramid,
    right pyramid or None)."""
    n = len(frames)
    F = (lk_pool_frame * max(n, 1))()
    for i, (sid, prev, nxt, right) in enumerate(frames):
        F[i] = lk_pool_frame(sid, 0, _hv(prev) if prev is not None else None, _hv(nxt),
                             _hv(right) if right is not None else None)
    _check(lib.lk_pool_step(pool, F, n, C.byref(temporal) if temporal is not None else None,
                            C.byref(stereo) if stereo is not None else None, C.byref(detect), _stream(stream)))


def lk_pool_reset(pool, stream=None):
    _check(lib.lk_pool_reset(pool, _stream(stream)))


def lk_pool_destroy(pool):
    _check(lib.lk_pool_destroy(pool))


def lk_epipolar_check(ctx, sets, threshold_px: float = 1.0, stream=None):
    """sets: sequence of dicts with p, q (float32 CUDA tensors, n x 2),
    samples (int32 CUDA tensor, h x 8), intr (fx, fy, cx, cy), counts (int32,
    h), inliers (uint8, n), best (int32, 2) and optionally model (float64, 9)."""
    n = len(sets)
    S = (lk_epi_set * max(n, 1))()
    for i, d in enumerate(sets):
        fx, fy, cx, cy = d["intr"]
        S[i] = lk_epi_set(_ptr(d["p"]), _ptr(d["q"]), d["p"].shape[0], d["samples"].shape[0], _ptr(d["samples"]),
                          fx, fy, cx, cy, _ptr(d["counts"]), _ptr(d["inliers"]), _ptr(d["best"]), _ptr(d.get("model")))
    _check(lib.lk_epipolar_check(ctx, S, n, threshold_px, _stream(stream)))


# ---------------------------------------------------------------- helpers

def pool_state(n_streams: int, cap: int, device="cuda") -> dict:
    """Zeroed state tensors of a pool (every stream empty)."""
    import torch
    return {"pts": torch.zeros((n_streams, cap, 2), dtype=torch.float32, device=device),
            "ids": torch.zeros((n_streams, cap), dtype=torch.int64, device=device),
            "right": torch.zeros((n_streams, cap, 2), dtype=torch.float32, device=device),
            "count": torch.zeros((n_streams,), dtype=torch.int32, device=device),
            "next_id": torch.zeros((n_streams,), dtype=torch.int64, device=device),
            "stats": torch.zeros((n_streams, 4), dtype=torch.int32, device=device)}


def pool_scratch(n_streams: int, cap: int, device="cuda") -> dict:
    """Caller-owned scratch of a pool, readable after each step."""
    import torch
    return {"t_pts": torch.zeros((n_streams, cap, 2), dtype=torch.float32, device=device),
            "t_status": torch.zeros((n_streams, cap), dtype=torch.uint8, device=device),
            "c_pts": torch.zeros((n_streams, cap, 2), dtype=torch.float32, device=device),
            "c_ids": torch.zeros((n_streams, cap), dtype=torch.int64, device=device),
            "c_count": torch.zeros((n_streams,), dtype=torch.int32, device=device),
            "s_pts": torch.zeros((n_streams, cap, 2), dtype=torch.float32, device=device),
            "s_status": torch.zeros((n_streams, cap), dtype=torch.uint8, device=device)}


def gftt_params(radius=1, min_dist=30, max_corners=200, border=0, quality=0.01) -> lk_gftt_params:
    return lk_gftt_params(radius, min_dist, max_corners, border, quality)


def server_config(max_streams=256, max_points=1500, levels=4, storage=LK_STORAGE_F16, params=None,
                  max_batch=256, inflight=2, queue_depth=4, hbm_budget_bytes=64 << 30) -> lk_server_config:
    prm = params if params is not None else make_params(31, levels, 30, 0.01, 1e-6, 1.0)
    return lk_server_config(max_streams, max_points, levels, storage, prm, max_batch, inflight, queue_depth, 0,
                            hbm_budget_bytes)



def make_params(win=21, levels=3, max_iters=30, eps=0.01, min_eig=1e-6, fb_thresh=0.0,
                use_guess=False) -> lk_params:
    return lk_params(win, levels, max_iters, int(use_guess), eps, min_eig, fb_thresh, 0)


def outputs(n: int, levels: int, device="cuda", with_iters=False):
    """Output tensors (points, status, residual, iters) for n points."""
    import torch
    return (torch.empty((n, 2), dtype=torch.float32, device=device),
            torch.empty((n,), dtype=torch.uint8, device=device),
            torch.empty((n,), dtype=torch.float32, device=device),
            torch.empty((n, 2, levels), dtype=torch.int32, device=device) if with_iters else None)
