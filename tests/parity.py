"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle point by point.

Comparison rule.  A point's oracle diagnostics give, for every decision the
method takes, how far the deciding quantity was from its threshold: the
eigenvalue ratio (relative), the distance to the out-of-bounds boxes (px),
| |eta| - eps | over all iterations (px) and | fb - fb_thresh | (px).  Where
one of them is within the band (1e-4 by default) the float32 path may take
the other branch, so that point is only checked loosely.  Points that ran
into the iteration cap at some level never converged, and points whose
oracle result moves when the input moves by a float32 rounding (a second
oracle run on perturbed points) are ill-conditioned; both are excluded too.
Every other point must have the same status as the oracle and, if tracked,
the same iteration counts, an end point within ``pos_tol`` and a residual
within ``res_abs + res_rel * residual``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle


@dataclass
class Report:
    n: int
    excluded: int
    compared_ok: int
    max_err: float
    p99_err: float
    max_res_err: float
    status_mismatch: int
    iter_mismatch: int
    loose_max_err: float
    notes: list = field(default_factory=list)

    def __str__(self):
        return ("n=%d excluded=%d ok=%d max_err=%.3g p99=%.3g res_err=%.3g status_mm=%d iter_mm=%d loose=%.3g"
                % (self.n, self.excluded, self.compared_ok, self.max_err, self.p99_err, self.max_res_err,
                   self.status_mismatch, self.iter_mismatch, self.loose_max_err))


def near_threshold(r: oracle.Result, band: float) -> np.ndarray:
    m = r.margins
    return (m[:, 0] <= band) | (m[:, 1] <= band) | (m[:, 2] <= band) | (m[:, 3] <= band)


def capped(r: oracle.Result, max_iters: int) -> np.ndarray:
    """Points where some level stopped at the iteration cap: the end point is
    not a converged fixed point and may depend on rounding."""
    return np.any(r.iters >= max_iters, axis=(1, 2))


def unstable(r: oracle.Result, r_perturbed: oracle.Result, tol: float) -> np.ndarray:
    """Points whose oracle result changes by more than ``tol`` (or changes
    status) when the inputs move by about one float32 rounding."""
    return (np.abs(r.pts - r_perturbed.pts).max(axis=1) > tol) | (r.status != r_perturbed.status)


def compare(pts, status, residual, iters, r: oracle.Result, *, band=1e-4, pos_tol=1e-3,
            res_abs=1e-3, res_rel=1e-4, check_iters=True, eps=0.01, max_iters=30,
            r_perturbed: oracle.Result | None = None, loose_tol=None, conv_band=None) -> Report:
    pts = np.asarray(pts, dtype=np.float64)
    status = np.asarray(status)
    residual = np.asarray(residual, dtype=np.float64)
    n = len(status)
    m = r.margins
    cb = band if conv_band is None else conv_band
    excl = ((m[:, 0] <= band) | (m[:, 1] <= band) | (m[:, 2] <= cb) | (m[:, 3] <= band)
            | capped(r, max_iters))
    if r_perturbed is not None:
        excl |= unstable(r, r_perturbed, pos_tol / 4)
    keep = ~excl
    st_mm = int(np.sum((status != r.status) & keep))
    both = keep & (status == 0) & (r.status == 0)
    err = np.abs(pts - r.pts).max(axis=1)
    e = err[both]
    res_err = np.abs(residual - r.residual)[both]
    it_mm = 0
    if check_iters and iters is not None:
        it = np.asarray(iters)
        it_mm = int(np.sum(np.any(it != r.iters, axis=(1, 2)) & both))
    near = (m[:, 0] <= band) | (m[:, 1] <= band) | (m[:, 2] <= cb) | (m[:, 3] <= band)
    loose = near & ~capped(r, max_iters) & (status == 0) & (r.status == 0)
    if r_perturbed is not None:
        loose &= ~unstable(r, r_perturbed, pos_tol / 4)
    rep = Report(n=n, excluded=int(excl.sum()), compared_ok=int(both.sum()),
                 max_err=float(e.max()) if e.size else 0.0,
                 p99_err=float(np.percentile(e, 99)) if e.size else 0.0,
                 max_res_err=float((res_err - res_rel * r.residual[both]).max()) if e.size else 0.0,
                 status_mismatch=st_mm, iter_mismatch=it_mm,
                 loose_max_err=float(err[loose].max()) if loose.any() else 0.0)
    assert st_mm == 0, "status differs on %d points away from thresholds: %s" % (st_mm, rep)
    assert rep.max_err <= pos_tol, "end point differs by %.3g px: %s" % (rep.max_err, rep)
    assert rep.max_res_err <= res_abs, "residual differs: %s" % rep
    assert it_mm == 0, "iteration counts differ on %d points: %s" % (it_mm, rep)
    # near a threshold the float path may take one step more or less
    assert rep.loose_max_err <= (4 * eps if loose_tol is None else loose_tol), \
        "near-threshold point moved %.3g px: %s" % (rep.loose_max_err, rep)
    return rep


class GpuTracker:
    """Uploads frames, builds pyramids and tracks through the C ABI."""

    def __init__(self, lk, ctx):
        self.lk = lk
        self.ctx = ctx

    def pyramid(self, img: np.ndarray, levels: int, storage: int):
        import torch
        t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
        h, w = img.shape
        p = self.lk.lk_pyramid_create(self.ctx, w, h, levels, storage)
        self.lk.lk_build_pyramid(self.ctx, p, t)
        return p, t

    def track(self, prev, nxt, pts, guess=None, *, win=21, levels=3, max_iters=30, eps=0.01, min_eig=1e-6,
              fb_thresh=0.0, storage=0, pyr_levels=None):
        import torch
        lk = self.lk
        pl = pyr_levels or levels
        pa, ta = self.pyramid(prev, pl, storage)
        pb, tb = self.pyramid(nxt, pl, storage)
        n = len(pts)
        d_pts = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).cuda()
        d_guess = None if guess is None else torch.from_numpy(np.ascontiguousarray(guess, dtype=np.float32)).cuda()
        prm = lk.make_params(win, levels, max_iters, eps, min_eig, fb_thresh, guess is not None)
        out, st, res, it = lk.outputs(max(n, 1), levels, with_iters=True)
        lk.lk_track(self.ctx, pa, pb, d_pts, d_guess, n, prm, out, st, res, it)
        torch.cuda.synchronize()
        result = (out[:n].cpu().numpy(), st[:n].cpu().numpy(), res[:n].cpu().numpy(), it[:n].cpu().numpy())
        lk.lk_pyramid_destroy(pa)
        lk.lk_pyramid_destroy(pb)
        del ta, tb
        return result
