"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle point by point.

Comparison rule.  Every point falls in exactly one class, decided from the
oracle alone:

* near: a decision of the method was taken within ``band`` of its threshold
  (the oracle's margins: eigenvalue ratio relative to min_eig, distance to
  the out-of-bounds boxes in level px, | |eta| - eps | in level px,
  | fb - fb_thresh | in px; ``conv_band`` may widen the convergence one).
  A float32 path may take the other branch there, so the status is free; a
  point tracked by both must still end within ``loose_tol`` (default
  4 eps: one Gauss-Newton step more or less).
* capped: some level of some pass stopped at the iteration cap, so the end
  point is an iterate, not a converged fixed point, and the float32 iterates
  may differ from the oracle's by up to ``cap_tol``.  End points within
  ``cap_tol``; the same status unless a decision lay within that distance of
  its threshold (a px margin <= cap_tol, or the eigenvalue margin <= band).
  A capped iteration that does not settle (it cycles or wanders, as on tiny
  windows) can also amplify rounding: where the perturbed oracle run shows
  it, the bound widens to that of the unstable class below.
* unstable: the oracle result moves by more than pos_tol / 4 (or changes
  status) when the input points move by 1e-5 px (a second oracle run,
  ``r_perturbed``).  Such a point amplifies input perturbations; a float32
  path perturbs its inputs by about a float32 rounding of the coordinates.
  End points within t = pos_tol + ``amp`` x (the oracle's own shift); the
  same status unless the perturbed oracle run changed it or a px margin is
  <= t.
* strict: everything else.  Same status and, if tracked, the same iteration
  counts per level and pass, an end point within ``pos_tol`` and a residual
  within ``res_abs + res_rel * residual``.

The report gives the size of every class and the largest error in it; the
tests bound the share of points outside the strict class.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle


@dataclass
class Report:
    n: int
    compared_ok: int          # strict points tracked by both
    max_err: float            # strict class
    p99_err: float
    max_res_err: float
    status_mismatch: int      # strict, capped and (stable-status) unstable points
    iter_mismatch: int
    n_near: int
    n_capped: int
    n_unstable: int
    loose_max_err: float      # near class, points tracked by both
    capped_max_err: float
    capped_max_ratio: float   # largest error / allowed error in the capped class (<= 1 passes)
    unstable_max_err: float   # largest error / allowed error in the unstable class (<= 1 passes)

    @property
    def excluded(self) -> int:
        """Points outside the strict class."""
        return self.n_near + self.n_capped + self.n_unstable

    @property
    def nonstrict_share(self) -> float:
        return self.excluded / self.n if self.n else 0.0

    def __str__(self):
        return ("n=%d strict_ok=%d max_err=%.3g p99=%.3g res_err=%.3g status_mm=%d iter_mm=%d | near=%d (max %.3g) "
                "capped=%d (max %.3g, max/allowed %.3g) unstable=%d (max/allowed %.3g)"
                % (self.n, self.compared_ok, self.max_err, self.p99_err, self.max_res_err, self.status_mismatch,
                   self.iter_mismatch, self.n_near, self.loose_max_err, self.n_capped, self.capped_max_err,
                   self.capped_max_ratio, self.n_unstable, self.unstable_max_err))


def near_threshold(r: oracle.Result, band: float, conv_band: float | None = None) -> np.ndarray:
    m = r.margins
    cb = band if conv_band is None else conv_band
    return (m[:, 0] <= band) | (m[:, 1] <= band) | (m[:, 2] <= cb) | (m[:, 3] <= band)


def near_px(r: oracle.Result, band: float, tol) -> np.ndarray:
    """A decision within ``tol`` px (oob, conv, fb) or ``band`` (eigenvalue
    ratio) of its threshold; ``tol`` may be per point."""
    m = r.margins
    return (m[:, 0] <= band) | (m[:, 1] <= tol) | (m[:, 2] <= tol) | (m[:, 3] <= tol)


def capped(r: oracle.Result, max_iters: int) -> np.ndarray:
    """Points where some level of some pass stopped at the iteration cap."""
    return np.any(r.iters >= max_iters, axis=(1, 2))


def oracle_shift(r: oracle.Result, r_perturbed: oracle.Result) -> np.ndarray:
    return np.abs(r.pts - r_perturbed.pts).max(axis=1)


def unstable(r: oracle.Result, r_perturbed: oracle.Result, tol: float) -> np.ndarray:
    """Points whose oracle result changes by more than ``tol`` (or changes
    status) when the inputs move by about one float32 rounding."""
    return (oracle_shift(r, r_perturbed) > tol) | (r.status != r_perturbed.status)


def _max(a) -> float:
    return float(np.max(a)) if np.size(a) else 0.0


def compare(pts, status, residual, iters, r: oracle.Result, *, band=1e-4, pos_tol=1e-3,
            res_abs=1e-3, res_rel=1e-4, check_iters=True, eps=0.01, max_iters=30,
            r_perturbed: oracle.Result | None = None, loose_tol=None, conv_band=None,
            cap_tol=0.05, amp=20.0, check=True) -> Report:
    pts = np.asarray(pts, dtype=np.float64)
    status = np.asarray(status)
    residual = np.asarray(residual, dtype=np.float64)
    n = len(status)
    with np.errstate(invalid="ignore"):
        err = np.abs(pts - r.pts).max(axis=1)
    both = (status == 0) & (r.status == 0)

    near = near_threshold(r, band, conv_band)
    cap = capped(r, max_iters) & ~near
    if r_perturbed is not None:
        unst = unstable(r, r_perturbed, pos_tol / 4) & ~near & ~cap
        shift = oracle_shift(r, r_perturbed)
        flips = r.status != r_perturbed.status
    else:
        unst = np.zeros(n, bool)
        shift = np.zeros(n)
        flips = np.zeros(n, bool)
    strict = ~(near | cap | unst)

    allowed = pos_tol + amp * shift
    cap_allowed = np.maximum(cap_tol, allowed) if r_perturbed is not None else np.full(n, cap_tol)
    # status: free near a threshold, and in the capped / unstable classes
    # where a decision lay within that class's position tolerance of its
    # threshold or the perturbed oracle itself changed it
    st_free = (near | (cap & (flips | near_px(r, band, cap_allowed)))
               | (unst & (flips | near_px(r, band, allowed))))
    st_mm = int(np.sum((status != r.status) & ~st_free))

    s_ok = strict & both
    e = err[s_ok]
    res_err = (np.abs(residual - r.residual) - res_rel * r.residual)[s_ok]
    it_mm = 0
    if check_iters and iters is not None:
        it = np.asarray(iters)
        it_mm = int(np.sum(np.any(it != r.iters, axis=(1, 2)) & s_ok))
    u_ok = unst & both
    c_ok = cap & both
    rep = Report(n=n, compared_ok=int(s_ok.sum()),
                 max_err=_max(e), p99_err=float(np.percentile(e, 99)) if e.size else 0.0,
                 max_res_err=_max(res_err), status_mismatch=st_mm, iter_mismatch=it_mm,
                 n_near=int(near.sum()), n_capped=int(cap.sum()), n_unstable=int(unst.sum()),
                 loose_max_err=_max(err[near & both]), capped_max_err=_max(err[c_ok]),
                 capped_max_ratio=_max(err[c_ok] / cap_allowed[c_ok]),
                 unstable_max_err=_max(err[u_ok] / allowed[u_ok]))
    if not check:
        return rep
    assert st_mm == 0, "status differs on %d points away from thresholds: %s" % (st_mm, rep)
    assert rep.max_err <= pos_tol, "end point differs by %.3g px: %s" % (rep.max_err, rep)
    assert rep.max_res_err <= res_abs, "residual differs: %s" % rep
    assert it_mm == 0, "iteration counts differ on %d points: %s" % (it_mm, rep)
    # near a threshold the float path may take one step more or less
    assert rep.loose_max_err <= (4 * eps if loose_tol is None else loose_tol), \
        "near-threshold point moved %.3g px: %s" % (rep.loose_max_err, rep)
    assert rep.capped_max_ratio <= 1.0, "capped point beyond its bound (%.3g px): %s" % (rep.capped_max_err, rep)
    assert rep.unstable_max_err <= 1.0, "ill-conditioned point beyond its bound: %s" % rep
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
