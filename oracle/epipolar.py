"""Epipolar check of tracked correspondences -- TEST INFRASTRUCTURE (oracle).

The geometric verification the paper applies to temporal correspondences
(Sec. III-C): the points are moved to the normalized image plane with the
camera intrinsics, an essential-matrix model is estimated robustly, and
correspondences farther than 1 px from their epipolar line are rejected.
Written out plainly, as hypothesis-and-score:

* a hypothesis is 8 correspondences (indices drawn by the caller: the
  random draws are inputs);
* its model is the linear eight-point estimate: the 3x3 matrix E with
  x_q^T E x_p = 0 for the 8 samples, x = K^-1 (u, v, 1) (the null vector of
  the 8 x 9 system, from an SVD); a system of rank < 8 gives no model;
* in pixels the model is F = K^-T E K^-1, the epipolar line of p in the later
  frame is l = F (p, 1), and the error of a correspondence is the distance of
  q to that line, |(q, 1) . l| / sqrt(l1^2 + l2^2); it is an inlier when the
  error is at most the threshold;
* the best hypothesis has the most inliers (ties: the lowest index); its
  inliers are the verified correspondences.
In exact arithmetic the pixel-space F does not depend on K (a change of
coordinates applied to both frames cancels in K^-T E K^-1); the intrinsics
condition the linear system.
"""
from __future__ import annotations

import numpy as np

RANK_TOL = 1e-10        # sigma_8 / sigma_1 at or below this: rank < 8, no model


def kinv(fx, fy, cx, cy):
    return np.array([[1.0 / fx, 0.0, -cx / fx], [0.0, 1.0 / fy, -cy / fy], [0.0, 0.0, 1.0]])


def hom(pts):
    pts = np.asarray(pts, np.float64).reshape(-1, 2)
    return np.concatenate([pts, np.ones((len(pts), 1))], axis=1)


def model(p, q, sample, intr):
    """Pixel-space F (unit Frobenius norm) of the eight-point estimate from
    the sampled correspondences, or None when the system has rank < 8."""
    ki = kinv(*intr)
    xp = hom(np.asarray(p, np.float64)[list(sample)]) @ ki.T
    xq = hom(np.asarray(q, np.float64)[list(sample)]) @ ki.T
    a = np.stack([np.kron(xq[i], xp[i]) for i in range(len(sample))])   # row: x_q^T E x_p = a . vec(E)
    _, sv, vt = np.linalg.svd(a)
    if len(sample) != 8 or sv[7] <= RANK_TOL * sv[0]:
        return None
    e = vt[-1].reshape(3, 3)
    f = ki.T @ e @ ki
    return f / np.linalg.norm(f)


def errors(f, p, q):
    """Distance (pixels) of every q to the epipolar line of its p."""
    l = hom(p) @ f.T
    return np.abs(np.sum(hom(q) * l, axis=1)) / np.sqrt(l[:, 0] ** 2 + l[:, 1] ** 2)


def check(p, q, samples, intr, threshold=1.0):
    """Returns (best index or -1, inlier count of every hypothesis (-1: no
    model), inlier mask of the best, per-hypothesis error arrays (None for no
    model))."""
    n = len(p)
    counts, errs = [], []
    for s in samples:
        s = [int(i) for i in s]
        ok = len(s) == 8 and all(0 <= i < n for i in s) and len(set(s)) == 8
        f = model(p, q, s, intr) if ok else None
        if f is None:
            counts.append(-1)
            errs.append(None)
            continue
        e = errors(f, p, q)
        errs.append(e)
        counts.append(int(np.sum(e <= threshold)))
    counts = np.asarray(counts, np.int64)
    valid = [i for i, e in enumerate(errs) if e is not None]
    if not valid:
        return -1, counts, np.zeros(n, bool), errs
    best = max(valid, key=lambda i: (counts[i], -i))
    return best, counts, errs[best] <= threshold, errs
