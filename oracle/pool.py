"""Track pool lifecycle of one camera stream -- TEST INFRASTRUCTURE (oracle).

The steps the front-end takes after the tracker, written out plainly:

* features associated from frame t-1 to frame t keep their track identity;
  the others end (Sec. III-C, feature matching: matched features retain their
  cached identities, the cache is then refreshed with the current features);
* unmatched new detections of frame t start new tracks (same passage), here
  Shi-Tomasi corners kept at least the minimum distance away from every
  surviving track, in rank order, until the pool holds ``target`` points;
* in stereo mode only the points that pass the cross-camera optical-flow
  check enter the temporal pool (Sec. V, the Botanic Garden discussion); in
  mono mode there is no gate and the pool is carried over by temporal
  tracking alone (the same passage's "forward rate").

Positions in the pool are binary32 (what the tracker returns); identities are
64-bit integers, dense per stream in the order tracks are admitted.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import OK, gftt, track

NEW = -1       # identity placeholder of a candidate not admitted yet


@dataclass
class Pool:
    pts: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.float32))
    ids: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    right: np.ndarray | None = None     # stereo positions of the pool points (stereo mode)
    next_id: int = 0


def carry(ids, tracked_pts, status):
    """Survivors of the temporal pass in pool order: a point survives when its
    tracking status is OK; it keeps its identity and moves to its end point."""
    ids = np.asarray(ids, np.int64)
    keep = np.asarray(status) == OK
    return np.asarray(tracked_pts, np.float32)[keep].reshape(-1, 2), ids[keep]


def candidates(img, surv_pts, surv_ids, target, *, r=1, quality=0.01, min_dist=30, border=0):
    """Survivors followed by new corners of ``img``: corners at least
    ``min_dist`` from every survivor (and from each other), in rank order,
    until there are ``target`` points (no new corner when the survivors
    already fill it).  New candidates carry the NEW identity."""
    s = len(surv_ids)
    room = max(int(target) - s, 0)
    new = gftt(img, r=r, quality=quality, min_dist=min_dist, max_corners=room, border=border,
               occupied=surv_pts if s else None)
    pts = np.concatenate([np.asarray(surv_pts, np.float32).reshape(-1, 2), new]).astype(np.float32)
    ids = np.concatenate([np.asarray(surv_ids, np.int64), np.full(len(new), NEW, np.int64)])
    return pts, ids


def commit(cand_pts, cand_ids, next_id, gate_status=None, right_pts=None):
    """The new pool: every candidate, or with a gate only those whose gate
    status is OK, in candidate order.  Admitted new candidates get the next
    identities in order.  Returns (pts, ids, right, next_id)."""
    cand_ids = np.asarray(cand_ids, np.int64)
    n = len(cand_ids)
    keep = np.ones(n, bool) if gate_status is None else (np.asarray(gate_status) == OK)
    ids = []
    nid = int(next_id)
    for i in range(n):
        if not keep[i]:
            continue
        if cand_ids[i] == NEW:
            ids.append(nid)
            nid += 1
        else:
            ids.append(int(cand_ids[i]))
    pts = np.asarray(cand_pts, np.float32).reshape(-1, 2)[keep]
    right = None if right_pts is None else np.asarray(right_pts, np.float32).reshape(-1, 2)[keep]
    return pts, np.asarray(ids, np.int64), right, nid


def step(pool: Pool, prev, nxt, right=None, *, target, track_kw=None, stereo_kw=None, gftt_kw=None):
    """One frame of one stream: temporal tracking of the pool from ``prev`` to
    ``nxt`` (skipped when ``prev`` is None), carry-over, top-up by detection
    on ``nxt``, and with a ``right`` frame the cross-camera gate.  Returns
    (new pool, stats) with stats = (previous count, carried, new candidates,
    admitted)."""
    track_kw = dict(track_kw or {})
    stereo_kw = dict(stereo_kw or {})
    gftt_kw = dict(gftt_kw or {})
    n0 = len(pool.ids)
    if prev is not None and n0:
        r = track(prev, nxt, pool.pts, **track_kw)
        sp, si = carry(pool.ids, r.pts.astype(np.float32), r.status)
    else:
        sp, si = np.zeros((0, 2), np.float32), np.zeros(0, np.int64)
    cp, ci = candidates(nxt, sp, si, target, **gftt_kw)
    gate = rp = None
    if right is not None and len(ci):
        rs = track(nxt, right, cp, **stereo_kw)
        gate, rp = rs.status, rs.pts.astype(np.float32)
    elif right is not None:
        gate, rp = np.zeros(0, np.uint8), np.zeros((0, 2), np.float32)
    pts, ids, rpts, nid = commit(cp, ci, pool.next_id, gate, rp)
    stats = (n0, len(si), len(ci) - len(si), len(ids))
    return Pool(pts, ids, rpts, nid), stats
