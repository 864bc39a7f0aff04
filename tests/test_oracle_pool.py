"""Pins of the track-pool oracle (oracle.pool): hand-worked carry and commit
cases, the reduction of a fresh pool to the detector, the distance and
prefix properties of the greedy top-up, the degenerate frames (identical,
flat), and identity invariants over a stereo sequence."""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
import synth

if os.environ.get("LKO_POOL_SRC"):
    # the mutation tests point this at a planted copy of oracle/pool.py
    _spec = importlib.util.spec_from_file_location("oracle._pool_planted", os.environ["LKO_POOL_SRC"])
    P = importlib.util.module_from_spec(_spec)
    sys.modules[_spec.name] = P
    _spec.loader.exec_module(P)
else:
    from oracle import pool as P

GK = dict(r=1, quality=0.01, min_dist=20, border=8)


def texture(h, w, seed):
    return synth.quantize_u8(synth.texture_canvas(h, w, seed))


def test_carry_hand_case():
    ids = np.array([7, 3, 9, 4], np.int64)
    pts = np.array([[1, 2], [3, 4], [5.5, 6], [7, 8]], np.float32)
    st = np.array([oracle.OK, oracle.LOST_EIG, oracle.OK, oracle.LOST_FB], np.uint8)
    sp, si = P.carry(ids, pts, st)
    assert si.tolist() == [7, 9]
    assert sp.tolist() == [[1, 2], [5.5, 6]]
    sp, si = P.carry(ids[:0], pts[:0], st[:0])
    assert sp.shape == (0, 2) and si.shape == (0,)


def test_commit_hand_cases():
    cp = np.arange(10, dtype=np.float32).reshape(5, 2)
    ci = np.array([5, 9, P.NEW, P.NEW, P.NEW], np.int64)
    gate = np.array([oracle.OK, oracle.LOST_FB, oracle.OK, oracle.LOST_OOB, oracle.OK], np.uint8)
    rp = cp + 100
    pts, ids, right, nid = P.commit(cp, ci, 20, gate, rp)
    assert ids.tolist() == [5, 20, 21] and nid == 22
    assert pts.tolist() == cp[[0, 2, 4]].tolist() and right.tolist() == rp[[0, 2, 4]].tolist()
    pts, ids, right, nid = P.commit(cp, ci, 20)
    assert ids.tolist() == [5, 9, 20, 21, 22] and nid == 23 and right is None
    assert np.array_equal(pts, cp)
    # nothing admitted: the identity counter does not move
    pts, ids, _, nid = P.commit(cp, ci, 20, np.full(5, oracle.LOST_EIG, np.uint8), rp)
    assert len(ids) == 0 and nid == 20


def test_fresh_pool_is_the_detector():
    im = texture(240, 320, 1)
    cp, ci = P.candidates(im, np.zeros((0, 2), np.float32), np.zeros(0, np.int64), 150, **GK)
    want = oracle.gftt(im, max_corners=150, **GK)
    assert np.array_equal(cp, want) and np.all(ci == P.NEW)
    pool, stats = P.step(P.Pool(), None, im, target=150, gftt_kw=GK)
    assert pool.ids.tolist() == list(range(len(want))) and pool.next_id == len(want)
    assert stats == (0, 0, len(want), len(want))


def test_topup_distance_and_prefix_properties():
    im = texture(240, 320, 2)
    rng = np.random.default_rng(3)
    surv = np.column_stack([rng.uniform(0, 319, 40), rng.uniform(0, 239, 40)]).astype(np.float32)
    sid = np.arange(100, 140, dtype=np.int64)
    full, fid = P.candidates(im, surv, sid, 400, **GK)
    s = len(sid)
    assert np.array_equal(full[:s], surv) and np.array_equal(fid[:s], sid)
    new = full[s:].astype(np.float64)
    d2 = ((new[:, None, :] - surv[None, :, :].astype(np.float64)) ** 2).sum(-1)
    assert np.all(d2 >= GK["min_dist"] ** 2)
    # greedy selection in rank order: a smaller target takes a prefix
    for t in (s, s + 1, s + 7, s + 30):
        part, pid = P.candidates(im, surv, sid, t, **GK)
        assert np.array_equal(part, full[:len(part)])
        assert len(part) == min(t, len(full))
    # survivors above the target are kept, nothing is added
    part, pid = P.candidates(im, surv, sid, 10, **GK)
    assert np.array_equal(part, surv) and np.array_equal(pid, sid)


def test_identical_frames_carry_every_trackable_point():
    im = texture(240, 320, 4)
    kw = dict(win=21, levels=3, min_eig=1e-6)
    pool, _ = P.step(P.Pool(), None, im, target=120, gftt_kw=GK)
    n = len(pool.ids)
    r = oracle.track(im, im, pool.pts, **kw)
    nxt, stats = P.step(pool, im, im, target=120, track_kw=kw, gftt_kw=GK)
    ok = r.status == oracle.OK
    assert stats[0] == n and stats[1] == int(ok.sum())
    # zero flow: survivors stay exactly where they were, with their identities
    assert np.array_equal(nxt.pts[:stats[1]], pool.pts[ok])
    assert np.array_equal(nxt.ids[:stats[1]], pool.ids[ok])
    assert nxt.next_id == pool.next_id + (len(nxt.ids) - stats[1])


def test_flat_template_ends_every_track():
    # the eigenvalue test reads the template frame: a flat frame t-1 ends
    # every track, and the pool restarts from the detector on frame t
    im = texture(240, 320, 5)
    flat = np.full_like(im, 90)
    pool, _ = P.step(P.Pool(), None, im, target=80, gftt_kw=GK)
    nxt, stats = P.step(pool, flat, im, target=80, track_kw=dict(min_eig=1e-6), gftt_kw=GK)
    want = oracle.gftt(im, max_corners=80, **GK)
    assert stats == (len(pool.ids), 0, len(want), len(want))
    assert np.array_equal(nxt.pts, want)
    assert nxt.ids.tolist() == list(range(pool.next_id, pool.next_id + len(want)))
    # nothing to detect on a flat frame
    empty, stats = P.step(P.Pool(), None, flat, target=80, gftt_kw=GK)
    assert len(empty.ids) == 0 and empty.next_id == 0 and stats == (0, 0, 0, 0)


def test_stereo_gate_with_identical_cameras_equals_mono():
    im = texture(240, 320, 6)
    kw = dict(win=21, levels=3, min_eig=1e-6)
    mono, _ = P.step(P.Pool(), None, im, target=100, gftt_kw=GK)
    st, _ = P.step(P.Pool(), None, im, im, target=100, stereo_kw=dict(kw, fb_thresh=1.0), gftt_kw=GK)
    r = oracle.track(im, im, mono.pts, **kw)
    keep = r.status == oracle.OK
    assert np.array_equal(st.pts, mono.pts[keep])
    assert st.ids.tolist() == list(range(int(keep.sum())))
    assert np.array_equal(st.right, st.pts)       # zero disparity, exactly


@pytest.mark.parametrize("stereo", [False, True])
def test_identity_invariants_over_a_sequence(stereo):
    seq = synth.StereoSequence(2, width=320, height=240, n_frames=12)
    kw = dict(win=21, levels=3, min_eig=1e-6)
    pool = P.Pool()
    seen = set()
    prev = None
    for t in range(6):
        left = seq.frame(t)
        right = seq.frame(t, 1) if stereo else None
        old = set(pool.ids.tolist())
        pool, (n0, carried, new, adm) = P.step(pool, prev, left, right, target=100, track_kw=kw,
                                               stereo_kw=dict(kw, fb_thresh=1.0), gftt_kw=GK)
        ids = pool.ids.tolist()
        assert len(ids) == len(set(ids)) == adm <= 100
        fresh = [i for i in ids if i not in old]
        assert all(i not in seen for i in fresh)             # never reused
        assert fresh == sorted(fresh)                         # dense and in order
        assert set(ids) - set(fresh) <= old
        if t:
            assert carried <= n0 and carried > 0.5 * n0       # smooth motion keeps most tracks
        seen |= set(ids)
        prev = left
