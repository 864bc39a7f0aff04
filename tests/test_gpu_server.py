"""The continuous-batching server: each frame's result is the same bits
alone and in a mix of streams (and the same as the plain lk_track path),
frames of a stream complete in order, admission honours the budget."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lk():
    import torch
    assert torch.cuda.is_available()
    from paper_2607_01757_amd import lk as _lk
    return _lk


@pytest.fixture(scope="module")
def ctx(lk):
    c = lk.lk_context_create(0, 0)
    yield c
    lk.lk_context_destroy(c)


def wait(lk, srv, ticket, maxp, timeout=30.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        r = lk.lk_server_poll(srv, ticket, maxp)
        if r is not None:
            return r
        time.sleep(0.0005)
    raise TimeoutError("ticket %d not done" % ticket)


def frames_for(seed, w, h, n):
    canvas = synth.texture_canvas(h + 64, w + 64, seed)
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        dx, dy = rng.integers(-6, 7, 2)
        out.append(synth.quantize_u8(canvas[32 + dy:32 + dy + h, 32 + dx:32 + dx + w]))
    return out


def run_stream_alone(lk, ctx, cfg, frames, pts):
    srv = lk.lk_server_create(ctx, cfg)
    sid = lk.lk_server_open_stream(srv, frames[0].shape[1], frames[0].shape[0])
    res = []
    for f in frames:
        t = lk.lk_server_submit(srv, sid, f, pts)
        res.append(wait(lk, srv, t, cfg.max_points))
    lk.lk_server_destroy(srv)
    return res


@pytest.mark.parametrize("storage", [0, 1])
def test_alone_equals_mix_equals_plain(lk, ctx, storage):
    import torch
    prm = lk.make_params(21, 3, 30, 0.01, 1e-6, 1.0)
    cfg = lk.server_config(max_streams=16, max_points=400, levels=3, storage=storage, params=prm, inflight=2)
    w, h = 320, 240
    frames = frames_for(1, w, h, 4)
    pts = synth.uniform_points(np.random.default_rng(0), 300, w, h)
    alone = run_stream_alone(lk, ctx, cfg, frames, pts)
    assert len(alone[0][0]) == 0                       # first frame only primes
    # the same stream in a mix of 9 others of other sizes, submitted interleaved
    srv = lk.lk_server_create(ctx, cfg)
    sid = lk.lk_server_open_stream(srv, w, h)
    others = []
    for k in range(9):
        ow, oh = [(160, 120), (400, 300), (256, 256)][k % 3]
        oid = lk.lk_server_open_stream(srv, ow, oh)
        others.append((oid, frames_for(100 + k, ow, oh, 4), synth.uniform_points(np.random.default_rng(k), 50 + 30 * k, ow, oh)))
    mine, theirs = [], []
    for i in range(4):
        for oid, ofr, opts in others[:5]:
            theirs.append(lk.lk_server_submit(srv, oid, ofr[i], opts))
        mine.append(lk.lk_server_submit(srv, sid, frames[i], pts))
        for oid, ofr, opts in others[5:]:
            theirs.append(lk.lk_server_submit(srv, oid, ofr[i], opts))
        mine[-1] = wait(lk, srv, mine[-1], cfg.max_points)
        theirs = [wait(lk, srv, t, cfg.max_points) if isinstance(t, int) else t for t in theirs]
    stats = lk.lk_server_get_stats(srv)
    assert stats.frames == 40 and stats.batches < 40       # frames were batched together
    lk.lk_server_destroy(srv)
    for a, b in zip(alone, mine):
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    # and the plain path on the same frames
    for i in range(1, 4):
        pa = lk.lk_pyramid_create(ctx, w, h, 3, storage)
        pb = lk.lk_pyramid_create(ctx, w, h, 3, storage)
        ta, tb = torch.from_numpy(frames[i - 1]).cuda(), torch.from_numpy(frames[i]).cuda()
        lk.lk_build_pyramid(ctx, pa, ta)
        lk.lk_build_pyramid(ctx, pb, tb)
        d_pts = torch.from_numpy(pts).cuda()
        out, st, res, _ = lk.outputs(len(pts), 3)
        lk.lk_track(ctx, pa, pb, d_pts, None, len(pts), prm, out, st, res)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), alone[i][0])
        assert np.array_equal(st.cpu().numpy(), alone[i][1])
        assert np.array_equal(res.cpu().numpy(), alone[i][2])
        lk.lk_pyramid_destroy(pa)
        lk.lk_pyramid_destroy(pb)


def test_queued_frames_complete_in_order(lk, ctx):
    cfg = lk.server_config(max_streams=4, max_points=200, levels=3, storage=0, params=lk.make_params(), queue_depth=6)
    w, h = 200, 160
    frames = frames_for(5, w, h, 6)
    pts = synth.uniform_points(np.random.default_rng(1), 150, w, h)
    srv = lk.lk_server_create(ctx, cfg)
    sid = lk.lk_server_open_stream(srv, w, h)
    tickets = [lk.lk_server_submit(srv, sid, f, pts) for f in frames]
    res = [wait(lk, srv, t, 200) for t in tickets]
    done = [r[3][2] for r in res]
    assert done == sorted(done)
    assert all(len(r[0]) == 150 for r in res[1:])
    # same as submitting one at a time
    ref = run_stream_alone(lk, ctx, cfg, frames, pts)
    for a, b in zip(ref, res):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    lk.lk_server_destroy(srv)


def test_admission_budget_and_errors(lk, ctx):
    # float32 storage, 3 levels: 640x480 holds ~1.4 MB, 1280x720 ~4.1 MB, 960x600 ~2.8 MB
    budget = 3584 << 10
    cfg = lk.server_config(max_streams=8, max_points=100, levels=3, storage=0, params=lk.make_params(),
                           hbm_budget_bytes=budget, queue_depth=1)
    srv = lk.lk_server_create(ctx, cfg)
    a = lk.lk_server_open_stream(srv, 640, 480)
    with pytest.raises(lk.LKError) as e:
        lk.lk_server_open_stream(srv, 1280, 720)                  # does not fit
    assert e.value.code == lk.LK_ERR_BUSY
    with pytest.raises(lk.LKError) as e:
        lk.lk_server_poll(srv, 12345, 100)
    assert e.value.code == lk.LK_ERR_NOT_FOUND
    f = frames_for(2, 640, 480, 2)
    pts = synth.uniform_points(np.random.default_rng(2), 100, 640, 480)
    t1 = lk.lk_server_submit(srv, a, f[0], pts)
    # one staging slot: a second frame is refused until the first is retired
    try:
        t2 = lk.lk_server_submit(srv, a, f[1], pts)
        wait(lk, srv, t1, 100)
        wait(lk, srv, t2, 100)
    except lk.LKError as err:
        assert err.code == lk.LK_ERR_BUSY
        wait(lk, srv, t1, 100)
    with pytest.raises(lk.LKError):
        lk.lk_server_poll(srv, t1, 100)                           # retired
    # close while a frame may be in flight, then the freed budget admits a bigger stream
    lk.lk_server_submit(srv, a, f[1], pts)
    lk.lk_server_close_stream(srv, a)
    b = lk.lk_server_open_stream(srv, 960, 600)
    with pytest.raises(lk.LKError):
        lk.lk_server_submit(srv, a, f[0], pts)                    # closed stream
    st = lk.lk_server_get_stats(srv)
    assert st.open_streams == 1 and st.resident_bytes <= budget
    lk.lk_server_close_stream(srv, b)
    lk.lk_server_destroy(srv)


def plain_track(lk, ctx, a, b, pts, prm, levels, storage):
    import torch
    h, w = a.shape
    pa = lk.lk_pyramid_create(ctx, w, h, levels, storage)
    pb = lk.lk_pyramid_create(ctx, w, h, levels, storage)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    lk.lk_build_pyramid(ctx, pa, ta)
    lk.lk_build_pyramid(ctx, pb, tb)
    d_pts = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    out, st, res, _ = lk.outputs(len(pts), levels)
    lk.lk_track(ctx, pa, pb, d_pts, None, len(pts), prm, out, st, res)
    torch.cuda.synchronize()
    r = out.cpu().numpy(), st.cpu().numpy(), res.cpu().numpy()
    lk.lk_pyramid_destroy(pa)
    lk.lk_pyramid_destroy(pb)
    return r


def test_failed_launch_reports_device_error_and_stream_recovers(lk, ctx):
    """A launch that fails on the host (its pyramid-table staging is made to
    fail after the frame's copy was enqueued) completes its frame with
    LK_ERR_DEVICE; the stream keeps its previous pyramid, so the next frame
    is tracked from the last frame that completed."""
    prm = lk.make_params(21, 3, 30, 0.01, 1e-6, 0.0)
    cfg = lk.server_config(max_streams=2, max_points=200, levels=3, storage=0, params=prm, inflight=1)
    w, h = 256, 192
    frames = frames_for(7, w, h, 4)
    pts = synth.uniform_points(np.random.default_rng(3), 120, w, h)
    srv = lk.lk_server_create(ctx, cfg)
    sid = lk.lk_server_open_stream(srv, w, h)
    wait(lk, srv, lk.lk_server_submit(srv, sid, frames[0], pts), 200)          # primes
    ok1 = wait(lk, srv, lk.lk_server_submit(srv, sid, frames[1], pts), 200)
    lk.lk_server_fail_next_launches(srv, 1)
    t2 = lk.lk_server_submit(srv, sid, frames[2], pts)
    with pytest.raises(lk.LKError) as e:
        wait(lk, srv, t2, 200)
    assert e.value.code == lk.LK_ERR_DEVICE
    with pytest.raises(lk.LKError) as e:
        lk.lk_server_poll(srv, t2, 200)                                          # retired
    assert e.value.code == lk.LK_ERR_NOT_FOUND
    ok3 = wait(lk, srv, lk.lk_server_submit(srv, sid, frames[3], pts), 200)
    st = lk.lk_server_get_stats(srv)
    assert st.frames == 3                                                        # the failed frame is not counted
    lk.lk_server_destroy(srv)
    for got, (a, b) in ((ok1, (0, 1)), (ok3, (1, 3))):
        ref = plain_track(lk, ctx, frames[a], frames[b], pts, prm, 3, 0)
        for x, y in zip(got[:3], ref):
            assert np.array_equal(x, y)


def test_close_while_submitting(lk, ctx):
    """Submits on a stream race with its close: every submit either gets a
    ticket or a clean error, closing waits for copies in progress, and the
    stream slot is reusable afterwards."""
    import threading
    prm = lk.make_params()
    cfg = lk.server_config(max_streams=2, max_points=300, levels=3, storage=0, params=prm, queue_depth=4)
    w, h = 640, 480
    frames = frames_for(9, w, h, 3)
    pts = synth.uniform_points(np.random.default_rng(4), 300, w, h)
    srv = lk.lk_server_create(ctx, cfg)
    for rnd in range(3):
        sid = lk.lk_server_open_stream(srv, w, h)
        codes, tickets = [], []
        stop = threading.Event()

        def submitter():
            k = 0
            while not stop.is_set():
                try:
                    tickets.append(lk.lk_server_submit(srv, sid, frames[k % 3], pts))
                except lk.LKError as err:
                    codes.append(err.code)
                    if err.code == lk.LK_ERR_NOT_FOUND:
                        return
                k += 1
        th = [threading.Thread(target=submitter) for _ in range(3)]
        for t in th:
            t.start()
        time.sleep(0.02 * (rnd + 1))
        lk.lk_server_close_stream(srv, sid)
        stop.set()
        for t in th:
            t.join(timeout=30)
            assert not t.is_alive()
        assert set(codes) <= {lk.LK_ERR_BUSY, lk.LK_ERR_NOT_FOUND}
        for t in tickets:                      # tickets of a closed stream are unknown or already done
            try:
                lk.lk_server_poll(srv, t, 300)
            except lk.LKError as err:
                assert err.code == lk.LK_ERR_NOT_FOUND
    # the slot is free again and serves a stream of another size
    sid = lk.lk_server_open_stream(srv, 320, 240)
    f = frames_for(10, 320, 240, 2)
    p2 = synth.uniform_points(np.random.default_rng(5), 100, 320, 240)
    wait(lk, srv, lk.lk_server_submit(srv, sid, f[0], p2), 300)
    r = wait(lk, srv, lk.lk_server_submit(srv, sid, f[1], p2), 300)
    assert len(r[0]) == 100
    assert lk.lk_server_get_stats(srv).open_streams == 1
    lk.lk_server_destroy(srv)


def test_served_c5_tracker_matches_oracle(lk, ctx):
    """The serving configuration's tracker (31x31 window, 4 levels, 30
    iterations, eps 0.01, forward-backward 1 px, binary16 storage) through
    the server on four streams of different sizes, submitted interleaved:
    every served frame follows the parity rule against the oracle with the
    same binary16 storage, and stays within 1e-2 px of the unrounded FP64
    oracle."""
    import oracle
    from parity import compare
    prm = lk.make_params(31, 4, 30, 0.01, 1e-6, 1.0)
    cfg = lk.server_config(max_streams=8, max_points=400, levels=4, storage=1, params=prm, inflight=2)
    seqs = [synth.StereoSequence(21 + k, width=w, height=h, n_frames=8)
            for k, (w, h) in enumerate([(752, 480), (640, 480), (960, 600), (400, 304)])]
    kps = [200, 150, 300, 120]
    frames = [[s.frame(t) for t in range(4)] for s in seqs]
    srv = lk.lk_server_create(ctx, cfg)
    sids = [lk.lk_server_open_stream(srv, s.width, s.height) for s in seqs]
    served = [[None] * 4 for _ in seqs]
    for t in range(4):
        tk = [lk.lk_server_submit(srv, sid, frames[k][t], seqs[k].points(t, kps[k])) for k, sid in enumerate(sids)]
        for k, ticket in enumerate(tk):
            served[k][t] = wait(lk, srv, ticket, cfg.max_points)
    stats = lk.lk_server_get_stats(srv)
    lk.lk_server_destroy(srv)
    assert stats.frames == 16 and stats.batches < 16
    worst64, n_cmp = 0.0, 0
    for k, s in enumerate(seqs):
        for t in range(1, 4):
            pts = s.points(t, kps[k])
            g = served[k][t][:3]
            r16 = oracle.track(frames[k][t - 1], frames[k][t], pts, win=31, levels=4, fb_thresh=1.0, min_eig=1e-6,
                               f16=True, nthreads=8)
            rep = compare(*g, None, r16, check_iters=False)
            r64 = oracle.track(frames[k][t - 1], frames[k][t], pts, win=31, levels=4, fb_thresh=1.0, min_eig=1e-6,
                               nthreads=8)
            both = (g[1] == 0) & (r64.status == 0)
            e64 = np.abs(g[0][both] - r64.pts[both]).max(axis=1)
            print("stream %d frame %d: %s | vs FP64: %d points, max %.3g px" % (k, t, rep, both.sum(), e64.max()))
            assert rep.compared_ok >= 0.8 * kps[k]
            assert e64.max() <= 1e-2
            worst64 = max(worst64, float(e64.max()))
            n_cmp += rep.compared_ok
    print("served C5 tracker: %d points compared, max %.3g px vs the unrounded oracle" % (n_cmp, worst64))
