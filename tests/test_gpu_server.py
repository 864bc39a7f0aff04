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
