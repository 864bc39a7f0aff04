"""Batched, prepared (graph / persistent) and plain tracking give the same
bits: every point's arithmetic is independent of the launch it is in."""
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


RES = ((160, 120), (333, 251), (640, 480), (97, 131))


def make_streams(seed, n=6):
    return synth.batch_streams(seed, n_streams=n, kp_range=(1, 300), resolutions=RES)


class Setup:
    def __init__(self, lk, ctx, streams, storage, win, levels, fb):
        import torch
        self.lk, self.ctx = lk, ctx
        self.prev = [torch.from_numpy(s.prev).cuda() for s in streams]
        self.next = [torch.from_numpy(s.next).cuda() for s in streams]
        self.pp = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
        self.pn = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
        lk.lk_build_pyramids(ctx, self.pp, self.prev)
        counts = [len(s.pts) for s in streams]
        self.counts = counts
        self.offs = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(int)
        self.n = int(sum(counts))
        self.pts = torch.from_numpy(np.concatenate([s.pts for s in streams])).cuda()
        self.params = lk.make_params(win, levels, 30, 0.01, 1e-6, fb)
        self.pairs = [(a, b, int(o), c) for a, b, o, c in zip(self.pp, self.pn, self.offs, counts)]
        self.levels = levels

    def outputs(self):
        return self.lk.outputs(self.n, self.levels, with_iters=True)

    def plain(self):
        import torch
        lk = self.lk
        out = self.outputs()
        for i, (a, b, o, c) in enumerate(self.pairs):
            lk.lk_build_pyramid(self.ctx, b, self.next[i])
            lk.lk_track(self.ctx, a, b, self.pts[o:o + c], None, c, self.params, out[0][o:o + c], out[1][o:o + c],
                        out[2][o:o + c], out[3][o:o + c])
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in out]

    def close(self):
        for p in self.pp + self.pn:
            self.lk.lk_pyramid_destroy(p)


def same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("storage,win,levels,fb", [(0, 21, 3, 0.0), (1, 31, 4, 1.0), (0, 9, 2, 1.0), (1, 21, 3, 0.0)])
def test_batched_equals_plain_bitwise(lk, ctx, storage, win, levels, fb):
    import torch
    st = Setup(lk, ctx, make_streams(storage * 10 + win), storage, win, levels, fb)
    ref = st.plain()
    out = st.outputs()
    lk.lk_build_pyramids(ctx, st.pn, st.next)
    lk.lk_track_batched(ctx, st.pairs, st.pts, None, st.params, *out)
    torch.cuda.synchronize()
    same(ref, [t.cpu().numpy() for t in out])
    assert (ref[1] == 0).mean() > 0.5
    st.close()


@pytest.mark.parametrize("persistent,bpc,graph,chunk,wpg,storage",
                         [(0, 0, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0), (1, 1, 1, 0, 0, 0), (1, 4, 0, 1, 0, 0),
                          (1, 16, 1, 32, 0, 0), (1, 20, 0, 8, 0, 1), (0, 0, 1, 0, 2, 0), (0, 0, 0, 0, 4, 0),
                          (0, 0, 1, 0, 4, 1), (0, 0, 0, 0, 1, 1)])
def test_prepared_batch_equals_plain(lk, ctx, persistent, bpc, graph, chunk, wpg, storage):
    """Every execution shape the tuner can pick (hardware dispatch with 1, 2
    or 4 wavefronts per workgroup, persistent grids with fine and coarse work
    fetches) gives the plain path's bits."""
    import torch
    st = Setup(lk, ctx, make_streams(7 + storage), storage, 21, 3, 1.0)
    ref = st.plain()
    out = st.outputs()
    cfg = lk.lk_exec_config(persistent, bpc, graph, chunk, wpg, 0)
    b = lk.lk_batch_create(ctx, st.pn, st.next, st.pairs, st.pts, None, st.params, *out, config=cfg)
    for rep in range(3):
        for t in out:
            t.zero_()
        lk.lk_batch_run(b)
        torch.cuda.synchronize()
        same(ref, [t.cpu().numpy() for t in out])
        # unrelated eager work between graph replays
        torch.ones(1 << 20, device="cuda").sum().item()
    lk.lk_batch_destroy(b)
    st.close()


def test_autotuner_picks_a_config_and_keeps_results(lk, ctx):
    import torch
    st = Setup(lk, ctx, make_streams(3, n=8), 0, 21, 3, 0.0)
    ref = st.plain()
    out = st.outputs()
    b = lk.lk_batch_create(ctx, st.pn, st.next, st.pairs, st.pts, None, st.params, *out)
    cfg, ms = lk.lk_batch_tune(b, reps=2)
    assert ms > 0 and cfg.persistent in (0, 1) and cfg.use_graph == 1
    got = lk.lk_batch_config(b)
    assert (got.persistent, got.blocks_per_cu) == (cfg.persistent, cfg.blocks_per_cu)
    for t in out:
        t.zero_()
    lk.lk_batch_run(b)
    torch.cuda.synchronize()
    same(ref, [t.cpu().numpy() for t in out])
    lk.lk_batch_destroy(b)
    st.close()


def test_invalid_batch_arguments(lk, ctx):
    st = Setup(lk, ctx, make_streams(1, n=2), 0, 21, 3, 0.0)
    out = st.outputs()
    for bad_cfg in (lk.lk_exec_config(2, 1, 0, 0), lk.lk_exec_config(0, 0, 1, 0, 3, 0),
                    lk.lk_exec_config(1, 4, 1, 0, 2, 0), lk.lk_exec_config(1, 4, 1, 2000, 0, 0),
                    lk.lk_exec_config(0, 0, 1, 0, 0, 1)):
        with pytest.raises(lk.LKError) as e:
            lk.lk_batch_create(ctx, st.pn, st.next, st.pairs, st.pts, None, st.params, *out, config=bad_cfg)
        assert e.value.code == lk.LK_ERR_INVALID_ARG
    bad = lk.make_params(win=22)
    with pytest.raises(lk.LKError):
        lk.lk_batch_create(ctx, st.pn, st.next, st.pairs, st.pts, None, bad, *out)
    st.close()


@pytest.mark.parametrize("levels_of", [[2, 2, 2, 3, 2, 2, 2], [3, 3, 3, 3, 3, 3, 3]])
def test_batched_build_writes_every_descriptor(lk, ctx, levels_of):
    """A batched build writes each pyramid's device descriptor either with the
    fused level-1/2 launch (one per workgroup, when it has a workgroup for
    each) or with a launch of its own (here: 2-level pyramids have no fused
    job, so the first case has more descriptors than fused workgroups).  The
    tracker reads those descriptors: tracking on the batch-built pyramids must
    equal tracking on singly built ones, bit for bit."""
    import torch
    streams = synth.batch_streams(21, n_streams=len(levels_of), kp_range=(20, 120),
                                  resolutions=((97, 131), (160, 120)))
    prev = [torch.from_numpy(s.prev).cuda() for s in streams]
    nxt = [torch.from_numpy(s.next).cuda() for s in streams]
    mk = lambda: [lk.lk_pyramid_create(ctx, s.width, s.height, L, 0) for s, L in zip(streams, levels_of)]
    pp, pn, qn = mk(), mk(), mk()
    lk.lk_build_pyramids(ctx, pp, prev)
    lk.lk_build_pyramids(ctx, pn, nxt)                   # batched
    for q, im in zip(qn, nxt):
        lk.lk_build_pyramid(ctx, q, im)                  # one at a time
    params = lk.make_params(21, 2, 30, 0.01, 1e-6, 0.0)
    for a, b, q, s in zip(pp, pn, qn, streams):
        n = len(s.pts)
        pts = torch.from_numpy(s.pts).cuda()
        got, ref = lk.outputs(n, 2, with_iters=True), lk.outputs(n, 2, with_iters=True)
        lk.lk_track(ctx, a, b, pts, None, n, params, *got)
        lk.lk_track(ctx, a, q, pts, None, n, params, *ref)
        torch.cuda.synchronize()
        same([t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got])
        assert (ref[1].cpu().numpy() == 0).mean() > 0.5
    for p in pp + pn + qn:
        lk.lk_pyramid_destroy(p)


def test_shape_table_row_is_used(lk, ctx, tmp_path, monkeypatch):
    """lk_batch_create without a shape takes the matching row of the table
    file (architecture, window, levels, storage, size and keypoint buckets),
    and the step keeps the plain path's bits; rows for other keys, comments
    and malformed lines are skipped."""
    import torch
    st = Setup(lk, ctx, make_streams(5, n=6), 0, 21, 3, 0.0)
    ref = st.plain()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    px = int(np.mean([w * h for (w, h) in [(s.width, s.height) for s in make_streams(5, n=6)]]))
    kp = int(np.mean(st.counts))
    rb, kb = lk.lk_exec_buckets(px, kp)
    table = tmp_path / "table.txt"
    table.write_text("# arch win levels storage res kp persistent bpc graph chunk wpg ms\n"
                     "%s 21 3 0 %d %d 1 7 1 5 0 0.5\n"
                     "%s 21 3 1 %d %d 0 0 1 0 2\n"
                     "not a row\n"
                     "%s 9 3 0 %d %d 0 0 1 0 4\n" % (arch, rb, kb, arch, rb, kb, arch, rb, kb))
    monkeypatch.setenv("LKMI_EXEC_TABLE", str(table))
    cfg, found = lk.lk_exec_table_lookup(ctx, st.pairs, st.params)
    assert found and (cfg.persistent, cfg.blocks_per_cu, cfg.use_graph, cfg.chunk, cfg.waves_per_group) == \
        (1, 7, 1, 5, 0)
    out = st.outputs()
    b = lk.lk_batch_create(ctx, st.pn, st.next, st.pairs, st.pts, None, st.params, *out)
    got = lk.lk_batch_config(b)
    assert (got.persistent, got.blocks_per_cu, got.chunk) == (1, 7, 5)
    lk.lk_batch_run(b)
    torch.cuda.synchronize()
    same(ref, [t.cpu().numpy() for t in out])
    lk.lk_batch_destroy(b)
    # another window: no row matches, the default shape
    cfg, found = lk.lk_exec_table_lookup(ctx, st.pairs, lk.make_params(win=15))
    assert not found and (cfg.persistent, cfg.use_graph, cfg.waves_per_group) == (0, 1, 0)
    monkeypatch.delenv("LKMI_EXEC_TABLE")
    st.close()
