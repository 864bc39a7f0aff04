"""GPU parity of the corner detector (lk_detect_corners) against the oracle.

The detector's result is exact by definition (integer tensor, binary64
response with one rounding per operation, a total order on candidates), so
the comparison is bit for bit: the response map, the number of corners, and
every corner in order.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2607_01757_amd import lk


@pytest.fixture(scope="module")
def det():
    ctx = lk.lk_context_create(0)
    d = lk.lk_detector_create(ctx, 64, 64 * 1920 * 1088)
    yield d
    lk.lk_detector_destroy(d)
    lk.lk_context_destroy(ctx)


def texture(h, w, seed):
    return synth.quantize_u8(synth.texture_canvas(h, w, seed))


def run(det, imgs, *, r=1, quality=0.01, min_dist=16, max_corners=200, border=0, occupied=None,
        response=False, pitch_pad=0):
    frames, outs = [], []
    for k, im in enumerate(imgs):
        h, w = im.shape
        buf = torch.zeros((h, w + pitch_pad), dtype=torch.uint8, device="cuda")
        buf[:, :w] = torch.from_numpy(im).cuda()
        f = {"img": buf[:, :w], "pitch": w + pitch_pad,
             "out_xy": torch.full((max(max_corners, 1), 2), -1.0, dtype=torch.float32, device="cuda"),
             "count": torch.full((1,), -1, dtype=torch.int32, device="cuda")}
        if occupied is not None and occupied[k] is not None and len(occupied[k]):
            f["occupied"] = torch.from_numpy(np.ascontiguousarray(occupied[k], np.float32)).cuda()
        if response:
            f["response"] = torch.empty((h, w), dtype=torch.float64, device="cuda")
        frames.append(f)
    lk.lk_detect_corners(det, frames, lk.gftt_params(r, min_dist, max_corners, border, quality))
    torch.cuda.synchronize()
    for f in frames:
        n = int(f["count"].item())
        outs.append((f["out_xy"][:n].cpu().numpy(), f["response"].cpu().numpy() if response else None))
    return outs


def oracle_corners(im, occ=None, **kw):
    return oracle.gftt(im, r=kw.get("r", 1), quality=kw.get("quality", 0.01), min_dist=kw.get("min_dist", 16),
                       max_corners=kw.get("max_corners", 200), border=kw.get("border", 0), occupied=occ)


# (129, 125): a last row of strips one row tall; (200, 61): a last column of
# strips one column wide, and strips away from the top and bottom edges
# (their walk rolls the separable gradient) between strips that touch them
@pytest.mark.parametrize("r", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(3, 3), (5, 70), (17, 65), (61, 83), (129, 125), (200, 61), (480, 752)])
def test_response_bitwise(det, r, shape):
    im = texture(*shape, 10 + r)
    print("response r=%d shape=%s" % (r, shape), flush=True)
    (_, R), = run(det, [im], r=r, response=True)
    want = oracle.gftt_response(im, r)
    assert np.array_equal(R.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("r", [0, 1])
def test_tall_strips_of_a_large_call(det, r):
    """A call of at least 8 Mi pixels walks 64-row strips (smaller calls 32):
    responses of two of its frames bit for bit, corners of all five exact."""
    shapes = [(1080, 1920)] * 4 + [(480, 752)]
    assert sum(h * w for h, w in shapes) >= 8 << 20
    imgs = [texture(h, w, 60 + 7 * r + i) for i, (h, w) in enumerate(shapes)]
    print("tall strips r=%d" % r, flush=True)
    kw = dict(r=r, quality=0.01, min_dist=30, max_corners=200)
    frames, outs = [], []
    for k, im in enumerate(imgs):
        h, w = im.shape
        f = {"img": torch.from_numpy(im).cuda(),
             "out_xy": torch.full((200, 2), -1.0, dtype=torch.float32, device="cuda"),
             "count": torch.full((1,), -1, dtype=torch.int32, device="cuda")}
        if k in (0, 4):
            f["response"] = torch.empty((h, w), dtype=torch.float64, device="cuda")
        frames.append(f)
    lk.lk_detect_corners(det, frames, lk.gftt_params(r, 30, 200, 0, 0.01))
    torch.cuda.synchronize()
    for k, (im, f) in enumerate(zip(imgs, frames)):
        if "response" in f:
            want = oracle.gftt_response(im, r)
            assert np.array_equal(f["response"].cpu().numpy().view(np.uint64), want.view(np.uint64)), k
        n = int(f["count"].item())
        assert np.array_equal(f["out_xy"][:n].cpu().numpy(), oracle_corners(im, **kw)), k


@pytest.mark.parametrize("r", [0, 1])
def test_response_bitwise_unaligned_pitch(det, r):
    """Rows whose pitch (145 bytes) is no multiple of 8: the staging loads bytes."""
    im = texture(200, 131, 40 + r)
    print("response unaligned pitch r=%d" % r, flush=True)
    (_, R), = run(det, [im], r=r, response=True, pitch_pad=14)
    want = oracle.gftt_response(im, r)
    assert np.array_equal(R.view(np.uint64), want.view(np.uint64))


CASES = [
    dict(r=1, quality=0.01, min_dist=30, max_corners=200),
    dict(r=1, quality=0.01, min_dist=16, max_corners=200, border=10),
    dict(r=2, quality=0.001, min_dist=8, max_corners=1000),
    dict(r=0, quality=0.05, min_dist=0, max_corners=300),
    dict(r=3, quality=0.0, min_dist=1, max_corners=4096),
    dict(r=1, quality=0.001, min_dist=5, max_corners=4096),
    dict(r=1, quality=0.01, min_dist=30, max_corners=0),
    dict(r=1, quality=0.01, min_dist=30, max_corners=1),
    dict(r=1, quality=2.0, min_dist=30, max_corners=50),
]


@pytest.mark.parametrize("kw", CASES, ids=[str(i) for i in range(len(CASES))])
@pytest.mark.parametrize("shape", [(480, 752), (97, 131), (200, 61)])
def test_corners_exact(det, kw, shape):
    im = texture(*shape, 3)
    print("corners %s shape=%s" % (kw, shape), flush=True)
    (got, _), = run(det, [im], **kw)
    want = oracle_corners(im, **kw)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_many_windows_large_frame(det):
    # ~40k candidates above the threshold: the selection walks many windows
    im = texture(720, 1280, 7)
    kw = dict(r=1, quality=0.0, min_dist=2, max_corners=4096)
    (got, _), = run(det, [im], **kw)
    want = oracle_corners(im, **kw)
    assert len(want) == 4096
    assert np.array_equal(got, want)


def test_candidates_exhausted_before_max_corners(det):
    # the frame cannot hold max_corners corners min_dist apart: every window
    # of candidates is gathered and decided, most of them already blocked by
    # corners of earlier windows (the case of a top-up beside many tracked
    # points); with and without occupied points, and a small min_dist whose
    # taken-corner grid needs cells larger than min_dist
    im = texture(480, 752, 11)
    rng = np.random.default_rng(4)
    occ = np.column_stack([rng.uniform(0, 752, 200), rng.uniform(0, 480, 200)]).astype(np.float32)
    for kw, o in ((dict(r=1, quality=0.001, min_dist=30, max_corners=4096), None),
                  (dict(r=1, quality=0.001, min_dist=30, max_corners=4096), occ),
                  (dict(r=1, quality=0.005, min_dist=3, max_corners=4096), occ)):
        (got, _), = run(det, [im], occupied=[o], **kw)
        want = oracle_corners(im, occ=o, **kw)
        assert len(want) < kw["max_corners"]
        assert np.array_equal(got, want), (kw, o is None)


def test_ties_and_plateaus(det):
    # a periodic pattern gives many exactly equal responses: ties are broken
    # by raster index, plateaus of equal maxima are all candidates
    y, x = np.mgrid[0:96, 0:160]
    im = np.where(((x // 4) + (y // 4)) % 2 == 0, 40, 210).astype(np.uint8)
    for kw in (dict(r=1, quality=0.01, min_dist=3, max_corners=4096),
               dict(r=2, quality=0.5, min_dist=0, max_corners=4096),
               dict(r=1, quality=0.01, min_dist=9, max_corners=37),
               # a threshold a few ulps below the maximum: the candidates are
               # the maxima, their R bits agree with the threshold's in all
               # but the last few, so their bucket is made of the last R bits
               # and the first bits of the index
               dict(r=1, quality=1.0 - 2.0 ** -50, min_dist=3, max_corners=4096),
               dict(r=1, quality=1.0 - 2.0 ** -50, min_dist=0, max_corners=25)):
        (got, _), = run(det, [im], **kw)
        want = oracle_corners(im, **kw)
        assert len(want) > 0 and np.array_equal(got, want), kw


def test_threshold_an_ulp_below_the_maximum(det):
    """quality 1 - 2^-50 on textured frames: the threshold's R bits agree
    with the maximum's in their first 59-61 bits, so the candidates' bucket
    straddles the R bits and the index bits of the rank key."""
    imgs = [texture(97, 131, 70 + k) for k in range(5)]
    kw = dict(r=1, quality=1.0 - 2.0 ** -50, min_dist=0, max_corners=10)
    outs = run(det, imgs, **kw)
    for im, (got, _) in zip(imgs, outs):
        want = oracle_corners(im, **kw)
        assert len(want) >= 1 and np.array_equal(got, want)


def test_flat_and_tiny_frames(det):
    flat = np.full((40, 50), 77, np.uint8)
    (got, R), = run(det, [flat], response=True)
    assert len(got) == 0 and np.all(R == 0.0)
    tiny = texture(3, 3, 1)
    (got, _), = run(det, [tiny], min_dist=0, max_corners=9, quality=0.0)
    assert np.array_equal(got, oracle_corners(tiny, min_dist=0, max_corners=9, quality=0.0))


def test_occupied_points(det):
    im = texture(480, 752, 5)
    rng = np.random.default_rng(0)
    occ = np.column_stack([rng.uniform(-5, 757, 1500), rng.uniform(-5, 485, 1500)]).astype(np.float32)
    for n in (1, 300, 1500):
        kw = dict(r=1, quality=0.001, min_dist=12, max_corners=400)
        (got, _), = run(det, [im], occupied=[occ[:n]], **kw)
        want = oracle_corners(im, occ=occ[:n], **kw)
        assert np.array_equal(got, want), n


def test_occupied_points_short_distances_and_full_cover(det):
    """Frames with occupied points (which the compaction filters by) beside
    frames without (which it marks in keep bits) in one call: occupied points
    with min_dist 0 (they block nothing), 1 and 5, and a 6-pixel grid of them
    that at min_dist 5 blocks every peak (no candidate is left)."""
    shapes = [(97, 131), (97, 131), (97, 131), (120, 90)]
    imgs = [texture(h, w, 60 + i) for i, (h, w) in enumerate(shapes)]
    rng = np.random.default_rng(7)
    scatter = np.column_stack([rng.uniform(-3, 134, 200), rng.uniform(-3, 100, 200)]).astype(np.float32)
    gx, gy = np.meshgrid(np.arange(0, 137, 6), np.arange(0, 103, 6))   # past the edges too
    cover = np.column_stack([gx.ravel(), gy.ravel()]).astype(np.float32)
    occ = [scatter, cover, None, scatter[:50]]
    for md in (0, 1, 5):
        kw = dict(r=1, quality=0.001, min_dist=md, max_corners=500)
        print("occupied short distances min_dist=%d" % md, flush=True)
        outs = run(det, imgs, occupied=occ, **kw)
        for k, (im, o, (got, _)) in enumerate(zip(imgs, occ, outs)):
            want = oracle_corners(im, occ=o, **kw)
            assert np.array_equal(got, want), (md, k)
        if md == 5:
            assert len(outs[1][0]) == 0


def test_batched_frames_of_mixed_sizes(det):
    shapes = [(480, 640), (480, 752), (600, 960), (720, 1280), (33, 47), (1080, 1920)]
    imgs = [texture(h, w, 20 + i) for i, (h, w) in enumerate(shapes)]
    rng = np.random.default_rng(1)
    occ = [None if i % 2 else np.column_stack([rng.uniform(0, w, 100), rng.uniform(0, h, 100)]).astype(np.float32)
           for i, (h, w) in enumerate(shapes)]
    kw = dict(r=1, quality=0.01, min_dist=20, max_corners=300, border=8)
    outs = run(det, imgs, occupied=occ, pitch_pad=13, **kw)
    for im, o, (got, _) in zip(imgs, occ, outs):
        assert np.array_equal(got, oracle_corners(im, occ=o, **kw))


def test_detector_argument_errors(det):
    im = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    out = torch.zeros((8, 2), dtype=torch.float32, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int32, device="cuda")
    f = [{"img": im, "out_xy": out, "count": cnt}]
    for bad in (lk.gftt_params(4, 1, 8, 0, 0.01), lk.gftt_params(1, -1, 8, 0, 0.01),
                lk.gftt_params(1, 1, 5000, 0, 0.01), lk.gftt_params(1, 1, 8, -1, 0.01),
                lk.gftt_params(1, 1, 8, 0, -0.5), lk.gftt_params(1, 1, 8, 0, float("nan"))):
        with pytest.raises(lk.LKError):
            lk.lk_detect_corners(det, f, bad)
    with pytest.raises(lk.LKError):
        lk.lk_detect_corners(det, [{"img": im[:2], "out_xy": out, "count": cnt}], lk.gftt_params())
    big = torch.zeros((2000, 2000), dtype=torch.uint8, device="cuda")
    ctx = lk.lk_context_create(0)
    small = lk.lk_detector_create(ctx, 1, 1000)
    try:
        with pytest.raises(lk.LKError):
            lk.lk_detect_corners(small, [{"img": big, "out_xy": out, "count": cnt}], lk.gftt_params())
    finally:
        lk.lk_detector_destroy(small)
        lk.lk_context_destroy(ctx)
