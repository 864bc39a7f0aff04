"""The synthetic generators are seed-deterministic and carry the shapes the
paper prints (Table III resolutions, Sec. IV keypoint caps)."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_workload_shapes.json")


def test_resolutions_cover_the_papers_cameras():
    g = json.load(open(GOLDEN))
    for name, wh in g["camera_resolutions"].items():
        assert tuple(wh) in synth.RESOLUTIONS, name
    # the single-pair and sequence workloads use the EuRoC camera
    p = synth.pair(0)
    assert (p.width, p.height) == tuple(g["camera_resolutions"]["EuRoC"])
    assert synth.StereoSequence.__dataclass_fields__["width"].default == 752


def test_keypoint_ranges_span_the_caps():
    g = json.load(open(GOLDEN))
    streams = synth.batch_streams(0, n_streams=8, resolutions=((64, 48),))
    n = [len(s.pts) for s in streams]
    assert min(n) >= 150 and max(n) <= 1500
    assert 150 <= g["keypoint_cap_subt"] <= g["keypoint_cap"] <= 1500


def test_pair_is_seed_deterministic_and_in_range():
    a, b = synth.pair(3), synth.pair(3)
    assert np.array_equal(a.prev, b.prev) and np.array_equal(a.next, b.next)
    assert np.array_equal(a.pts, b.pts)
    assert a.prev.dtype == np.uint8 and a.pts.dtype == np.float32
    assert np.all(a.pts >= 16) and np.all(a.pts[:, 0] <= a.width - 17) and np.all(a.pts[:, 1] <= a.height - 17)
    assert np.all(np.abs(np.array(a.shift)) <= 8.0)
    np.testing.assert_allclose(a.gt - a.pts, np.tile(a.shift, (len(a.pts), 1)), atol=1e-5)
    c = synth.pair(4)
    assert not np.array_equal(a.prev, c.prev)


def test_stereo_sequence_motion_bounds():
    s = synth.StereoSequence(1, n_frames=200)
    pts = s.points(10, 50)
    for t in range(1, 200, 13):
        d = s.temporal_gt(t, pts) - pts
        assert np.abs(d).max() <= 12.0 + 0.2 * 752 * np.deg2rad(3.0)
    st = s.stereo_gt(10, pts) - pts
    assert 8.0 <= -st[:, 0].mean() <= 40.0
    f0 = s.frame(3)
    assert f0.shape == (480, 752) and f0.dtype == np.uint8


def test_serving_trace_rates():
    tr = synth.ServingTrace(0, n_streams=32, duration_s=4.0)
    counts = np.bincount([e[1] for e in tr.events], minlength=32)
    rates = np.array([sp.rate_hz for sp in tr.streams])
    assert np.all((rates >= 20) & (rates <= 30))
    assert abs(counts.sum() / 4.0 - rates.sum()) < 0.2 * rates.sum()
    times = [e[0] for e in tr.events]
    assert times == sorted(times)
