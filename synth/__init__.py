"""Seeded synthetic inputs (textures, motion, arrival traces).  Shared by the
tests, the benchmark and the oracle checks; contains none of the tracker's
arithmetic."""
from .texture import make_rng, quantize_u8, texture_canvas  # noqa: F401
from .workloads import (RESOLUTIONS, FramePool, Pair, ServingTrace,  # noqa: F401
                        StereoSequence, TwoView, batch_streams, pair, ransac_samples, two_view, uniform_points)
