#!/usr/bin/env python3
"""Benchmark of the pyramidal LK hot path on one MI355X.

Default workload ("batched"): 64 independent camera streams, resolution
uniform over {640x480, 752x480, 960x600, 1280x720, 1920x1080}, U[150, 1500]
keypoints per frame, sub-pixel shifts up to 8 px with noise sigma 2;
21x21 window, 3 levels, 30 iterations, eps 0.01, float32 storage.  One step
is the steady state of all streams: the new frame of every stream gets its
pyramid (one launch per level for all frames) and every keypoint is tracked
from the resident previous pyramid in one launch.  The same frames are also
run through the plain per-frame path (one pyramid build and one tracker
launch per stream) for comparison.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, GB/s
PEAK_FP32_TFLOPS = 157.3       # MI355X fp32 vector (packed); 78.6 without packed FP32
# algorithmic flops per window pixel: 29 per level for the template (three
# bilinear samples, the normal matrix), 13 per Gauss-Newton iteration (one
# bilinear sample, the mismatch and its two products)
FLOP_TEMPLATE, FLOP_ITER = 29, 13


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else 0.0


def level_dims(w, h, levels):
    out = [(w, h)]
    for _ in range(1, levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        out.append((w, h))
    return out


def footprint_bytes(pts, ends, w, h, levels, win, store_bytes):
    """Unique bytes of the window footprints the tracker must read: template
    windows (win+3)^2 around p / 2^l in the previous pyramid and target
    windows (win+1)^2 covering start and end in the next one."""
    hw = (win - 1) // 2
    total = 0
    for l, (lw, lh) in enumerate(level_dims(w, h, levels)):
        s = 1 if l == 0 else store_bytes
        for pts_l, ext in ((pts / 2 ** l, hw + 2), (None, hw + 1)):
            diff = np.zeros((lh + 1, lw + 1), np.int32)
            if pts_l is not None:
                x0 = np.floor(pts_l[:, 0]) - ext + 1
                x1 = np.floor(pts_l[:, 0]) + ext + 1
                y0 = np.floor(pts_l[:, 1]) - ext + 1
                y1 = np.floor(pts_l[:, 1]) + ext + 1
            else:
                a, b = pts / 2 ** l, ends / 2 ** l
                lo, hi = np.minimum(a, b), np.maximum(a, b)
                x0 = np.floor(lo[:, 0]) - ext
                x1 = np.floor(hi[:, 0]) + ext + 2
                y0 = np.floor(lo[:, 1]) - ext
                y1 = np.floor(hi[:, 1]) + ext + 2
            x0 = np.clip(x0, 0, lw).astype(int); x1 = np.clip(x1, 0, lw).astype(int)
            y0 = np.clip(y0, 0, lh).astype(int); y1 = np.clip(y1, 0, lh).astype(int)
            np.add.at(diff, (y0, x0), 1); np.add.at(diff, (y0, x1), -1)
            np.add.at(diff, (y1, x0), -1); np.add.at(diff, (y1, x1), 1)
            cover = np.cumsum(np.cumsum(diff, 0), 1)[:lh, :lw] > 0
            total += int(cover.sum()) * s
    return total


def flops_from_iters(iters, win, fb):
    """Algorithmic flops of the tracker from per-point iteration counts
    (N x 2 x L: forward / backward)."""
    nw = win * win
    it = iters.astype(np.int64)
    L = it.shape[2]
    passes = 1 + (1 if fb else 0)
    per = nw * FLOP_TEMPLATE * L * passes
    return float(len(it) * per + nw * FLOP_ITER * it.sum())


# ---------------------------------------------------------------- workloads

def make_streams(n_streams, seed):
    import synth
    t0 = time.time()
    streams = synth.batch_streams(seed, n_streams=n_streams)
    log("generated %d streams in %.1fs (%d keypoints)" % (n_streams, time.time() - t0,
                                                        sum(len(s.pts) for s in streams)))
    return streams


class BatchedWorkload:
    def __init__(self, lk, ctx, streams, win=21, levels=3, storage=0, fb=0.0):
        import torch
        self.lk, self.ctx, self.streams = lk, ctx, streams
        self.win, self.levels, self.storage, self.fb = win, levels, storage, fb
        self.prev_img = [torch.from_numpy(s.prev).cuda() for s in streams]
        self.next_img = [torch.from_numpy(s.next).cuda() for s in streams]
        self.prev_pyr = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
        self.next_pyr = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
        lk.lk_build_pyramids(ctx, self.prev_pyr, self.prev_img)
        counts = [len(s.pts) for s in streams]
        self.offsets = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
        self.n = int(sum(counts))
        self.pts = torch.from_numpy(np.concatenate([s.pts for s in streams])).cuda()
        self.pairs = [(a, b, int(o), c) for a, b, o, c in zip(self.prev_pyr, self.next_pyr, self.offsets, counts)]
        self.params = lk.make_params(win, levels, 30, 0.01, 1e-6, fb)
        self.out, self.st, self.res, self.it = lk.outputs(self.n, levels, with_iters=True)
        torch.cuda.synchronize()

    def build(self):
        self.lk.lk_build_pyramids(self.ctx, self.next_pyr, self.next_img)

    def track(self, iters=False):
        self.lk.lk_track_batched(self.ctx, self.pairs, self.pts, None, self.params, self.out, self.st,
                                 self.res, self.it if iters else None)

    def step(self):
        self.build()
        self.track()

    def plain_frame(self, i):
        lk, s = self.lk, self.streams[i]
        lk.lk_build_pyramid(self.ctx, self.next_pyr[i], self.next_img[i])
        o, c = int(self.offsets[i]), len(s.pts)
        lk.lk_track(self.ctx, self.prev_pyr[i], self.next_pyr[i], self.pts[o:o + c], None, c, self.params,
                    self.out[o:o + c], self.st[o:o + c], self.res[o:o + c], None)

    def close(self):
        for p in self.prev_pyr + self.next_pyr:
            self.lk.lk_pyramid_destroy(p)


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def cpu_baseline(streams, n_sample, win, levels, fb):
    import oracle
    threads = os.cpu_count() or 1
    sample = streams[:n_sample]
    npts = sum(len(s.pts) for s in sample)
    t0 = time.perf_counter()
    for s in sample:
        oracle.track(s.prev, s.next, s.pts, win=win, levels=levels, min_eig=1e-6, fb_thresh=fb, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": npts / dt, "unit": "keypoints/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d streams, all %d of their keypoints; the oracle builds both pyramids of "
                      "each pair (FP64) and tracks on %d threads; %.1f s wall" % (n_sample, len(streams), npts,
                                                                                  threads, dt)}


def run_batched(args):
    import torch
    from paper_2607_01757_amd import lk

    streams = make_streams(args.streams, args.seed)
    ctx = lk.lk_context_create(0, 0)
    wl = BatchedWorkload(lk, ctx, streams)
    log("resident: %.1f MB of pyramids, %d keypoints" % (lk.lk_context_bytes_in_use(ctx) / 1e6, wl.n))
    # one untimed step with iteration counts (deterministic: same counts when timed)
    wl.step()
    wl.track(iters=True)
    torch.cuda.synchronize()
    iters = wl.it.cpu().numpy()
    status = wl.st.cpu().numpy()
    ends = wl.out.cpu().numpy()
    f_alg = flops_from_iters(iters, wl.win, False)

    # tracker kernel alone (the dominant kernel), HIP events on the launch stream
    _, trk = time_steps(wl.track, args.steps, args.warmup)
    t_trk = float(np.mean(trk)) * 1e-3
    # pyramid build alone
    _, pyr = time_steps(wl.build, args.steps, args.warmup)
    # whole step
    wall, per = time_steps(wl.step, args.steps, args.warmup)
    kps = wl.n * args.steps / wall
    log("batched: %.3f ms/step  %.3g kp/s  tracker %.3f ms  pyramids %.3f ms" %
        (wall / args.steps * 1e3, kps, t_trk * 1e3, np.mean(pyr)))

    # plain per-frame launches over the same frames
    plain = None
    if not args.no_plain:
        def plain_step():
            for i in range(len(streams)):
                wl.plain_frame(i)
        pw, pper = time_steps(plain_step, max(2, args.steps // 4), max(1, args.warmup // 2))
        # per-frame latency of the plain path: each frame alone, events around it
        lat = []
        for i in range(len(streams)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(); wl.plain_frame(i); b.record()
            torch.cuda.synchronize()
            lat.append(a.elapsed_time(b))
        plain = {"value": wl.n * max(2, args.steps // 4) / pw, "unit": "keypoints/s",
                 "ms_per_step": pw / max(2, args.steps // 4) * 1e3,
                 "p50_frame_ms": percentile(lat, 50), "p99_frame_ms": percentile(lat, 99)}
        log("plain: %.3f ms/step  %.3g kp/s" % (plain["ms_per_step"], plain["value"]))

    # algorithmic bytes of one step (whole path)
    b_frames = sum(s.width * s.height for s in streams)
    b_levels = sum(4 * sum(w * h for (w, h) in level_dims(s.width, s.height, 3)[1:]) for s in streams)
    b_windows = 0
    off = 0
    for s in streams:
        c = len(s.pts)
        b_windows += footprint_bytes(s.pts.astype(np.float64), ends[off:off + c].astype(np.float64),
                                     s.width, s.height, 3, 21, 4)
        off += c
    b_io = wl.n * (8 + 8 + 1 + 4)
    b_alg = b_frames + b_levels + b_windows + b_io
    step_s = wall / args.steps

    result = {
        "metric": "tracked keypoints/sec (batched, 64 streams) + p50/p99 frame latency",
        "value": kps, "unit": "keypoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 64 streams, resolutions {640x480..1920x1080}, U[150,1500] keypoints, "
                               "21x21 window, 3 levels, 30 iterations, eps 0.01, float32 storage",
                   "streams": len(streams), "keypoints_per_step": wl.n, "seed": args.seed},
        "p50_frame_ms": percentile(per, 50), "p99_frame_ms": percentile(per, 99),
        "tracked_fraction": float(np.mean(status == 0)),
        "roofline": {"bound": "alu", "kernel": "k_track_batched", "achieved": f_alg / t_trk / 1e12,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": f_alg / t_trk / 1e12 / PEAK_FP32_TFLOPS,
                     "traffic": None, "flops_per_launch": f_alg, "kernel_ms": t_trk * 1e3},
        "path_hbm": {"algorithmic_bytes": b_alg, "achieved_GBs": b_alg / step_s / 1e9,
                     "frac": b_alg / step_s / 1e9 / PEAK_HBM_GBS},
        "pyramid_ms": float(np.mean(pyr)),
        "plain": plain,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        result["cpu_baseline"] = cpu_baseline(streams, args.cpu_streams, 21, 3, 0.0)
    wl.close()
    lk.lk_context_destroy(ctx)
    return result


def run_copy(args):
    """Plain device copy of a known size (calibrates rocprof byte counters)."""
    import torch
    n = 256 << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"metric": "device copy", "bytes_read": n, "bytes_written": n, "launches": 3}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched", choices=["batched", "copy"])
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-streams", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (streams would be sharded "
              "across GPUs with no exchange, see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        res = run_copy(args)
    else:
        res = run_batched(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
