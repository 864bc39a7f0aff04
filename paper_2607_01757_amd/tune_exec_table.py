"""Writes lk_exec_table.txt, the table of tuned execution shapes that
lk_batch_create reads when it is given no shape.

For every tracker configuration in CONFIGS and every cell of the bucket grid
(mean frame size per pair x mean keypoint count per pair, lk_exec_buckets),
one batch of synthetic streams of that cell is built, lk_batch_tune times
every candidate shape on it on this GPU, and the winner becomes the cell's
row.  Cells are represented by streams of one resolution (640x480, 960x600,
1280x720, 1920x1080) and one keypoint count (160, 384, 768, 1500); the cell
of the mixed 64-stream workload (resolutions 640x480 .. 1920x1080, 150-1500
keypoints) is tuned on that mixed set itself.

    python -m paper_2607_01757_amd.tune_exec_table [--out PATH] [--streams N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (window, levels, storage): the batched float32 and binary16 forms, and the
# binary16 form of the precision / serving configuration
CONFIGS = ((21, 3, 0), (21, 3, 1), (31, 4, 1))
CELL_RES = ((640, 480), (960, 600), (1280, 720), (1920, 1080))
CELL_KP = (160, 384, 768, 1500)


def tune_set(lk, ctx, streams, win, levels, storage, reps):
    import torch
    prev = [torch.from_numpy(s.prev).cuda() for s in streams]
    nxt = [torch.from_numpy(s.next).cuda() for s in streams]
    pp = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
    pn = [lk.lk_pyramid_create(ctx, s.width, s.height, levels, storage) for s in streams]
    lk.lk_build_pyramids(ctx, pp, prev)
    counts = [len(s.pts) for s in streams]
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(int)
    n = int(sum(counts))
    pts = torch.from_numpy(np.concatenate([s.pts for s in streams])).cuda()
    pairs = [(a, b, int(o), c) for a, b, o, c in zip(pp, pn, offs, counts)]
    params = lk.make_params(win, levels, 30, 0.01, 1e-6, 1.0 if win == 31 else 0.0)
    out, st, res, _ = lk.outputs(n, levels)
    b = lk.lk_batch_create(ctx, pn, nxt, pairs, pts, None, params, out, st, res, None,
                           config=lk.lk_exec_config(0, 0, 1, 0, 0, 0))
    cfg, ms = lk.lk_batch_tune(b, reps=reps)
    lk.lk_batch_destroy(b)
    for p in pp + pn:
        lk.lk_pyramid_destroy(p)
    mean_px = int(np.mean([s.width * s.height for s in streams]))
    rb, kb = lk.lk_exec_buckets(mean_px, int(np.mean(counts)))
    return rb, kb, cfg, ms


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=os.path.join(PKG, "lk_exec_table.txt"))
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    import synth
    from paper_2607_01757_amd import lk

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    ctx = lk.lk_context_create(0, 0)
    rows = {}
    t0 = time.time()
    sets = []
    for ri, (w, h) in enumerate(CELL_RES):
        base = synth.batch_streams(40 + ri, n_streams=args.streams, kp_range=(max(CELL_KP), max(CELL_KP)),
                                   resolutions=((w, h),))
        for kp in CELL_KP:
            sets.append(("%dx%d, %d keypoints" % (w, h, kp),
                         [synth.Pair(s.prev, s.next, s.pts[:kp]) for s in base]))
        print("streams of %dx%d ready (%.0f s)" % (w, h, time.time() - t0), flush=True)
    sets.append(("mixed 640x480..1920x1080, 150-1500 keypoints", synth.batch_streams(0, n_streams=args.streams)))
    for win, levels, storage in CONFIGS:
        for name, streams in sets:
            rb, kb, cfg, ms = tune_set(lk, ctx, streams, win, levels, storage, args.reps)
            rows[(win, levels, storage, rb, kb)] = (cfg, ms, name)
            print("win %d L%d %s, %s -> buckets (%d, %d): persistent %d bpc %d chunk %d wpg %d, %.3f ms" % (
                win, levels, "f16" if storage else "f32", name, rb, kb, cfg.persistent, cfg.blocks_per_cu,
                cfg.chunk, cfg.waves_per_group, ms), flush=True)
    lk.lk_context_destroy(ctx)
    with open(args.out, "w") as f:
        f.write("# Tuned execution shapes of prepared batched steps (lk_batch_create with no shape).\n")
        f.write("# Written by: python -m paper_2607_01757_amd.tune_exec_table --streams %d --reps %d\n"
                % (args.streams, args.reps))
        f.write("# arch win levels storage res_bucket kp_bucket persistent blocks_per_cu use_graph chunk "
                "waves_per_group ms_per_step  # tuned on\n")
        for key in sorted(rows):
            cfg, ms, name = rows[key]
            f.write("%s %d %d %d %d %d %d %d 1 %d %d %.4f  # %s\n" % (
                arch, *key, cfg.persistent, cfg.blocks_per_cu, cfg.chunk, cfg.waves_per_group, ms, name))
    print("wrote %d rows to %s" % (len(rows), args.out))


if __name__ == "__main__":
    main()
