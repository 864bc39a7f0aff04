"""The ctypes mirrors of the ABI structs have exactly the C layout of
include/lk.h (sizes and field offsets, printed by a C program compiled
here with gcc)."""
import ctypes as C
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "lk_params": ["win", "levels", "max_iters", "use_guess", "eps", "min_eig", "fb_thresh", "reserved"],
    "lk_pair": ["prev", "next", "pt_offset", "n", "reserved"],
    "lk_batch_desc": ["n_builds", "build_pyrs", "build_imgs", "build_pitches", "n_pairs", "pairs", "d_pts",
                      "d_guess", "params", "d_out_pts", "d_status", "d_residual", "d_iters"],
    "lk_exec_config": ["persistent", "blocks_per_cu", "use_graph", "chunk", "waves_per_group", "reserved"],
    "lk_server_config": ["max_streams", "max_points", "levels", "storage", "params", "max_batch", "inflight",
                         "queue_depth", "reserved", "hbm_budget_bytes"],
    "lk_timing": ["submit_ns", "launch_ns", "done_ns"],
    "lk_server_stats": ["frames", "batches", "points", "resident_bytes", "open_streams", "reserved"],
    "lk_gftt_params": ["radius", "min_dist", "max_corners", "border", "quality"],
    "lk_gftt_frame": ["img", "w", "h", "pitch", "n_occupied", "occupied", "out_xy", "count", "response"],
    "lk_pool_state": ["pts", "ids", "right", "count", "next_id", "stats"],
    "lk_pool_scratch": ["t_pts", "t_status", "c_pts", "c_ids", "c_count", "s_pts", "s_status"],
    "lk_pool_frame": ["stream", "reserved", "prev", "next", "right"],
    "lk_epi_set": ["p", "q", "n", "h", "samples", "fx", "fy", "cx", "cy", "counts", "inliers", "best", "model"],
}


@pytest.fixture(scope="module")
def c_layout():
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lk.h"', "int main(void) {"]
    for s, fields in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (s, s))
        for f in fields:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (s, f, s, f))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.check_output([exe]).decode()
    table = {}
    for line in out.splitlines():
        k, *rest = line.split()
        table[k if not rest[0] == "size" else k + ".size"] = int(rest[-1])
    return table


def test_struct_layouts(c_layout):
    from paper_2607_01757_amd import lk
    for s, fields in STRUCTS.items():
        cls = getattr(lk, s)
        assert C.sizeof(cls) == c_layout[s + ".size"], s
        for f in fields:
            assert getattr(cls, f).offset == c_layout["%s.%s" % (s, f)], (s, f)
