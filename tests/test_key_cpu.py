"""The detector's rank-key helpers (paper_2607_01757_amd/csrc/lk_key.h),
built for the host, against Python integers: the 96-bit key (R bits, then
the complemented raster index), its 8-bit digits at any bit position, prefix
equality, the key order and the least key with a given prefix and digit --
the arithmetic the bucket layout and the radix selection rest on."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2607_01757_amd", "csrc")
M96 = (1 << 96) - 1


def digit(K, p):
    # bits [p, p + 8) counted from the most significant of 96; zeros past the end
    return ((K << 8) >> (96 - p)) & 0xFF


def with_digit(Q, p, v):
    head = (Q >> (96 - p)) << (96 - p) if p else 0
    return (head | ((v << 88) >> p)) & M96


def test_key_helpers_against_integers(tmp_path):
    exe = str(tmp_path / "key_driver")
    build = subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I" + CSRC, os.path.join(HERE, "key_cpu", "key_driver.cpp"),
                            "-o", exe], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    out = subprocess.run([exe, "20000", "7"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.split("\n")[:-1]
    assert len(lines) == 20000
    shared = 0
    for line in lines:
        f = line.split()
        K = (int(f[0], 16) << 32) | int(f[1], 16)
        Q = (int(f[2], 16) << 32) | int(f[3], 16)
        p, pe, v, d, eq, less = (int(x) for x in f[4:10])
        W = (int(f[10], 16) << 32) | int(f[11], 16)
        assert d == digit(K, p), line
        assert eq == int(pe == 0 or ((K ^ Q) >> (96 - pe)) == 0), line
        assert less == int(K < Q), line
        assert W == with_digit(Q, p, v), line
        # W is the least key with Q's leading p bits and digit v at p (where
        # the digit lies inside the key): W has them, and any key that has
        # them is at least W
        if p <= 88:
            assert digit(W, p) == v and (p == 0 or (W ^ Q) >> (96 - p) == 0), line
            low = (1 << (96 - p - 8)) - 1
            assert W & low == 0, line
        shared += eq
    assert shared > 1000        # the prefix cases were exercised
