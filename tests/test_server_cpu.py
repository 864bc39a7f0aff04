"""The serving scheduler (paper_2607_01757_amd/csrc/lk_sched.cpp) on the CPU:
tests/server_cpu/sched_driver.cpp runs it over a fake device backend (a CPU
executor that tracks with the FP64 oracle after an injected latency and can
fail launches) through every case of the scheduler's contract -- results
and per-stream order, timing fields, continuous batching, admission by
resident bytes, full staging, close while in flight, unknown tickets,
device errors and host-side launch failures, invalid arguments, several
submitting threads.  Built plain, with AddressSanitizer +
UndefinedBehaviorSanitizer (leak checking on) and with ThreadSanitizer; any
failed check or sanitizer report fails the test."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2607_01757_amd", "csrc")
DRIVER = os.path.join(HERE, "server_cpu", "sched_driver.cpp")
ORACLE = os.path.join(ROOT, "oracle", "lk_oracle.c")
VARIANTS = {
    "plain": (["-O2"], {}),
    "asan_ubsan": (["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"],
                   {"ASAN_OPTIONS": "detect_leaks=1"}),
    "tsan": (["-O1", "-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


@pytest.mark.parametrize("kind", sorted(VARIANTS))
def test_scheduler_with_fake_backend(kind, tmp_path):
    flags, env_extra = VARIANTS[kind]
    obj = str(tmp_path / "lk_oracle.o")
    exe = str(tmp_path / ("sched_" + kind))
    steps = [
        ["gcc", "-g", "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off", *flags, "-c", ORACLE, "-o", obj],
        ["g++", "-g", "-std=c++17", "-Wall", *flags, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, DRIVER,
         os.path.join(CSRC, "lk_sched.cpp"), os.path.join(CSRC, "lk_errors.cpp"), obj, "-o", exe, "-lpthread", "-lm"],
    ]
    for cmd in steps:
        build = subprocess.run(cmd, capture_output=True, text=True)
        if build.returncode != 0 and "cannot find" in build.stderr:
            pytest.skip("sanitizer runtime not installed: " + build.stderr.strip()[:200])
        assert build.returncode == 0, build.stderr
    env = dict(os.environ, **env_extra)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-3000:]
    for marker in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in out, out[-3000:]
    assert "sched cpu run ok" in run.stdout
