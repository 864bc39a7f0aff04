"""The FP64 oracle under host sanitizers: tests/san/oracle_driver.c (which
compiles oracle/lk_oracle.c into itself) built with AddressSanitizer +
UndefinedBehaviorSanitizer (leak checking on) and, separately, with
ThreadSanitizer (the oracle tracks keypoints on several threads), then run;
any sanitizer report fails the run."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "san", "oracle_driver.c")
BASE = ["gcc", "-O1", "-g", "-std=c99", "-D_GNU_SOURCE", "-fno-omit-frame-pointer", "-ffp-contract=off"]
SANITIZERS = {
    "asan_ubsan": (["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], {"ASAN_OPTIONS": "detect_leaks=1"}),
    "tsan": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_oracle_clean_under_sanitizer(kind, tmp_path):
    flags, env_extra = SANITIZERS[kind]
    exe = str(tmp_path / ("oracle_" + kind))
    build = subprocess.run(BASE + flags + [DRIVER, "-o", exe, "-lm", "-lpthread"], capture_output=True, text=True)
    if build.returncode != 0 and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtime not installed: " + build.stderr.strip()[:200])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, **env_extra)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-3000:]
    for marker in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:", "WARNING: ThreadSanitizer"):
        assert marker not in out, out[-3000:]
    assert "oracle sanitizer run ok" in run.stdout
