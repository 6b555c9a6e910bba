"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc),
driven by tests/native/oracle_sanitize_driver.c over seeded problems and its edge
cases (one variable, no inequalities, no equalities, a replayed step count, a
non-finite input): every call returns the expected status with no sanitizer
report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-o", exe,
           os.path.join(ROOT, "tests", "native", "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "qp_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "FAILED" not in run.stdout and "runtime error" not in run.stderr, run.stdout + run.stderr
    assert run.stdout.count(" ok") == 7, run.stdout
