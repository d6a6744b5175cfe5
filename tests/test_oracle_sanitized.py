"""The C oracle built with AddressSanitizer + UndefinedBehaviorSanitizer (host code only) and run
on closed-form, edge and invalid-argument cases by tests/sanitized/oracle_driver.c: any
out-of-bounds access or undefined arithmetic on those paths aborts the driver, and the driver's
exit status counts failed checks."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp",
           str(ROOT / "oracle" / "demap_oracle.c"), str(ROOT / "tests" / "sanitized" / "oracle_driver.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(res.stdout[-3000:], res.stderr[-3000:])
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "0 failure(s)" in res.stdout
