"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its sources and
a driver that calls every entry point at small sizes (L = 2 .. 10, both precisions,
Metropolis, heat bath, over-relaxation, renormalisation, taint tracking, replica
exchange, the own elementary functions) are built with gcc's sanitizers and run; any
out-of-bounds access, use of freed memory or undefined operation aborts the run."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def test_oracle_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preloaded library would precede the sanitizer runtime")
    exe = tmp_path / "oracle_sanitized"
    srcs = [os.path.join(ORACLE, f) for f in ("hsgo_common.c", "hsgo_f32.c", "hsgo_f64.c")]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-std=gnu11",
           "-I", ORACLE, *srcs, os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
           "-lm", "-lquadmath", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle sanitizer run: ok" in r.stdout
