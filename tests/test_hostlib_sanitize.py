"""The host side of libhsg under AddressSanitizer and UndefinedBehaviorSanitizer:
`api.hip` is rebuilt with the sanitizers on its host code only (the kernels are the
library's own objects), linked with a driver that calls every entry point with the
arguments its checks must reject, every lattice size, the chain-table check and the tile
table (tests/hostlib_sanitize_driver.cpp); any out-of-bounds access, use of freed memory
or undefined operation aborts the run.  (It found a signed overflow in the chain-table
check: an offset near the int64 limit plus the chain's size.)  CPU only: the driver
reaches no kernel."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1006_2566_amd", "csrc")
OBJS = os.path.join(ROOT, "paper_1006_2566_amd", "_build")
KERNELS = ["kernels_sweep", "kernels_lattice", "kernels_batch", "kernels_march",
           "kernels_observe", "kernels_phase"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_host_library_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and shutil.which("g++")):
        pytest.skip("hipcc or g++ not available")
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a preloaded library would precede the sanitizer runtime")
    objs = [os.path.join(OBJS, f"{k}.hip.o") for k in KERNELS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("the library's objects are not built (paper_1006_2566_amd.build)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    api = str(tmp_path / "api_sanitized.o")
    subprocess.run(
        [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", *inc,
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
         "-c", os.path.join(CSRC, "api.hip"), "-o", api], check=True, capture_output=True)
    drv = str(tmp_path / "driver.o")
    subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
         "-I", "/opt/rocm/include", *inc, "-c",
         os.path.join(ROOT, "tests", "hostlib_sanitize_driver.cpp"), "-o", drv],
        check=True, capture_output=True)
    exe = str(tmp_path / "hostlib_sanitized")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address", "-fsanitize=undefined",
                    "-fno-gpu-sanitize", drv, api, *objs, "-o", exe],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed expectations" in r.stdout
