"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C solvers (oracle/pcg_oracle.c) run on small systems, and the
library's host-side tile cutting (build_tiles in csrc/tiles.hpp) on ragged
row-length patterns, each built with -fsanitize=address,undefined and
-fno-sanitize-recover so that any finding fails the run.  The HIP file is
built for the host only (the sanitizer flags apply to the host pass; no
kernel is launched).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


def test_oracle_c_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    cmd = [gcc, *SAN, "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    assert "0 failed checks" in _run(exe)


def test_tile_cutting_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tiles_driver")
    host = []
    for f in SAN:
        host += ["-Xarch_host", f]
    cmd = [hipcc, "--offload-arch=gfx950", "-std=c++17", "-I", os.path.join(ROOT, "include"), *host,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "sanitize", "tiles_driver.hip"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 of 15 patterns failed" in _run(exe)
