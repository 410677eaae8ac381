"""Sanitizer builds (CPU only).

The oracle: gcc builds oracle/pnref.c (serially: OpenMP pragmas ignored)
with tests/sanitize_oracle.c, which calls every oracle entry point on small
seeded systems (N = 2, 3, 7, 33; c = 30, inf, 3; eps = 1e-4, 0, 1e-2) and
on invalid arguments.

The library's host code: hipcc builds csrc/pn_api.hip with
tests/sanitize_host.cpp, sanitizers on the host pass only; without a GPU the
driver reaches argument validation of every entry point, the launch-shape
table and its queries across N = 2 ... 2^28, the error strings, and a valid
call that must fail cleanly at device set-up.

AddressSanitizer (with leak detection) and UndefinedBehaviorSanitizer abort
either run on any out-of-bounds access, use after free, leak, signed
overflow or other undefined behaviour."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe, marker):
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("no sanitizer runtime: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert run.returncode == 0, run.stdout[-1000:] + run.stderr[-3000:]
    assert marker in run.stdout


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    cmd = [gcc, "-O1", "-g", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-ffp-contract=off", "-o", exe,
           os.path.join(ROOT, "tests", "sanitize_oracle.c"),
           os.path.join(ROOT, "oracle", "pnref.c"), "-lm"]
    _build_and_run(cmd, exe, "all calls ok")


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "sanitize_host")
    pkg = os.path.join(ROOT, "paper_1801_07986_amd")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(pkg, "csrc"),
           os.path.join(ROOT, "tests", "sanitize_host.cpp"),
           os.path.join(pkg, "csrc", "pn_api.hip"), "-o", exe]
    _build_and_run(cmd, exe, "all calls ok")
