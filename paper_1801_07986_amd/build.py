"""Build libpn.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1801_07986_amd.build`` (also called by
``__graft_entry__.build()``).  The library is written next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpn.so")
SOURCES = [os.path.join(HERE, "csrc", "pn_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "pn_kernels.h"), os.path.join(ROOT, "include", "pn.h")]

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU
# instructions (v_pk_fma_f32 & co.); the host pass warns that it does not know
# the feature, which is harmless.
# -ffp-contract=off: every fused multiply-add in the kernels is an explicit
# fma(); the compiler may not fuse a*b + c on its own, which it otherwise
# decides per kernel, so that one source function inlined into two kernels
# (a single system's step and the batched step, say) rounds identically.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


def assembly(out: str) -> None:
    """Write the gfx950 assembly of the device code (for inspection)."""
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-S",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"), "-o", out,
           *SOURCES]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)


if __name__ == "__main__":
    print(build(verbose=True))
    if len(sys.argv) > 1:
        assembly(sys.argv[1])
