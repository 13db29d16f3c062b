"""Builds libhc.so (the C-ABI library with the gfx950 kernels) in the package directory.

    python -m paper_2112_03444_amd.build

hipcc compiles the kernels for gfx950 only.  Packed-FP32 instructions are switched
off (-packed-fp32-ops): plain float code is compiled to scalar FP32 VALU ops.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhc.so")
SOURCES = [os.path.join(CSRC, "hc_api.cpp"), os.path.join(CSRC, "hc_server.cpp"),
           os.path.join(CSRC, "hc_kernels.hip"), os.path.join(CSRC, "hc_track_group.hip")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def compile_cmd(out: str):
    return [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-fPIC", "-shared", "-pthread", "-I", INCLUDE, "-I", CSRC, *SOURCES, "-o", out]


def build(verbose: bool = False) -> str:
    """Always compiles (the caller asked for a build); returns the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = compile_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
