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
           os.path.join(CSRC, "hc_kernels.hip"), os.path.join(CSRC, "hc_track_group.hip"),
           os.path.join(CSRC, "hc_terms_q16.hip"), os.path.join(CSRC, "hc_terms_g16.hip"),
           os.path.join(CSRC, "hc_terms_g20.hip"), os.path.join(CSRC, "hc_terms_q14.hip"),
           os.path.join(CSRC, "hc_terms_g18.hip"), os.path.join(CSRC, "hc_terms_q10.hip"),
           os.path.join(CSRC, "hc_terms_g32.hip"),
           os.path.join(CSRC, "hc_lu.hip"),
           os.path.join(CSRC, "hc_peak.hip"), os.path.join(CSRC, "hc_scratch.hip"),
           os.path.join(CSRC, "hc_endgame.hip"), os.path.join(CSRC, "hc_distinct.hip"),
           os.path.join(CSRC, "hc_wave.hip"), os.path.join(CSRC, "hc_eval.hip")]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fPIC"]
# The 32-row group LUs of the standalone solver and of the 32-row term-list
# tracker are larger than the unroller's default budget for #pragma unroll;
# rolled, their register rows would go to scratch memory.  The matrix-core evaluation keeps its accumulators in
# ordinary VGPRs (gfx950 allows either file) rather than in AGPRs, which would
# cost a copy of every result before the Euler sums read it.
EXTRA_FLAGS = {"hc_lu.hip": ["-mllvm", "-pragma-unroll-threshold=65536"],
               "hc_terms_g32.hip": ["-mllvm", "-pragma-unroll-threshold=65536"],
               "hc_eval.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def build(verbose: bool = False) -> str:
    """Always compiles (the caller asked for a build); returns the library path.
    The sources compile to objects in parallel, then link into libhc.so."""
    import concurrent.futures
    import tempfile

    with tempfile.TemporaryDirectory(prefix="hc_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[hipcc(), *FLAGS, *EXTRA_FLAGS.get(os.path.basename(src), []), "-pthread", "-I", INCLUDE, "-I", CSRC,
                 "-c", src, "-o", obj]
                for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        workers = max(1, min(len(cmds), os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
