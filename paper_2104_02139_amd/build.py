"""Build libhyperlag.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2104_02139_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhyperlag.so")
SELFTEST_LIB = os.path.join(PKG, "libhl_selftest.so")
SELFTEST_SRC = os.path.join(CSRC, "hl_selftest.hip")
SOURCES = [os.path.join(CSRC, "hl_kernels.hip"), os.path.join(CSRC, "hl_adjoint.hip"),
           os.path.join(CSRC, "hl_refine.hip"), os.path.join(CSRC, "hl_mesh.hip"), os.path.join(CSRC, "hl_noalloc.hip"),
           os.path.join(CSRC, "hl_peaks.hip"), os.path.join(CSRC, "hl_api.hip")]
ARCH = os.environ.get("HL_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # host-side finite-difference self-test of the adjoint building blocks
    tmp = SELFTEST_LIB + ".tmp"
    cmd = [hipcc, *FLAGS, SELFTEST_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SELFTEST_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
