"""Compile the HIP library ``libmrcm.so`` for gfx950 (in-tree).

Usage: ``python -m paper_2104_04653_amd.build`` (or ``build()`` from Python).
The shared library is written next to this file and loaded by the ctypes
binding in ``paper_2104_04653_amd.mrcm``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmrcm.so")
SOURCES = ["api.hip", "local.hip", "local_mfma.hip", "interface.hip", "surrogate.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # the one-wavefront kernels keep their tiles in registers only when their
    # block loops are fully unrolled
    "-mllvm", "-pragma-unroll-threshold=60000",
]


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every source into libmrcm.so; returns the library path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra_flags or []), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed with exit code %d" % res.returncode)
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
