"""Compile the HIP library ``libmrcm.so`` for gfx950 (in-tree).

Usage: ``python -m paper_2104_04653_amd.build`` (or ``build()`` from Python).
The shared library is written next to this file and loaded by the ctypes
binding in ``paper_2104_04653_amd.mrcm``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmrcm.so")
SOURCES = ["api.hip", "local.hip", "local_mfma.hip", "local_mfma32.hip", "interface.hip", "surrogate.hip",
           "transport.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # the one-wavefront kernels keep their tiles in registers only when their
    # block loops are fully unrolled
    "-mllvm", "-pragma-unroll-threshold=60000",
]
# per-source additions: the local solves (latency-bound Gauss-Jordan chains
# at two wavefronts per SIMD) run about 1.5% faster with the ILP-maximising
# instruction scheduler; the interface kernels run slower with it
SOURCE_FLAGS = {
    "local_mfma.hip": ["-mllvm", "--amdgpu-sched-strategy=max-ilp"],
}


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every source (in parallel, one object each) and link
    libmrcm.so; returns the library path."""
    with tempfile.TemporaryDirectory(prefix="mrcm_build_") as tmpdir:
        procs = []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s + ".o")
            cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(s, []), *(extra_flags or []), "-c",
                   os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                   text=True)))
        objs, failed = [], []
        for s, obj, pr in procs:
            out, err = pr.communicate()
            if pr.returncode != 0:
                failed.append(s)
                sys.stderr.write(out + err)
            elif verbose and err.strip():
                sys.stderr.write(err)
            objs.append(obj)
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("linking libmrcm.so failed with exit code %d" % res.returncode)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
