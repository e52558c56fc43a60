"""Builds libgdsw.so (host analysis + HIP kernels for gfx950) in the package
directory.  Run as ``python -m paper_2304_04876_amd.build``."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgdsw.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-fopenmp", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    tmp = tempfile.mkdtemp(prefix="gdsw_build_")
    try:
        objs = []
        for src in ("symbolic.cpp", "nd.cpp", "capi.cpp"):
            o = os.path.join(tmp, src + ".o")
            _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
            objs.append(o)
        o = os.path.join(tmp, "device.o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "device.hip"), "-o", o])
        objs.append(o)
        out = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", out, "-lgomp"])
        os.replace(out, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
