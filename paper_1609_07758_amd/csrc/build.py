"""Build libhofem.so in-tree: HIP kernels for gfx950 plus the binary128 host
precompute.  Usage: ``python paper_1609_07758_amd/csrc/build.py`` (or build()).

Every invocation recompiles all sources (a few tens of seconds).
"""
import os
import subprocess
import sys

CSRC = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(CSRC)
ROOT = os.path.dirname(PKG)
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhofem.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
CXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-Wall",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True):
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    o = os.path.join(OUT_DIR, "plan1d.o")
    _run(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, "plan1d.cpp"), "-o", o])
    objs.append(o)
    for src in ("kernels.hip", "operator.hip", "pcg.hip", "capi.hip"):
        o = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
