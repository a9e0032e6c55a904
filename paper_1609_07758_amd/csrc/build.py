"""Build libhofem.so in-tree: HIP kernels for gfx950 plus the binary128 host
precompute.  Usage: ``python paper_1609_07758_amd/csrc/build.py`` (or build()).

Every invocation recompiles all sources (a few tens of seconds).
"""
import concurrent.futures
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


def kernel_hash():
    """Hash of the line-pass sources (keys the autotuner's cache)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("linepass.h", "linepass.hip", "linepass_dispatch.hip", "kernels.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _jobs():
    """(command, object) for every translation unit; the line passes are
    compiled once per element order."""
    jobs = []
    o = os.path.join(OUT_DIR, "plan1d.o")
    jobs.append((["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, "plan1d.cpp"), "-o", o], o))
    for n in range(1, 10):
        o = os.path.join(OUT_DIR, f"linepass_{n}.o")
        jobs.append(([HIPCC] + HIP_FLAGS + [f"-DHOFEM_ORDER={n}", "-c",
                                            os.path.join(CSRC, "linepass.hip"), "-o", o], o))
    for src in ("linepass_dispatch.hip", "operator.hip", "pcg.hip", "capi.hip", "batch.hip",
                "timestep.hip", "banded.hip", "periodic.hip", "neumann.hip", "dense.hip"):
        o = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        extra = [f'-DHOFEM_KERNEL_HASH="{kernel_hash()}"'] if src == "capi.hip" else []
        jobs.append(([HIPCC] + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", o], o))
    return jobs


def build(verbose=True, jobs=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    todo = _jobs()
    workers = jobs or max(1, min(len(todo), os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda job: _run(job[0]), todo))
    objs = [o for _, o in todo]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
