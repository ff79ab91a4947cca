"""Builds libcj.so (HIP kernels for gfx950 + host runtime) in the package directory.

    python -m paper_1705_00103_amd.build

Device code: -O3 for gfx950, no fast-math, no floating-point contraction
(the kernels write every fma explicitly, so all kernels that evaluate the
update produce the same bits), and no packed FP32 instructions.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcj.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = os.environ.get("CJ_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HIP_SOURCES = ["kernels.hip"]
HOST_SOURCES = ["plan.cpp", "runtime.cpp", "batch.cpp"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False, save_temps=False):
    """Compiles every source and links libcj.so; returns its path."""
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        extra = ["-save-temps=obj"] if save_temps else []
        _run([cc, "-x", "hip", "-c"] + COMMON + DEVICE + extra + [os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        # host-only sources: plain C++ against the HIP runtime headers
        _run([cc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c"] + COMMON
             + [os.path.join(CSRC, src), "-o", obj],
             verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([cc, "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, save_temps="--save-temps" in sys.argv)
