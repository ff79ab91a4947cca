"""Builds the C part of the CPU oracle (cj_oracle.c -> _cj_oracle.so).

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU library; the library never
loads it.  Flags: -O3 without -march=native (the shared object travels to other
hosts), no fast-math and no floating-point contraction, so every operation is a
separately rounded IEEE double operation.  OpenMP parallelises the sweep over
rows only; each node is computed independently, so results do not depend on
the thread count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cj_oracle.c")
LIB = os.path.join(HERE, "_cj_oracle.so")

CFLAGS = ["-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose=False):
    """Compiles the oracle; returns the path of the shared object."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
