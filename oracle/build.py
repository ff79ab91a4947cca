"""Builds the C part of the CPU oracle (cj_oracle.c -> _cj_oracle.so).

TEST INFRASTRUCTURE ONLY: the oracle checks the GPU library; the library never
loads it.  Flags: -O3, no fast-math and no floating-point contraction, so every
operation is a separately rounded IEEE double operation.  OpenMP parallelises
the sweep over rows only; each node is computed independently, so results do
not depend on the thread count.

Two builds: _cj_oracle.so without -march=native (built once, it travels to
other hosts), and _cj_oracle_native.so with -march=native, built on the host
that runs it, for timing the oracle as a CPU baseline (same operations and
the same results: vector instructions change neither the rounding nor, with
contraction off, the operations).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cj_oracle.c")
LIB = os.path.join(HERE, "_cj_oracle.so")
LIB_NATIVE = os.path.join(HERE, "_cj_oracle_native.so")

CFLAGS = ["-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def build(verbose=False, native=False):
    """Compiles the oracle (native: with -march=native for this host); returns
    the path of the shared object."""
    out = LIB_NATIVE if native else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + (["-march=native"] if native else []) + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
