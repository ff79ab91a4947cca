"""The C ABI from C: include/cj.h compiles as strict C99, and a plain C caller
(tests/c_abi_caller.c) links libcj.so, makes the host-only calls on the CPU
and, on the GPU, solves through device buffers it allocates with hipMalloc."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1705_00103_amd")
ROCM = "/opt/rocm"


def _gcc():
    g = shutil.which("gcc")
    if not g:
        pytest.skip("no C compiler")
    return g


@pytest.fixture(scope="module")
def caller(tmp_path_factory):
    if not os.path.exists(cj.LIB_PATH):
        pytest.skip("libcj.so is not built")
    out = str(tmp_path_factory.mktemp("cabi") / "c_abi_caller")
    cmd = [_gcc(), "-std=c99", "-Wall", "-Wextra", "-Werror", "-O1", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_caller.c"), "-L", PKG, "-lcj", "-L", os.path.join(ROCM, "lib"),
           "-lamdhip64", "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return out


def test_header_is_strict_c99(tmp_path):
    src = tmp_path / "h.c"
    src.write_text('#include "cj.h"\nint main(void) { cj_options o; cj_options_init(&o); return o.M; }\n')
    r = subprocess.run([_gcc(), "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr


def test_c_caller_host_calls(caller):
    """Plan, plan info and launch info from C give what the binding reads for the
    same plan; an invalid stencil comes back as CJ_ERR_ARG with a message."""
    r = subprocess.run([caller, "host"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    m = re.search(r"plan M (\d+) cycles (\d+) kmin (\S+) kmax (\S+) w0 (\S+) w1 (\S+) workspace (\d+) K (\d+)",
                  r.stdout)
    p = cj.plan(129, 100, 9, 1e-10)
    assert (int(m.group(1)), int(m.group(2))) == (p.M, p.cycles_pred)
    assert float(m.group(3)) == p.kmin and float(m.group(4)) == p.kmax == 1.6
    assert (float(m.group(5)), float(m.group(6))) == (p.weights[0], p.weights[1])
    assert int(m.group(7)) == p.workspace_bytes and int(m.group(8)) == p.sweeps_per_launch
    assert "stencil 7: CJ_ERR_ARG (stencil must be 5, 9 or 17), plan null" in r.stdout


@pytest.mark.gpu
@pytest.mark.parametrize("st,nx,ny", [(9, 200, 150), (17, 97, 131)])
def test_c_caller_solves_on_the_gpu(caller, tmp_path, st, nx, ny):
    """A C program with hipMalloc'd buffers and the default stream solves to tol
    and returns the oracle's solution."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tol = 1e-10
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=60 + st)
    fin, uout = tmp_path / "f.bin", tmp_path / "u.bin"
    np.ascontiguousarray(f, dtype=np.float64).tofile(fin)
    print("case: C caller, %d-point %dx%d" % (st, nx, ny), flush=True)
    r = subprocess.run([caller, "solve", str(nx), str(ny), str(st), repr(tol), str(fin), str(uout)],
                       capture_output=True, text=True, timeout=120)
    print(r.stdout.strip(), flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "solve: CJ_OK" in r.stdout
    u = np.fromfile(uout, dtype=np.float64).reshape(ny, nx)
    ref = cjm.solve(f, nx, ny, st, tol)
    assert ref["status"] == "ok"
    err = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    print("rel-L2 vs oracle %.3e, relres (oracle) %.3e" % (err, cjm.relative_residual(st, f, u, nx, ny)), flush=True)
    assert err <= 1e-12
    assert cjm.relative_residual(st, f, u, nx, ny) <= tol * 1.01
