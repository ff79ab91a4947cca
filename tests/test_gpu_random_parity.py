"""Seeded random launch configurations through the C ABI, against the oracle.

Each case draws a grid (1..399 x 1..299 interior nodes), a stencil, homogeneous
data or a boundary frame, Chebyshev-Jacobi or plain Jacobi, a cycle length, a
blocking depth K, a tile height and a sweep count, so that strips, tile seams,
ragged edges, cycle ends and the shorter launch that finishes a cycle fall in
every position.  Bars: the single-sweep kernel within 1e-12 relative L2 of the
oracle's sweeps; the blocked kernel bit-identical to it (FP64 and FP32); the
frame returned as it was given.
"""
import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu

K64 = {5: (2, 3, 4, 6, 8, 10), 9: (2, 3, 4, 6, 8, 10), 17: (2, 3, 4)}
K32 = {5: (2, 4, 8), 9: (2, 4, 8), 17: (2, 3, 4)}
ROWS = (0, 1, 2, 3, 8, 16, 33, 64, 100)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _draw(seed, k_table):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(1, 400)), int(rng.integers(1, 300))
    st = int(rng.choice([5, 9, 17]))
    frame = bool(rng.integers(0, 2))
    M = int(rng.choice([4, 8, 16, 32]))
    K = int(rng.choice(k_table[st]))
    rows = int(rng.choice(ROWS))
    n = int(rng.integers(1, 2 * M + 6))
    return rng, nx, ny, st, frame, M, K, rows, n


@pytest.mark.parametrize("seed", range(48))
def test_random_fp64_sweeps(torch_cuda, seed):
    torch = torch_cuda
    rng, nx, ny, st, frame, M, K, rows, n = _draw(1000 + seed, K64)
    method = cj.JACOBI if rng.integers(0, 4) == 0 else cj.CHEBYSHEV
    print("case seed %d: %dx%d st %d frame %d method %d M %d K %d rows %d n %d"
          % (seed, nx, ny, st, frame, method, M, K, rows, n), flush=True)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=seed)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    if frame:
        G = inputs.frame_width(st)
        u0 = inputs.expxy_frame(nx, ny, G, interior=inputs.random_field(nx, ny, seed + 7))
    else:
        u0 = inputs.random_field(nx, ny, seed + 7)
    kw = dict(M=M, bc=bc, method=method)
    one = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-8, sweeps_per_launch=1, **kw), _dev(torch, f), one, n)
    blk = _dev(torch, u0)
    pk = cj.plan(nx, ny, st, 1e-8, sweeps_per_launch=K, tile_rows=rows, **kw)
    assert pk.sweeps_per_launch == K
    cj.sweeps(pk, _dev(torch, f), blk, n)
    got1, gotk = _host(one), _host(blk)
    assert np.array_equal(gotk, got1)
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-8, n, M=M, u0=u0, bc=cjm.BC_FRAME if frame else cjm.BC_ZERO,
                         method="jacobi" if method == cj.JACOBI else "chebyshev")
    assert _rel(got1, ref) <= 1e-12
    if frame:
        mask = np.ones(u0.shape, dtype=bool)
        mask[G:ny + G, G:nx + G] = False
        assert np.array_equal(gotk[mask], u0[mask])


@pytest.mark.parametrize("seed", range(16))
def test_random_fp32_blocked_sweeps_bitwise(torch_cuda, seed):
    torch = torch_cuda
    rng, nx, ny, st, frame, M, K, rows, n = _draw(2000 + seed, K32)
    print("case seed %d: FP32 %dx%d st %d M %d K %d rows %d n %d" % (seed, nx, ny, st, M, K, rows, n), flush=True)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=seed)
    u0 = inputs.random_field(nx, ny, seed + 3)
    kw = dict(M=M, precision=cj.F32_REFINE, inner_M=M)
    one = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-6, sweeps_per_launch=1, **kw), _dev(torch, f), one, n)
    blk = _dev(torch, u0)
    pk = cj.plan(nx, ny, st, 1e-6, sweeps_per_launch=K, tile_rows=rows, **kw)
    assert pk.sweeps_per_launch == K
    cj.sweeps(pk, _dev(torch, f), blk, n)
    assert np.array_equal(_host(blk), _host(one))


@pytest.mark.parametrize("seed", range(10))
def test_random_double_double_solves(torch_cuda, seed):
    """cj_solve_dd on seeded random grids, stencils, data and inner precisions:
    the oracle's extended-precision residual of u + u_lo meets the tolerance
    (below the FP64 floor of the grid) and u_lo is a low part."""
    torch = torch_cuda
    rng = np.random.default_rng(3000 + seed)
    nx, ny = int(rng.integers(1, 220)), int(rng.integers(1, 160))
    st = int(rng.choice([5, 9, 17]))
    frame = bool(rng.integers(0, 2))
    precision = cj.F64 if rng.integers(0, 2) else cj.F32_REFINE
    tol = 1e-14
    print("case seed %d: %dx%d st %d frame %d precision %d" % (seed, nx, ny, st, frame, precision), flush=True)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=seed)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    if frame:
        u0 = inputs.expxy_frame(nx, ny, inputs.frame_width(st))
    else:
        u0 = np.zeros((ny, nx))
    p = cj.plan(nx, ny, st, tol, precision=precision, bc=bc, max_cycles=60)
    u = _dev(torch, u0)
    lo = torch.zeros_like(u)
    r = cj.solve_dd(p, _dev(torch, f), u, lo)
    hi, lo = _host(u), _host(lo)
    ext = cjm.relative_residual_ext(st, f, hi, lo, nx, ny, bc=cjm.BC_FRAME if frame else cjm.BC_ZERO)
    print("  status %s, outer %d, relres %.3e, oracle (extended) %.3e" % (r["status"], r["cycles"],
                                                                          r["rel_residual"], ext), flush=True)
    assert r["status"] == "ok"
    assert ext <= 1.5 * tol
    assert np.all(np.abs(lo) <= np.spacing(np.abs(hi)) / 2)
