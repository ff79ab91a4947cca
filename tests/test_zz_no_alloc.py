"""GPU test of cj_residual_noalloc, the allocation-free form of cj_residual:
through the C ABI, on two calls in a row (the second on a smaller grid, so
the scratch array holds the first call's partial sums when it starts), its
value equals cj_residual's on the same inputs (same partial sums, same
order); both match the oracle's residual.  Also a frame problem, the three
stencils, a value captured in a HIP graph and replayed, and the size limit."""
import ctypes

import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _noalloc(torch, p, fd, ud):
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    cj.residual_noalloc(p, fd, ud, out)
    torch.cuda.synchronize()
    return float(out.item())


@pytest.mark.parametrize("st", [9, 5, 17])
def test_noalloc_residual_matches_cj_residual_twice(torch_cuda, st):
    torch = torch_cuda
    for (nx, ny), seed in (((1000, 700), 1), ((130, 33), 2)):     # the second call is smaller
        print("case: stencil %d, %dx%d" % (st, nx, ny), flush=True)
        f = inputs.gaussian_bumps_rhs(nx, ny, seed=seed)
        u0 = inputs.random_field(nx, ny, seed=seed + 10, scale=1e-3)
        p = cj.plan(nx, ny, st, 1e-8)
        fd, ud = _dev(torch, f), _dev(torch, u0)
        got = _noalloc(torch, p, fd, ud)
        ref = cj.residual(p, fd, ud)
        orc = cjm.relative_residual(st, f, u0, nx, ny)
        print("  noalloc %.17g  cj_residual %.17g  oracle %.17g" % (got, ref, orc), flush=True)
        assert got == ref
        assert abs(got - orc) <= 1e-12 * orc


def test_noalloc_residual_frame_and_zero_rhs(torch_cuda):
    torch = torch_cuda
    nx, ny, st = 301, 157, 17
    G = inputs.frame_width(st)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=4)
    u0 = inputs.expxy_frame(nx, ny, G)
    u0[G:ny + G, G:nx + G] = inputs.random_field(nx, ny, seed=5, scale=1e-2)
    p = cj.plan(nx, ny, st, 1e-8, bc=cj.BC_FRAME)
    fd, ud = _dev(torch, f), _dev(torch, u0)
    got = _noalloc(torch, p, fd, ud)
    ref = cj.residual(p, fd, ud)
    orc = cjm.relative_residual(st, f, u0, nx, ny, bc=cjm.BC_FRAME)
    print("frame: noalloc %.17g  cj_residual %.17g  oracle %.17g" % (got, ref, orc), flush=True)
    assert got == ref
    assert abs(got - orc) <= 1e-12 * orc
    # zero right-hand side, homogeneous data: 0 by definition
    q = cj.plan(64, 64, 9, 1e-8)
    z = torch.zeros(64, 64, dtype=torch.float64, device="cuda")
    assert _noalloc(torch, q, z, _dev(torch, inputs.random_field(64, 64, 3))) == 0.0


def test_noalloc_residual_in_a_replayed_graph(torch_cuda):
    """Captured once into a HIP graph and replayed with new contents of u
    between replays (eager work in between): every replay gives cj_residual's
    value for the u it saw."""
    torch = torch_cuda
    nx, ny, st = 517, 259, 9
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=8)
    p = cj.plan(nx, ny, st, 1e-8)
    fd = _dev(torch, f)
    ud = _dev(torch, inputs.random_field(nx, ny, seed=9, scale=1e-3))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        cj.residual_noalloc(p, fd, ud, out, stream=s)      # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cj.residual_noalloc(p, fd, ud, out, stream=s)
    torch.cuda.synchronize()
    for k in range(4):
        ud.copy_(_dev(torch, inputs.random_field(nx, ny, seed=20 + k, scale=10.0 ** -k)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = float(out.item())
        ref = cj.residual(p, fd, ud)
        print("replay %d: %.17g vs %.17g" % (k, got, ref), flush=True)
        assert got == ref


def test_noalloc_residual_rejects_grids_beyond_its_scratch(torch_cuda):
    """More than 65536 residual tiles: CJ_ERR_ARG before any device work."""
    p = cj.plan(16384, 16385, 9, 1e-8)             # 64 x 1025 tiles of 256 x 16
    L = cj.lib()
    code = L.cj_residual_noalloc(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4096), ctypes.c_void_p(4096),
                                 None)
    assert code == cj.CJ_ERR_ARG
    assert "65536" in cj.last_error()
