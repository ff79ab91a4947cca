"""GPU tests of chained blocked launches: consecutive K-sweep launches of a
cycle fused into one launch whose workgroups take (launch, tile) items in
order and wait for the neighbour tiles of the previous launch.  The result
must be bit-identical to separate launches (and so to one-sweep launches) for
every stencil, boundary kind, tile height (including heights that make the
tiles wait on each other all the time) and chain length; a solve with chained
launches must give the separate launches' bits, status and cycle count."""
import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

# The chained launch path these tests exercised was removed: its first GPU run
# (test_chained_sweeps_are_bitwise_separate_launches, 9-point K = 10 on
# 517 x 203 with 16-row tiles) did not finish within the 120 s test limit,
# its per-wait time limit did not end it either, and no cause was found by
# reading the kernel and its assembly.  The plan option they use no longer
# exists; they stay here, skipped, as the record of that case.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="chained launches removed after their first GPU run did not finish "
                                      "(cause not found)")]


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


CASES = [
    # stencil, K, nx, ny, tile rows, M, sweeps
    (9, 10, 517, 203, 16, 64, 2 * 64 + 3),       # odd number of whole launches per cycle, a K = 4 remainder
    (9, 8, 1000, 700, 64, 32, 3 * 32),
    (5, 10, 300, 1200, 24, 128, 128 + 41),
    (17, 4, 517, 203, 16, 32, 2 * 32 + 5),       # homogeneous data: reflected outer ring
    (17, 3, 260, 260, 12, 16, 3 * 16 + 2),
    (9, 2, 64, 64, 1, 16, 40),                   # one-row tiles: every item waits on its neighbours
    (9, 10, 1, 1, 0, 32, 70),
    (5, 6, 2100, 33, 33, 64, 64),
]


@pytest.mark.parametrize("st,K,nx,ny,rows,M,n", CASES)
@pytest.mark.parametrize("frame", [False, True])
def test_chained_sweeps_are_bitwise_separate_launches(torch_cuda, st, K, nx, ny, rows, M, n, frame):
    torch = torch_cuda
    print("case: stencil %d K %d %dx%d rows %d M %d sweeps %d frame %d" % (st, K, nx, ny, rows, M, n, frame),
          flush=True)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    f = _dev(torch, inputs.gaussian_bumps_rhs(nx, ny, seed=nx + ny))
    if frame:
        u0 = inputs.expxy_frame(nx, ny, inputs.frame_width(st))
        G = inputs.frame_width(st)
        u0[G:ny + G, G:nx + G] = inputs.random_field(nx, ny, seed=3, scale=1e-2)
    else:
        u0 = inputs.random_field(nx, ny, seed=3, scale=1e-2)
    outs = []
    for chain in (-1, 1):
        p = cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=K, tile_rows=rows, chain=chain, bc=bc)
        u = _dev(torch, u0)
        cj.sweeps(p, f, u, n)
        outs.append(_host(u))
        p.destroy()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("st", [9, 17])
def test_chained_solve_matches_separate_launches_and_the_oracle(torch_cuda, st):
    torch = torch_cuda
    nx, ny, tol = 611, 409, 1e-10
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=12)
    fd = _dev(torch, f)
    res = []
    for chain in (-1, 1):
        p = cj.plan(nx, ny, st, tol, chain=chain, tile_rows=32)
        u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
        r = cj.solve(p, fd, u)
        res.append((r["status"], r["cycles"], _host(u)))
    assert res[0][:2] == res[1][:2]
    assert np.array_equal(res[0][2], res[1][2])
    ref = cjm.solve(f, nx, ny, st, tol)
    assert (res[1][0], res[1][1]) == (ref["status"], ref["cycles"])
    assert np.linalg.norm(res[1][2] - ref["u"]) / np.linalg.norm(ref["u"]) <= 1e-12


def test_chained_tuned_solve_at_4096(torch_cuda):
    """The automatic configuration on a large grid (chained launches, tile height
    timed on chains at the first solve) gives the bits of separate launches at a
    fixed height."""
    torch = torch_cuda
    n, st, tol = 4096, 9, 1e-10
    fd = _dev(torch, inputs.gaussian_bumps_rhs(n, n, seed=1714))
    pa = cj.plan(n, n, st, tol)                       # chained, tuned
    pb = cj.plan(n, n, st, tol, chain=-1, tile_rows=128)
    ua = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    ub = torch.zeros_like(ua)
    ra = cj.solve(pa, fd, ua)
    rb = cj.solve(pb, fd, ub)
    print("tuned rows %d: %s %d cycles %.3f s; separate: %.3f s"
          % (pa.refresh_launch_info()[1], ra["status"], ra["cycles"], ra["seconds"], rb["seconds"]), flush=True)
    assert (ra["status"], ra["cycles"]) == (rb["status"], rb["cycles"])
    assert torch.equal(ua, ub)


def test_chained_batch_matches_separate_launches(torch_cuda):
    """Batched solves whose super-steps run as chained launches give the same
    bits, statuses and outer-step counts as separate launches; mixed stencils,
    tiny and thin grids included."""
    torch = torch_cuda
    shapes = inputs.log_uniform_shapes(30, seed=5, lo=16, hi=300) + [(1, 1), (517, 3), (3, 400)]
    stencils = [(5, 9, 17)[i % 3] for i in range(len(shapes))]
    tols = [(1e-6, 1e-8, 1e-10)[i % 3] for i in range(len(shapes))]
    fs = [_dev(torch, inputs.gaussian_bumps_rhs(nx, ny, seed=100 + i)) for i, (nx, ny) in enumerate(shapes)]
    out = []
    for chain in (-1, 1):
        b = cj.Batch(shapes, stencils, tols, chain=chain)
        us = [torch.zeros_like(f) for f in fs]
        res, stats = b.solve(fs, us)
        out.append((res, us, stats))
        b.destroy()
    (ra, ua, sa), (rb, ub, sb) = out
    print("separate: %d launches; chained: %d launches, %d super-steps" % (sa["launches"], sb["launches"],
                                                                           sb["supersteps"]), flush=True)
    assert sa["supersteps"] == sb["supersteps"]
    for i in range(len(shapes)):
        assert (ra[i]["status"], ra[i]["cycles"], ra[i]["sweeps"]) == (rb[i]["status"], rb[i]["cycles"],
                                                                        rb[i]["sweeps"])
        assert torch.equal(ua[i], ub[i])
