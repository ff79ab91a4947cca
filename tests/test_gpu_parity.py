"""GPU parity: libcj.so (through its C ABI) against the CPU oracle.

Bar (FP64 path): relative L2 difference <= 1e-12 on the same inputs and the same
weight schedule; statuses and cycle counts identical.  Inputs come from
paper_1705_00103_amd.inputs; expected values from oracle/ only.
"""
import ctypes
import math
import sys

import numpy as np
import pytest

from oracle import cjm, dense
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu

REL_L2 = 1e-12       # FP64 parity bar


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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c1_manufactured_full_solve(torch_cuda):
    """128 x 128 interior, 9-point, f = -Delta(sin pi x sin pi y), tol 1e-10."""
    torch = torch_cuda
    n, st, tol = 128, 9, 1e-10
    _say("case: C1 128x128 9-point")
    f = inputs.sinsin_rhs(n, n)
    ref = cjm.solve(f, n, n, st, tol)
    p = cj.plan(n, n, st, tol)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    assert r["status"] == "ok" == ref["status"]
    assert r["cycles"] == ref["cycles"] == 8
    # Near convergence r = g - D^{-1}A u cancels terms of size |u| ~ |g| / kmin, so the
    # two residual evaluations differ by rounding noise ~ eps * kmax / kmin.
    noise = 50 * np.finfo(float).eps * p.kmax / p.kmin
    assert abs(r["rel_residual"] - ref["relres"]) <= 1e-6 * ref["relres"] + noise
    assert _rel(_host(u), ref["u"]) <= REL_L2


SHAPES = [(1, 1), (2, 3), (1, 70), (70, 1), (17, 5), (63, 47), (130, 64), (257, 33), (300, 70)]


@pytest.mark.parametrize("st", [5, 9, 17])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_full_solve_parity(torch_cuda, st, nx, ny):
    """Full solves on shapes that span several tiles, ragged tails and degenerate strips."""
    torch = torch_cuda
    tol = 1e-10
    _say("case: solve", st, nx, ny)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=1705 + nx * 7 + ny)
    ref = cjm.solve(f, nx, ny, st, tol)
    p = cj.plan(nx, ny, st, tol)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    assert r["status"] == ref["status"]
    assert r["cycles"] == ref["cycles"]
    assert _rel(_host(u), ref["u"]) <= REL_L2


@pytest.mark.parametrize("st", [5, 9, 17])
def test_sweep_prefix_from_rough_guess(torch_cuda, st):
    """A fixed prefix of sweeps (crossing a cycle boundary) from a random guess,
    compared element by element."""
    torch = torch_cuda
    nx, ny = 301, 157
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=5)
    u0 = inputs.random_field(nx, ny, seed=6)
    p = cj.plan(nx, ny, st, 1e-6, M=16)
    n = 37
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=16, u0=u0)
    u = _dev(torch, u0)
    cj.sweeps(p, _dev(torch, f), u, n)
    got = _host(u)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# cycles of M = 8 (K <= 8) or 32 (K = 10): K = 3, 6 and 10 also exercise the
# shorter blocked launch that finishes a cycle
BLOCKED = [(5, 2), (5, 3), (5, 4), (5, 6), (5, 8), (5, 10), (9, 2), (9, 3), (9, 4), (9, 6), (9, 8), (9, 10),
           (17, 2), (17, 3), (17, 4)]


@pytest.mark.parametrize("st,K", BLOCKED)
@pytest.mark.parametrize("nx,ny,rows", [(517, 203, 16), (1, 1, 0), (3, 2, 0), (40, 7, 0), (250, 300, 64)])
def test_blocked_sweeps_match_single_sweeps_bitwise(torch_cuda, st, K, nx, ny, rows):
    """K sweeps per launch (temporal blocking) give the same bits as K launches of
    one sweep, across strips, tile seams, ragged edges and cycle ends; and both
    match the oracle."""
    torch = torch_cuda
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=21)
    u0 = inputs.random_field(nx, ny, seed=22)
    M = 32 if K >= 10 else 8
    n = 2 * M + 3
    ref1 = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=1), _dev(torch, f), ref1, n)
    pk = cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=K, tile_rows=rows)
    assert pk.sweeps_per_launch == K
    uk = _dev(torch, u0)
    cj.sweeps(pk, _dev(torch, f), uk, n)
    assert np.array_equal(_host(uk), _host(ref1))
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=M, u0=u0)
    assert np.abs(_host(uk) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("st", [5, 9])
@pytest.mark.parametrize("frame", [False, True])
@pytest.mark.parametrize("nx,ny,rows", [(985, 61, 16), (1476, 23, 0), (493, 40, 7)])
def test_wide_strips_bitwise_at_their_seams(torch_cuda, st, frame, nx, ny, rows):
    """K = 10 runs FP64 5- and 9-point sweeps in 512-lane strips (492 output
    columns): widths of one strip plus a column, two strips plus one and three
    strips, with homogeneous and frame data, give the bits of single sweeps and
    the oracle's values."""
    torch = torch_cuda
    K, M = 10, 32
    n = 2 * M + 3
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=23)
    kw, obc = {}, cjm.BC_ZERO
    if frame:
        G = inputs.frame_width(st)
        u0 = inputs.expxy_frame(nx, ny, G, interior=inputs.random_field(nx, ny, 24))
        kw, obc = {"bc": cj.BC_FRAME}, cjm.BC_FRAME
    else:
        u0 = inputs.random_field(nx, ny, seed=24)
    ref1 = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=1, **kw), _dev(torch, f), ref1, n)
    pk = cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=K, tile_rows=rows, **kw)
    k, r, wg = pk.refresh_launch_info()
    assert k == K and wg == -(-nx // 492) * -(-ny // r)
    uk = _dev(torch, u0)
    cj.sweeps(pk, _dev(torch, f), uk, n)
    assert np.array_equal(_host(uk), _host(ref1))
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=M, u0=u0, bc=obc)
    assert np.abs(_host(uk) - ref).max() <= 1e-12 * np.abs(ref).max()


# (K, nx): the boundary column nx + 1 in the last lane of a wave, in the first
# lane of the next one, and in the highest lane that can hold it (the last
# output lane plus KR: lane 502 of 512, 248 of 256), for 512-lane (K = 10) and
# 256-lane (K = 8) strips of FP64 5- and 9-point sweeps, in the first and in a
# second strip; column 0 is lane KR - 1 of the first strip.
WAVE_EDGE_CASES = [(10, 53), (10, 54), (10, 117), (10, 118), (10, 492),
                   (8, 55), (8, 56), (8, 240), (8, 295), (8, 296)]


@pytest.mark.parametrize("st", [5, 9])
@pytest.mark.parametrize("frame", [False, True])
@pytest.mark.parametrize("K,nx", WAVE_EDGE_CASES)
def test_boundary_columns_at_wave_edges_bitwise(torch_cuda, st, frame, K, nx):
    """Only the wave that holds column 0 or nx + 1 applies the column
    boundary rule, and only the row blocks that reach a y-boundary apply the
    row rule; with the boundary column at either side of a wave edge, and
    tiles whose first and last row blocks touch the boundary rows, K blocked
    sweeps still give the bits of K single sweeps and the oracle's values."""
    torch = torch_cuda
    M = 32
    n = 2 * M + 3
    ny, rows = (37, 16) if nx % 2 else (45, 0)
    lanes = 512 if K >= 10 else 256
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=29)
    kw, obc = {}, cjm.BC_ZERO
    if frame:
        G = inputs.frame_width(st)
        u0 = inputs.expxy_frame(nx, ny, G, interior=inputs.random_field(nx, ny, 30))
        kw, obc = {"bc": cj.BC_FRAME}, cjm.BC_FRAME
    else:
        u0 = inputs.random_field(nx, ny, seed=30)
    ref1 = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=1, **kw), _dev(torch, f), ref1, n)
    pk = cj.plan(nx, ny, st, 1e-6, M=M, sweeps_per_launch=K, tile_rows=rows, **kw)
    k, r, wg = pk.refresh_launch_info()
    assert k == K and wg == -(-nx // (lanes - 2 * K)) * -(-ny // r)
    uk = _dev(torch, u0)
    cj.sweeps(pk, _dev(torch, f), uk, n)
    assert np.array_equal(_host(uk), _host(ref1))
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=M, u0=u0, bc=obc)
    assert np.abs(_host(uk) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("st,K", [(9, 1), (9, 8), (9, 10), (5, 1), (17, 1), (17, 4)])
def test_full_solve_parity_launch_depths(torch_cuda, st, K):
    torch = torch_cuda
    nx, ny, tol = 211, 143, 1e-10
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=77)
    ref = cjm.solve(f, nx, ny, st, tol)
    p = cj.plan(nx, ny, st, tol, sweeps_per_launch=K)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    assert (r["status"], r["cycles"]) == (ref["status"], ref["cycles"])
    assert _rel(_host(u), ref["u"]) <= REL_L2


def test_zero_sweeps_round_trip_is_exact(torch_cuda):
    torch = torch_cuda
    for st in (5, 9, 17):
        nx, ny = 259, 67
        u0 = inputs.random_field(nx, ny, seed=st)
        p = cj.plan(nx, ny, st, 1e-8)
        u = _dev(torch, u0)
        cj.sweeps(p, _dev(torch, inputs.random_field(nx, ny, 1)), u, 0)
        assert np.array_equal(_host(u), u0)


@pytest.mark.parametrize("st", [5, 9, 17])
def test_residual_and_apply(torch_cuda, st):
    torch = torch_cuda
    nx, ny = 190, 77
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=9)
    u0 = inputs.random_field(nx, ny, seed=10, scale=1e-3)
    p = cj.plan(nx, ny, st, 1e-8)
    fd, ud = _dev(torch, f), _dev(torch, u0)
    rr = cj.residual(p, fd, ud)
    rr2 = cj.residual(p, fd, ud)
    assert rr == rr2                         # deterministic reduction
    ref = cjm.relative_residual(st, f, u0, nx, ny)
    assert abs(rr - ref) <= 1e-12 * ref
    au = torch.empty_like(ud)
    cj.apply(p, ud, au)
    ref_au = cjm.apply(st, u0, nx, ny)
    h = cjm.spacing(nx, ny)
    scale = np.abs(u0).max() * 8.0 / (h * h)   # magnitude of the terms summed
    assert np.abs(_host(au) - ref_au).max() <= 1e-14 * scale


def test_status_paths(torch_cuda):
    torch = torch_cuda
    n = 40
    f = inputs.random_field(n, n, 5)
    p = cj.plan(n, n, 9, 1e-8)
    g = f.copy()
    g[3, 4] = np.nan
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    assert cj.solve(p, _dev(torch, g), u)["status"] == "nonfinite"
    u = _dev(torch, inputs.random_field(n, n, 1))
    r = cj.solve(p, torch.zeros(n, n, dtype=torch.float64, device="cuda"), u)
    assert r["status"] == "ok" and not _host(u).any()
    p1 = cj.plan(n, n, 9, 1e-12, max_cycles=1)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p1, _dev(torch, f), u)
    ref = cjm.solve(f, n, n, 9, 1e-12, max_cycles=1)
    assert r["status"] == "not_converged" == ref["status"] and r["cycles"] == 1
    assert _rel(_host(u), ref["u"]) <= REL_L2
    p2 = cj.plan(n, n, 9, 1e-17)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p2, _dev(torch, f), u)
    assert r["status"] == "stagnated"
    assert r["cycles"] >= p2.cycles_pred and r["floor_estimate"] > 0
    # a converged guess costs no cycle
    ref = cjm.solve(f, n, n, 9, 1e-12)["u"]
    u = _dev(torch, ref)
    r = cj.solve(p, _dev(torch, f), u)
    assert r["status"] == "ok" and r["cycles"] == 0
    assert np.array_equal(_host(u), ref)


def _sample_points(nx, ny, rng, k=24):
    pts = [(1, 1), (nx, 1), (1, ny), (nx, ny), (2, ny // 2), (nx // 2, 2), (nx - 1, ny - 1),
           (256, 64), (257, 65), (256 * 3, 64 * 5 + 1)]
    pts += [(int(rng.integers(1, nx + 1)), int(rng.integers(1, ny + 1))) for _ in range(k)]
    return [(min(i, nx), min(j, ny)) for (i, j) in pts]


@pytest.mark.parametrize("st", [9, 17, 5])
@pytest.mark.parametrize("n", [4096, 8192])
def test_full_size_sampled_sweeps(torch_cuda, st, n):
    """At the benchmark sizes and launch configuration: a prefix of sweeps from a
    rough guess, sampled at edges, corners, tile seams and random nodes; each
    sample is computed by the oracle on its own domain of dependence."""
    torch = torch_cuda
    _say("case: full-size sampled", st, n)
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    u0 = inputs.random_field(n, n, seed=17, scale=1e-3)
    p = cj.plan(n, n, st, 1e-10)
    nsw = 6
    u = _dev(torch, u0)
    cj.sweeps(p, _dev(torch, f), u, nsw)
    got = _host(u)
    pts = _sample_points(n, n, np.random.default_rng(n + st))
    ref = cjm.sampled_sweeps(f, u0, n, n, st, 1e-10, nsw, pts)
    vals = np.array([got[j - 1, i - 1] for (i, j) in pts])
    scale = np.abs(ref).max()
    assert np.abs(vals - ref).max() <= 1e-12 * scale


def test_full_size_solve_against_exact_solution(torch_cuda):
    """4096 x 4096, 9-point, bumps: the full GPU solve against the exact discrete
    solution (sine transform) and its residual recomputed by the oracle."""
    torch = torch_cuda
    n, st = 4096, 9
    _say("case: 4096 full solve vs DST")
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    p = cj.plan(n, n, st, 1e-10)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    assert r["status"] in ("ok", "stagnated")
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, n, n)
    taps, s = cjm.taps(st)
    h = cjm.spacing(n, n)
    exact = dense.dst_solve(taps, s, f, n, n, h)
    err = _rel(got, exact)
    _say("gpu relres %.3e  oracle relres %.3e  rel err vs DST %.3e  status %s cycles %d"
         % (r["rel_residual"], rr, err, r["status"], r["cycles"]))
    # Two FP64 evaluations of r = g - D^{-1}A u differ by rounding noise of order
    # eps * ||u|| / ||g|| (terms of size |u| cancel down to |r|).
    D = -dense.centre(taps) / (s * h * h)
    noise = 8 * np.finfo(float).eps * np.linalg.norm(got) * D / np.linalg.norm(f)
    assert abs(rr - r["rel_residual"]) <= 1e-3 * rr + noise
    assert rr <= 5e-10          # FP64 floor at this size: the stored iterate cannot do better
    assert err <= 1e-8


@pytest.mark.parametrize("st,nx,ny", [(9, 128, 128), (5, 300, 77), (17, 200, 150), (9, 1000, 1000)])
def test_graph_replayed_cycles_match_eager_launches(torch_cuda, st, nx, ny):
    """Each cycle's plain launches replayed as one captured graph give the same bits
    as launching them one by one; the graph is replayed across cycles and across
    solves, with eager work (another plan's solve) in between."""
    torch = torch_cuda
    f = _dev(torch, inputs.gaussian_bumps_rhs(nx, ny, seed=31))
    # launched cycles (small grids otherwise take the single-workgroup solve)
    pg = cj.plan(nx, ny, st, 1e-10, graph=1, single_workgroup=-1)
    pe = cj.plan(nx, ny, st, 1e-10, graph=-1, single_workgroup=-1)
    ref = None
    for rep in range(3):
        ue = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
        re = cj.solve(pe, f, ue)
        ug = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
        rg = cj.solve(pg, f, ug)
        assert (rg["status"], rg["cycles"]) == (re["status"], re["cycles"])
        assert rg["cycles"] >= 2
        assert torch.equal(ug, ue)
        if ref is None:
            ref = ue.clone()
        assert torch.equal(ug, ref)


@pytest.mark.parametrize("st,precision", [(9, cj.F64), (17, cj.F64), (9, cj.F32_REFINE)])
def test_tuned_tile_height_gives_the_same_bits(torch_cuda, st, precision):
    """Grids above 2^18 points pick the blocked kernels' tile height on the
    device at the first solve; the result is bit-identical to a fixed height."""
    torch = torch_cuda
    nx, ny, tol = 2100, 2050, 1e-6
    f = _dev(torch, inputs.gaussian_bumps_rhs(nx, ny, seed=5))
    p_auto = cj.plan(nx, ny, st, tol, precision=precision)
    p_fix = cj.plan(nx, ny, st, tol, precision=precision, tile_rows=128)
    ua = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    uf = torch.zeros_like(ua)
    ra = cj.solve(p_auto, f, ua)
    rf = cj.solve(p_fix, f, uf)
    L = cj.lib()
    rows = ctypes.c_int()
    assert L.cj_plan_launch_info(p_auto.handle, None, ctypes.byref(rows), None) == 0
    print("st %d precision %d: tuned rows %d, %s / %s" % (st, precision, rows.value, ra["status"], rf["status"]),
          flush=True)
    assert 16 <= rows.value <= 2048
    assert (ra["status"], ra["cycles"]) == (rf["status"], rf["cycles"])
    assert torch.equal(ua, uf)


@pytest.mark.parametrize("st", [5, 9, 17])
@pytest.mark.parametrize("nx,ny", [(1 << 20, 2), (3, 1 << 17), (70001, 5)])
def test_extreme_aspect_ratios(torch_cuda, st, nx, ny):
    """The largest axis the planner accepts (2^20 nodes), long thin strips and
    single-tile widths: blocked sweeps still match the oracle and the single sweep."""
    torch = torch_cuda
    n = 13
    f = inputs.random_field(nx, ny, seed=3)
    u0 = inputs.random_field(nx, ny, seed=4)
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=16, u0=u0)
    outs = []
    for K in (1, 0):
        p = cj.plan(nx, ny, st, 1e-6, M=16, sweeps_per_launch=K)
        u = _dev(torch, u0)
        cj.sweeps(p, _dev(torch, f), u, n)
        outs.append(_host(u))
        p.destroy()
    assert np.array_equal(outs[0], outs[1])
    assert np.abs(outs[0] - ref).max() <= 1e-12 * np.abs(ref).max()


SMALL = [(9, 128, 128, False, "chebyshev"), (5, 128, 128, False, "chebyshev"), (9, 1, 1, False, "chebyshev"),
         (9, 3, 2, False, "chebyshev"), (5, 100, 37, True, "chebyshev"), (9, 1000, 10, False, "chebyshev"),
         (9, 64, 256, True, "chebyshev"), (5, 70, 70, False, "jacobi"), (9, 130, 64, False, "chebyshev"),
         # bands of at most four rows: the variant that keeps g in registers
         (9, 32, 32, True, "chebyshev"), (5, 64, 64, False, "chebyshev"), (9, 256, 16, False, "jacobi"),
         (5, 65, 61, False, "chebyshev"),
         # bands of five to eight rows: the middle variant (g in registers)
         (9, 96, 64, False, "chebyshev"), (9, 1000, 8, True, "chebyshev"), (5, 150, 40, False, "jacobi")]


@pytest.mark.parametrize("st,nx,ny,frame,method", SMALL)
def test_single_workgroup_solve_matches_launched_cycles(torch_cuda, st, nx, ny, frame, method):
    """Small 5- and 9-point grids solved in one workgroup with the grid in LDS
    give the bits, status and cycle count of the launched cycles (the residual
    that decides is summed in another order, so it agrees to rounding), and
    the oracle's solution."""
    torch = torch_cuda
    tol = 1e-10
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=40 + nx + ny)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    obc = cjm.BC_FRAME if frame else cjm.BC_ZERO
    m = cj.JACOBI if method == "jacobi" else cj.CHEBYSHEV
    u0 = inputs.expxy_frame(nx, ny, 1) if frame else np.zeros((ny, nx))
    out = []
    for sw in (1, -1):
        p = cj.plan(nx, ny, st, tol, bc=bc, method=m, single_workgroup=sw)
        u = _dev(torch, u0)
        r = cj.solve(p, _dev(torch, f), u)
        out.append((r, _host(u)))
    (r1, u1), (r2, u2) = out
    print("%d-point %dx%d %s: %s %d cycles, relres %.6e / %.6e, %.3f / %.3f ms"
          % (st, nx, ny, method, r1["status"], r1["cycles"], r1["rel_residual"], r2["rel_residual"],
             r1["seconds"] * 1e3, r2["seconds"] * 1e3), flush=True)
    assert (r1["status"], r1["cycles"], r1["sweeps"]) == (r2["status"], r2["cycles"], r2["sweeps"])
    assert np.array_equal(u1, u2)
    assert abs(r1["rel_residual"] - r2["rel_residual"]) <= 1e-9 * r2["rel_residual"] + 1e-15
    ref = cjm.solve(f, nx, ny, st, tol, u0=u0 if frame else None, bc=obc, method=method)
    assert (r1["status"], r1["cycles"]) == (ref["status"], ref["cycles"])
    assert _rel(u1, ref["u"]) <= REL_L2
