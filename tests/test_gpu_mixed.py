"""GPU tests of the FP32-sweep / FP64-refinement path (CJ_PRECISION_F32_REFINE).

Bars: FP32 sweeps agree with the FP64 oracle to the FP32 rounding they carry
(bounded below); blocked FP32 sweeps are bit-identical to single FP32 sweeps;
refined solves meet the FP64 tolerance as recomputed by the oracle and agree
with the oracle's FP64 solution to within the tolerance's error scale.
"""
import sys

import numpy as np
import pytest

from oracle import cjm, dense
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("st", [5, 9, 17])
def test_f32_sweeps_track_the_fp64_oracle(torch_cuda, st):
    """A prefix of FP32 sweeps from a rough guess stays within FP32 rounding of the
    FP64 oracle: per sweep each value carries a relative error of a few eps32 of the
    magnitudes it is formed from, amplified at most by the weights."""
    torch = torch_cuda
    nx, ny, M, n = 301, 157, 8, 11
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=5)
    u0 = inputs.random_field(nx, ny, seed=6)
    p = cj.plan(nx, ny, st, 1e-6, M=M, precision=cj.F32_REFINE, inner_M=M, sweeps_per_launch=1)
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-6, n, M=M, u0=u0)
    u = _dev(torch, u0)
    cj.sweeps(p, _dev(torch, f), u, n)
    got = _host(u)
    wmax = max(cjm.plan(nx, ny, st, 1e-6, M=M).weights)
    bound = 8 * n * EPS32 * (1 + wmax) * np.abs(ref).max()
    err = np.abs(got - ref).max()
    print("st %d: max err %.3e, bound %.3e" % (st, err, bound), flush=True)
    assert err <= bound
    assert err > 0          # it really ran in FP32


@pytest.mark.parametrize("st,K", [(5, 2), (5, 4), (5, 8), (9, 2), (9, 4), (9, 8), (17, 2), (17, 3), (17, 4)])
def test_f32_blocked_sweeps_bitwise(torch_cuda, st, K):
    torch = torch_cuda
    nx, ny, n = 517, 203, 19
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=21)
    u0 = inputs.random_field(nx, ny, seed=22)
    a = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-6, M=8, precision=cj.F32_REFINE, inner_M=8, sweeps_per_launch=1),
              _dev(torch, f), a, n)
    b = _dev(torch, u0)
    pk = cj.plan(nx, ny, st, 1e-6, M=8, precision=cj.F32_REFINE, inner_M=8, sweeps_per_launch=K, tile_rows=16)
    assert pk.sweeps_per_launch == K
    cj.sweeps(pk, _dev(torch, f), b, n)
    assert np.array_equal(_host(a), _host(b))


@pytest.mark.parametrize("st", [5, 9, 17])
@pytest.mark.parametrize("nx,ny", [(127, 127), (255, 96), (33, 300)])
def test_refined_solve_meets_fp64_tolerance(torch_cuda, st, nx, ny):
    torch = torch_cuda
    tol = 1e-10
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=1705 + nx + ny)
    p = cj.plan(nx, ny, st, tol, precision=cj.F32_REFINE)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, nx, ny)
    ref = cjm.solve(f, nx, ny, st, tol)
    err = _rel(got, ref["u"])
    print("st %d %dx%d: status %s, outer %d, relres %.3e (oracle %.3e), err vs FP64 oracle %.3e"
          % (st, nx, ny, r["status"], r["cycles"], r["rel_residual"], rr, err), flush=True)
    assert r["status"] == "ok"
    assert rr <= tol * 1.01
    # two solutions that both meet tol differ by at most ~ tol * (kmax/kmin) in the
    # worst case; for a smooth right-hand side the error follows the residual
    assert err <= 50 * tol


def test_refined_solve_special_cases(torch_cuda):
    torch = torch_cuda
    n = 40
    p = cj.plan(n, n, 9, 1e-8, precision=cj.F32_REFINE)
    u = _dev(torch, inputs.random_field(n, n, 1))
    r = cj.solve(p, torch.zeros(n, n, dtype=torch.float64, device="cuda"), u)
    assert r["status"] == "ok" and not _host(u).any()
    g = inputs.random_field(n, n, 5)
    g[1, 2] = np.inf
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    assert cj.solve(p, _dev(torch, g), u)["status"] == "nonfinite"
    p2 = cj.plan(n, n, 9, 1e-17, precision=cj.F32_REFINE)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p2, _dev(torch, inputs.random_field(n, n, 5)), u)
    assert r["status"] == "stagnated" and r["floor_estimate"] > 0


@pytest.mark.parametrize("n", [2047, 4095])
def test_refined_solve_large(torch_cuda, n):
    """Larger grids where eps32 * kmax / kmin approaches 1e-1: the refinement still
    meets the FP64 tolerance (at 4095^2 only with the accurately evaluated outer
    residual; the plain sweep expression stagnates near 1.1e-10 there), checked
    against the exact discrete solution."""
    torch = torch_cuda
    st, tol = 9, 1e-10
    f = inputs.gaussian_bumps_rhs(n, n, seed=99)
    p = cj.plan(n, n, st, tol, precision=cj.F32_REFINE)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p, _dev(torch, f), u)
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, n, n)
    taps, s = cjm.taps(st)
    exact = dense.dst_solve(taps, s, f, n, n, cjm.spacing(n, n))
    err = _rel(got, exact)
    print("n %d: status %s, outer %d, FP32 sweeps %d, relres %.3e (oracle %.3e), err vs exact %.3e"
          % (n, r["status"], r["cycles"], r["sweeps"], r["rel_residual"], rr, err), flush=True)
    sys.stdout.flush()
    assert r["status"] == "ok"
    assert rr <= 2e-10      # the oracle's own FP64 evaluation adds ~7e-11 at 4095^2
    assert err <= 1e-8


DD_PRECISIONS = [pytest.param(cj.F32_REFINE, id="f32inner"), pytest.param(cj.F64, id="f64inner")]


@pytest.mark.parametrize("precision", DD_PRECISIONS)
@pytest.mark.parametrize("st", [5, 9, 17])
@pytest.mark.parametrize("frame", [False, True])
def test_double_double_solve_below_the_fp64_floor(torch_cuda, st, frame, precision):
    """cj_solve_dd carries the iterate as u + u_lo: it meets a tolerance far
    below what an FP64 iterate can reach, measured by the oracle's residual of
    u + u_lo in extended precision; u_lo is the low part (|u_lo| <= ulp(u)/2),
    the frame comes back as given and u_lo's frame is zero.  Inner FP32 cycles
    (refinement plans) and FP64 cycles (FP64 plans)."""
    torch = torch_cuda
    nx, ny, tol = 301, 233, 3e-15
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=40 + st)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    if frame:
        G = inputs.frame_width(st)
        u0 = inputs.expxy_frame(nx, ny, G)
    else:
        u0 = np.zeros((ny, nx))
    p = cj.plan(nx, ny, st, tol, precision=precision, bc=bc, max_cycles=60)
    u = _dev(torch, u0)
    lo = torch.full_like(u, 7.0)       # written only
    r = cj.solve_dd(p, _dev(torch, f), u, lo)
    hi, lo = _host(u), _host(lo)
    obc = cjm.BC_FRAME if frame else cjm.BC_ZERO
    ext = cjm.relative_residual_ext(st, f, hi, lo, nx, ny, bc=obc)
    ext_hi = cjm.relative_residual_ext(st, f, hi, np.zeros_like(lo), nx, ny, bc=obc)
    print("st %d frame %d precision %d: status %s, outer %d, relres %.3e, oracle (extended) %.3e, of u alone %.3e"
          % (st, frame, precision, r["status"], r["cycles"], r["rel_residual"], ext, ext_hi), flush=True)
    assert r["status"] == "ok" and r["rel_residual"] <= tol
    assert ext <= 1.5 * tol
    assert np.all(np.abs(lo) <= np.spacing(np.abs(hi)) / 2)
    if frame:
        mask = np.ones(u0.shape, dtype=bool)
        mask[G:ny + G, G:nx + G] = False
        assert np.array_equal(hi[mask], u0[mask])
        assert np.all(lo[mask] == 0.0)
    # the plain solve of the same plan stops at the floor of an FP64 iterate
    u2 = _dev(torch, u0)
    r2 = cj.solve(p, _dev(torch, f), u2)
    print("  FP64 iterate: status %s, relres %.3e" % (r2["status"], r2["rel_residual"]), flush=True)
    assert ext < r2["rel_residual"]


@pytest.mark.parametrize("precision", DD_PRECISIONS)
def test_double_double_solve_large(torch_cuda, precision):
    """2047^2, 9-point: tol 1e-12, below the floor of an FP64 iterate there
    (about 2e-11)."""
    torch = torch_cuda
    n, st, tol = 2047, 9, 1e-12
    f = inputs.gaussian_bumps_rhs(n, n, seed=99)
    p = cj.plan(n, n, st, tol, precision=precision)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    lo = torch.zeros_like(u)
    r = cj.solve_dd(p, _dev(torch, f), u, lo)
    ext = cjm.relative_residual_ext(st, f, _host(u), _host(lo), n, n)
    print("n %d precision %d: status %s, outer %d, sweeps %d, relres %.3e, oracle (extended) %.3e"
          % (n, precision, r["status"], r["cycles"], r["sweeps"], r["rel_residual"], ext), flush=True)
    assert r["status"] == "ok"
    assert ext <= 1.5 * tol


def test_double_double_argument_errors(torch_cuda):
    torch = torch_cuda
    n = 40
    f = _dev(torch, inputs.gaussian_bumps_rhs(n, n, seed=1))
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    pj = cj.plan(n, n, 9, 1e-10, method=cj.JACOBI)
    with pytest.raises(cj.CJError) as e:
        cj.solve_dd(pj, f, u, torch.zeros_like(u))
    assert e.value.code == cj.CJ_ERR_ARG
    p = cj.plan(n, n, 9, 1e-10, precision=cj.F32_REFINE)
    with pytest.raises(cj.CJError) as e:
        cj.solve_dd(p, f, u, u)
    assert e.value.code == cj.CJ_ERR_ARG
    # f = 0: u and u_lo come back zero
    for q in (p, cj.plan(n, n, 9, 1e-10)):
        lo = torch.full_like(u, 3.0)
        u.fill_(1.0)
        r = cj.solve_dd(q, torch.zeros_like(f), u, lo)
        assert r["status"] == "ok" and not bool(u.any()) and not bool(lo.any())


@pytest.mark.parametrize("precision", DD_PRECISIONS)
@pytest.mark.parametrize("st,frame", [(17, True), (17, False), (9, True)])
def test_plain_solve_after_double_double_is_unchanged(torch_cuda, st, frame, precision):
    """cj_solve_dd keeps the low parts in the plan's second iterate; a later
    cj_solve and cj_sweeps on the same plan give the bits of a fresh plan."""
    torch = torch_cuda
    nx, ny, tol = 97, 83, 1e-9
    f = _dev(torch, inputs.gaussian_bumps_rhs(nx, ny, seed=st))
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    if frame:
        u0 = inputs.expxy_frame(nx, ny, inputs.frame_width(st))
    else:
        u0 = np.zeros((ny, nx))
    used = cj.plan(nx, ny, st, tol, precision=precision, bc=bc)
    fresh = cj.plan(nx, ny, st, tol, precision=precision, bc=bc)
    u, lo = _dev(torch, u0), _dev(torch, u0)
    cj.solve_dd(used, f, u, lo)
    a, b = _dev(torch, u0), _dev(torch, u0)
    ra = cj.solve(used, f, a)
    rb = cj.solve(fresh, f, b)
    assert (ra["status"], ra["cycles"]) == (rb["status"], rb["cycles"])
    assert torch.equal(a, b)
    a, b = _dev(torch, u0), _dev(torch, u0)
    cj.sweeps(used, f, a, 11)
    cj.sweeps(fresh, f, b, 11)
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", DD_PRECISIONS)
def test_double_double_not_converged_returns_the_last_iterate(torch_cuda, precision):
    """max_cycles outer steps without meeting tol: status not_converged, and the
    pair returned is the iterate whose residual was reported (checked by the
    oracle's extended-precision residual)."""
    torch = torch_cuda
    nx, ny, st = 150, 131, 9
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=8)
    p = cj.plan(nx, ny, st, 1e-15, precision=precision, max_cycles=1)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    lo = torch.zeros_like(u)
    r = cj.solve_dd(p, _dev(torch, f), u, lo)
    ext = cjm.relative_residual_ext(st, f, _host(u), _host(lo), nx, ny)
    print("precision %d: status %s, outer %d, relres %.6e, oracle (extended) %.6e"
          % (precision, r["status"], r["cycles"], r["rel_residual"], ext), flush=True)
    assert r["status"] == "not_converged" and r["cycles"] == 1
    assert abs(ext - r["rel_residual"]) <= 1e-6 * ext + 1e-15


@pytest.mark.parametrize("st", [5, 9, 17])
@pytest.mark.parametrize("frame", [False, True])
def test_refinement_with_fp64_inner_cycles(torch_cuda, st, frame):
    """A refinement plan with FP64 inner cycles (forced here; chosen
    automatically where eps32 * kmax / kmin > 4): its sweeps are the FP64
    plan's bits, cj_solve meets the tolerance by the oracle's residual and
    agrees with the FP64 oracle's solution, and cj_solve_dd meets a tolerance
    below the FP64 floor by the oracle's extended-precision residual."""
    torch = torch_cuda
    nx, ny = 211, 143
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=300 + st)
    fd = _dev(torch, f)
    bc = cj.BC_FRAME if frame else cj.BC_ZERO
    obc = cjm.BC_FRAME if frame else cjm.BC_ZERO
    u0 = inputs.expxy_frame(nx, ny, inputs.frame_width(st)) if frame else np.zeros((ny, nx))
    p = cj.plan(nx, ny, st, 1e-10, precision=cj.F32_REFINE, inner_precision=cj.INNER_F64, bc=bc)
    q = cj.plan(nx, ny, st, 1e-10, bc=bc)
    assert (p.M, p.sweeps_per_launch) == (q.M, q.sweeps_per_launch)
    a, b = _dev(torch, u0), _dev(torch, u0)
    cj.sweeps(p, fd, a, 23)
    cj.sweeps(q, fd, b, 23)
    assert torch.equal(a, b)
    u = _dev(torch, u0)
    r = cj.solve(p, fd, u)
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, nx, ny, bc=obc)
    ref = cjm.solve(f, nx, ny, st, 1e-10, u0=u0 if frame else None, bc=obc)
    err = _rel(got, ref["u"])
    print("st %d frame %d: status %s, outer %d, sweeps %d, relres %.3e (oracle %.3e), err vs FP64 oracle %.3e"
          % (st, frame, r["status"], r["cycles"], r["sweeps"], r["rel_residual"], rr, err), flush=True)
    assert r["status"] == "ok" and rr <= 1e-10 * 1.01
    assert err <= 50 * 1e-10
    pd = cj.plan(nx, ny, st, 1e-14, precision=cj.F32_REFINE, inner_precision=cj.INNER_F64, bc=bc, max_cycles=30)
    u = _dev(torch, u0)
    lo = torch.zeros_like(u)
    r = cj.solve_dd(pd, fd, u, lo)
    ext = cjm.relative_residual_ext(st, f, _host(u), _host(lo), nx, ny, bc=obc)
    print("  double-double: status %s, outer %d, relres %.3e, oracle (extended) %.3e"
          % (r["status"], r["cycles"], r["rel_residual"], ext), flush=True)
    assert r["status"] == "ok" and ext <= 1.5e-14
