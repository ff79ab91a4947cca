"""GPU parity of the paper's own test problem: Dirichlet data carried in a frame
around the interior (CJ_BC_DIRICHLET_FRAME; for 17 points two layers, the
second of analytic ghosts) and plain Jacobi (CJ_METHOD_JACOBI), against the
oracle on the same inputs.

Bars: FP64 prefixes and full solves within 1e-12 relative L2 of the oracle;
blocked and single-sweep launches bit-identical; the frame is returned as it
was given; FP32-refined solves meet the FP64 tolerance as the oracle measures
it.
"""
import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu
STENCILS = (5, 9, 17)


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


def _frame(nx, ny, st, seed):
    G = inputs.frame_width(st)
    return inputs.expxy_frame(nx, ny, G, interior=inputs.random_field(nx, ny, seed))


@pytest.mark.parametrize("st", STENCILS)
@pytest.mark.parametrize("nx,ny", [(97, 61), (300, 257), (1, 5), (517, 33)])
def test_frame_sweeps_match_oracle(torch_cuda, st, nx, ny):
    torch = torch_cuda
    n = 21
    f = inputs.expxy_rhs(nx, ny)
    u0 = _frame(nx, ny, st, nx + ny)
    ref = cjm.run_sweeps(f, nx, ny, st, 1e-8, n, M=16, u0=u0, bc=cjm.BC_FRAME)
    outs = []
    for K in (1, 0):
        p = cj.plan(nx, ny, st, 1e-8, M=16, bc=cj.BC_FRAME, sweeps_per_launch=K)
        u = _dev(torch, u0)
        cj.sweeps(p, _dev(torch, f), u, n)
        outs.append(_host(u))
    print("st %d %dx%d: rel err %.3e" % (st, nx, ny, _rel(outs[0], ref)), flush=True)
    assert np.array_equal(outs[0], outs[1])            # blocked == single, bitwise
    assert _rel(outs[0], ref) <= 1e-12
    G = inputs.frame_width(st)
    frame_mask = np.ones(u0.shape, dtype=bool)
    frame_mask[G:ny + G, G:nx + G] = False
    assert np.array_equal(outs[0][frame_mask], u0[frame_mask])


@pytest.mark.parametrize("st,K", [(5, 2), (5, 4), (5, 8), (9, 3), (9, 6), (9, 8), (17, 2), (17, 3), (17, 4)])
def test_frame_blocked_bitwise(torch_cuda, st, K):
    torch = torch_cuda
    nx, ny, n = 411, 203, 2 * K + 1
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=3)
    u0 = _frame(nx, ny, st, 4)
    a = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-8, M=64, bc=cj.BC_FRAME, sweeps_per_launch=1), _dev(torch, f), a, n)
    b = _dev(torch, u0)
    cj.sweeps(cj.plan(nx, ny, st, 1e-8, M=64, bc=cj.BC_FRAME, sweeps_per_launch=K, tile_rows=16),
              _dev(torch, f), b, n)
    assert np.array_equal(_host(a), _host(b))


@pytest.mark.parametrize("st", STENCILS)
@pytest.mark.parametrize("nx,ny", [(127, 127), (90, 143)])
def test_frame_solve_matches_oracle(torch_cuda, st, nx, ny):
    torch = torch_cuda
    tol = 1e-10
    G = inputs.frame_width(st)
    f = inputs.expxy_rhs(nx, ny)
    u0 = inputs.expxy_frame(nx, ny, G)
    ref = cjm.solve(f, nx, ny, st, tol, u0=u0, bc=cjm.BC_FRAME)
    p = cj.plan(nx, ny, st, tol, bc=cj.BC_FRAME)
    u = _dev(torch, u0)
    r = cj.solve(p, _dev(torch, f), u)
    got = _host(u)
    err = _rel(got, ref["u"])
    print("st %d %dx%d: %s/%s cycles %d/%d relres %.3e/%.3e rel err %.3e"
          % (st, nx, ny, r["status"], ref["status"], r["cycles"], ref["cycles"], r["rel_residual"],
             ref["relres"], err), flush=True)
    assert r["status"] == ref["status"] == "ok"
    assert r["cycles"] == ref["cycles"]
    assert abs(r["rel_residual"] - ref["relres"]) <= 1e-6 * ref["relres"] + 1e-14
    assert err <= 1e-12
    # and the discrete solution approximates -e^{xy} at the stencil's order
    exact = inputs.expxy_exact(nx, ny)
    assert np.abs(got[G:ny + G, G:nx + G] - exact).max() < (1e-8 if st == 17 else 1e-5)


@pytest.mark.parametrize("st", STENCILS)
def test_frame_residual_and_apply(torch_cuda, st):
    torch = torch_cuda
    nx, ny = 203, 77
    f = inputs.expxy_rhs(nx, ny)
    u0 = _frame(nx, ny, st, 8)
    p = cj.plan(nx, ny, st, 1e-8, bc=cj.BC_FRAME)
    rr = cj.residual(p, _dev(torch, f), _dev(torch, u0))
    assert abs(rr - cjm.relative_residual(st, f, u0, nx, ny, bc=cjm.BC_FRAME)) <= 1e-12 * rr
    au = torch.empty(ny, nx, dtype=torch.float64, device="cuda")
    cj.apply(p, _dev(torch, u0), au)
    ref = cjm.apply(st, u0, nx, ny, bc=cjm.BC_FRAME)
    assert _rel(_host(au), ref) <= 1e-14


@pytest.mark.parametrize("st", STENCILS)
def test_frame_special_cases(torch_cuda, st):
    torch = torch_cuda
    nx, ny = 50, 41
    G = inputs.frame_width(st)
    p = cj.plan(nx, ny, st, 1e-10, bc=cj.BC_FRAME)
    # zero data and zero f: the zero interior, frame untouched
    u0 = np.zeros((ny + 2 * G, nx + 2 * G))
    u0[G:ny + G, G:nx + G] = inputs.random_field(nx, ny, 2)
    u = _dev(torch, u0)
    r = cj.solve(p, torch.zeros(ny, nx, dtype=torch.float64, device="cuda"), u)
    assert r["status"] == "ok" and not _host(u).any()
    # Laplace's equation with data from a harmonic cubic: the cubic is the discrete solution
    x = np.arange(1 - G, nx + G + 1) * inputs.spacing(nx, ny)
    y = np.arange(1 - G, ny + G + 1) * inputs.spacing(nx, ny)
    X, Y = np.meshgrid(x, y)
    harm = X ** 3 - 3 * X * Y * Y + X * Y
    u0 = harm.copy()
    u0[G:ny + G, G:nx + G] = 0.0
    u = _dev(torch, u0)
    r = cj.solve(p, torch.zeros(ny, nx, dtype=torch.float64, device="cuda"), u)
    assert r["status"] == "ok"
    assert np.abs(_host(u) - harm).max() < 1e-9


@pytest.mark.parametrize("st", STENCILS)
def test_jacobi_sweeps_and_solve_match_oracle(torch_cuda, st):
    torch = torch_cuda
    nx, ny = 63, 47
    G = inputs.frame_width(st)
    f = inputs.expxy_rhs(nx, ny)
    u0 = inputs.expxy_frame(nx, ny, G)
    tol = 1e-6
    ref = cjm.solve(f, nx, ny, st, tol, u0=u0, bc=cjm.BC_FRAME, method="jacobi")
    p = cj.plan(nx, ny, st, tol, bc=cj.BC_FRAME, method=cj.JACOBI)
    assert (p.M, p.cycles_pred) == (ref["plan"].M, ref["plan"].cycles_pred)
    u = _dev(torch, u0)
    r = cj.solve(p, _dev(torch, f), u)
    err = _rel(_host(u), ref["u"])
    print("st %d: jacobi %s/%s checks %d/%d sweeps %d rel err %.3e" % (st, r["status"], ref["status"], r["cycles"],
                                                                      ref["cycles"], r["sweeps"], err), flush=True)
    assert r["status"] == ref["status"] == "ok"
    assert r["cycles"] == ref["cycles"]
    assert err <= 1e-12
    # homogeneous data too, prefix of blocked sweeps
    g = inputs.gaussian_bumps_rhs(nx, ny, seed=9)
    pj = cj.plan(nx, ny, st, tol, method=cj.JACOBI)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    cj.sweeps(pj, _dev(torch, g), u, 37)
    assert _rel(_host(u), cjm.run_sweeps(g, nx, ny, st, tol, 37, method="jacobi")) <= 1e-13


@pytest.mark.parametrize("st", STENCILS)
def test_frame_refined_solve(torch_cuda, st):
    torch = torch_cuda
    nx, ny, tol = 255, 200, 1e-10
    G = inputs.frame_width(st)
    f = inputs.expxy_rhs(nx, ny)
    u0 = inputs.expxy_frame(nx, ny, G)
    p = cj.plan(nx, ny, st, tol, bc=cj.BC_FRAME, precision=cj.F32_REFINE)
    u = _dev(torch, u0)
    r = cj.solve(p, _dev(torch, f), u)
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, nx, ny, bc=cjm.BC_FRAME)
    ref = cjm.solve(f, nx, ny, st, tol, u0=u0, bc=cjm.BC_FRAME)
    err = _rel(got, ref["u"])
    print("st %d: refined %s outer %d relres %.3e (oracle %.3e) err vs FP64 oracle %.3e"
          % (st, r["status"], r["cycles"], r["rel_residual"], rr, err), flush=True)
    assert r["status"] == "ok"
    assert rr <= tol * 1.01
    assert err <= 50 * tol
    mask = np.ones(u0.shape, dtype=bool)
    mask[G:ny + G, G:nx + G] = False
    assert np.array_equal(got[mask], u0[mask])
    # the FP32 sweeps leave the refinement's corrections clean for the next solve
    v = _dev(torch, u0)
    cj.sweeps(p, _dev(torch, f), v, 9)
    u = _dev(torch, u0)
    r2 = cj.solve(p, _dev(torch, f), u)
    assert r2["status"] == "ok" and np.array_equal(_host(u), got)


def test_frame_status_paths(torch_cuda):
    torch = torch_cuda
    nx, ny = 60, 45
    for st in (9, 17):
        G = inputs.frame_width(st)
        f = _dev(torch, inputs.expxy_rhs(nx, ny))
        # a NaN in the boundary data reaches the lifted right-hand side
        bad = inputs.expxy_frame(nx, ny, G)
        bad[0, 7] = np.nan
        p = cj.plan(nx, ny, st, 1e-10, bc=cj.BC_FRAME)
        assert cj.solve(p, f, _dev(torch, bad))["status"] == "nonfinite"
        # Jacobi stopped after one check far above tol
        pj = cj.plan(nx, ny, st, 1e-12, bc=cj.BC_FRAME, method=cj.JACOBI, M=16, max_cycles=1)
        r = cj.solve(pj, f, _dev(torch, inputs.expxy_frame(nx, ny, G)))
        assert r["status"] == "not_converged" and r["cycles"] == 1 and r["sweeps"] == 16
