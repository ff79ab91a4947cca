"""Host-side checks of libcj.so: it loads, exports every function include/cj.h
declares, and its planner (host only, no GPU needed) agrees with the oracle's."""
import ctypes
import math
import os
import re

import pytest

from oracle import cjm
from paper_1705_00103_amd import cj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cj.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cj_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(cj.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = cj.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_status_strings():
    for code, name in [(0, "CJ_OK"), (1, "CJ_STAGNATED"), (-1, "CJ_ERR_ARG"), (-2, "CJ_ERR_NOMEM"),
                       (-3, "CJ_ERR_HIP"), (-4, "CJ_ERR_NOT_CONVERGED"), (-5, "CJ_ERR_NONFINITE"),
                       (-6, "CJ_ERR_DEVICE")]:
        assert cj.status_string(code) == name
    assert cj.status_string(42) == "CJ_UNKNOWN_STATUS"


CASES = [(5, 1, 1, 1e-10), (9, 1, 300, 1e-8), (17, 2, 3, 1e-10), (9, 128, 128, 1e-10),
         (5, 4096, 4096, 1e-10), (9, 4096, 4096, 1e-10), (17, 4096, 4096, 1e-10),
         (5, 8192, 8192, 1e-10), (9, 8192, 8192, 1e-10), (17, 8192, 8192, 1e-10),
         (9, 16384, 4096, 1e-10), (9, 300, 77, 1e-6), (17, 1000, 999, 1e-12), (5, 64, 2048, 1e-8)]


@pytest.mark.parametrize("st,nx,ny,tol", CASES)
def test_plan_matches_oracle(st, nx, ny, tol):
    p = cj.plan(nx, ny, st, tol)
    o = cjm.plan(nx, ny, st, tol)
    assert (p.M, p.cycles_pred) == (o.M, o.cycles_pred)
    assert p.kmax == o.kmax
    assert abs(p.kmin - o.kmin) <= 4e-16 * o.kmin
    for a, b in zip(p.weights, o.weights):
        assert abs(a - b) <= 1e-14 * abs(b)
    Lp = cj.lib()
    del Lp
    pitch_min = (nx + 18) * (ny + 4) * 8 * 3
    assert p.workspace_bytes >= pitch_min


def test_plan_explicit_M_and_options():
    p = cj.plan(100, 50, 9, 1e-8, M=64)
    o = cjm.plan(100, 50, 9, 1e-8, M=64)
    assert (p.M, p.cycles_pred) == (64, o.cycles_pred)
    h = 0.01
    p2 = cj.plan(100, 50, 9, 1e-8, h=h)
    assert p2.M == cjm.plan(100, 50, 9, 1e-8, h=h).M


@pytest.mark.parametrize("args,kw", [
    ((0, 5, 9, 1e-8), {}), ((5, 0, 9, 1e-8), {}), ((5, 5, 7, 1e-8), {}), ((5, 5, 9, 0.0), {}),
    ((5, 5, 9, -1.0), {}), ((5, 5, 9, float("nan")), {}), ((5, 5, 9, 1e-8), {"M": 6}),
    ((5, 5, 9, 1e-8), {"M": -2}), ((5, 5, 9, 1e-8), {"bc": 2}), ((5, 5, 9, 1e-8), {"max_cycles": -1}),
    ((5, 5, 9, 1e-8), {"h": -0.5}), ((5, 5, 9, 1e-8), {"method": 2}),
    ((5, 5, 9, 1e-8), {"method": 1, "precision": 1}), ((5, 5, 9, 1e-8), {"method": 1, "M": 3}),
    (((1 << 20) + 1, 5, 9, 1e-8), {}), ((5, (1 << 20) + 1, 17, 1e-8), {}), ((5, 5, 9, float("inf")), {}),
    ((5, 5, 9, 1e-8), {"sweeps_per_launch": 5}), ((5, 5, 17, 1e-8), {"sweeps_per_launch": 6}),
])
def test_plan_rejects_bad_arguments(args, kw):
    with pytest.raises(cj.CJError) as e:
        cj.plan(*args, **kw)
    assert e.value.code == cj.CJ_ERR_ARG
    assert cj.last_error()


def test_null_arguments_are_errors_not_crashes():
    L = cj.lib()
    assert L.cj_plan(5, 5, 9, 0, 1e-8, None) == cj.CJ_ERR_ARG
    assert L.cj_plan_info(None, None, None, None, None, None, None) == cj.CJ_ERR_ARG
    assert L.cj_solve(None, None, None, None, None) == cj.CJ_ERR_ARG
    p = cj.plan(8, 8, 9, 1e-8)
    # NULL and misaligned device pointers are rejected before any device work
    assert L.cj_solve(p.handle, None, ctypes.c_void_p(4096), None, None) == cj.CJ_ERR_ARG
    assert L.cj_sweeps(p.handle, ctypes.c_void_p(4097), ctypes.c_void_p(4096), 1, None) == cj.CJ_ERR_ARG
    assert L.cj_sweeps(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4096), -1, None) == cj.CJ_ERR_ARG
    assert L.cj_residual(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4096), None, None) == cj.CJ_ERR_ARG
    assert L.cj_apply(p.handle, None, None, None) == cj.CJ_ERR_ARG
    assert L.cj_solve_dd(None, None, None, None, None, None) == cj.CJ_ERR_ARG
    assert L.cj_solve_dd(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(8192), None, None, None) == cj.CJ_ERR_ARG
    L.cj_plan_destroy(None)
    p.destroy()
    p.destroy()


def test_weights_are_positive_and_span_the_interval():
    p = cj.plan(255, 255, 17, 1e-10)
    assert min(p.weights) > 1.0 / p.kmax * 0.99
    assert max(p.weights) < 1.0 / p.kmin * 1.01
    assert len(set(p.weights)) == p.M
    assert math.isclose(sum(1.0 / w for w in p.weights) / p.M, (p.kmax + p.kmin) / 2, rel_tol=1e-12)


def test_batch_create_host_side():
    shapes = [(64, 80), (300, 17), (1, 1), (129, 129)]
    b = cj.Batch(shapes, [9, 5, 17, 9], [1e-8, 1e-6, 1e-10, 1e-8])
    for i, (nx, ny) in enumerate(shapes):
        inf = b.info(i)
        st = [9, 5, 17, 9][i]
        p = cj.plan(nx, ny, st, [1e-8, 1e-6, 1e-10, 1e-8][i], precision=cj.F32_REFINE)
        assert inf["M"] == max(p.M, 16)
        assert inf["sweeps_per_launch"] == (4 if st == 17 else 8)
    assert b.info(0)["workspace_bytes"] > 0
    b.destroy()
    with pytest.raises(cj.CJError):
        cj.Batch([(10, 10)], [7], [1e-8])
    with pytest.raises(cj.CJError):
        cj.Batch([(10, 10)], [9], [0.0])
    with pytest.raises(cj.CJError):
        cj.Batch([(10, 10)], [9], [1e-8], sweeps_per_launch=3)
    L = cj.lib()
    assert L.cj_batch_create(0, None, None, None, None, None, ctypes.byref(ctypes.c_void_p())) == cj.CJ_ERR_ARG
    assert L.cj_batch_solve(None, None, None, None, None, None) == cj.CJ_ERR_ARG
    L.cj_batch_destroy(None)


@pytest.mark.parametrize("st,n,tol", [(5, 1023, 9.5e-7), (9, 1023, 9.5e-7), (17, 1023, 9.5e-7), (9, 100, 1e-10),
                                      (17, 31, 1e-3), (5, 1, 0.5)])
def test_jacobi_plan_matches_oracle(st, n, tol):
    p = cj.plan(n, n, st, tol, method=cj.JACOBI)
    o = cjm.plan(n, n, st, tol, method="jacobi")
    assert (p.M, p.cycles_pred) == (o.M, o.cycles_pred)
    assert p.weights == [1.0] * p.M
    p2 = cj.plan(n, n, st, tol, method=cj.JACOBI, M=64)
    assert (p2.M, p2.cycles_pred) == (64, cjm.plan(n, n, st, tol, M=64, method="jacobi").cycles_pred)


def test_frame_plans_on_the_host():
    for st in (5, 9, 17):
        p = cj.plan(40, 30, st, 1e-8, bc=cj.BC_FRAME)
        assert p.frame == (2 if st == 17 else 1)
        q = cj.plan(40, 30, st, 1e-8)
        assert (p.M, p.cycles_pred, p.weights) == (q.M, q.cycles_pred, q.weights)
        cj.plan(40, 30, st, 1e-8, bc=cj.BC_FRAME, precision=cj.F32_REFINE)
    # batches run Chebyshev-Jacobi only
    L = cj.lib()
    o = cj.Options()
    L.cj_options_init(ctypes.byref(o))
    o.precision, o.method = cj.F32_REFINE, cj.JACOBI
    h = ctypes.c_void_p()
    code = L.cj_batch_create(1, (ctypes.c_int * 1)(10), (ctypes.c_int * 1)(10), (ctypes.c_int * 1)(9),
                             (ctypes.c_double * 1)(1e-8), ctypes.byref(o), ctypes.byref(h))
    assert code == cj.CJ_ERR_ARG and not h.value


def test_default_blocking_depth():
    """K = 10 for the 5- and 9-point stencils above 2^22 points, 8 up to it (whole
    launches per cycle); 4 for the 17-point stencil."""
    for st, big, small in ((5, 10, 8), (9, 10, 8), (17, 4, 4)):
        assert cj.plan(4096, 1025, st, 1e-8).sweeps_per_launch == big
        assert cj.plan(2048, 2048, st, 1e-8).sweeps_per_launch == small


def test_refinement_inner_precision_on_the_host():
    """Refinement plans take FP64 inner cycles where eps32 * kmax / kmin > 4
    (16384^2, 9-point: 8.6) and FP32 ones below (8192^2: 2.2); either can be
    forced.  FP64 inner cycles report the FP64 schedule and blocking depth."""
    eps32 = 2.0 ** -23
    big = cj.plan(16384, 16384, 9, 1e-10, precision=cj.F32_REFINE)
    o = cjm.plan(16384, 16384, 9, 1e-10)
    assert eps32 * o.kmax / o.kmin > 4
    assert (big.M, big.cycles_pred) == (o.M, o.cycles_pred)
    assert big.sweeps_per_launch == 10                      # the FP64 default above 2^22 points
    mid = cj.plan(8192, 8192, 9, 1e-10, precision=cj.F32_REFINE)
    assert mid.sweeps_per_launch == 8                       # FP32 inner cycles
    forced = cj.plan(8192, 8192, 9, 1e-10, precision=cj.F32_REFINE, inner_precision=cj.INNER_F64)
    assert forced.sweeps_per_launch == 10 and forced.M == cjm.plan(8192, 8192, 9, 1e-10).M
    f32 = cj.plan(16384, 16384, 9, 1e-10, precision=cj.F32_REFINE, inner_precision=cj.INNER_F32)
    assert f32.sweeps_per_launch == 8
    # FP64 inner cycles hold three more padded FP64 arrays instead of three FP32 ones
    assert forced.workspace_bytes > mid.workspace_bytes
    small = cj.plan(40, 30, 9, 1e-8, precision=cj.F32_REFINE, inner_precision=cj.INNER_F64, inner_M=64)
    assert small.M == 64
    for kw in ({"inner_precision": 3}, {"inner_precision": -1}, {"inner_precision": cj.INNER_F64, "precision": cj.F64}):
        with pytest.raises(cj.CJError) as e:
            cj.plan(40, 30, 9, 1e-8, **kw)
        assert e.value.code == cj.CJ_ERR_ARG
    # batches and servers run FP32 inner cycles only
    L = cj.lib()
    opt = cj.Options()
    L.cj_options_init(ctypes.byref(opt))
    opt.precision, opt.inner_precision = cj.F32_REFINE, cj.INNER_F64
    h = ctypes.c_void_p()
    code = L.cj_batch_create(1, (ctypes.c_int * 1)(10), (ctypes.c_int * 1)(10), (ctypes.c_int * 1)(9),
                             (ctypes.c_double * 1)(1e-8), ctypes.byref(opt), ctypes.byref(h))
    assert code == cj.CJ_ERR_ARG and not h.value


def test_single_workgroup_option_on_the_host():
    cj.plan(128, 128, 9, 1e-10, single_workgroup=1)
    cj.plan(1000, 10, 5, 1e-10, single_workgroup=1)
    for args in ((129, 129, 9), (1025, 2, 9), (64, 300, 9), (128, 128, 17)):
        with pytest.raises(cj.CJError) as e:
            cj.plan(*args, 1e-10, single_workgroup=1)
        assert e.value.code == cj.CJ_ERR_ARG
    with pytest.raises(cj.CJError):
        cj.plan(128, 128, 9, 1e-10, precision=cj.F32_REFINE, single_workgroup=1)
    with pytest.raises(cj.CJError):
        cj.plan(64, 64, 9, 1e-10, single_workgroup=2)


@pytest.mark.parametrize("st,precision,K,lanes", [
    (9, "f64", 10, 512), (5, "f64", 10, 512), (9, "f64", 8, 256), (17, "f64", 4, 256),
    (9, "f32", 8, 256), (5, "f32", 8, 256)])
def test_blocked_strip_width_on_the_host(st, precision, K, lanes):
    """The blocked kernel's strips: 512 lanes (512 - 2KR output columns) for FP64
    radius-1 stencils at K = 10, 256 lanes otherwise; the plan's launch geometry
    (before any solve: the default tile height) says which."""
    n = 8192
    prec = cj.F64 if precision == "f64" else cj.F32_REFINE
    p = cj.plan(n, n, st, 1e-10, sweeps_per_launch=K, precision=prec, tile_rows=100)
    k, rows, wg = p.refresh_launch_info()
    R = 2 if st == 17 else 1
    assert (k, rows) == (K, 100)
    assert wg == -(-n // (lanes - 2 * K * R)) * -(-n // rows)
