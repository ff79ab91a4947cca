"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the mistake it would catch.  None of them needs a GPU.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cjm, dense
from paper_1705_00103_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STENCILS = (5, 9, 17)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(v) for v in line.split()])
    return rows


def _ring(di, dj):
    a, b = abs(di), abs(dj)
    return (max(a, b), min(a, b))


# --------------------------------------------------------------------------- stencils


def test_taps_match_figure_one():
    """The oracle's tap tables (transcribed from the stencil equations) equal the
    second printing of the coefficients (Figure 1, Table tab:ste2).  Catches a
    mistyped coefficient, a wrong prefactor or a tap in the wrong ring."""
    want = {}
    for st, a, b, num, den in _read_golden("stencil_coefficients.txt"):
        want[(st, (a, b))] = Fraction(num, den)
    for st in STENCILS:
        taps, s = cjm.taps(st)
        seen = {}
        for di, dj, c in taps:
            key = (st, _ring(di, dj))
            got = Fraction(c).limit_denominator(1000) / Fraction(s).limit_denominator(1000)
            assert key in want, key
            assert got == want[key], (key, got, want[key])
            seen[key] = seen.get(key, 0) + 1
        for key in want:
            if key[0] == st:
                assert seen[key] == (1 if key[1] == (0, 0) else 4), key
        assert len(taps) == st


@pytest.mark.parametrize("st,exact_degree", [(5, 3), (9, 3), (17, 5)])
def test_taps_consistency_order(st, exact_degree):
    """Delta_h p equals Delta p for every polynomial up to the stencil's exactness
    degree (3 for the second-order 5- and 9-point stencils, 5 for the fourth-order
    17-point one) and not beyond.  Catches a dropped term or a wrong sign."""
    taps, s = cjm.taps(st)
    h, x0, y0 = 0.125, 0.3, -0.7

    def lap_h(p):
        return sum(c * p(x0 + di * h, y0 + dj * h) for di, dj, c in taps) / (s * h * h)

    for deg in range(0, exact_degree + 2):
        for a in range(deg + 1):
            b = deg - a
            p = (lambda a, b: lambda x, y: x ** a * y ** b)(a, b)
            lap = (a * (a - 1) * x0 ** max(a - 2, 0) * y0 ** b if a >= 2 else 0.0) + \
                  (b * (b - 1) * y0 ** max(b - 2, 0) * x0 ** a if b >= 2 else 0.0)
            err = abs(lap_h(p) - lap)
            if deg <= exact_degree:
                assert err < 1e-9, (st, a, b, err)
    # the first degree beyond exactness is not reproduced for x^(d+1)
    d = exact_degree + 1
    p = lambda x, y: x ** d
    lap = d * (d - 1) * x0 ** (d - 2)
    assert abs(lap_h(p) - lap) > 1e-6


def test_kappa_max_printed_values():
    """kappa_max equals the printed 8/5 and 128/75 and the symbol's supremum at (pi, pi)."""
    for st, num, den in _read_golden("kappa_max.txt"):
        assert cjm.KAPPA_MAX[st] == num / den
    for st in STENCILS:
        taps, _ = cjm.taps(st)
        t = np.linspace(0.0, math.pi, 401)
        TX, TY = np.meshgrid(t, t)
        sym = dense.symbol(taps, TX, TY)
        assert abs(sym.max() - cjm.KAPPA_MAX[st]) < 1e-14
        assert abs(dense.symbol(taps, math.pi, math.pi) - cjm.KAPPA_MAX[st]) < 1e-14


GRIDS = [(1, 1), (2, 3), (3, 2), (6, 6), (9, 5), (12, 7), (5, 11)]


def _dense_from_C(st, nx, ny, h):
    n = nx * ny
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = cjm.apply(st, e.reshape(ny, nx), nx, ny, h).ravel()
    return A


@pytest.mark.parametrize("st", STENCILS)
@pytest.mark.parametrize("nx,ny", GRIDS)
def test_kappa_closed_forms_equal_dense_spectrum(st, nx, ny):
    """The smallest eigenvalue of D^{-1}A (dense, from the oracle's own node loops)
    equals the paper's kappa_min closed form with N = n + 1; the largest stays
    below kappa_max; A is symmetric and equals the Kronecker-product assembly.
    Catches a wrong coefficient, a wrong D, an index slip in the loops, a wrong
    second-ring closure and the N = n misreading."""
    h = cjm.spacing(nx, ny)
    taps, s = cjm.taps(st)
    A = _dense_from_C(st, nx, ny, h)
    K = dense.laplacian_matrix(taps, s, nx, ny, h).toarray()
    assert np.abs(A - K).max() <= 1e-14 * np.abs(K).max()
    assert np.array_equal(A, A.T)
    D = -dense.centre(taps) / (s * h * h)
    ev = np.linalg.eigvalsh(A / D)
    kmin, kmax = cjm.kappa_bounds(st, nx, ny)
    assert abs(ev[0] - kmin) < 2e-15 * max(1.0, kmin) + 1e-15
    assert ev[-1] < kmax
    # the symbol gives the whole spectrum
    sym = np.sort(dense.eigenvalues_DinvA(taps, nx, ny).ravel())
    assert np.abs(sym - ev).max() < 1e-13


def test_interval_count_reading():
    """With N = n (interior count) the closed form misses the smallest eigenvalue
    by a wide margin (reading R1 of the oracle)."""
    st, n = 5, 6
    taps, s = cjm.taps(st)
    h = cjm.spacing(n, n)
    A = _dense_from_C(st, n, n, h)
    D = -dense.centre(taps) / (s * h * h)
    lam = np.linalg.eigvalsh(A / D)[0]
    wrong = cjm.kappa_bounds(st, n - 1, n - 1)[0]   # formula evaluated with N = n
    assert wrong / lam > 1.3


# --------------------------------------------------------------------------- weights


@pytest.mark.parametrize("M", [1, 2, 4, 8, 16, 64, 256])
def test_weights_product_is_scaled_chebyshev(M):
    """prod_j (1 - omega_j kappa) = T_M((b + a - 2 kappa)/(b - a)) / T_M((b + a)/(b - a)).
    Catches a wrong map of the Chebyshev zeros (factor 2, sign, interval ends)."""
    a, b = 3.0e-3, 1.6
    w = cjm.weights(a, b, M)
    kap = np.concatenate([np.linspace(a, b, 57), [0.5 * a, 1.2 * b, 0.0]])
    prod = np.ones_like(kap)
    for wj in w:
        prod *= 1.0 - wj * kap
    ref = dense.chebyshev_T(M, (b + a - 2 * kap) / (b - a)) / dense.chebyshev_T(M, np.array([(b + a) / (b - a)]))[0]
    assert np.allclose(prod, ref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("st,n,tol", [(9, 128, 1e-10), (5, 255, 1e-8), (17, 100, 1e-10), (9, 1023, 1e-10)])
def test_bound_per_cycle_equals_max_of_cycle_polynomial(st, n, tol):
    """rho(M) = 1/cosh(M beta) equals max over [kmin, kmax] of |prod (1 - omega kappa)|,
    evaluated from the weights themselves.  Pins the cycle rule's bound."""
    p = cjm.plan(n, n, st, tol)
    kap = np.linspace(p.kmin, p.kmax, 20001)
    prod = np.ones_like(kap)
    for wj in p.weights:
        prod *= 1.0 - wj * kap
    assert abs(np.abs(prod).max() - p.rho) <= 1e-6 * p.rho
    assert p.rho ** p.cycles_pred <= tol * (1 + 1e-12)
    assert p.cycles_pred == 1 or p.rho ** (p.cycles_pred - 1) > tol


def test_lf_order_small_cases_and_permutation():
    assert cjm.lf_order(1) == [1]
    assert cjm.lf_order(2) == [1, 3]
    assert cjm.lf_order(4) == [1, 7, 3, 5]
    assert cjm.lf_order(8) == [1, 15, 7, 9, 3, 13, 5, 11]
    for p in range(0, 15):
        M = 1 << p
        assert sorted(cjm.lf_order(M)) == list(range(1, 2 * M, 2))
    with pytest.raises(ValueError):
        cjm.lf_order(6)


@pytest.mark.parametrize("st,n", [(9, 127), (5, 511), (17, 1023)])
def test_ordering_keeps_every_tail_product_bounded(st, n):
    """Every suffix product prod_{i >= j} (1 - omega_i kappa) stays <= 1 on
    [kmin, kmax]: a rounding error made mid-cycle is never amplified by the rest
    of the cycle.  The monotone order, by contrast, overflows (reading R7)."""
    p = cjm.plan(n, n, st, 1e-10)
    M = p.M
    kap = np.linspace(p.kmin, p.kmax, 4001)
    suffix = np.ones_like(kap)
    worst = 0.0
    for wj in reversed(p.weights):
        suffix *= 1.0 - wj * kap
        worst = max(worst, np.abs(suffix).max())
    assert worst <= 1.0 + 1e-9, worst
    mono = sorted(p.weights, reverse=True)
    with np.errstate(over="ignore", invalid="ignore"):
        prefix = np.ones_like(kap)
        growth = 0.0
        for wj in mono:
            prefix *= 1.0 - wj * kap
            growth = max(growth, np.nanmax(np.abs(prefix)))
    if M >= 2048:
        assert not np.isfinite(growth) or growth > 1e100


def test_cycle_rule_minimises_work():
    for st in STENCILS:
        for n in (31, 128, 1000, 4095):
            for tol in (1e-6, 1e-8, 1e-10):
                kmin, kmax = cjm.kappa_bounds(st, n, n)
                M, c = cjm.choose_cycle(kmin, kmax, tol)
                b = cjm.beta(kmin, kmax)
                for p in range(0, 22):
                    Mp = 1 << p
                    assert cjm.cycles_needed(Mp, b, tol) * Mp >= c * M


# --------------------------------------------------------------------------- solves


@pytest.mark.parametrize("st", STENCILS)
@pytest.mark.parametrize("nx,ny", [(3, 3), (8, 5), (16, 16), (13, 9)])
def test_dense_direct_solve_tiny(st, nx, ny):
    """A converged CJM solve equals numpy's dense direct solve of A u = f."""
    taps, s = cjm.taps(st)
    h = cjm.spacing(nx, ny)
    f = inputs.random_field(nx, ny, seed=nx * 100 + ny)
    r = cjm.solve(f, nx, ny, st, 1e-14)
    assert r["status"] == "ok", r["status"]
    A = dense.laplacian_matrix(taps, s, nx, ny, h).toarray()
    u = np.linalg.solve(A, f.ravel()).reshape(ny, nx)
    assert np.linalg.norm(r["u"] - u) <= 1e-11 * np.linalg.norm(u)


@pytest.mark.parametrize("st", STENCILS)
def test_cycles_match_spectral_prediction(st):
    """From u0 = 0 the iterate after c cycles is A^{-1}(I - P(D^{-1}A)^c) f, with
    P(kappa) = T_M((b+a-2kappa)/(b-a)) / T_M((b+a)/(b-a)) applied per sine mode.
    Pins the sweep, D, the weights and the cycle loop together."""
    nx, ny = 47, 33
    taps, s = cjm.taps(st)
    h = cjm.spacing(nx, ny)
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=7)
    p = cjm.plan(nx, ny, st, 1e-6)
    ncyc = 2
    u = cjm.run_sweeps(f, nx, ny, st, 1e-6, ncyc * p.M)
    a, b = p.kmin, p.kmax
    kap = dense.eigenvalues_DinvA(taps, nx, ny)
    P = dense.chebyshev_T(p.M, (b + a - 2 * kap) / (b - a)) / dense.chebyshev_T(p.M, np.array([(b + a) / (b - a)]))[0]
    D = -dense.centre(taps) / (s * h * h)
    fh = dense.dst_forward(f)
    pred = dense.dst_forward(fh * (1.0 - P ** ncyc) / (D * kap))
    assert np.linalg.norm(u - pred) <= 1e-11 * np.linalg.norm(pred)


def test_manufactured_solution_c1():
    """128 x 128, 9-point, f = -Delta(sin pi x sin pi y): the RHS is the (1,1) sine
    mode, so each cycle divides the residual by exactly T_M(x0) = 1/rho(M), and the
    iterate's relative error against the exact discrete solution
    [2 pi^2 / (D kmin)] sin pi x sin pi y equals its relative residual."""
    n, st = 128, 9
    f = inputs.sinsin_rhs(n, n)
    r = cjm.solve(f, n, n, st, 1e-10)
    p = r["plan"]
    assert r["status"] == "ok" and r["relres"] <= 1e-10
    assert (p.M, p.cycles_pred, r["cycles"]) == (128, 8, 8)
    hist = r["history"]
    for c in range(1, 5):
        assert abs(hist[c] / hist[c - 1] - p.rho) <= 1e-8 * p.rho
    taps, s = cjm.taps(st)
    D = -dense.centre(taps) / (s * p.h * p.h)
    uh = (2 * math.pi ** 2 / (D * p.kmin)) * inputs.sinsin_exact(n, n)
    relerr = np.linalg.norm(r["u"] - uh) / np.linalg.norm(uh)
    assert abs(relerr - r["relres"]) <= 0.01 * r["relres"]


@pytest.mark.parametrize("st", STENCILS)
def test_chebyshev_bound_random_rhs(st):
    """For any f (A symmetric, D scalar) the residual after c cycles from u0 = 0 is
    at most rho(M)^c times the initial one."""
    nx, ny = 40, 29
    f = inputs.random_field(nx, ny, seed=3)
    r = cjm.solve(f, nx, ny, st, 1e-9)
    p = r["plan"]
    for c, rr in enumerate(r["history"]):
        assert rr <= p.rho ** c * (1 + 1e-8) + 1e-15


@pytest.mark.parametrize("st", STENCILS)
def test_unit_weight_is_textbook_jacobi(st):
    """omega = 1 gives u_new = D^{-1}(f - (A - D) u), the classical Jacobi step, with
    D the scalar centre coefficient (reading R2).  For 5 and 9 points D is also the
    matrix diagonal; for 17 points the second-ring reflection changes the diagonal
    of the rows next to the boundary, and the method keeps the scalar D."""
    nx, ny = 11, 8
    taps, s = cjm.taps(st)
    h = cjm.spacing(nx, ny)
    f = inputs.random_field(nx, ny, 1)
    u = inputs.random_field(nx, ny, 2)
    p = cjm.plan(nx, ny, st, 1e-6)
    a = cjm.pad(u, nx, ny)
    b = np.zeros_like(a)
    cjm.sweep(p, f, a, b, 1.0)
    A = dense.laplacian_matrix(taps, s, nx, ny, h).toarray()
    D = -dense.centre(taps) / (s * h * h)
    if st != 17:
        assert np.allclose(np.diag(A), D, rtol=1e-15)
    ref = (f.ravel() - (A - D * np.eye(nx * ny)) @ u.ravel()) / D
    assert np.allclose(cjm.unpad(b, nx, ny).ravel(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("st", STENCILS)
def test_exact_solution_by_sine_transform(st):
    """A solve to 1e-12 agrees with the exact discrete solution (DST-I) to within the
    residual scale for a smooth right-hand side."""
    n = 95
    taps, s = cjm.taps(st)
    f = inputs.gaussian_bumps_rhs(n, n, seed=11)
    r = cjm.solve(f, n, n, st, 1e-12)
    assert r["status"] == "ok"
    u = dense.dst_solve(taps, s, f, n, n, cjm.spacing(n, n))
    assert np.linalg.norm(r["u"] - u) <= 100 * 1e-12 * np.linalg.norm(u)
    # and the DST solution itself has a tiny residual under the oracle's operator
    assert cjm.relative_residual(st, f, u, n, n) < 1e-13


@pytest.mark.parametrize("st,slope", [(5, 2.0), (9, 2.0), (17, 4.0)])
def test_discretisation_order(st, slope):
    """Manufactured u = sin pi x sin pi y: max error of the CJM solution against the
    continuous u falls like h^2 (5- and 9-point) and h^4 (17-point)."""
    errs, hs = [], []
    for n in (15, 31, 63):
        f = inputs.sinsin_rhs(n, n)
        r = cjm.solve(f, n, n, st, 1e-14)
        assert r["status"] in ("ok", "stagnated")
        errs.append(np.abs(r["u"] - inputs.sinsin_exact(n, n)).max())
        hs.append(cjm.spacing(n, n))
    k = math.log(errs[-2] / errs[-1]) / math.log(hs[-2] / hs[-1])
    assert abs(k - slope) < 0.05, (st, k, errs)


def test_nine_point_fourth_order_needs_corrected_rhs():
    """The 9-point stencil reaches fourth order only with the RHS f + (h^2/12) Delta_5 f
    (not in the paper); plain f gives second order (see the oracle's readings)."""
    errs, hs = [], []
    taps5, s5 = cjm.taps(5)
    for n in (15, 31, 63):
        h = cjm.spacing(n, n)
        f = inputs.sinsin_rhs(n, n)
        # Delta_5 f with the exact boundary values of f (zero on the boundary)
        f_corr = f - (h * h / 12.0) * cjm.apply(5, f, n, n)
        r = cjm.solve(f_corr, n, n, 9, 1e-14)
        errs.append(np.abs(r["u"] - inputs.sinsin_exact(n, n)).max())
        hs.append(h)
    k = math.log(errs[-2] / errs[-1]) / math.log(hs[-2] / hs[-1])
    assert abs(k - 4.0) < 0.05, k


# --------------------------------------------------------------------------- stopping rule


def test_stopping_special_cases():
    n = 20
    f = inputs.random_field(n, n, 5)
    g = f.copy()
    g[3, 4] = np.nan
    assert cjm.solve(g, n, n, 9, 1e-8)["status"] == "nonfinite"
    z = cjm.solve(np.zeros((n, n)), n, n, 9, 1e-8, u0=inputs.random_field(n, n, 1))
    assert z["status"] == "ok" and not z["u"].any()
    r = cjm.solve(f, n, n, 9, 1e-12, max_cycles=1)
    assert r["status"] == "not_converged" and r["cycles"] == 1
    r = cjm.solve(f, n, n, 9, 1e-17)
    assert r["status"] == "stagnated"
    assert r["cycles"] >= r["plan"].cycles_pred
    # a guess that already meets the tolerance costs no cycle
    u = cjm.solve(f, n, n, 9, 1e-12)["u"]
    r = cjm.solve(f, n, n, 9, 1e-8, u0=u)
    assert r["status"] == "ok" and r["cycles"] == 0


@pytest.mark.parametrize("st", STENCILS)
def test_sampled_sweeps_match_full_sweeps(st):
    """Values computed on each point's domain of dependence equal the full sweeps,
    including points next to edges and corners."""
    nx, ny = 37, 26
    f = inputs.gaussian_bumps_rhs(nx, ny, 3)
    u0 = inputs.random_field(nx, ny, 4)
    n = 7
    full = cjm.run_sweeps(f, nx, ny, st, 1e-8, n, u0=u0)
    pts = [(1, 1), (nx, ny), (1, ny), (nx, 1), (2, 13), (19, 2), (18, 13), (nx - 1, 12)]
    vals = cjm.sampled_sweeps(f, u0, nx, ny, st, 1e-8, n, pts)
    ref = np.array([full[j - 1, i - 1] for (i, j) in pts])
    assert np.array_equal(vals, ref)


def _reordered_sweep9(u, g, w):
    """A second FP64 evaluation of the 9-point weighted sweep (homogeneous data,
    u padded by one zero ring), summing the taps in another order than the
    oracle: r = (S / 20 + g) - u with S = 4 (axis pairs) + (diagonal pairs)."""
    C = u[1:-1, 1:-1]
    axis = (u[1:-1, :-2] + u[1:-1, 2:]) + (u[:-2, 1:-1] + u[2:, 1:-1])
    diag = (u[:-2, :-2] + u[:-2, 2:]) + (u[2:, :-2] + u[2:, 2:])
    r = ((4.0 * axis + diag) * (1.0 / 20.0) + g) - C
    out = np.zeros_like(u)
    out[1:-1, 1:-1] = C + w * r
    return out


@pytest.mark.parametrize("n", [128, 256])
def test_rounding_order_spread_over_one_cycle(n):
    """Two FP64 evaluations of one full cycle that round in different orders end
    about 0.17 eps max(omega) apart (rel-L2): the cycle's largest weight,
    ~1/kappa_min, multiplies the rounding of the residuals that follow.  This is
    the bar of the GPU's full-cycle parity test at the benchmark sizes; the
    measured constant holds from 128^2 to 4096^2 (0.169-0.177)."""
    st, tol = 9, 1e-10
    f = inputs.gaussian_bumps_rhs(n, n, seed=1714)
    p = cjm.plan(n, n, st, tol)
    h = cjm.spacing(n, n)
    g = f * (6.0 * h * h / 20.0)          # D^{-1} f, D = 20 / (6 h^2)
    ref = cjm.run_sweeps(f, n, n, st, tol, p.M)
    u = np.zeros((n + 2, n + 2))
    for k in range(p.M):
        u = _reordered_sweep9(u, g, p.weights[k])
    rel = np.linalg.norm(u[1:-1, 1:-1] - ref) / np.linalg.norm(ref)
    c = rel / (np.finfo(float).eps * max(p.weights))
    assert 0.1 <= c <= 0.25, c
