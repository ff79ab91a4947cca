"""Pins of the oracle's extended-precision residual (relative_residual_ext).

The reference is exact rational arithmetic (fractions.Fraction) on tiny grids:
the discrete operator written out from its definition (the stencil taps and
1 / (s h^2), §2.1; odd reflection beyond the Dirichlet nodes for homogeneous
data, R3; a frame of data, R9), and the exact discrete solution from Gaussian
elimination over the rationals.  Two properties are checked:
  * on generic data the extended evaluation equals the exact residual to FP64
    rounding of the result;
  * at the exact solution split as a double-double hi + lo, it resolves the
    residual of hi alone (about 1e-16, which an FP64 evaluation cannot
    resolve) to 1e-3, and the residual of hi + lo comes out below 1e-18.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import cjm

GRIDS = [(6, 5), (5, 7)]


def _pad_exact(interior, frame, nx, ny, stencil, bc):
    """(ny + 4) x (nx + 4) lists of Fractions, interior at [2 + j][2 + i]."""
    P = [[Fr(0)] * (nx + 4) for _ in range(ny + 4)]
    if bc == cjm.BC_FRAME:
        G = cjm.RADIUS[stencil]
        for j in range(ny + 2 * G):
            for i in range(nx + 2 * G):
                P[2 - G + j][2 - G + i] = Fr(float(frame[j, i]))
    for j in range(ny):
        for i in range(nx):
            P[2 + j][2 + i] = interior[j][i]
    if bc == cjm.BC_ZERO:
        # Dirichlet nodes zero; the node beyond each is the odd reflection of
        # the first interior node (columns first, then rows, corners included)
        for j in range(0, ny + 2):
            P[1 + j][1] = Fr(0)
            P[1 + j][nx + 2] = Fr(0)
        for i in range(0, nx + 2):
            P[1][1 + i] = Fr(0)
            P[ny + 2][1 + i] = Fr(0)
        for j in range(0, ny + 2):
            P[1 + j][0] = -P[1 + j][2]
            P[1 + j][nx + 3] = -P[1 + j][nx + 1]
        for i in range(-1, nx + 3):
            P[0][1 + i] = -P[2][1 + i]
            P[ny + 3][1 + i] = -P[ny + 1][1 + i]
    return P


def _residual_exact(stencil, f, interior, frame, nx, ny, bc, h):
    """f + Delta_h u on the interior, exactly."""
    tp, s = cjm.taps(stencil)
    k = 1 / (Fr(s) * Fr(h) * Fr(h))
    P = _pad_exact(interior, frame, nx, ny, stencil, bc)
    return [[Fr(float(f[j, i])) + k * sum(Fr(c) * P[2 + j + dj][2 + i + di] for di, dj, c in tp)
             for i in range(nx)] for j in range(ny)]


def _norm2(rows):
    return math.sqrt(float(sum(v * v for row in rows for v in row)))


def _exact_solution(stencil, f, frame, nx, ny, bc, h):
    """Interior x with f + Delta_h x = 0 exactly (Gaussian elimination over Q)."""
    n = nx * ny
    zero = [[Fr(0)] * nx for _ in range(ny)]
    r0 = _residual_exact(stencil, f, zero, frame, nx, ny, bc, h)
    cols = []
    zf = np.zeros_like(f)
    zframe = None if frame is None else np.zeros_like(frame)
    for k in range(n):
        e = [[Fr(1) if j * nx + i == k else Fr(0) for i in range(nx)] for j in range(ny)]
        rk = _residual_exact(stencil, zf, e, zframe, nx, ny, bc, h)
        cols.append([rk[j][i] for j in range(ny) for i in range(nx)])
    # rows of the augmented system J x = -r0, J[:, k] = cols[k]
    M = [[cols[k][q] for k in range(n)] + [-r0[q // nx][q % nx]] for q in range(n)]
    for c in range(n):
        piv = next(q for q in range(c, n) if M[q][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for q in range(n):
            if q != c and M[q][c] != 0:
                fac = M[q][c]
                M[q] = [a - fac * b for a, b in zip(M[q], M[c])]
    x = [M[q][n] for q in range(n)]
    return [[x[j * nx + i] for i in range(nx)] for j in range(ny)]


def _case(stencil, bc, nx, ny, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((ny, nx))
    frame = None
    if bc == cjm.BC_FRAME:
        G = cjm.RADIUS[stencil]
        frame = rng.standard_normal((ny + 2 * G, nx + 2 * G))
        frame[G:ny + G, G:nx + G] = 0.0
    return f, frame


def _frame_array(frame, interior, stencil, bc):
    if bc != cjm.BC_FRAME:
        return interior
    G = cjm.RADIUS[stencil]
    out = frame.copy()
    ny, nx = interior.shape
    out[G:ny + G, G:nx + G] = interior
    return out


def _rhs_norm_exact(stencil, f, frame, nx, ny, bc, h):
    zero = [[Fr(0)] * nx for _ in range(ny)]
    return _norm2(_residual_exact(stencil, f, zero, frame, nx, ny, bc, h))


@pytest.mark.parametrize("stencil", [5, 9, 17])
@pytest.mark.parametrize("bc", [cjm.BC_ZERO, cjm.BC_FRAME])
@pytest.mark.parametrize("nx,ny", GRIDS)
def test_ext_residual_equals_exact_on_generic_data(stencil, bc, nx, ny):
    f, frame = _case(stencil, bc, nx, ny, seed=stencil * 10 + bc)
    rng = np.random.default_rng(7)
    hi = rng.standard_normal((ny, nx))
    lo = hi * 1e-17 * rng.standard_normal((ny, nx))
    h = cjm.spacing(nx, ny)
    exact = _residual_exact(stencil, f, [[Fr(float(hi[j, i])) + Fr(float(lo[j, i])) for i in range(nx)]
                                         for j in range(ny)], frame, nx, ny, bc, h)
    want = _norm2(exact) / _rhs_norm_exact(stencil, f, frame, nx, ny, bc, h)
    zlo = np.zeros_like(frame) if bc == cjm.BC_FRAME else None
    got = cjm.relative_residual_ext(stencil, f, _frame_array(frame, hi, stencil, bc),
                                    _frame_array(zlo, lo, stencil, bc), nx, ny, bc=bc)
    assert abs(got - want) <= 1e-14 * want


@pytest.mark.parametrize("stencil", [5, 9, 17])
@pytest.mark.parametrize("bc", [cjm.BC_ZERO, cjm.BC_FRAME])
def test_ext_residual_resolves_below_the_fp64_floor(stencil, bc):
    nx, ny = GRIDS[0]
    f, frame = _case(stencil, bc, nx, ny, seed=100 + stencil + bc)
    h = cjm.spacing(nx, ny)
    x = _exact_solution(stencil, f, frame, nx, ny, bc, h)
    hi = np.array([[float(v) for v in row] for row in x])
    lo = np.array([[float(x[j][i] - Fr(float(hi[j, i]))) for i in range(nx)] for j in range(ny)])
    assert np.all(np.abs(lo) <= np.spacing(np.abs(hi)) / 2)
    den = _rhs_norm_exact(stencil, f, frame, nx, ny, bc, h)
    hi_exact = _norm2(_residual_exact(stencil, f, [[Fr(float(v)) for v in row] for row in hi], frame, nx, ny,
                                      bc, h)) / den
    zlo = np.zeros_like(frame) if bc == cjm.BC_FRAME else None
    z = np.zeros_like(hi)
    ext_hi = cjm.relative_residual_ext(stencil, f, _frame_array(frame, hi, stencil, bc),
                                       _frame_array(zlo, z, stencil, bc), nx, ny, bc=bc)
    ext_dd = cjm.relative_residual_ext(stencil, f, _frame_array(frame, hi, stencil, bc),
                                       _frame_array(zlo, lo, stencil, bc), nx, ny, bc=bc)
    assert 1e-18 < hi_exact < 1e-14
    assert abs(ext_hi - hi_exact) <= 1e-3 * hi_exact
    assert ext_dd < 1e-18
