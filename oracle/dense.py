"""Plain definitions that pin the CJM oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

  laplacian_matrix   A = -Delta_h assembled from Kronecker products of 1D
                     shift matrices (a textbook construction, independent of
                     the node loops in cj_oracle.c);
  symbol             eigenvalue of D^{-1}A on the sine mode (k, l): for a
                     stencil symmetric in both axes it is
                     sum_taps c cos(di tx) cos(dj ty) / c_centre;
  dst_solve          the exact discrete solution A^{-1} f by the type-I
                     discrete sine transform, which diagonalises A (Dirichlet
                     data, odd reflection for the second ring);
  chebyshev_T        T_M(x) = cos(M arccos x) (|x| <= 1), cosh(M arccosh |x|)
                     with sign (-1)^M for x < -1.
The stencil enters only as a list of taps (di, dj, c) and the denominator s of
Delta_h u = (1/(s h^2)) sum c u(i+di, j+dj), so every routine here works on
whatever coefficients a test passes in.
"""
import math

import numpy as np
import scipy.fft
import scipy.sparse as sp


def shift_matrix(n, d):
    """n x n matrix S_d with (S_d u)_i = u_{i-d} + u_{i+d}, for 1-based nodes 1..n,
    u_0 = u_{n+1} = 0 (Dirichlet) and odd reflection u_{-k} = -u_k, u_{n+1+k} = -u_{n+1-k}.
    S_0 is the identity."""
    if d == 0:
        return sp.identity(n, format="csr")
    rows, cols, vals = [], [], []
    for i in range(1, n + 1):
        for k in (i - d, i + d):
            sgn = 1.0
            if k < 0:
                k, sgn = -k, -1.0
            elif k > n + 1:
                k, sgn = 2 * (n + 1) - k, -1.0
            if 1 <= k <= n:
                rows.append(i - 1)
                cols.append(k - 1)
                vals.append(sgn)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def _classes(taps):
    """Groups symmetric taps by (|di|, |dj|); each class must share one coefficient."""
    cls = {}
    for di, dj, c in taps:
        key = (abs(di), abs(dj))
        cls.setdefault(key, set()).add(c)
    out = {}
    for key, cs in cls.items():
        if len(cs) != 1:
            raise ValueError("stencil not symmetric in class %r" % (key,))
        out[key] = cs.pop()
    return out


def laplacian_matrix(taps, s, nx, ny, h):
    """A = -Delta_h as a sparse (nx*ny)^2 matrix, unknowns ordered x fastest."""
    L = sp.csr_matrix((nx * ny, nx * ny))
    for (a, b), c in _classes(taps).items():
        L = L + c * sp.kron(shift_matrix(ny, b), shift_matrix(nx, a), format="csr")
    # Class (a, 0) with a > 0 has taps (+-a, 0): S_a already sums both.  Same for (0, b).
    # Class (a, b) with a, b > 0 has four taps (+-a, +-b): S_b (x) S_a sums all four.
    # Class (0, 0) is the centre: S_0 (x) S_0 = I.
    return (-1.0 / (s * h * h)) * L


def centre(taps):
    return [c for di, dj, c in taps if di == 0 and dj == 0][0]


def symbol(taps, tx, ty):
    """Eigenvalue of D^{-1}A on the sine mode with angles (tx, ty) = (k pi/N_x, l pi/N_y)."""
    acc = 0.0
    for (a, b), c in _classes(taps).items():
        fa = 1.0 if a == 0 else 2.0 * np.cos(a * tx)
        fb = 1.0 if b == 0 else 2.0 * np.cos(b * ty)
        acc = acc + c * fa * fb
    return acc / centre(taps)


def mode_angles(nx, ny):
    tx = np.arange(1, nx + 1) * math.pi / (nx + 1)
    ty = np.arange(1, ny + 1) * math.pi / (ny + 1)
    return np.meshgrid(tx, ty)      # (ny, nx) arrays


def eigenvalues_DinvA(taps, nx, ny):
    """All eigenvalues of D^{-1}A, shape (ny, nx), by the symbol."""
    TX, TY = mode_angles(nx, ny)
    return symbol(taps, TX, TY)


def dst_forward(x):
    return scipy.fft.dstn(x, type=1, norm="ortho", workers=-1)


def dst_solve(taps, s, f, nx, ny, h):
    """Exact discrete solution of A u = f (FP64 sine transform)."""
    D = -centre(taps) / (s * h * h)
    lam = D * eigenvalues_DinvA(taps, nx, ny)
    fh = dst_forward(np.asarray(f, dtype=np.float64).reshape(ny, nx))
    return dst_forward(fh / lam)       # the orthonormal DST-I is its own inverse


def chebyshev_T(M, x):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(M * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** M * np.cosh(M * np.arccosh(np.abs(xo)))
    return out
