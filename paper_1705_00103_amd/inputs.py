"""Seeded synthetic right-hand sides for the 2D Poisson problem A u = f.

This module holds input generation only: no part of the solver's arithmetic.
Both the GPU library's tests and the CPU oracle's tests draw their inputs here,
so the two sides see bit-identical data.

Grid convention: nx x ny interior nodes (i, j), 1 <= i <= nx, 1 <= j <= ny, at
x_i = i h, y_j = j h with h = 1 / max(nx + 1, ny + 1); arrays are (ny, nx),
x fastest, float64.
"""
import math

import numpy as np


def spacing(nx, ny):
    return 1.0 / max(nx + 1, ny + 1)


def coords(nx, ny):
    h = spacing(nx, ny)
    return np.arange(1, nx + 1) * h, np.arange(1, ny + 1) * h


def sinsin_rhs(nx, ny):
    """f = -Delta u for u = sin(pi x) sin(pi y): f = 2 pi^2 sin(pi x) sin(pi y)."""
    x, y = coords(nx, ny)
    return (2.0 * math.pi ** 2) * np.outer(np.sin(math.pi * y), np.sin(math.pi * x))


def sinsin_exact(nx, ny):
    x, y = coords(nx, ny)
    return np.outer(np.sin(math.pi * y), np.sin(math.pi * x))


def bump_params(nx, ny, seed, nbumps=16):
    """Centres uniform in the domain [0, (nx+1)h] x [0, (ny+1)h], widths sigma uniform
    in [0.02, 0.1], amplitudes N(0, 1); drawn in that order from default_rng(seed)."""
    h = spacing(nx, ny)
    Lx, Ly = (nx + 1) * h, (ny + 1) * h
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, Lx, nbumps)
    cy = rng.uniform(0.0, Ly, nbumps)
    sigma = rng.uniform(0.02, 0.1, nbumps)
    amp = rng.normal(0.0, 1.0, nbumps)
    return cx, cy, sigma, amp


def gaussian_bumps_rhs(nx, ny, seed, nbumps=16):
    """f = sum_k A_k exp(-((x - cx_k)^2 + (y - cy_k)^2) / (2 sigma_k^2)), evaluated
    as a sum of separable outer products."""
    x, y = coords(nx, ny)
    cx, cy, sigma, amp = bump_params(nx, ny, seed, nbumps)
    f = np.zeros((ny, nx), dtype=np.float64)
    for k in range(nbumps):
        gx = np.exp(-((x - cx[k]) ** 2) / (2.0 * sigma[k] ** 2))
        gy = amp[k] * np.exp(-((y - cy[k]) ** 2) / (2.0 * sigma[k] ** 2))
        f += np.outer(gy, gx)
    return f


def random_field(nx, ny, seed, scale=1.0):
    """Uniform(-scale, scale) values, e.g. a rough initial guess or a rough RHS."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, (ny, nx))


def log_uniform_shapes(n, seed, lo=64, hi=2048):
    """n grid shapes (nx, ny), each drawn independently log-uniform over [lo, hi]
    (rounded to integers) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(math.log(lo), math.log(hi), (n, 2)))
    return [(int(round(x)), int(round(y))) for x, y in a]


# ------------------------------------------------------------ the paper's test problem
# Delta u = -(x^2 + y^2) e^{xy} on the unit square with the Dirichlet data of its
# analytic solution u = -e^{xy} (test-problem subsection of the results).  In the
# form A u = f with A = -Delta_h: f = (x^2 + y^2) e^{xy}.  The boundary data
# travel in a frame of width G around the interior (G = 1 for the 5- and 9-point
# stencils, 2 for the 17-point one, whose second layer holds analytic ghost
# values outside the square).

def frame_width(stencil):
    return 2 if stencil == 17 else 1


def expxy_rhs(nx, ny):
    """f = (x^2 + y^2) e^{xy} at the interior nodes, (ny, nx)."""
    x, y = coords(nx, ny)
    X, Y = np.meshgrid(x, y)
    return (X * X + Y * Y) * np.exp(X * Y)


def expxy_exact(nx, ny):
    """u = -e^{xy} at the interior nodes, (ny, nx)."""
    x, y = coords(nx, ny)
    X, Y = np.meshgrid(x, y)
    return -np.exp(X * Y)


def expxy_frame(nx, ny, G, interior=0.0):
    """(ny + 2G, nx + 2G) array over nodes 1-G .. n+G: -e^{xy} on the frame of
    width G, `interior` (a scalar or an (ny, nx) array, e.g. an initial guess)
    inside."""
    h = spacing(nx, ny)
    x = np.arange(1 - G, nx + G + 1) * h
    y = np.arange(1 - G, ny + G + 1) * h
    X, Y = np.meshgrid(x, y)
    out = -np.exp(X * Y)
    out[G:ny + G, G:nx + G] = interior
    return out


def frame_from_function(fn, nx, ny, G, interior=0.0):
    """Like expxy_frame for any function fn(X, Y) of the node coordinates."""
    h = spacing(nx, ny)
    x = np.arange(1 - G, nx + G + 1) * h
    y = np.arange(1 - G, ny + G + 1) * h
    X, Y = np.meshgrid(x, y)
    out = np.asarray(fn(X, Y), dtype=np.float64)
    out = np.array(np.broadcast_to(out, X.shape))
    out[G:ny + G, G:nx + G] = interior
    return out
