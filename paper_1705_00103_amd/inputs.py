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
