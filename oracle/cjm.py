"""Plain FP64 Chebyshev-Jacobi method (CJM): plan and cycle loop.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the paper
(Adsuara et al., arXiv 1705.00103), §2.1, with the readings listed below where
the paper is silent or ambiguous.

The method (§2.1): a weighted Jacobi iteration
    u <- u + omega_n * D^{-1} (f - A u)
whose weights omega_n change at every iteration and are precomputed, before the
iteration starts, from the zeros of a Chebyshev polynomial mapped onto the
interval [kappa_min, kappa_max] that bounds the spectrum of D^{-1} A.  The
bounds come from the smallest and largest sine waves the mesh supports and have
closed forms for the 9-point (Eq. for kappa^(9)) and 17-point (Eq. for
kappa^(17)) stencils.  One pass over the M weights is a "cycle"; the cycle is
repeated until the tolerance is met (§3.4 speaks of M weights per cycle).

Readings (the paper does not fix these; each is pinned by the tests):
  R1  N_x, N_y in the kappa closed forms count intervals: nx interior unknowns
      give N_x = nx + 1, and h = 1 / max(N_x, N_y) (uniform mesh, §2.1).
  R2  D is the scalar centre coefficient of A (A = -Delta_h, SPD).
  R3  The 17-point stencil's second ring is closed by odd reflection about the
      Dirichlet node (see cj_oracle.c).
  R4  The weights are the reciprocals of the Chebyshev zeros mapped onto
      [kappa_min, kappa_max] (Richardson's method with Chebyshev parameters):
      omega_j = 2 / ((kmax + kmin) - (kmax - kmin) cos((2j - 1) pi / (2M))).
  R5  The 5-point bounds, not printed here, follow from the stencil symbol:
      kappa_min = sin^2(pi/2N_x) + sin^2(pi/2N_y), kappa_max = 2.
  R6  The cycle length is a power of two, M = 2^p, chosen to minimise
      (cycles x M) where cycles = ceil(ln(1/tol) / ln cosh(M beta)) is the
      number of cycles the Chebyshev bound 1/cosh(M beta) needs,
      beta = arccosh((kmax + kmin) / (kmax - kmin)); ties go to the smaller M.
  R7  Within a cycle the weights are applied in the recursive symmetric-pair
      (Lebedev-Finogenov type) order: S_1 = [1], S_2m = [s_1, 4m - s_1, s_2,
      4m - s_2, ...]; weight k of the cycle uses theta = S_M[k] in
      cos(theta pi / (2M)).  A monotone order overflows for large M.
  R8  Stopping is tested at cycle ends only, on the relative residual
      ||f - A u||_2 / ||f||_2: stop when <= tol; report "stagnated" when, at or
      after the predicted cycle count, a cycle fails to halve the residual;
      report "not_converged" after max_cycles (default predicted + 4) cycles.
      A zero right-hand side has the solution u = 0.
  R9  Non-homogeneous Dirichlet data (the paper's test problem takes them from
      the analytic solution) travel in a frame of width G around the interior,
      G = the stencil radius: for the 17-point stencil the second layer holds
      prescribed ghost values instead of the reflection of R3.  The relative
      residual is then taken against the residual of the zero interior, i.e.
      the norm of the lifted right-hand side f - A_IB u_B.
  R10 Jacobi, the paper's reference method, is the same sweep with omega = 1.
      It is checked every M sweeps, M = 2^p the largest power of two not above
      max(1, n_J / 32), where n_J = ceil(ln(1/tol) / -ln(1 - kappa_min)) sweeps
      meet tol under the bound (1 - kappa_min)^n; the predicted check count is
      ceil(n_J / M) and the stopping rule is R8's.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STENCILS = (5, 9, 17)
# kappa_max: supremum of the symbol of D^{-1}A, printed for 9 and 17 points (§2.1); 2 for 5 points (R5).
KAPPA_MAX = {5: 2.0, 9: 8.0 / 5.0, 17: 128.0 / 75.0}
# Stencil radius: the 17-point stencil reaches two nodes out.
RADIUS = {5: 1, 9: 1, 17: 2}
# Boundary data (R3, R9).
BC_ZERO, BC_FRAME = 0, 1


def lib():
    """The compiled loops of cj_oracle.c (built on first use if absent).  With
    CJ_ORACLE_NATIVE=1 in the environment, the build for this host's CPU
    (-march=native), used to time the oracle as a CPU baseline."""
    global _LIB
    if _LIB is None:
        native = os.environ.get("CJ_ORACLE_NATIVE") == "1"
        path = os.path.join(_HERE, "_cj_oracle_native.so" if native else "_cj_oracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build(native=native)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.cjo_ntaps.argtypes = [c_int]
        L.cjo_ntaps.restype = c_int
        L.cjo_tap.argtypes = [c_int, c_int, ip, ip, dp, dp]
        L.cjo_tap.restype = c_int
        L.cjo_fill_ring.argtypes = [c_int, c_int, dp]
        L.cjo_fill_ring.restype = None
        L.cjo_apply.argtypes = [c_int, c_int, c_int, c_double, dp, dp]
        L.cjo_apply.restype = c_int
        L.cjo_sweep.argtypes = [c_int, c_int, c_int, c_double, dp, dp, dp, c_double,
                                c_int, c_int, c_int, c_int]
        L.cjo_sweep.restype = c_int
        L.cjo_residual_sumsq.argtypes = [c_int, c_int, c_int, c_double, dp, dp]
        L.cjo_residual_sumsq.restype = c_double
        L.cjo_residual_sumsq_ext.argtypes = [c_int, c_int, c_int, c_double, dp, dp, dp]
        L.cjo_residual_sumsq_ext.restype = c_double
        L.cjo_sumsq.argtypes = [ctypes.c_size_t, dp]
        L.cjo_sumsq.restype = c_double
        L.cjo_threads.argtypes = []
        L.cjo_threads.restype = c_int
        _LIB = L
    return _LIB


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def taps(stencil):
    """The stencil as the C loops hold it: list of (di, dj, c) and the denominator s,
    with Delta_h u = (1/(s h^2)) sum c u(i+di, j+dj)."""
    L = lib()
    n = L.cjo_ntaps(stencil)
    if n == 0:
        raise ValueError("unknown stencil %r" % (stencil,))
    out = []
    s = ctypes.c_double()
    for k in range(n):
        di, dj, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        L.cjo_tap(stencil, k, ctypes.byref(di), ctypes.byref(dj), ctypes.byref(c), ctypes.byref(s))
        out.append((di.value, dj.value, c.value))
    return out, s.value


def threads():
    return lib().cjo_threads()


# ----------------------------------------------------------------------------- grid


def spacing(nx, ny):
    """h = 1 / max(N_x, N_y) with N = n + 1 intervals (R1)."""
    return 1.0 / max(nx + 1, ny + 1)


def pad(u, nx, ny):
    """Unpadded (ny, nx) array -> padded (ny+4, nx+4) array with the ring filled."""
    p = np.zeros((ny + 4, nx + 4), dtype=np.float64)
    p[2:ny + 2, 2:nx + 2] = np.asarray(u, dtype=np.float64).reshape(ny, nx)
    lib().cjo_fill_ring(nx, ny, _ptr(p))
    return p


def unpad(p, nx, ny):
    return np.ascontiguousarray(p[2:ny + 2, 2:nx + 2])


def pad_frame(uf, nx, ny, stencil):
    """Frame array (ny + 2G, nx + 2G) over nodes 1-G .. n+G (R9) -> padded
    (ny+4, nx+4) array; nodes beyond the frame (the second ring of the 5- and
    9-point stencils, which they never read) are zero."""
    G = RADIUS[stencil]
    uf = np.asarray(uf, dtype=np.float64)
    if uf.shape != (ny + 2 * G, nx + 2 * G):
        raise ValueError("frame array must be (ny + 2G, nx + 2G) = %r" % ((ny + 2 * G, nx + 2 * G),))
    p = np.zeros((ny + 4, nx + 4), dtype=np.float64)
    p[2 - G:ny + 2 + G, 2 - G:nx + 2 + G] = uf
    return p


def unpad_frame(p, nx, ny, stencil):
    G = RADIUS[stencil]
    return np.ascontiguousarray(p[2 - G:ny + 2 + G, 2 - G:nx + 2 + G])


def _padded(u, nx, ny, stencil, bc):
    return pad_frame(u, nx, ny, stencil) if bc == BC_FRAME else pad(u, nx, ny)


def _zero_interior(p, nx, ny):
    z = p.copy()
    z[2:ny + 2, 2:nx + 2] = 0.0
    return z


# ----------------------------------------------------------------------------- plan


def kappa_bounds(stencil, nx, ny):
    """[kappa_min, kappa_max] of D^{-1}A (§2.1 closed forms; 5-point per R5)."""
    Nx, Ny = nx + 1, ny + 1
    ax, ay = math.pi / (2 * Nx), math.pi / (2 * Ny)   # pi / 2N
    bx, by = math.pi / Nx, math.pi / Ny               # pi / N

    def s2(a):
        return math.sin(a) ** 2

    if stencil == 5:
        kmin = s2(ax) + s2(ay)
    elif stencil == 9:
        kmin = (4.0 / 5.0) * (s2(ax) + s2(ay)) + (1.0 / 5.0) * (s2(ax + ay) + s2(ax - ay))
    elif stencil == 17:
        kmin = (-(4.0 / 75.0) * (s2(bx) + s2(by))
                + (64.0 / 75.0) * (s2(ax) + s2(ay))
                - (1.0 / 75.0) * (s2(bx + by) + s2(bx - by))
                + (16.0 / 75.0) * (s2(ax + ay) + s2(ax - ay)))
    else:
        raise ValueError("unknown stencil %r" % (stencil,))
    return kmin, KAPPA_MAX[stencil]


def beta(kmin, kmax):
    return math.acosh((kmax + kmin) / (kmax - kmin))


def log_cosh(x):
    """ln cosh x without overflow."""
    x = abs(x)
    return x + math.log1p(math.exp(-2.0 * x)) - math.log(2.0)


def cycles_needed(M, b, tol):
    """Cycles of length M the Chebyshev bound 1/cosh(M beta) per cycle needs to reach tol (R6)."""
    if tol >= 1.0:
        return 1
    return max(1, math.ceil(math.log(1.0 / tol) / log_cosh(M * b)))


def choose_cycle(kmin, kmax, tol, max_log2=24):
    """(M, predicted cycles) per R6."""
    b = beta(kmin, kmax)
    best = None
    for p in range(0, max_log2 + 1):
        M = 1 << p
        c = cycles_needed(M, b, tol)
        if best is None or c * M < best[0] * best[1]:
            best = (c, M)
        if c == 1:
            break
    return best[1], best[0]


def lf_order(M):
    """Recursive symmetric-pair ordering S_M of the odd integers 1..2M-1 (R7)."""
    if M < 1 or (M & (M - 1)):
        raise ValueError("the ordering needs M = 2^p, got %d" % M)
    S = [1]
    m = 1
    while m < M:
        S = [v for s in S for v in (s, 4 * m - s)]
        m *= 2
    return S


def weight(theta, M, kmin, kmax):
    """omega for odd theta = 2j - 1 (R4)."""
    return 2.0 / ((kmax + kmin) - (kmax - kmin) * math.cos(theta * math.pi / (2.0 * M)))


def weights(kmin, kmax, M):
    """The M weights of one cycle, in applied order (R4, R7)."""
    return [weight(t, M, kmin, kmax) for t in lf_order(M)]


def jacobi_sweeps_needed(kmin, tol):
    """n_J of R10: sweeps after which (1 - kappa_min)^n <= tol."""
    if tol >= 1.0:
        return 1
    return max(1, math.ceil(math.log(1.0 / tol) / -math.log1p(-kmin)))


def jacobi_check(kmin, tol, max_log2=24):
    """(M, predicted checks) of R10."""
    nj = jacobi_sweeps_needed(kmin, tol)
    M = 1
    while 2 * M <= max(1, nj // 32) and M < (1 << max_log2):
        M *= 2
    return M, math.ceil(nj / M)


class Plan:
    def __init__(self, nx, ny, stencil, tol, M=None, h=None, method="chebyshev", bc=BC_ZERO):
        if nx < 1 or ny < 1:
            raise ValueError("nx, ny must be >= 1")
        if not (tol > 0.0):
            raise ValueError("tol must be > 0")
        if method not in ("chebyshev", "jacobi"):
            raise ValueError("method must be 'chebyshev' or 'jacobi'")
        if bc not in (BC_ZERO, BC_FRAME):
            raise ValueError("bc must be BC_ZERO or BC_FRAME")
        self.nx, self.ny, self.stencil, self.tol = nx, ny, stencil, tol
        self.method, self.bc = method, bc
        self.h = spacing(nx, ny) if h is None else float(h)
        self.kmin, self.kmax = kappa_bounds(stencil, nx, ny)
        if method == "jacobi":
            # R10: omega = 1 throughout; M is the check interval
            if M is None:
                self.M, self.cycles_pred = jacobi_check(self.kmin, tol)
            else:
                self.M, self.cycles_pred = M, math.ceil(jacobi_sweeps_needed(self.kmin, tol) / M)
            self.weights = [1.0] * self.M
            self.rho = math.exp(self.M * math.log1p(-self.kmin))   # (1 - kappa_min)^M
            return
        b = beta(self.kmin, self.kmax)
        if M is None:
            self.M, self.cycles_pred = choose_cycle(self.kmin, self.kmax, tol)
        else:
            self.M, self.cycles_pred = M, cycles_needed(M, b, tol)
        self.weights = weights(self.kmin, self.kmax, self.M)
        self.rho = math.exp(-log_cosh(self.M * b))   # Chebyshev bound per cycle


def plan(nx, ny, stencil, tol, M=None, h=None, method="chebyshev", bc=BC_ZERO):
    return Plan(nx, ny, stencil, tol, M=M, h=h, method=method, bc=bc)


# ----------------------------------------------------------------------------- loops


def sweep(p, f, u_in, u_out, omega, region=None):
    """One weighted Jacobi sweep of the padded iterate u_in into u_out.  With
    homogeneous data the ring of u_out is refilled (zeros, reflections); with a
    frame (R9) it is data, and both buffers already hold it."""
    nx, ny = p.nx, p.ny
    i0, i1, j0, j1 = region if region is not None else (1, nx, 1, ny)
    L = lib()
    L.cjo_sweep(nx, ny, p.stencil, p.h, _ptr(f), _ptr(u_in), _ptr(u_out), omega, i0, i1, j0, j1)
    if p.bc == BC_ZERO:
        L.cjo_fill_ring(nx, ny, _ptr(u_out))


def sumsq(x):
    """Sum of squares, accumulated serially in storage order."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().cjo_sumsq(ctypes.c_size_t(x.size), _ptr(x))


def residual_sumsq(p, f, u_pad):
    return lib().cjo_residual_sumsq(p.nx, p.ny, p.stencil, p.h, _ptr(f), _ptr(u_pad))


def apply(stencil, u, nx, ny, h=None, bc=BC_ZERO):
    """A u = -Delta_h u on the interior, (ny, nx); u is (ny, nx), or the frame
    array for bc = BC_FRAME (its frame values enter the stencil)."""
    h = spacing(nx, ny) if h is None else h
    up = _padded(u, nx, ny, stencil, bc)
    out = np.empty((ny, nx), dtype=np.float64)
    if lib().cjo_apply(nx, ny, stencil, h, _ptr(up), _ptr(out)) != 0:
        raise ValueError("unknown stencil")
    return out


def rhs_norm(p, f, u_pad):
    """The denominator of the relative residual: ||f|| for homogeneous data
    (R8), the residual norm of the zero interior inside the frame for a frame
    (R9)."""
    if p.bc == BC_FRAME:
        return math.sqrt(residual_sumsq(p, f, _zero_interior(u_pad, p.nx, p.ny)))
    return math.sqrt(sumsq(f))


def relative_residual(stencil, f, u, nx, ny, h=None, bc=BC_ZERO):
    """||f - A u||_2 / ||f - A u_0||_2 with u_0 the zero interior (R8, R9),
    accumulated serially in FP64.  With bc = BC_FRAME, u is the frame array."""
    p = Plan(nx, ny, stencil, 1.0, M=1, h=h, bc=bc)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(ny, nx)
    up = _padded(u, nx, ny, stencil, bc)
    return math.sqrt(residual_sumsq(p, f, up)) / rhs_norm(p, f, up)


def relative_residual_ext(stencil, f, u, u_lo, nx, ny, h=None, bc=BC_ZERO):
    """relative_residual of the unevaluated sum u + u_lo (a double-double
    iterate), the numerator evaluated in x87 extended precision (long double,
    64-bit significand; cjo_residual_sumsq_ext): about 2^-11 of the rounding
    of an FP64 evaluation, so it resolves residuals below the FP64 floor of
    the grid.  The denominator is rhs_norm (FP64).  u_lo has u's shape (with
    bc = BC_FRAME, its frame is zero)."""
    h = spacing(nx, ny) if h is None else h
    p = Plan(nx, ny, stencil, 1.0, M=1, h=h, bc=bc)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(ny, nx)
    hi = _padded(u, nx, ny, stencil, bc)
    lo = _padded(u_lo, nx, ny, stencil, bc)
    num = math.sqrt(lib().cjo_residual_sumsq_ext(nx, ny, stencil, h, _ptr(f), _ptr(hi), _ptr(lo)))
    return num / rhs_norm(p, f, hi)


def solve(f, nx, ny, stencil, tol, M=None, u0=None, max_cycles=None, h=None, method="chebyshev", bc=BC_ZERO):
    """Full solve (R8; R9 with bc = BC_FRAME, where u0 is the frame array and is
    required; R10 with method = 'jacobi').  Returns a dict: u (the frame array
    for a frame), status, cycles, sweeps, relres, history, plan."""
    p = Plan(nx, ny, stencil, tol, M=M, h=h, method=method, bc=bc)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(ny, nx)
    if max_cycles is None:
        max_cycles = p.cycles_pred + 4
    if bc == BC_FRAME:
        if u0 is None:
            raise ValueError("a frame solve needs u0 (the frame array with the boundary data)")
        a = pad_frame(u0, nx, ny, stencil)
    else:
        a = pad(np.zeros((ny, nx)) if u0 is None else u0, nx, ny)

    def result(pad_arr):
        return unpad_frame(pad_arr, nx, ny, stencil) if bc == BC_FRAME else unpad(pad_arr, nx, ny)

    fnorm = rhs_norm(p, f, a)
    out = dict(plan=p, cycles=0, sweeps=0, history=[])
    if not math.isfinite(fnorm):
        out.update(u=np.full(result(a).shape, np.nan), status="nonfinite", relres=float("nan"))
        return out
    if fnorm == 0.0:
        out.update(u=result(_zero_interior(a, nx, ny)), status="ok", relres=0.0)
        return out
    b = a.copy()
    hist = out["history"]
    c = 0
    while True:
        rr = math.sqrt(residual_sumsq(p, f, a)) / fnorm
        hist.append(rr)
        if not math.isfinite(rr):
            status = "nonfinite"
            break
        if rr <= tol:
            status = "ok"
            break
        if c >= 1 and c >= p.cycles_pred and rr > 0.5 * hist[-2]:
            status = "stagnated"
            break
        if c >= max_cycles:
            status = "not_converged"
            break
        for w in p.weights:
            sweep(p, f, a, b, w)
            a, b = b, a
        c += 1
    out.update(u=result(a), status=status, relres=hist[-1], cycles=c, sweeps=c * p.M)
    return out


def run_sweeps(f, nx, ny, stencil, tol, n, M=None, u0=None, h=None, method="chebyshev", bc=BC_ZERO):
    """The iterate after the first n sweeps of the schedule (weights taken
    cyclically); the frame array for bc = BC_FRAME (u0 required then)."""
    p = Plan(nx, ny, stencil, tol, M=M, h=h, method=method, bc=bc)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(ny, nx)
    if bc == BC_FRAME:
        a = pad_frame(u0, nx, ny, stencil)
    else:
        a = pad(np.zeros((ny, nx)) if u0 is None else u0, nx, ny)
    b = a.copy()
    for k in range(n):
        sweep(p, f, a, b, p.weights[k % p.M])
        a, b = b, a
    return unpad_frame(a, nx, ny, stencil) if bc == BC_FRAME else unpad(a, nx, ny)


def sampled_sweeps(f, u0, nx, ny, stencil, tol, n, points, M=None, h=None, first=0, method="chebyshev",
                   bc=BC_ZERO):
    """Values of the iterate after n sweeps (weights first .. first+n-1, cyclic) at the
    given (i, j) nodes, 1-based.  Each value is computed on its domain of dependence
    only: sweep t updates the nodes within radius*(n - t) of each point, which is all
    the next sweep reads.  Works at any grid size in seconds.  u0 is the frame
    array for bc = BC_FRAME."""
    p = Plan(nx, ny, stencil, tol, M=M, h=h, method=method, bc=bc)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(ny, nx)
    r = RADIUS[stencil]
    L = lib()
    a = _padded(u0, nx, ny, stencil, bc)
    b = a.copy()
    for t in range(1, n + 1):
        w = p.weights[(first + t - 1) % p.M]
        e = r * (n - t)
        for (i, j) in points:
            L.cjo_sweep(nx, ny, p.stencil, p.h, _ptr(f), _ptr(a), _ptr(b), w,
                        i - e, i + e, j - e, j + e)
        if bc == BC_ZERO:
            L.cjo_fill_ring(nx, ny, _ptr(b))
        a, b = b, a
    return np.array([a[j + 1, i + 1] for (i, j) in points])
