"""Python binding of libcj.so (include/cj.h): argument marshalling only.

Every computation runs in the library's HIP kernels.  Grids are torch tensors
on the GPU: float64, contiguous, shape (ny, nx) (x fastest).  torch provides
device memory and the current HIP stream; nothing else.

    import torch
    from paper_1705_00103_amd import cj
    p = cj.plan(nx, ny, stencil=9, tol=1e-10)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    res = cj.solve(p, f, u)        # u now holds the solution

With bc=BC_FRAME, u is (ny + 2G, nx + 2G) and carries the Dirichlet data in
its frame of width G = plan.frame (1, or 2 for the 17-point stencil).
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcj.so")

CJ_OK = 0
CJ_STAGNATED = 1
CJ_ERR_ARG = -1
CJ_ERR_NOMEM = -2
CJ_ERR_HIP = -3
CJ_ERR_NOT_CONVERGED = -4
CJ_ERR_NONFINITE = -5
CJ_ERR_DEVICE = -6

F64 = 0             # CJ_PRECISION_F64
F32_REFINE = 1      # CJ_PRECISION_F32_REFINE
BC_ZERO = 0         # CJ_BC_DIRICHLET0
BC_FRAME = 1        # CJ_BC_DIRICHLET_FRAME: u carries the boundary data in a frame
CHEBYSHEV = 0       # CJ_METHOD_CHEBYSHEV
JACOBI = 1          # CJ_METHOD_JACOBI
INNER_AUTO = 0      # CJ_INNER_AUTO: inner cycles of a refinement plan chosen from eps32 * kmax / kmin
INNER_F32 = 1       # CJ_INNER_F32
INNER_F64 = 2       # CJ_INNER_F64

STATUS_NAMES = {
    CJ_OK: "ok", CJ_STAGNATED: "stagnated", CJ_ERR_ARG: "arg", CJ_ERR_NOMEM: "nomem",
    CJ_ERR_HIP: "hip", CJ_ERR_NOT_CONVERGED: "not_converged", CJ_ERR_NONFINITE: "nonfinite",
    CJ_ERR_DEVICE: "device",
}

# Function names declared in include/cj.h (checked against the header by the tests).
EXPORTS = ("cj_options_init", "cj_plan", "cj_plan_ex", "cj_plan_info", "cj_plan_launch_info", "cj_solve",
           "cj_solve_dd", "cj_sweeps", "cj_residual", "cj_residual_noalloc", "cj_apply", "cj_plan_destroy",
           "cj_status_string", "cj_last_error",
           "cj_batch_create", "cj_batch_info", "cj_batch_solve", "cj_batch_destroy",
           "cj_server_create", "cj_server_submit", "cj_server_step", "cj_server_stats", "cj_server_destroy")


class Options(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("sweeps_per_launch", ctypes.c_int), ("tile_rows", ctypes.c_int),
                ("h", ctypes.c_double), ("precision", ctypes.c_int), ("inner_M", ctypes.c_int),
                ("graph", ctypes.c_int), ("method", ctypes.c_int), ("inner_precision", ctypes.c_int),
                ("single_workgroup", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("sweeps", ctypes.c_longlong),
                ("rel_residual", ctypes.c_double), ("floor_estimate", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sweep_seconds", ctypes.c_double),
                ("sweep_launches", ctypes.c_longlong)]

    def as_dict(self):
        return dict(status=STATUS_NAMES.get(self.status, str(self.status)), code=self.status,
                    cycles=self.cycles, sweeps=self.sweeps, rel_residual=self.rel_residual,
                    floor_estimate=self.floor_estimate, seconds=self.seconds,
                    sweep_seconds=self.sweep_seconds, sweep_launches=self.sweep_launches)


class BatchStats(ctypes.Structure):
    _fields_ = [("supersteps", ctypes.c_int), ("launches", ctypes.c_longlong), ("points", ctypes.c_longlong),
                ("updates", ctypes.c_double), ("seconds", ctypes.c_double),
                ("sweeps_per_launch", ctypes.c_int * 3), ("tile_rows", ctypes.c_int * 3),
                ("reserved", ctypes.c_int * 2)]

    def as_dict(self):
        return dict(supersteps=self.supersteps, launches=self.launches, points=self.points, updates=self.updates,
                    seconds=self.seconds, sweeps_per_launch=dict(zip((5, 9, 17), self.sweeps_per_launch)),
                    tile_rows=dict(zip((5, 9, 17), self.tile_rows)))


class CJError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed: %s (%s)" % (where, STATUS_NAMES.get(code, code), msg))
        self.code = code


_lib = None


def lib():
    """Loads libcj.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcj.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_1705_00103_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.cj_options_init.argtypes = [ctypes.POINTER(Options)]
        L.cj_options_init.restype = None
        L.cj_plan.argtypes = [c_int, c_int, c_int, c_int, c_double, ctypes.POINTER(vp)]
        L.cj_plan.restype = c_int
        L.cj_plan_ex.argtypes = [c_int, c_int, c_int, c_int, c_double, ctypes.POINTER(Options),
                                 ctypes.POINTER(vp)]
        L.cj_plan_ex.restype = c_int
        L.cj_plan_info.argtypes = [vp, dp, dp, ip, ip, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_size_t)]
        L.cj_plan_info.restype = c_int
        L.cj_plan_launch_info.argtypes = [vp, ip, ip, ip]
        L.cj_plan_launch_info.restype = c_int
        L.cj_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Result)]
        L.cj_solve.restype = c_int
        L.cj_solve_dd.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(Result)]
        L.cj_solve_dd.restype = c_int
        L.cj_sweeps.argtypes = [vp, vp, vp, ctypes.c_longlong, vp]
        L.cj_sweeps.restype = c_int
        L.cj_residual.argtypes = [vp, vp, vp, vp, dp]
        L.cj_residual.restype = c_int
        L.cj_residual_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.cj_residual_noalloc.restype = c_int
        L.cj_apply.argtypes = [vp, vp, vp, vp]
        L.cj_apply.restype = c_int
        L.cj_plan_destroy.argtypes = [vp]
        L.cj_plan_destroy.restype = None
        L.cj_batch_create.argtypes = [c_int, ip, ip, ip, dp, ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.cj_batch_create.restype = c_int
        L.cj_batch_info.argtypes = [vp, c_int, ip, ip, ctypes.POINTER(ctypes.c_size_t)]
        L.cj_batch_info.restype = c_int
        L.cj_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.POINTER(Result),
                                     ctypes.POINTER(BatchStats)]
        L.cj_batch_solve.restype = c_int
        L.cj_batch_destroy.argtypes = [vp]
        L.cj_batch_destroy.restype = None
        L.cj_server_create.argtypes = [ctypes.POINTER(Options), ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.cj_server_create.restype = c_int
        L.cj_server_submit.argtypes = [vp, c_int, c_int, c_int, c_double, vp, vp, ctypes.POINTER(ctypes.c_longlong)]
        L.cj_server_submit.restype = c_int
        L.cj_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(Result), c_int, ip]
        L.cj_server_step.restype = c_int
        L.cj_server_stats.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_size_t)]
        L.cj_server_stats.restype = c_int
        L.cj_server_destroy.argtypes = [vp]
        L.cj_server_destroy.restype = None
        L.cj_status_string.argtypes = [c_int]
        L.cj_status_string.restype = ctypes.c_char_p
        L.cj_last_error.argtypes = []
        L.cj_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def last_error():
    return lib().cj_last_error().decode()


def status_string(code):
    return lib().cj_status_string(code).decode()


def _check(code, where, ok=(CJ_OK,)):
    if code not in ok:
        raise CJError(code, where, last_error())
    return code


class Plan:
    """Owns a cj_plan_t.  Attributes mirror cj_plan_info."""

    def __init__(self, nx, ny, stencil=9, tol=1e-10, M=0, max_cycles=0, sweeps_per_launch=0,
                 tile_rows=0, h=0.0, bc=BC_ZERO, precision=F64, inner_M=0, graph=0, method=CHEBYSHEV,
                 inner_precision=INNER_AUTO, single_workgroup=0):
        L = lib()
        o = Options()
        L.cj_options_init(ctypes.byref(o))
        o.M, o.max_cycles, o.sweeps_per_launch, o.tile_rows, o.h = M, max_cycles, sweeps_per_launch, tile_rows, h
        o.precision, o.inner_M, o.graph, o.method = precision, inner_M, graph, method
        o.inner_precision, o.single_workgroup = inner_precision, single_workgroup
        self.precision, self.bc, self.method = precision, bc, method
        # width of u's boundary frame (CJ_BC_DIRICHLET_FRAME)
        self.frame = (2 if stencil == 17 else 1) if bc == BC_FRAME else 0
        handle = ctypes.c_void_p()
        _check(L.cj_plan_ex(nx, ny, stencil, bc, tol, ctypes.byref(o), ctypes.byref(handle)), "cj_plan_ex")
        self._h = handle
        self.nx, self.ny, self.stencil, self.tol = nx, ny, stencil, tol
        kmin, kmax = ctypes.c_double(), ctypes.c_double()
        Mo, cp = ctypes.c_int(), ctypes.c_int()
        w = ctypes.POINTER(ctypes.c_double)()
        ws = ctypes.c_size_t()
        _check(L.cj_plan_info(handle, ctypes.byref(kmin), ctypes.byref(kmax), ctypes.byref(Mo),
                              ctypes.byref(cp), ctypes.byref(w), ctypes.byref(ws)), "cj_plan_info")
        self.kmin, self.kmax, self.M, self.cycles_pred = kmin.value, kmax.value, Mo.value, cp.value
        self.weights = [w[k] for k in range(self.M)]
        self.workspace_bytes = ws.value
        self.refresh_launch_info()

    def refresh_launch_info(self):
        """Re-reads cj_plan_launch_info (the tile height is chosen at the first
        solve)."""
        k, rows, wg = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().cj_plan_launch_info(self.handle, ctypes.byref(k), ctypes.byref(rows), ctypes.byref(wg)),
               "cj_plan_launch_info")
        self.sweeps_per_launch, self.tile_rows, self.workgroups = k.value, rows.value, wg.value
        return self.sweeps_per_launch, self.tile_rows, self.workgroups

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    def destroy(self):
        if self._h is not None and _lib is not None:
            _lib.cj_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def plan(nx, ny, stencil=9, tol=1e-10, **opts):
    return Plan(nx, ny, stencil, tol, **opts)


def _grid_ptr(t, p, name, framed=False):
    """framed: the array is u of a CJ_BC_DIRICHLET_FRAME plan, (ny + 2G) x (nx + 2G)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 GPU tensor" % name)
    G = p.frame if framed else 0
    need = (p.nx + 2 * G) * (p.ny + 2 * G)
    if t.numel() != need:
        raise ValueError("%s has %d elements, the plan needs %d" % (name, t.numel(), need))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def solve(p, f, u, stream=None, raise_on_error=False):
    """Solves A u = f in place (u: guess in, solution out).  Returns the result dict;
    status 'stagnated' and 'not_converged' are results, not exceptions, unless
    raise_on_error is set.  Argument and runtime errors raise CJError."""
    r = Result()
    code = lib().cj_solve(p.handle, _grid_ptr(f, p, "f"), _grid_ptr(u, p, "u", True), _stream(stream),
                          ctypes.byref(r))
    if code in (CJ_ERR_ARG, CJ_ERR_NOMEM, CJ_ERR_HIP, CJ_ERR_DEVICE) or (raise_on_error and code != CJ_OK):
        raise CJError(code, "cj_solve", last_error())
    return r.as_dict()


def solve_dd(p, f, u, u_lo, stream=None, raise_on_error=False):
    """cj_solve_dd: iterative refinement with the iterate carried as u + u_lo
    (inner FP32 cycles for an F32_REFINE plan, FP64 cycles for an F64 plan).
    u: guess in, high parts out; u_lo (same shape, must not overlap u or f):
    low parts out.  Result as for solve."""
    r = Result()
    code = lib().cj_solve_dd(p.handle, _grid_ptr(f, p, "f"), _grid_ptr(u, p, "u", True),
                             _grid_ptr(u_lo, p, "u_lo", True), _stream(stream), ctypes.byref(r))
    if code in (CJ_ERR_ARG, CJ_ERR_NOMEM, CJ_ERR_HIP, CJ_ERR_DEVICE) or (raise_on_error and code != CJ_OK):
        raise CJError(code, "cj_solve_dd", last_error())
    return r.as_dict()


def sweeps(p, f, u, n, stream=None):
    """Applies the first n sweeps of the plan's schedule to u in place."""
    _check(lib().cj_sweeps(p.handle, _grid_ptr(f, p, "f"), _grid_ptr(u, p, "u", True), int(n), _stream(stream)),
           "cj_sweeps")


def residual(p, f, u, stream=None):
    """||f - A u|| / ||f||."""
    out = ctypes.c_double()
    _check(lib().cj_residual(p.handle, _grid_ptr(f, p, "f"), _grid_ptr(u, p, "u", True), _stream(stream),
                             ctypes.byref(out)), "cj_residual")
    return out.value


def residual_noalloc(p, f, u, out, stream=None):
    """cj_residual_noalloc: ||f - A u|| / ||f|| written to out (a float64 GPU
    tensor with one element) on the stream, without waiting and without any
    device allocation."""
    import torch
    if not isinstance(out, torch.Tensor) or out.device.type != "cuda" or out.dtype != torch.float64 \
            or out.numel() < 1:
        raise ValueError("out must be a float64 GPU tensor")
    _check(lib().cj_residual_noalloc(p.handle, _grid_ptr(f, p, "f"), _grid_ptr(u, p, "u", True),
                                     ctypes.c_void_p(out.data_ptr()), _stream(stream)), "cj_residual_noalloc")


def apply(p, u, au, stream=None):
    """au = A u."""
    _check(lib().cj_apply(p.handle, _grid_ptr(u, p, "u", True), _grid_ptr(au, p, "au"), _stream(stream)),
           "cj_apply")


class Batch:
    """Owns a cj_batch_t: n problems given as lists of (nx, ny), stencils and tolerances."""

    def __init__(self, shapes, stencils, tols, sweeps_per_launch=0, tile_rows=0, max_cycles=0):
        L = lib()
        n = len(shapes)
        if not (len(stencils) == len(tols) == n):
            raise ValueError("shapes, stencils and tols must have the same length")
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        IA = ctypes.c_int * n
        nx = IA(*[a for a, _ in self.shapes])
        ny = IA(*[b for _, b in self.shapes])
        st = IA(*[int(v) for v in stencils])
        tl = (ctypes.c_double * n)(*[float(v) for v in tols])
        o = Options()
        L.cj_options_init(ctypes.byref(o))
        o.precision = F32_REFINE
        o.sweeps_per_launch, o.tile_rows, o.max_cycles = sweeps_per_launch, tile_rows, max_cycles
        h = ctypes.c_void_p()
        _check(L.cj_batch_create(n, nx, ny, st, tl, ctypes.byref(o), ctypes.byref(h)), "cj_batch_create")
        self._h = h
        self.n = n

    def info(self, i):
        M, k, ws = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().cj_batch_info(self._h, i, ctypes.byref(M), ctypes.byref(k), ctypes.byref(ws)), "cj_batch_info")
        return dict(M=M.value, sweeps_per_launch=k.value, workspace_bytes=ws.value)

    def solve(self, fs, us, stream=None):
        """Solves every problem in place (us[i]: guess in, solution out).  Returns
        (list of per-problem result dicts, stats dict)."""
        import torch
        if len(fs) != self.n or len(us) != self.n:
            raise ValueError("need %d f and u tensors" % self.n)
        VA = ctypes.c_void_p * self.n
        fp, up = VA(), VA()
        for i, ((nx, ny), f, u) in enumerate(zip(self.shapes, fs, us)):
            for name, t in (("f", f), ("u", u)):
                if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
                        or not t.is_contiguous() or t.numel() != nx * ny:
                    raise ValueError("problem %d: %s must be a contiguous float64 GPU tensor of %d elements"
                                     % (i, name, nx * ny))
            fp[i] = f.data_ptr()
            up[i] = u.data_ptr()
        res = (Result * self.n)()
        stats = BatchStats()
        code = lib().cj_batch_solve(self._h, fp, up, _stream(stream), res, ctypes.byref(stats))
        if code in (CJ_ERR_ARG, CJ_ERR_NOMEM, CJ_ERR_HIP, CJ_ERR_DEVICE):
            raise CJError(code, "cj_batch_solve", last_error())
        return [r.as_dict() for r in res], stats.as_dict()

    def destroy(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.cj_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Owns a cj_server_t (continuous batching of solve requests)."""

    def __init__(self, hbm_budget_bytes, stream=None, sweeps_per_launch=0, tile_rows=0, max_cycles=0):
        L = lib()
        o = Options()
        L.cj_options_init(ctypes.byref(o))
        o.precision = F32_REFINE
        o.sweeps_per_launch, o.tile_rows, o.max_cycles = sweeps_per_launch, tile_rows, max_cycles
        h = ctypes.c_void_p()
        _check(L.cj_server_create(ctypes.byref(o), int(hbm_budget_bytes), _stream(stream), ctypes.byref(h)),
               "cj_server_create")
        self._h = h
        self._keep = {}     # ticket -> (f, u) kept alive until done

    def submit(self, nx, ny, stencil, tol, f, u):
        import torch
        for name, t in (("f", f), ("u", u)):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
                    or not t.is_contiguous() or t.numel() != nx * ny:
                raise ValueError("%s must be a contiguous float64 GPU tensor of nx*ny elements" % name)
        tk = ctypes.c_longlong()
        _check(lib().cj_server_submit(self._h, nx, ny, stencil, tol, ctypes.c_void_p(f.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr()), ctypes.byref(tk)), "cj_server_submit")
        self._keep[tk.value] = (f, u)
        return tk.value

    def step(self, max_done=256):
        """One server step; returns a list of (ticket, result dict) finished in it."""
        tks = (ctypes.c_longlong * max_done)()
        res = (Result * max_done)()
        nd = ctypes.c_int()
        code = lib().cj_server_step(self._h, tks, res, max_done, ctypes.byref(nd))
        out = []
        for k in range(nd.value):
            self._keep.pop(tks[k], None)
            out.append((tks[k], res[k].as_dict()))
        if code in (CJ_ERR_ARG, CJ_ERR_NOMEM, CJ_ERR_HIP, CJ_ERR_DEVICE):
            raise CJError(code, "cj_server_step", last_error())
        return out

    def stats(self):
        a, q, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().cj_server_stats(self._h, ctypes.byref(a), ctypes.byref(q), ctypes.byref(b)), "cj_server_stats")
        return dict(active=a.value, queued=q.value, bytes_in_use=b.value)

    def destroy(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.cj_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
