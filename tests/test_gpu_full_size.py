"""GPU parity at the benchmark sizes, in the launch configuration the benchmark
times: the first solve on a plan picks the blocked kernel's tile height on the
device, and every comparison below runs on that same plan afterwards.

- 4096^2, 9-point: one full weight cycle (M = 4096 sweeps: K = 10 launches and
  the shorter launch that ends the cycle), bitwise equal to M one-sweep launches
  and against the oracle element by element.  Over a whole cycle no FP64
  evaluation can meet 1e-12 against another that rounds in a different order:
  the first weight of the cycle is the largest (about 1/kappa_min), and the two
  end the cycle about 0.17 eps max(omega) apart (9.3e-11 at 4096^2), the same
  for the oracle against a reordered CPU sweep; the bar is three times that.
  The norm-fused first launch of a cycle gives the same bits.
- 8192^2, all three stencils: the full solve against the exact discrete solution
  (type-I sine transform) and its residual recomputed by the oracle; then 3K + 3
  sweeps from a rough guess sampled on the blocked kernel's strip seams
  (lanes - 2KR output columns per strip) and tuned tile seams, each sample computed
  by the oracle on its own domain of dependence, bar 1e-12 of the sample scale.
- Mixed precision at 8192^2 and 16384 x 4096 (FP32 sweeps inside FP64
  refinement, and the double-double iterate of cj_solve_dd): the oracle's
  extended-precision residual and the error against the exact discrete solution.
"""
import sys

import numpy as np
import pytest

from oracle import cjm, dense
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu

REL_L2 = 1e-12
# rel-L2 distance between two FP64 rounding orders after one full cycle, in
# units of eps * max(omega) (measured on the CPU; test_oracle_pins.py)
CYCLE_SPREAD = 0.17


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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _residual_noise(st, f, u, nx, ny):
    """Two FP64 evaluations of r = g - D^{-1}A u cancel terms of size |u| down to
    |r|, so they differ by about eps * ||D u|| / ||f||."""
    taps, s = cjm.taps(st)
    h = cjm.spacing(nx, ny)
    D = -dense.centre(taps) / (s * h * h)
    return 8 * np.finfo(float).eps * np.linalg.norm(u) * D / np.linalg.norm(f)


def test_c2_4096_one_full_cycle_in_the_bench_launch_configuration(torch_cuda):
    torch = torch_cuda
    n, st, tol = 4096, 9, 1e-10
    _say("case: 4096^2 9-point, one full cycle after the tuning solve")
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    fd = _dev(torch, f)
    p = cj.plan(n, n, st, tol)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    cj.solve(p, fd, u)                       # picks the tile height on the device
    K, rows, wg = p.refresh_launch_info()
    M = p.M
    _say("K %d, tuned rows %d, workgroups %d, M %d (%d launches of K and one of %d)"
         % (K, rows, wg, M, M // K, M % K))
    assert K == 10 and M % K != 0
    u.zero_()
    cj.sweeps(p, fd, u, M)
    got = _host(u)
    # bitwise: the same cycle as M launches of the one-sweep kernel
    p_single = cj.plan(n, n, st, tol, sweeps_per_launch=1)
    u.zero_()
    cj.sweeps(p_single, fd, u, M)
    assert np.array_equal(_host(u), got)
    # against the oracle: the largest weight of the cycle multiplies the
    # rounding of every later residual evaluation, so two FP64 evaluations in
    # different orders end a cycle CYCLE_SPREAD * eps * max(omega) apart
    # (test_oracle_pins.py measures this between the oracle and a reordered
    # sweep); the bar allows three times that
    ref = cjm.run_sweeps(f, n, n, st, tol, M)
    rel = _rel(got, ref)
    spread = np.finfo(float).eps * max(p.weights)
    _say("one cycle: rel-L2 vs oracle %.3e = %.3f eps max(omega)" % (rel, rel / spread))
    assert rel <= 3 * CYCLE_SPREAD * spread
    # the solve's first launch of a cycle also reduces the residual of its input;
    # it gives the same bits, and the residual it reports for the end of cycle 1
    # is the oracle's evaluation of the same iterate up to evaluation noise
    p1 = cj.plan(n, n, st, tol, max_cycles=1, tile_rows=rows)
    assert p1.refresh_launch_info()[:2] == (K, rows)
    u1 = torch.zeros_like(u)
    r1 = cj.solve(p1, fd, u1)
    assert r1["status"] == "not_converged" and r1["cycles"] == 1
    assert np.array_equal(_host(u1), got)
    rr = cjm.relative_residual(st, f, got, n, n)
    _say("cycle-1 relres: GPU %.6e, oracle %.6e" % (r1["rel_residual"], rr))
    assert abs(r1["rel_residual"] - rr) <= 1e-6 * rr + _residual_noise(st, f, got, n, n)


def _strip_lanes(n, K, R, rows, workgroups):
    """Lanes per workgroup of the blocked launch (256 or 512 columns per strip),
    read off the plan's workgroup count: strips of lanes - 2KR output columns
    by tiles of `rows` rows."""
    fits = [w for w in (256, 512)
            if -(-n // (w - 2 * K * R)) * -(-n // rows) == workgroups]
    assert len(fits) == 1, (n, K, R, rows, workgroups)
    return fits[0]


def _seam_points(n, K, R, rows, rng, lanes=256):
    """Nodes on both sides of the blocked kernel's strip seams (strips of
    lanes - 2KR output columns; also those of a K = 3 launch, which ends a short
    run in 256-lane strips) and of the tile seams (tuned height, and the 128-row
    default of the shorter launch), plus corners and random nodes."""
    wout = lanes - 2 * K * R
    xs = set()
    for w in (wout, 256 - 2 * 3 * R):
        for k in (1, 2, 5, n // w - 1, n // w):
            xs.update({k * w, k * w + 1})
    ys = set()
    for hgt in (rows, 128):
        for k in (1, 2, n // hgt // 2, n // hgt - 1, n // hgt):
            ys.update({k * hgt, k * hgt + 1})
    xs = sorted(x for x in xs if 1 <= x <= n)
    ys = sorted(y for y in ys if 1 <= y <= n)
    pts = {(1, 1), (n, 1), (1, n), (n, n), (2, n // 2), (n - 1, n - 1)}
    for x in xs:
        pts.add((x, int(rng.integers(1, n + 1))))
    for y in ys:
        pts.add((int(rng.integers(1, n + 1)), y))
    for k in range(12):
        pts.add((xs[int(rng.integers(len(xs)))], ys[int(rng.integers(len(ys)))]))
    for k in range(8):
        pts.add((int(rng.integers(1, n + 1)), int(rng.integers(1, n + 1))))
    return sorted(pts)


@pytest.mark.parametrize("st", [9, 5, 17])
def test_c2_8192_solve_and_blocked_seams(torch_cuda, st):
    torch = torch_cuda
    n, tol = 8192, 1e-10
    _say("case: 8192^2 %d-point full solve" % st)
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    fd = _dev(torch, f)
    p = cj.plan(n, n, st, tol)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p, fd, u)
    K, rows, wg = p.refresh_launch_info()
    got = _host(u)
    del u
    rr = cjm.relative_residual(st, f, got, n, n)
    taps, s = cjm.taps(st)
    exact = dense.dst_solve(taps, s, f, n, n, cjm.spacing(n, n))
    err = _rel(got, exact)
    _say("K %d rows %d: status %s cycles %d, relres GPU %.3e oracle %.3e, rel err vs DST %.3e"
         % (K, rows, r["status"], r["cycles"], r["rel_residual"], rr, err))
    assert r["status"] in ("ok", "stagnated")
    assert r["cycles"] >= p.cycles_pred
    assert abs(rr - r["rel_residual"]) <= 1e-3 * rr + _residual_noise(st, f, got, n, n)
    assert rr <= 5e-9           # the FP64 floor at this size (1.98e-9 for 9 points)
    assert err <= 1e-8
    del got, exact

    R = 2 if st == 17 else 1
    nsw = 3 * K + 3             # three full K-launches and a K = 3 launch
    _say("case: 8192^2 %d-point, %d sweeps sampled at seams" % (st, nsw))
    u0 = inputs.random_field(n, n, seed=17, scale=1e-3)
    u = _dev(torch, u0)
    cj.sweeps(p, fd, u, nsw)
    got = _host(u)
    p_single = cj.plan(n, n, st, tol, sweeps_per_launch=1)
    u.copy_(_dev(torch, u0))
    cj.sweeps(p_single, fd, u, nsw)
    assert np.array_equal(_host(u), got)
    lanes = _strip_lanes(n, K, R, rows, wg)
    pts = _seam_points(n, K, R, rows, np.random.default_rng(n + st), lanes)
    _say("strips of %d lanes (%d output columns), %d-row tiles" % (lanes, lanes - 2 * K * R, rows))
    ref = cjm.sampled_sweeps(f, u0, n, n, st, tol, nsw, pts)
    vals = np.array([got[j - 1, i - 1] for (i, j) in pts])
    dev = np.abs(vals - ref).max()
    scale = np.abs(ref).max()
    _say("%d sampled nodes: max |GPU - oracle| %.3e of scale %.3e" % (len(pts), dev, scale))
    assert dev <= 1e-12 * scale


def test_c3_16384_blocked_seams(torch_cuda):
    """The largest grid (16384^2, 9-point, the C3 size) in the plain FP64 path's own
    launch configuration: one cycle tunes the tile height, then 3K + 3 sweeps are
    bitwise equal to single sweeps and match the oracle at the blocked kernel's
    strip and tile seams."""
    torch = torch_cuda
    n, st, tol = 16384, 9, 1e-10
    _say("case: 16384^2 9-point, one cycle (tile tuning)")
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    fd = _dev(torch, f)
    p = cj.plan(n, n, st, tol, max_cycles=1)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    r = cj.solve(p, fd, u)
    K, rows, wg = p.refresh_launch_info()
    _say("K %d rows %d workgroups %d: status %s after %d cycle(s), relres %.3e"
         % (K, rows, wg, r["status"], r["cycles"], r["rel_residual"]))
    assert r["status"] == "not_converged" and r["cycles"] == 1 and np.isfinite(r["rel_residual"])
    nsw = 3 * K + 3
    _say("case: 16384^2 9-point, %d sweeps sampled at seams" % nsw)
    u0 = inputs.random_field(n, n, seed=19, scale=1e-3)
    u.copy_(_dev(torch, u0))
    cj.sweeps(p, fd, u, nsw)
    got = _host(u)
    p_single = cj.plan(n, n, st, tol, sweeps_per_launch=1)
    u.copy_(_dev(torch, u0))
    cj.sweeps(p_single, fd, u, nsw)
    assert np.array_equal(_host(u), got)
    lanes = _strip_lanes(n, K, 1, rows, wg)
    pts = _seam_points(n, K, 1, rows, np.random.default_rng(n + st), lanes)
    _say("strips of %d lanes (%d output columns), %d-row tiles" % (lanes, lanes - 2 * K, rows))
    ref = cjm.sampled_sweeps(f, u0, n, n, st, tol, nsw, pts)
    vals = np.array([got[j - 1, i - 1] for (i, j) in pts])
    dev = np.abs(vals - ref).max()
    scale = np.abs(ref).max()
    _say("%d sampled nodes: max |GPU - oracle| %.3e of scale %.3e" % (len(pts), dev, scale))
    assert dev <= 1e-12 * scale


C3_SHAPES = [pytest.param(8192, 8192, id="8192x8192"), pytest.param(16384, 4096, id="16384x4096")]


@pytest.mark.parametrize("nx,ny", C3_SHAPES)
def test_c3_refinement_at_full_size(torch_cuda, nx, ny):
    """FP32 sweeps inside FP64 refinement, 9-point, tol 1e-10: the double-double
    iterate (cj_solve_dd on the refinement plan) meets the tolerance by the
    oracle's extended-precision residual; the FP64 iterate of cj_solve reaches
    what an FP64 array holds there.  Both are compared with the exact discrete
    solution."""
    torch = torch_cuda
    st, tol = 9, 1e-10
    _say("case: C3 %dx%d" % (nx, ny))
    f = inputs.gaussian_bumps_rhs(nx, ny, seed=1705 + st)
    fd = _dev(torch, f)
    p = cj.plan(nx, ny, st, tol, precision=cj.F32_REFINE)
    u = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
    lo = torch.zeros_like(u)
    r = cj.solve_dd(p, fd, u, lo)
    hi, lo_h = _host(u), _host(lo)
    ext = cjm.relative_residual_ext(st, f, hi, lo_h, nx, ny)
    taps, s = cjm.taps(st)
    exact = dense.dst_solve(taps, s, f, nx, ny, cjm.spacing(nx, ny))
    err = _rel(hi, exact)
    _say("double-double: status %s outer %d FP32 sweeps %d relres %.3e oracle (extended) %.3e err vs DST %.3e"
         % (r["status"], r["cycles"], r["sweeps"], r["rel_residual"], ext, err))
    assert r["status"] == "ok" and r["rel_residual"] <= tol
    assert ext <= 1.5 * tol
    assert np.all(np.abs(lo_h) <= np.spacing(np.abs(hi)) / 2)
    assert err <= 1e-8
    del hi, lo_h, lo
    u.zero_()
    r2 = cj.solve(p, fd, u)
    got = _host(u)
    rr = cjm.relative_residual(st, f, got, nx, ny)
    err2 = _rel(got, exact)
    _say("FP64 iterate: status %s outer %d relres %.3e oracle %.3e err vs DST %.3e"
         % (r2["status"], r2["cycles"], r2["rel_residual"], rr, err2))
    assert r2["status"] in ("ok", "stagnated")
    assert abs(rr - r2["rel_residual"]) <= 1e-3 * rr + _residual_noise(st, f, got, nx, ny)
    assert rr <= 5e-10
    assert err2 <= 1e-8


def test_c3_16384_refinement_takes_fp64_inner_cycles(torch_cuda):
    """16384^2, 9-point, tol 1e-10: eps32 * kmax / kmin = 8.6, where FP32 inner
    cycles stagnate near 4e-10; the refinement plan takes FP64 inner cycles by
    itself, and its double-double iterate meets the tolerance by the oracle's
    extended-precision residual."""
    torch = torch_cuda
    n, st, tol = 16384, 9, 1e-10
    _say("case: C3 16384^2")
    f = inputs.gaussian_bumps_rhs(n, n, seed=1705 + st)
    p = cj.plan(n, n, st, tol, precision=cj.F32_REFINE)
    q = cj.plan(n, n, st, tol)
    assert (p.M, p.sweeps_per_launch) == (q.M, q.sweeps_per_launch)   # the FP64 schedule and kernel
    q.destroy()
    fd = _dev(torch, f)
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    lo = torch.zeros_like(u)
    r = cj.solve_dd(p, fd, u, lo)
    hi, lo_h = _host(u), _host(lo)
    del u, lo, fd
    p.destroy()
    ext = cjm.relative_residual_ext(st, f, hi, lo_h, n, n)
    _say("double-double, FP64 inner cycles: status %s outer %d sweeps %d %.1f s relres %.3e oracle (extended) %.3e"
         % (r["status"], r["cycles"], r["sweeps"], r["seconds"], r["rel_residual"], ext))
    assert r["status"] == "ok" and r["rel_residual"] <= tol
    assert ext <= 1.5 * tol
    assert np.all(np.abs(lo_h) <= np.spacing(np.abs(hi)) / 2)
