"""GPU tests of batched solves (cj_batch_*): many problems of uneven size in
shared launches.  Each problem's result equals the single-problem refined solve
of the same problem (same kernels, same decisions) and meets its tolerance as
recomputed by the FP64 oracle."""
import numpy as np
import pytest

from oracle import cjm
from paper_1705_00103_amd import cj, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _run_batch(torch, shapes, stencils, tols, seed=0, zero=(), infos=None):
    fs, us, hf = [], [], []
    for i, (nx, ny) in enumerate(shapes):
        f = np.zeros((ny, nx)) if i in zero else inputs.gaussian_bumps_rhs(nx, ny, seed=seed + i)
        hf.append(f)
        fs.append(_dev(torch, f))
        us.append(torch.zeros(ny, nx, dtype=torch.float64, device="cuda"))
    b = cj.Batch(shapes, stencils, tols)
    if infos is not None:
        infos.extend(b.info(i) for i in range(len(shapes)))
    res, stats = b.solve(fs, us)
    b.destroy()
    return hf, fs, us, res, stats


def test_batch_matches_single_problem_solves(torch_cuda):
    torch = torch_cuda
    shapes = [(64, 64), (300, 41), (17, 260), (129, 129), (1, 1), (3, 2), (511, 70), (200, 200), (90, 33),
              (40, 40), (257, 65), (64, 300)]
    stencils = [9, 5, 17, 9, 9, 17, 9, 5, 17, 9, 9, 5]
    tols = [1e-8, 1e-10, 1e-8, 1e-10, 1e-8, 1e-8, 1e-9, 1e-6, 1e-10, 1e-8, 1e-8, 1e-10]
    infos = []
    hf, fs, us, res, stats = _run_batch(torch, shapes, stencils, tols, seed=100, zero=(9,), infos=infos)
    print("batch stats", stats, flush=True)
    assert stats["supersteps"] > 0
    for i, ((nx, ny), st, tol) in enumerate(zip(shapes, stencils, tols)):
        got = us[i].cpu().numpy()
        r = res[i]
        if i == 9:
            assert r["status"] == "ok" and not got.any()
            continue
        # the batch runs inner cycles of at least 16 sweeps: the single-problem
        # solve it is compared with uses the same inner cycle and depth
        p = cj.plan(nx, ny, st, tol, precision=cj.F32_REFINE, inner_M=infos[i]["M"],
                    sweeps_per_launch=infos[i]["sweeps_per_launch"])
        u1 = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
        r1 = cj.solve(p, fs[i], u1)
        one = u1.cpu().numpy()
        print(i, (nx, ny), st, tol, r["status"], r["cycles"], r1["cycles"], r["rel_residual"], flush=True)
        assert r["status"] == r1["status"] == "ok"
        assert r["cycles"] == r1["cycles"] and r["sweeps"] == r1["sweeps"]
        assert np.array_equal(got, one)
        rr = cjm.relative_residual(st, hf[i], got, nx, ny)
        assert rr <= tol * 1.01


def test_batch_of_many_uneven_problems(torch_cuda):
    torch = torch_cuda
    shapes = inputs.log_uniform_shapes(48, seed=7, lo=16, hi=400)
    stencils = [9 if i % 3 else 5 for i in range(len(shapes))]
    tols = [1e-8] * len(shapes)
    hf, fs, us, res, stats = _run_batch(torch, shapes, stencils, tols, seed=500)
    print("batch stats", stats, flush=True)
    for i, ((nx, ny), st) in enumerate(zip(shapes, stencils)):
        assert res[i]["status"] == "ok", (i, res[i])
        if i % 6 == 0:
            rr = cjm.relative_residual(st, hf[i], us[i].cpu().numpy(), nx, ny)
            assert rr <= 1.01e-8


def test_batch_at_the_c4_shape_range(torch_cuda):
    """64 problems with nx, ny log-uniform over [64, 2048] (the batched
    workload's range), 9-point, tol 1e-8: every result is bit-identical to the
    single-problem refined solve of the same problem and meets its tolerance
    by the oracle's residual."""
    torch = torch_cuda
    shapes = inputs.log_uniform_shapes(64, seed=1705, lo=64, hi=2048)
    stencils = [9] * len(shapes)
    tols = [1e-8] * len(shapes)
    infos = []
    hf, fs, us, res, stats = _run_batch(torch, shapes, stencils, tols, seed=2000, infos=infos)
    print("batch stats", stats, "points", sum(nx * ny for nx, ny in shapes), flush=True)
    worst = 0.0
    for i, (nx, ny) in enumerate(shapes):
        r = res[i]
        assert r["status"] == "ok", (i, r)
        p = cj.plan(nx, ny, 9, 1e-8, precision=cj.F32_REFINE, inner_M=infos[i]["M"],
                    sweeps_per_launch=infos[i]["sweeps_per_launch"])
        u1 = torch.zeros(ny, nx, dtype=torch.float64, device="cuda")
        r1 = cj.solve(p, fs[i], u1)
        p.destroy()
        assert (r["cycles"], r["sweeps"]) == (r1["cycles"], r1["sweeps"])
        assert torch.equal(us[i], u1)
        rr = cjm.relative_residual(9, hf[i], us[i].cpu().numpy(), nx, ny)
        worst = max(worst, rr)
        assert rr <= 1.01e-8
    print("largest oracle relres %.3e" % worst, flush=True)
