"""The other workloads at their full sizes, against the exact discrete solution.

* Upwind DG-Q1 on 1024 x 1024 cells (theta pi/5, element-block scaled,
  permuted; 4.19M unknowns): the FP64 solve and the V-cycles in FP32 and in
  BF16 storage inside the FP64 outer FGMRES.
* 64 right-hand sides of the FV 2048 x 2048 matrix (FP32 V-cycle), one outer
  process per column.
* 48 FV problems with sides drawn from {128, 256, 512, 1024} and angles from
  U(0, pi/2) in one block-diagonal hierarchy (FP32 and BF16 V-cycles), one
  outer process per problem.

The exact discrete solution comes from the oracle's flow-order sweep (one
Gauss-Seidel pass in flow order solves an upwind system exactly).  Every
result must reach the FP64 true relative residual 1e-10; its distance to the
exact solution is then bounded by the condition number times that residual,
and the test prints it (the figures the design notes quote)."""
import math

import numpy as np
import pytest

import oracle
from airg_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _err(x, u):
    return (float(np.abs(x - u).max() / np.abs(u).max()),
            float(np.linalg.norm(x - u) / np.linalg.norm(u)))


@pytest.fixture(scope="module")
def dg1024():
    _needs_gpu()
    print("building dg1024", flush=True)
    p = workloads.dg1024()
    u = oracle.sweep_solve(p.scipy(), p.b, p.level)
    return p, u


@pytest.mark.parametrize("prec,name", [(0, "fp64"), (1, "fp32"), (2, "bf16")])
def test_dg1024_against_the_exact_solution(dg1024, prec, name):
    from paper_2508_17517_amd import Solver
    p, u = dg1024
    s = Solver(p.indptr, p.indices, p.data, precision=prec)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    xg = x.cpu().numpy()
    rel = np.linalg.norm(p.b - p.scipy() @ xg) / np.linalg.norm(p.b)
    emax, e2 = _err(xg, u)
    print(f"dg1024 {name}: {info['iterations']} iterations, true rel residual {rel:.2e}, "
          f"error vs exact: max {emax:.2e}, 2-norm {e2:.2e}", flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert rel <= 1e-10 * (1 + 1e-6)
    assert e2 <= 1e-7
    s.close()


def test_fv2048_64_columns_against_the_exact_solution():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    print("building fv2048 and 64 right-hand sides", flush=True)
    p = workloads.fv2048()
    B = workloads.rhs_batch(p, 64)
    s = Solver(p.indptr, p.indices, p.data, precision=1)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    A = p.scipy()
    assert all(i["converged"] == 1 and i["rel_residual"] <= 1e-10 for i in infos)
    worst = 0.0
    for c in (0, 21, 42, 63):
        xc = X[c].cpu().numpy()
        assert np.linalg.norm(B[c] - A @ xc) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(B[c])
        u = oracle.sweep_solve(A, B[c], p.level)
        emax, e2 = _err(xc, u)
        worst = max(worst, e2)
        assert e2 <= 1e-7, c
    print(f"fv2048 x 64 columns (FP32 V-cycle): iterations {min(i['iterations'] for i in infos)}-"
          f"{max(i['iterations'] for i in infos)}, worst 2-norm error vs exact over the 4 "
          f"checked columns {worst:.2e}", flush=True)
    s.close()


@pytest.mark.parametrize("prec,name", [(1, "fp32"), (2, "bf16")])
def test_48_problems_against_the_exact_solution(prec, name):
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver
    print(f"building the 48 problems ({name} V-cycle)", flush=True)
    probs = workloads.batch_problems(48)
    mats = [(q.indptr, q.indices, q.data) for q in probs]
    sb = BatchSolver(mats, precision=prec)
    xs, infos = sb.solve([torch.from_numpy(q.b).cuda() for q in probs])
    worst = 0.0
    for q, x, i in zip(probs, xs, infos):
        xq = x.cpu().numpy()
        A = q.scipy()
        assert i["converged"] == 1 and i["rel_residual"] <= 1e-10
        assert np.linalg.norm(q.b - A @ xq) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(q.b)
        u = oracle.sweep_solve(A, q.b, q.level)
        emax, e2 = _err(xq, u)
        worst = max(worst, e2)
        assert e2 <= 1e-7
    print(f"48 problems ({sum(q.n for q in probs)} unknowns, {name} V-cycle): iterations "
          f"{min(i['iterations'] for i in infos)}-{max(i['iterations'] for i in infos)}, worst "
          f"2-norm error vs exact {worst:.2e}", flush=True)
    sb.close()
