"""The coarsest level's Newton polynomial in one persistent launch
(params.coarse_persistent = 1): the coarsest matrix stays in registers across
the steps and a grid-wide barrier separates them.  The steps are those of the
per-step launches and only the order of each row's sum differs, so solves
must match the oracle (same iteration count, elementwise 1e-10) in FP64 and
with FP32 / BF16 storage, over one workgroup and over many, repeat bit for
bit, replay bit for bit from a captured graph, and fall back to the per-step
launches where the coarsest level does not fit."""
import math

import numpy as np
import pytest

import oracle
from airg_inputs import workloads
from parity import assert_elementwise, mmatrix_inverse_inf_norm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {
    # name: (problem, solver options)
    "fv128_perm": (lambda: workloads.fv_random(128, 0.3, True), {}),
    "fv100_theta1": (lambda: workloads.fv_random(100, 1.0, True), {}),
    "dg24_perm": (lambda: workloads.dg_random(24, math.pi / 5, True), {}),
    # one level: the coarsest matrix is the whole 25,600-row matrix, 25
    # workgroups of 1024 rows
    "fv160_one_level": (lambda: workloads.fv_random(160, 0.4, True),
                        dict(max_levels=1, coarse_poly_order=8, restart=40)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_persistent_coarse_solve_matches_the_oracle_and_repeats(case):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    make, kw = CASES[case]
    p = make()
    print(f"persistent coarse solve: {case} n={p.n}", flush=True)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, oracle.Params(**kw))
    s = Solver(p.indptr, p.indices, p.data, coarse_persistent=1, **kw)
    b = torch.from_numpy(p.b).cuda()
    x, info = s.solve(b)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert_elementwise(x.cpu().numpy(), xo)
    x2, info2 = s.solve(b)
    assert info2["iterations"] == info["iterations"]
    assert torch.equal(x2, x)
    s.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_persistent_coarse_solve_in_lower_storage_precision(prec):
    # the FP32 / BF16 V-cycle with the persistent coarse solve reaches the
    # FP64 tolerance in the FP64 oracle's count, within the bound of the
    # FP64 residuals' difference
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(128, 0.3, True)
    A = p.scipy()
    xo, its, rel, levels, _ = oracle.solve(A, p.b)
    s = Solver(p.indptr, p.indices, p.data, precision=prec, coarse_persistent=1)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    xg = x.cpu().numpy()
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    bound = mmatrix_inverse_inf_norm(A, p.level) * np.abs((p.b - A @ xo) - (p.b - A @ xg)).max()
    assert np.abs(xg - xo).max() <= 1.01 * bound + 1e-14 * np.abs(xo).max()
    s.close()


def test_persistent_and_per_step_coarse_solves_agree():
    # the same hierarchy's V-cycles with either form of the coarse solve:
    # the same iteration counts, solutions equal to rounding
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(256, 0.3, True)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, coarse_persistent=0)
    s1 = Solver(p.indptr, p.indices, p.data, coarse_persistent=1)
    x0, i0 = s0.solve(b)
    x1, i1 = s1.solve(b)
    assert i0["iterations"] == i1["iterations"]
    assert float((x1 - x0).abs().max()) <= 1e-12 * float(x0.abs().max())
    s0.close()
    s1.close()


def test_persistent_coarse_solve_replays_from_a_graph():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(128, 0.6, True)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, coarse_persistent=1, graph=0)
    s1 = Solver(p.indptr, p.indices, p.data, coarse_persistent=1, graph=1)
    x0, i0 = s0.solve(b)
    for rep in range(3):
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).cumsum(0)
        torch.cuda.synchronize()
        x1, i1 = s1.solve(b)
        assert i1["iterations"] == i0["iterations"], rep
        assert torch.equal(x1, x0), rep
        del junk
    s0.close()
    s1.close()


def test_coarsest_level_too_large_falls_back_to_per_step_launches():
    # one level of 67,600 rows: more than the 16-bit columns of the
    # persistent form address, so the per-step launches run, bit for bit
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(260, 0.4, True)
    kw = dict(max_levels=1, coarse_poly_order=20, restart=40)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, coarse_persistent=0, **kw)
    s1 = Solver(p.indptr, p.indices, p.data, coarse_persistent=1, **kw)
    x0, i0 = s0.solve(b)
    x1, i1 = s1.solve(b)
    assert i0["converged"] == 1 and i1["iterations"] == i0["iterations"]
    assert torch.equal(x1, x0)
    s0.close()
    s1.close()
