"""The outer FGMRES's look-ahead (params.lookahead = 1): Arnoldi step j + 1 is
queued on the device before the host reads step j's coefficients, its basis
vector divided by the device's own square root of |w|^2.  The host's and the
device's square roots are both correctly rounded, so a solve with the
look-ahead gives the same iteration counts and the same bits as one without,
in FP64 and with FP32 / BF16 storage, across restarts and past the fused
sweeps' 32 basis vectors, from zero and from a guess."""
import math

import pytest

from airg_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {
    "fv128_fp64": (lambda: workloads.fv_random(128, 0.3, True), {}),
    "fv96_fp32": (lambda: workloads.fv_random(96, 0.8, True), dict(precision=1)),
    "dg24_bf16": (lambda: workloads.dg_random(24, math.pi / 5, True), dict(precision=2)),
    # a weak preconditioner: 40-step cycles, restarts, separate sweeps past 32
    "fv64_restarts": (lambda: workloads.fv_random(64, 0.4, True),
                      dict(max_levels=1, coarse_poly_order=3, restart=40)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_lookahead_gives_the_same_bits(case):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    make, kw = CASES[case]
    p = make()
    print(f"look-ahead: {case} n={p.n}", flush=True)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, lookahead=0, **kw)
    s1 = Solver(p.indptr, p.indices, p.data, lookahead=1, **kw)
    x0, i0 = s0.solve(b)
    x1, i1 = s1.solve(b)
    assert i0["converged"] == 1
    assert i1["iterations"] == i0["iterations"] and i1["restarts"] == i0["restarts"]
    assert i1["rel_residual"] == i0["rel_residual"]
    assert torch.equal(x1, x0)
    # from a guess (half the solution): a shorter solve, the same bits
    g0, j0 = s0.solve(b, x=0.5 * x0, guess=True)
    g1, j1 = s1.solve(b, x=0.5 * x0, guess=True)
    assert j1["iterations"] == j0["iterations"]
    assert torch.equal(g1, g0)
    s0.close()
    s1.close()
