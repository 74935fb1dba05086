"""V-cycles replayed from captured HIP graphs (params.graph = 1).

A captured V-cycle holds exactly the launches of the direct path (the same
kernels, launch shapes and arguments), so every solve must give the same
iteration counts and the same bits as launching the kernels one by one: for
single solves in FP64 and lower storage precision, with C-point smoothing,
for column and problem batches (whose activity masks switch the masked
products on), over several replays with other GPU work in between, and after
launch shapes change.  Also the outer loop's absolute tolerance against the
oracle's."""
import math

import numpy as np
import pytest

import oracle
from airg_inputs import workloads
from parity import assert_elementwise

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = {
    "fv128_fp64": (lambda: workloads.fv_random(128, 0.3, True), {}),
    "fv96_fp32_assembled": (lambda: workloads.fv_random(96, 0.8, True), dict(precision=1, smoother=1)),
    "dg24_bf16": (lambda: workloads.dg_random(24, math.pi / 5, True), dict(precision=2)),
    "fv64_fcf": (lambda: workloads.fv_random(64, 1.1, True), dict(smooth_type=2)),
    "fv64_richardson_nair": (lambda: workloads.fv_random(64, 0.5, True), dict(outer=1, inverse_type=1)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_graph_replay_is_bitwise_the_direct_launches(case):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    make, kw = CASES[case]
    p = make()
    print(f"graph replay: {case} n={p.n}", flush=True)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, graph=0, **kw)
    s1 = Solver(p.indptr, p.indices, p.data, graph=1, **kw)
    x0, i0 = s0.solve(b)
    assert i0["converged"] == 1
    for rep in range(3):
        # eager work and a synchronisation between the replays
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).cumsum(0)
        torch.cuda.synchronize()
        x1, i1 = s1.solve(b)
        assert i1["iterations"] == i0["iterations"], rep
        assert torch.equal(x1, x0), rep
        del junk
    s0.close()
    s1.close()


def test_graph_replay_on_column_and_problem_batches():
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver, Solver
    p = workloads.fv_random(64, 0.6, True)
    B = torch.from_numpy(workloads.rhs_batch(p, 4)).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, graph=0, precision=1)
    s1 = Solver(p.indptr, p.indices, p.data, graph=1, precision=1)
    X0, inf0 = s0.solve(B)
    for rep in range(2):
        X1, inf1 = s1.solve(B)
        assert [i["iterations"] for i in inf1] == [i["iterations"] for i in inf0]
        assert torch.equal(X1, X0)
    s0.close()
    s1.close()
    probs = [workloads.fv_random(24, 0.2, True, seed=101), workloads.fv_random(40, 1.3, True, seed=102),
             workloads.fv_random(64, 0.7, True, seed=103), workloads.fv_random(8, 1.0, True, seed=106)]
    mats = [(q.indptr, q.indices, q.data) for q in probs]
    bs = [torch.from_numpy(q.b).cuda() for q in probs]
    b0 = BatchSolver(mats, graph=0)
    b1 = BatchSolver(mats, graph=1)
    xs0, infos0 = b0.solve(bs)
    its = [i["iterations"] for i in infos0]
    assert len(set(its)) >= 2  # problems stop at different counts: the masks switch on
    for rep in range(2):
        xs1, infos1 = b1.solve(bs)
        assert [i["iterations"] for i in infos1] == its
        for a, c in zip(xs1, xs0):
            assert torch.equal(a, c)
    b0.close()
    b1.close()


def test_graph_follows_launch_shape_changes():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(96, 0.4, True)
    b = torch.from_numpy(p.b).cuda()
    s0 = Solver(p.indptr, p.indices, p.data, graph=0)
    s1 = Solver(p.indptr, p.indices, p.data, graph=1)
    s1.solve(b)  # captures with the default shapes
    for s in (s0, s1):
        s.set_lanes(0, "ff", 4, 1)
        s.set_lanes(0, "top", 2, 0)
    x0, i0 = s0.solve(b)
    x1, i1 = s1.solve(b)
    assert i1["iterations"] == i0["iterations"] and torch.equal(x1, x0)
    tuned = s1.autotune(reps=2)
    s0.pin_shapes(tuned)
    s1.pin_shapes(tuned)
    x0, i0 = s0.solve(b)
    x1, i1 = s1.solve(b)
    assert i1["iterations"] == i0["iterations"] and torch.equal(x1, x0)
    s0.close()
    s1.close()


def test_absolute_tolerance_matches_the_oracle():
    # with rtol negligible, atol = c |b| stops FGMRES where the oracle stops
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(64, 0.3, True)
    A = p.scipy()
    atol = 1e-7 * np.linalg.norm(p.b)
    prm = oracle.Params(rtol=1e-300, atol=atol)
    xo, its, rel, _, _ = oracle.solve(A, p.b, prm)
    s = Solver(p.indptr, p.indices, p.data, rtol=1e-300, atol=atol)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["iterations"] == its
    assert info["converged"] == 1
    assert np.linalg.norm(p.b - A @ x.cpu().numpy()) <= atol * (1 + 1e-6)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()
