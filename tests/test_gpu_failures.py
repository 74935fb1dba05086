"""Failure handling forced from the host: an allocation budget that makes
the library's device allocations fail as out-of-memory, the stagnation
check of the outer loop on a system where FGMRES(1) cannot make progress,
and a poll limit that makes the grid barriers of persistent launches give up
(the persistent coarse solve fails; the breadth-first passes of the locality
order run again with one launch per step)."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from airg_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

AIRG_ERR_NOMEM = -5
AIRG_NOT_CONVERGED = 1
AIRG_ERR_INTERNAL = -7


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _budget(lib, nbytes):
    in_use = ctypes.c_int64()
    assert lib.airg_set_alloc_budget(nbytes, ctypes.byref(in_use)) == 0
    return in_use.value


def test_allocation_budget_turns_allocations_into_nomem():
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, Solver, binding
    lib = binding.load()
    p = workloads.fv_random(64, 0.3, True)
    base = _budget(lib, 0)
    try:
        _budget(lib, base + (1 << 20))  # 1 MiB more than the library holds now
        with pytest.raises(AirgError) as e:
            Solver(p.indptr, p.indices, p.data)
        assert e.value.code == AIRG_ERR_NOMEM
        assert "budget" in str(e.value)
        assert _budget(lib, base + (1 << 20)) == base  # the failed setup released everything
        _budget(lib, 0)
        s = Solver(p.indptr, p.indices, p.data)
        held = _budget(lib, 0)
        # a multi-column solve makes its workspace on first use: past the budget
        _budget(lib, held + 1024)
        B = torch.from_numpy(workloads.rhs_batch(p, 4)).cuda()
        with pytest.raises(AirgError) as e:
            s.solve(B)
        assert e.value.code == AIRG_ERR_NOMEM
        # the handle stays usable: its single-column workspace exists already
        x, info = s.solve(torch.from_numpy(p.b).cuda())
        assert info["converged"] == 1
        _budget(lib, 0)
        X, infos = s.solve(B)
        assert all(i["converged"] == 1 for i in infos)
        s.close()
    finally:
        _budget(lib, 0)


def _cyclic(n, eps):
    # eps I plus the cyclic shift: (r, A r) = eps |r|^2 for r = e_0, so one
    # minimal-residual step with a scalar preconditioner barely moves
    rows = np.concatenate([np.arange(n), np.arange(n)])
    cols = np.concatenate([np.arange(n), (np.arange(n) - 1) % n])
    vals = np.concatenate([np.full(n, eps), np.ones(n)])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A


def test_stagnation_check_stops_a_stagnating_solve():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    A = _cyclic(64, 0.05)
    kw = dict(max_levels=1, coarse_poly_order=0, restart=1, max_it=60)
    B = np.zeros((2, 64))
    B[0, 0] = 1.0
    B[1, 5] = 1.0
    for stag in (0, 1):
        s = Solver(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data,
                   stagnation_check=stag, **kw)
        x, info = s.solve(torch.from_numpy(B[0]).cuda())
        assert info["converged"] == 0
        if stag:
            assert info["stagnated"] == 1 and info["iterations"] < 10
        else:
            assert info["stagnated"] == 0 and info["iterations"] == 60
        # one process per column: each column stops on its own
        X, infos = s.solve(torch.from_numpy(B).cuda())
        for i in infos:
            assert i["converged"] == 0 and i["stagnated"] == stag
            assert (i["iterations"] < 10) if stag else (i["iterations"] == 60)
        s.close()


def test_persistent_coarse_barrier_that_gives_up_fails_the_solve():
    # the persistent coarse solve's grid barrier waits a bounded number of
    # polls; with one poll allowed, the waits give up, every workgroup still
    # finishes, and the solve reports AIRG_ERR_INTERNAL instead of hanging;
    # with the default limit the same handle then solves as before
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, Solver, binding
    lib = binding.load()
    p = workloads.fv_random(160, 0.4, True)  # one level: 25 workgroups
    s = Solver(p.indptr, p.indices, p.data, max_levels=1, coarse_poly_order=8, restart=40,
               coarse_persistent=1)
    b = torch.from_numpy(p.b).cuda()
    x0, i0 = s.solve(b)
    assert i0["converged"] == 1
    try:
        assert lib.airg_set_spin_limit(1) == 0
        with pytest.raises(AirgError) as e:
            s.solve(b)
        assert e.value.code == AIRG_ERR_INTERNAL
        assert "barrier" in str(e.value)
    finally:
        assert lib.airg_set_spin_limit(0) == 0
    x1, i1 = s.solve(b)
    assert i1["iterations"] == i0["iterations"]
    assert torch.equal(x1, x0)
    s.close()


BFS_CASES = {
    # one connected graph: the two-distance key of one component
    "fv256_perm": lambda: [workloads.fv_random(256, 0.3, True)],
    # a flow along the grid lines: 96 components, keyed all at once
    "fv96_theta0_perm": lambda: [workloads.fv_random(96, 0.0, True, seed=301)],
    # a block-diagonal batch: every problem's passes at once
    "batch3": lambda: [workloads.fv_random(96, 0.0, True, seed=301),
                       workloads.fv_random(48, 0.5, True, seed=302),
                       workloads.fv_random(64, 0.3, True, seed=303)],
}


@pytest.mark.parametrize("case", list(BFS_CASES))
def test_breadth_first_barrier_that_gives_up_falls_back_to_per_step_launches(case):
    # the locality order's breadth-first passes run many steps per launch
    # behind a grid barrier; with one poll allowed the barrier gives up and
    # the pass runs again with one launch per step.  Breadth-first distances
    # are unique, so both give the same order: the same iteration counts and
    # bit-for-bit the same solutions
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver, Solver, binding
    lib = binding.load()
    probs = BFS_CASES[case]()
    print(f"breadth-first fallback: {case}, n = {[q.n for q in probs]}", flush=True)

    def run():
        if len(probs) == 1:
            q = probs[0]
            s = Solver(q.indptr, q.indices, q.data)
            x, info = s.solve(torch.from_numpy(q.b).cuda())
            s.close()
            return [x], [info]
        s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs])
        xs, infos = s.solve([torch.from_numpy(q.b).cuda() for q in probs])
        s.close()
        return xs, infos

    x0, i0 = run()
    try:
        assert lib.airg_set_spin_limit(1) == 0
        x1, i1 = run()
    finally:
        assert lib.airg_set_spin_limit(0) == 0
    for a, b, ia, ib in zip(x0, x1, i0, i1):
        assert ia["converged"] == 1 and ia["iterations"] == ib["iterations"]
        assert torch.equal(a, b)
