"""Batched solves through the C ABI (needs an MI355X).

Two kinds of batching: several right-hand sides of one matrix (K interleaved
columns, one FGMRES process per column over shared V-cycle launches) and
several independent problems in one block-diagonal hierarchy (one process
per problem).  Every column or problem must reach the FP64
tolerance in its own residual, checked here on the CPU, and agree with the
exact discrete solution from the oracle's sweep.
"""
import ctypes

import numpy as np
import pytest

import oracle
from airg_inputs import workloads
from parity import assert_elementwise, mmatrix_inverse_inf_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RTOL = 1e-10


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel_residual(A, x, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(b - A @ x) / nb if nb > 0 else np.linalg.norm(x)


def _check_columns(p, B, X, infos, single=None):
    A = p.scipy()
    for k in range(B.shape[0]):
        x = X[k]
        rr = _rel_residual(A, x, B[k])
        assert infos[k]["converged"] == 1, k
        assert rr <= RTOL * (1 + 1e-6), (k, rr)
        u = oracle.sweep_solve(A, B[k], p.level)
        assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u), k
        if single is not None:
            assert np.linalg.norm(x - single[k]) <= 1e-8 * np.linalg.norm(single[k]), k


def test_column_batch_matches_single_solves():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(96, 0.4, True)
    B = workloads.rhs_batch(p, 11)  # padded to 16 interleaved columns
    print(f"fv96 perm, 11 columns", flush=True)
    s = Solver(p.indptr, p.indices, p.data)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    ones = [s.solve(torch.from_numpy(B[k]).cuda()) for k in range(11)]
    single = [x.cpu().numpy() for x, _ in ones]
    _check_columns(p, B, X.cpu().numpy(), infos, single)
    # each column runs its own FGMRES: the single solve's iteration count
    assert [i["iterations"] for i in infos] == [i["iterations"] for _, i in ones]
    # the workspaces come back after a trim, with the same results
    s.trim()
    X2, _ = s.solve(torch.from_numpy(B).cuda())
    assert torch.equal(X, X2)
    s.close()


@pytest.mark.parametrize("outer", [0, 1])
def test_each_column_iterates_like_the_oracle(outer):
    # one outer process per column: every column stops at its own count, the
    # one the oracle's single-column solve from the same guess takes
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(64, 0.4, True)
    A = p.scipy()
    B = workloads.rhs_batch(p, 6)
    B[4] *= 1e3
    pr = oracle.Params(outer=("fgmres", "richardson")[outer])
    levels = oracle.setup(A, pr)
    X0 = np.zeros_like(B)
    # a guess near column 2's solution and a rough one for column 5
    u2 = oracle.sweep_solve(A, B[2], p.level)
    X0[2] = u2 * (1.0 + 1e-7 * np.cos(np.arange(p.n)))
    X0[5] = 0.5 * oracle.sweep_solve(A, B[5], p.level)
    print(f"fv64 perm, 6 columns, outer {outer}", flush=True)
    s = Solver(p.indptr, p.indices, p.data, outer=outer)
    X, infos = s.solve(torch.from_numpy(B).cuda(), x=torch.from_numpy(X0).cuda(), guess=True)
    Xh = X.cpu().numpy()
    its = []
    for k in range(B.shape[0]):
        xo, ik, rel, _, _ = oracle.solve(A, B[k], pr, levels, x0=X0[k].copy())
        its.append(ik)
        assert infos[k]["converged"] == 1, k
        assert infos[k]["iterations"] == ik, (k, infos[k]["iterations"], ik)
        assert np.linalg.norm(Xh[k] - xo) <= 1e-10 * np.linalg.norm(xo), k
        assert_elementwise(Xh[k], xo)
    assert its[2] < its[0] and len(set(its)) >= 2
    s.close()


def test_column_batch_above_64_is_chunked():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(32, 1.1, True)
    B = workloads.rhs_batch(p, 70)  # 64 columns, then 6 padded to 8
    print("fv32 perm, 70 columns", flush=True)
    s = Solver(p.indptr, p.indices, p.data)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    assert len(infos) == 70
    _check_columns(p, B, X.cpu().numpy(), infos)
    s.close()


def test_column_batch_with_a_zero_column_and_guesses():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(64, 0.9, True)
    B = workloads.rhs_batch(p, 5)
    B[2] = 0.0
    s = Solver(p.indptr, p.indices, p.data)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    Xh = X.cpu().numpy()
    assert float(np.abs(Xh[2]).max()) == 0.0 and infos[2]["converged"] == 1
    keep = [0, 1, 3, 4]
    _check_columns(p, B[keep], Xh[keep], [infos[k] for k in keep])
    # restarting every column from its converged solution needs no iteration
    X2, infos2 = s.solve(torch.from_numpy(B).cuda(), x=X.clone(), guess=True)
    assert all(i["iterations"] == 0 and i["converged"] == 1 for i in infos2)
    s.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_column_batch_mixed_precision(prec):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(128, 0.3, True)
    B = workloads.rhs_batch(p, 8)
    s = Solver(p.indptr, p.indices, p.data, precision=prec)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    _check_columns(p, B, X.cpu().numpy(), infos)
    s.close()


def _problems():
    return [workloads.fv_random(24, 0.2, True, seed=101),
            workloads.fv_random(40, 1.3, True, seed=102),
            workloads.fv_random(64, 0.7, True, seed=103),
            workloads.fv_random(33, 0.4, True, seed=104, ny=17),
            workloads.fv_random(50, 0.0, False, seed=105),
            workloads.fv_random(8, 1.0, True, seed=106)]


def test_problem_batch_solves_every_problem():
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver
    probs = _problems()
    print("batch of", [q.n for q in probs], flush=True)
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs])
    assert s.n == sum(q.n for q in probs)
    bs = [torch.from_numpy(q.b).cuda() for q in probs]
    xs, infos = s.solve(bs)
    assert len(infos) == len(probs)
    for q, x, info in zip(probs, xs, infos):
        A = q.scipy()
        xh = x.cpu().numpy()
        assert info["converged"] == 1
        assert _rel_residual(A, xh, q.b) <= RTOL * (1 + 1e-6)
        u = oracle.sweep_solve(A, q.b, q.level)
        assert np.linalg.norm(xh - u) <= 1e-8 * np.linalg.norm(u)
    # from the converged solutions no iteration is needed
    xs2, infos2 = s.solve(bs, xs=[x.clone() for x in xs], guess=True)
    assert all(i["iterations"] == 0 for i in infos2)
    s.close()


@pytest.mark.parametrize("outer", [0, 1])
def test_problem_batch_runs_one_process_per_problem(outer):
    # each problem stops at its own count: the oracle's solve of that
    # problem alone (its right-hand side embedded, zeros elsewhere) with the
    # V-cycle of the same block-diagonal hierarchy
    _needs_gpu()
    import scipy.sparse as sp
    from paper_2508_17517_amd import BatchSolver
    probs = _problems()
    A = sp.csr_matrix(sp.block_diag([q.scipy() for q in probs]))
    A.sort_indices()
    pr = oracle.Params(outer=("fgmres", "richardson")[outer])
    levels = oracle.setup(A, pr)
    seg = np.concatenate([[0], np.cumsum([q.n for q in probs])])
    its, xo = [], []
    for k, q in enumerate(probs):
        b = np.zeros(A.shape[0])
        b[seg[k]:seg[k + 1]] = q.b
        x, ik, rel, _, _ = oracle.solve(A, b, pr, levels)
        its.append(ik)
        xo.append(x[seg[k]:seg[k + 1]])
    print("batch of", [q.n for q in probs], "outer", outer, "oracle its", its, flush=True)
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs], outer=outer)
    xs, infos = s.solve([torch.from_numpy(q.b).cuda() for q in probs])
    assert [i["iterations"] for i in infos] == its
    for k, (x, i) in enumerate(zip(xs, infos)):
        assert i["converged"] == 1
        assert np.linalg.norm(x.cpu().numpy() - xo[k]) <= 1e-10 * np.linalg.norm(xo[k]), k
        assert_elementwise(x.cpu().numpy(), xo[k])
    assert len(set(its)) >= 2
    s.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_problem_batch_low_precision_with_the_assembled_smoother(prec):
    # FP32 / BF16 storage and the assembled fixed-sparsity smoother on a
    # problem batch: each problem lies within the bound the two FP64
    # residuals give, |A^-1|_inf |r_o - r_g|_inf (A^-1 >= 0 for these upwind
    # M-matrices, so |A^-1|_inf is one sweep of ones), against the FP64
    # oracle with the assembled smoother on the same block-diagonal
    # hierarchy.  FP32 (6e-8 relative perturbation of the V-cycle) takes the
    # oracle's count; BF16 (4e-3) may cross the tolerance one outer step
    # earlier or later, as it does on the smallest problem here
    _needs_gpu()
    import scipy.sparse as sp
    from paper_2508_17517_amd import BatchSolver
    probs = _problems()
    A = sp.csr_matrix(sp.block_diag([q.scipy() for q in probs]))
    A.sort_indices()
    pr = oracle.Params(smoother="assembled")
    levels = oracle.setup(A, pr)
    seg = np.concatenate([[0], np.cumsum([q.n for q in probs])])
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs], precision=prec, smoother=1)
    xs, infos = s.solve([torch.from_numpy(q.b).cuda() for q in probs])
    for k, q in enumerate(probs):
        b = np.zeros(A.shape[0])
        b[seg[k]:seg[k + 1]] = q.b
        xo, ik, rel, _, _ = oracle.solve(A, b, pr, levels)
        xo = xo[seg[k]:seg[k + 1]]
        Aq = q.scipy()
        xg = xs[k].cpu().numpy()
        assert infos[k]["converged"] == 1, k
        if prec == 1:
            assert infos[k]["iterations"] == ik, k
        else:
            assert abs(infos[k]["iterations"] - ik) <= 1, k
        assert np.linalg.norm(q.b - Aq @ xg) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(q.b), k
        bound = mmatrix_inverse_inf_norm(Aq, q.level) * np.abs((q.b - Aq @ xo) - (q.b - Aq @ xg)).max()
        assert np.abs(xg - xo).max() <= 1.01 * bound + 1e-14 * np.abs(xo).max(), k
    s.close()


def test_problem_batch_with_decoupled_lines():
    # a theta = 0 problem (one component per grid line) next to coupled ones:
    # every problem still reaches the tolerance and its exact solution
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver
    probs = [workloads.fv_random(96, 0.0, True, seed=301), workloads.fv_random(48, 0.5, True, seed=302),
             workloads.fv_random(64, 0.0, False, seed=303, ny=40)]
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs])
    xs, infos = s.solve([torch.from_numpy(q.b).cuda() for q in probs])
    for q, x, i in zip(probs, xs, infos):
        A = q.scipy()
        xh = x.cpu().numpy()
        assert i["converged"] == 1
        u = oracle.sweep_solve(A, q.b, q.level)
        assert np.linalg.norm(xh - u) <= 1e-8 * np.linalg.norm(u)
    s.close()


def test_problem_batch_of_one_matches_the_single_solver():
    # one problem: the same matrix, the same hierarchy, the same iterates
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver, Solver
    p = workloads.fv_random(80, 0.6, True)
    s1 = Solver(p.indptr, p.indices, p.data)
    sb = BatchSolver([(p.indptr, p.indices, p.data)])
    b = torch.from_numpy(p.b).cuda()
    x1, i1 = s1.solve(b)
    xb, ib = sb.solve([b])
    assert ib[0]["iterations"] == i1["iterations"]
    assert float(torch.linalg.norm(xb[0] - x1) / torch.linalg.norm(x1)) <= 1e-12
    s1.close()
    sb.close()


def test_batch_argument_errors():
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, BatchSolver, Solver, binding
    probs = _problems()[:2]
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs])
    lib = binding.load()
    B = torch.zeros(2, s.n, dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    infos = (binding.SolveInfo * 2)()
    code = lib.airg_solve(s.h, 2, ctypes.c_void_p(B.data_ptr()), s.n,
                          ctypes.c_void_p(X.data_ptr()), s.n, 0, infos)
    assert code == -1
    # a batch handle takes its problems through airg_solve_batch only
    code = lib.airg_solve(s.h, 1, ctypes.c_void_p(B.data_ptr()), s.n,
                          ctypes.c_void_p(X.data_ptr()), s.n, 0, infos)
    assert code == -1
    code = lib.airg_adjoint_solve(s.h, 1, ctypes.c_void_p(B.data_ptr()), s.n,
                                  ctypes.c_void_p(X.data_ptr()), s.n, 0, infos)
    assert code == -1
    q = probs[0]
    single = Solver(q.indptr, q.indices, q.data)
    vp = ctypes.c_void_p * 1
    b = torch.from_numpy(q.b).cuda()
    x = torch.zeros_like(b)
    code = lib.airg_solve_batch(single.h, vp(b.data_ptr()), vp(x.data_ptr()), 0, infos)
    assert code == -1
    with pytest.raises(ValueError):
        s.solve([b])
    bad = q.data.copy()
    bad[0] = np.nan
    with pytest.raises(AirgError):
        BatchSolver([(q.indptr, q.indices, q.data), (q.indptr, q.indices, bad)])
    s.close()
    single.close()


def test_autotuned_shapes_keep_the_solution_and_can_be_pinned():
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, Solver
    p = workloads.fv_random(128, 0.5, True)
    s = Solver(p.indptr, p.indices, p.data)
    b = torch.from_numpy(p.b).cuda()
    x0, i0 = s.solve(b)
    tuned = s.autotune(reps=3)
    st = s.stats()
    assert len(tuned) == 3 * (st["levels"] - 1) + 2
    assert all(t["lanes"] in (0, 1, 2, 4, 8, 16, 32, 64) for t in tuned)
    assert all(t["xcd_map"] in (0, 1) for t in tuned)
    assert all(t["best_us"] <= t["default_us"] for t in tuned)
    x1, i1 = s.solve(b)
    # tuned shapes sum rows in another order: the same iterations, the
    # solution to rounding
    assert i1["converged"] == 1 and i1["iterations"] == i0["iterations"]
    assert float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)) <= 1e-10
    assert_elementwise(x1.cpu().numpy(), x0.cpu().numpy())
    # pinned shapes give bit-identical solves
    for t in tuned:
        s.set_lanes(t["level"], t["op"], 64 if t["op"] == "a" else 1, t["xcd_map"])
    x2, _ = s.solve(b)
    x3, _ = s.solve(b)
    assert torch.equal(x2, x3)
    # the LDS-staged product sums like the row kernel with the same lanes
    staged = 0
    for t in tuned:
        s.set_lanes(t["level"], t["op"], 4)
    x4, _ = s.solve(b)
    for t in tuned:
        try:
            s.set_lanes(t["level"], t["op"], 4, 1, 1)
            staged += 1
        except AirgError:
            pass
    assert staged >= 1
    x5, _ = s.solve(b)
    assert torch.equal(x4, x5)
    with pytest.raises(AirgError):
        s.set_lanes(0, "ff", 3)
    s.close()


def test_masked_row_block_and_staged_kernels_on_a_problem_batch():
    # problems that stop at different counts switch the V-cycle's products to
    # their masked versions (rows of stopped problems skipped); pinned to the
    # row-block kernel or to LDS staging, those versions must sum like the
    # one-lane and the row kernels with the same lanes, bit for bit, and
    # every problem must keep the oracle's iteration count
    _needs_gpu()
    import scipy.sparse as sp
    from paper_2508_17517_amd import AirgError, BatchSolver
    probs = _problems()
    A = sp.csr_matrix(sp.block_diag([q.scipy() for q in probs]))
    A.sort_indices()
    pr = oracle.Params()
    levels = oracle.setup(A, pr)
    seg = np.concatenate([[0], np.cumsum([q.n for q in probs])])
    its = []
    for k, q in enumerate(probs):
        b = np.zeros(A.shape[0])
        b[seg[k]:seg[k + 1]] = q.b
        its.append(oracle.solve(A, b, pr, levels)[1])
    assert len(set(its)) >= 2
    s = BatchSolver([(q.indptr, q.indices, q.data) for q in probs])
    bs = [torch.from_numpy(q.b).cuda() for q in probs]
    ops = [(e["level"], e["op"]) for e in s.autotune(reps=1)]

    def run(lanes, xcd, lds, fallback_lanes=None):
        switched = 0
        for l, op in ops:
            try:
                s.set_lanes(l, op, lanes, xcd, lds)
                switched += 1
            except AirgError:
                s.set_lanes(l, op, fallback_lanes if fallback_lanes is not None else lanes, xcd, 0)
        xs, infos = s.solve(bs)
        assert [i["iterations"] for i in infos] == its
        return [x.clone() for x in xs], switched

    x1, _ = run(1, 0, 0)
    x0, nrb = run(0, 1, 0, fallback_lanes=1)
    assert nrb >= 1, "no operator took the row-block kernel"
    for a, b in zip(x0, x1):
        assert torch.equal(a, b)
    x4, _ = run(4, 1, 0)
    x4s, nlds = run(4, 1, 1)
    assert nlds >= 1, "no operator took the LDS-staged kernel"
    for a, b in zip(x4s, x4):
        assert torch.equal(a, b)
    # the entry-staged kernel sums like the one-lane kernel
    xe, ne = run(1, 1, 2)
    assert ne == len(ops)
    for a, b in zip(xe, x1):
        assert torch.equal(a, b)
    s.close()


def test_row_block_kernel_sums_like_one_lane_per_row():
    # the row-block product adds each row's products in the one-lane order,
    # so pinning it instead of one lane per row changes no bit of the solve
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, Solver
    p = workloads.dg_random(48, 0.4, True)
    s = Solver(p.indptr, p.indices, p.data)
    st = s.stats()
    ops = [(l, op) for l in range(st["levels"] - 1) for op in ("ff", "b", "z")]
    ops += [(st["levels"] - 1, "a"), (0, "top")]
    for l, op in ops:
        s.set_lanes(l, op, 1)
    b = torch.from_numpy(p.b).cuda()
    x1, i1 = s.solve(b)
    switched = 0
    for l, op in ops:
        try:
            s.set_lanes(l, op, 0, 1)
            switched += 1
        except AirgError:
            pass
    assert switched >= 1
    x0, i0 = s.solve(b)
    assert i0["iterations"] == i1["iterations"]
    assert torch.equal(x0, x1)
    s.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_entry_staged_kernel_sums_like_one_lane_per_row(prec):
    # the entry-staged product (256 rows per workgroup, entries loaded at
    # consecutive addresses, products in LDS) adds each row's products in the
    # one-lane order: pinning it on every operator changes no bit of the solve
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(150, 0.4, True, ny=97)
    b = torch.from_numpy(p.b).cuda()
    s = Solver(p.indptr, p.indices, p.data, precision=prec)
    ops = [(e["level"], e["op"]) for e in s.autotune(reps=1)]
    for l, op in ops:
        s.set_lanes(l, op, 1, 0, 0)
    x1, i1 = s.solve(b)
    for l, op in ops:
        s.set_lanes(l, op, 1, 1, 2)
    x2, i2 = s.solve(b)
    assert i2["iterations"] == i1["iterations"]
    assert torch.equal(x1, x2)
    s.close()


@pytest.mark.parametrize("opts", [
    dict(precision=1, smoother=1),
    dict(precision=2, inverse_type=1),
    dict(outer=1, smoother=1, inverse_type=1),
    dict(outer=1, precision=1),
])
def test_option_combinations_on_column_batches(opts):
    # every combination of storage precision, smoother, polynomial and outer
    # loop reaches the FP64 tolerance on each of several columns
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(64, 0.7, True)
    B = workloads.rhs_batch(p, 3)
    print("options", opts, flush=True)
    s = Solver(p.indptr, p.indices, p.data, **opts)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    _check_columns(p, B, X.cpu().numpy(), infos)
    s.close()


def test_long_arnoldi_cycles_in_column_and_problem_batches():
    # a weak preconditioner (one level, degree-3 Newton polynomial) and
    # restart 40: every process's Arnoldi cycle passes 32 basis vectors,
    # where the fused per-column and per-problem Gram-Schmidt sweeps give
    # way to the separate ones, and then restarts
    _needs_gpu()
    import scipy.sparse as sp
    from paper_2508_17517_amd import BatchSolver, Solver
    kw = dict(max_levels=1, coarse_poly_order=3, restart=40)
    pr = oracle.Params(**kw)
    p = workloads.fv_random(64, 0.4, True)
    A = p.scipy()
    B = workloads.rhs_batch(p, 2)
    print("fv64 perm, 2 columns, restart 40", flush=True)
    s = Solver(p.indptr, p.indices, p.data, **kw)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    Xh = X.cpu().numpy()
    levels = oracle.setup(A, pr)
    for k in range(2):
        xo, ik, rel, _, _ = oracle.solve(A, B[k], pr, levels)
        assert ik > 40
        assert infos[k]["converged"] == 1 and infos[k]["restarts"] >= 1, k
        assert infos[k]["iterations"] == ik, (k, infos[k]["iterations"], ik)
        assert np.linalg.norm(Xh[k] - xo) <= 1e-10 * np.linalg.norm(xo), k
        assert_elementwise(Xh[k], xo)
    s.close()
    probs = [workloads.fv_random(48, 0.4, True, seed=311), workloads.fv_random(64, 0.9, True, seed=312)]
    Ab = sp.csr_matrix(sp.block_diag([q.scipy() for q in probs]))
    Ab.sort_indices()
    levels = oracle.setup(Ab, pr)
    seg = np.concatenate([[0], np.cumsum([q.n for q in probs])])
    print("batch of", [q.n for q in probs], "restart 40", flush=True)
    sb = BatchSolver([(q.indptr, q.indices, q.data) for q in probs], **kw)
    xs, infos = sb.solve([torch.from_numpy(q.b).cuda() for q in probs])
    for k, q in enumerate(probs):
        b = np.zeros(Ab.shape[0])
        b[seg[k]:seg[k + 1]] = q.b
        xo, ik, rel, _, _ = oracle.solve(Ab, b, pr, levels)
        xo = xo[seg[k]:seg[k + 1]]
        assert ik > 32
        assert infos[k]["converged"] == 1, k
        assert infos[k]["restarts"] >= (1 if ik > 41 else 0), k
        assert infos[k]["iterations"] == ik, (k, infos[k]["iterations"], ik)
        assert np.linalg.norm(xs[k].cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo), k
        assert_elementwise(xs[k].cpu().numpy(), xo)
    sb.close()
