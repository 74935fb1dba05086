"""GPU path vs the CPU oracle, through the C ABI (needs an MI355X).

The setup follows the same summation orders as the oracle, so every discrete
decision (CF split, prolongator, drops) and every assembled operator is
compared bit for bit level by level; the Newton roots come from different
eigenvalue codes and are compared to a tolerance.  Solutions must agree with
the oracle's to a relative 1e-10 with the same FGMRES iteration count.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from airg_inputs import workloads, fv_advection, fd_advection
from parity import assert_elementwise, mmatrix_inverse_inf_norm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(p, **kw):
    from paper_2508_17517_amd import Solver
    return Solver(p.indptr, p.indices, p.data, **kw)


CASES = {
    "fv64": lambda: workloads.fv64(),
    "fv48_perm": lambda: workloads.fv_random(48, 0.3, True),
    "fv128_perm": lambda: workloads.fv_random(128, 0.3, True),
    "fv100_theta1": lambda: workloads.fv_random(100, 1.0, True),
    "fv80x40_rect": lambda: workloads.fv_random(80, 0.7, True, ny=40),
    "dg24_perm": lambda: workloads.dg_random(24, math.pi / 5, True),
    "fd48_paper_g05": lambda: fd_advection(48, math.pi / 4, 0.5),
    "dg20x12_rect": lambda: workloads.dg_random(20, 1.2, True, ny=12),
}


def _csr_equal(name, got, want, l):
    rp, col, val = got
    want = sp.csr_matrix(want)
    want.sort_indices()
    assert np.array_equal(rp, want.indptr), f"level {l} {name}: row pointers differ"
    assert np.array_equal(col, want.indices), f"level {l} {name}: columns differ"
    if not np.array_equal(val, want.data):
        d = np.abs(val - want.data).max() / np.abs(want.data).max()
        raise AssertionError(f"level {l} {name}: values differ (max rel {d:.3e})")


def compare_hierarchy(s, levels):
    st = s.stats()
    assert st["levels"] == len(levels), (st["levels"], len(levels))
    for l, L in enumerate(levels):
        g = s.export_level(l)
        assert g["n"] == L.A.shape[0]
        if l > 0 or L.coarsest:
            _csr_equal("A", g["a"], L.A, l)
        if L.coarsest:
            assert g["is_coarsest"]
            want = np.array(L.roots)
            got = g["roots"]
            assert len(got) == len(want), f"coarsest: {len(got)} roots vs {len(want)}"
            assert np.allclose(np.sort_complex(got), np.sort_complex(want), rtol=1e-9, atol=1e-12)
            continue
        assert np.array_equal(g["state"], L.state), f"level {l}: CF split differs"
        _csr_equal("A_ff", g["ff"], L.Aff, l)
        _csr_equal("A_fc", g["fc"], L.Afc, l)
        assert np.array_equal(g["alpha"], L.alpha), f"level {l}: smoother coefficients differ"
        _csr_equal("Z", g["z"], L.Z, l)
        assert np.array_equal(g["cmap"], L.cmap), f"level {l}: prolongator differs"
        if L.trunc_rel is not None:
            assert st["trunc_rel"][l] == pytest.approx(L.trunc_rel, rel=1e-8)


@pytest.mark.parametrize("case", list(CASES))
def test_hierarchy_is_the_oracles_level_by_level(case):
    _needs_gpu()
    p = CASES[case]()
    print(f"case {case} n={p.n}", flush=True)
    levels = oracle.setup(p.scipy())
    s = _solver(p, keep_setup_data=1)
    compare_hierarchy(s, levels)
    s.close()


@pytest.mark.parametrize("case", list(CASES))
def test_solve_matches_oracle(case):
    _needs_gpu()
    p = CASES[case]()
    print(f"case {case} n={p.n}", flush=True)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b)
    s = _solver(p)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    xg = x.cpu().numpy()
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(xg, xo)
    # against the exact discrete solution too
    u = oracle.sweep_solve(p.scipy(), p.b, p.level)
    assert np.linalg.norm(xg - u) <= 1e-8 * np.linalg.norm(u)
    s.close()


def test_imported_oracle_hierarchy_solves_like_the_oracle():
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(96, 0.3, True)
    A = p.scipy()
    xo, its, rel, levels, _ = oracle.solve(A, p.b)

    def trip(M):
        M = sp.csr_matrix(M)
        M.sort_indices()
        return (M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)

    lv = []
    for l, L in enumerate(levels):
        d = {}
        if l == 0 or L.coarsest:
            d["a"] = trip(L.A)
        if L.coarsest:
            d["roots"] = np.array(L.roots)
        else:
            d.update(state=L.state, ff=trip(L.Aff), fc=trip(L.Afc), z=trip(L.Z),
                     cmap=L.cmap.astype(np.int32), alpha=L.alpha)
        lv.append(d)
    s = Solver.from_hierarchy(lv)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


def test_import_rejects_out_of_range_indices():
    _needs_gpu()
    from paper_2508_17517_amd import Solver, AirgError
    p = workloads.fv_random(32, 0.3, True)
    levels = oracle.setup(p.scipy())
    L0, Lc = levels[0], levels[-1]
    if len(levels) < 2:
        pytest.skip("single level")
    trip = lambda M: (M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)
    cm = L0.cmap.astype(np.int32).copy()
    cm[0] = 10 ** 6
    lv = [dict(a=trip(L0.A), state=L0.state, ff=trip(L0.Aff), fc=trip(L0.Afc), z=trip(L0.Z),
               cmap=cm, alpha=L0.alpha)]
    lv.append(dict(a=trip(levels[1].A), roots=np.array(levels[1].roots if levels[1].coarsest
                                                         else oracle.hierarchy.newton_for_level(
                                                             levels[1].A, 1, oracle.Params()))))
    with pytest.raises(AirgError):
        Solver.from_hierarchy(lv)


def test_adjoint_solve_matches_oracle_and_sweep():
    _needs_gpu()
    p = workloads.fv_random(64, 0.3, True)
    A = p.scipy()
    w = np.random.default_rng(3).standard_normal(p.n)
    lo, its, rel, _, _ = oracle.adjoint_solve(A, w)
    s = _solver(p)
    lam, info = s.adjoint_solve(torch.from_numpy(w).cuda())
    lg = lam.cpu().numpy()
    assert info["converged"] == 1 and info["iterations"] == its
    assert np.linalg.norm(lg - lo) <= 1e-10 * np.linalg.norm(lo)
    assert_elementwise(lg, lo, what="adjoint solution")
    ls = oracle.sweep_solve(A, w, p.level, transpose=True)
    assert np.linalg.norm(lg - ls) <= 1e-8 * np.linalg.norm(ls)
    s.close()


def test_several_right_hand_sides_and_initial_guess():
    _needs_gpu()
    p = workloads.fv_random(64, 0.5, True)
    B = workloads.rhs_batch(p, 3)
    s = _solver(p)
    X, infos = s.solve(torch.from_numpy(B).cuda())
    for k in range(3):
        u = oracle.sweep_solve(p.scipy(), B[k], p.level)
        assert infos[k]["converged"] == 1
        assert np.linalg.norm(X[k].cpu().numpy() - u) <= 1e-8 * np.linalg.norm(u)
    # restarting from the converged solution needs no iteration
    x2, info2 = s.solve(torch.from_numpy(B[0]).cuda(), x=X[0].clone(), guess=True)
    assert info2["iterations"] == 0 and info2["converged"] == 1
    # a zero right-hand side gives zero
    xz, infz = s.solve(torch.zeros(p.n, dtype=torch.float64, device="cuda"))
    assert infz["iterations"] == 0 and float(xz.abs().max()) == 0.0
    s.close()


def test_setup_is_deterministic_run_to_run():
    _needs_gpu()
    p = workloads.fv_random(128, 1.2, True)
    s1 = _solver(p, keep_setup_data=1)
    s2 = _solver(p, keep_setup_data=1)
    st1, st2 = s1.stats(), s2.stats()
    assert st1["levels"] == st2["levels"]
    for l in range(st1["levels"]):
        a, b = s1.export_level(l), s2.export_level(l)
        for k in a:
            if isinstance(a[k], tuple):
                for u, v in zip(a[k], b[k]):
                    assert np.array_equal(u, v)
            elif isinstance(a[k], np.ndarray):
                assert np.array_equal(a[k], b[k])
    x1, i1 = s1.solve(torch.from_numpy(p.b).cuda())
    x2, i2 = s2.solve(torch.from_numpy(p.b).cuda())
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x2)
    s1.close()
    s2.close()


def test_error_codes():
    _needs_gpu()
    from paper_2508_17517_amd import Solver, AirgError
    p = workloads.fv_random(16, 0.3, False)
    bad = p.data.copy()
    bad[p.indptr[5] + 0] = np.nan
    with pytest.raises(AirgError) as e:
        Solver(p.indptr, p.indices, bad)
    assert e.value.code == -3
    # zero diagonal: the last entry of each FV row is its diagonal
    z = p.data.copy()
    z[p.indptr[8] - 1] = 0.0
    with pytest.raises(AirgError) as e:
        Solver(p.indptr, p.indices, z)
    assert e.value.code == -2
    # unsorted columns
    ix = p.indices.copy()
    r = 20
    a, b = p.indptr[r], p.indptr[r + 1]
    ix[a:b] = ix[a:b][::-1].copy()
    with pytest.raises(AirgError) as e:
        Solver(p.indptr, ix, p.data)
    assert e.value.code == -1
    # a parameter out of range
    with pytest.raises(AirgError) as e:
        Solver(p.indptr, p.indices, p.data, strong_threshold=1.5)
    assert e.value.code == -1
    # non-finite right-hand side
    s = Solver(p.indptr, p.indices, p.data)
    bb = torch.from_numpy(p.b).cuda()
    bb[3] = float("inf")
    with pytest.raises(AirgError) as e:
        s.solve(bb)
    assert e.value.code == -3
    # an iteration cap that cannot be met reports not-converged with the iterate
    s2 = Solver(p.indptr, p.indices, p.data, max_it=1)
    x, info = s2.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 0 and info["iterations"] == 1
    s.close()
    s2.close()


def test_stats_are_consistent():
    _needs_gpu()
    p = workloads.fv_random(128, 0.3, True)
    s = _solver(p)
    st = s.stats()
    levels = oracle.setup(p.scipy())
    assert st["n"] == [L.A.shape[0] for L in levels]
    assert st["nnz"] == [L.A.nnz for L in levels]
    assert st["grid_complexity"] == pytest.approx(sum(L.A.shape[0] for L in levels) / p.n)
    assert st["cycle_complexity"] > 1 and st["storage_complexity"] > 1
    assert st["coarse_roots"] == len(levels[-1].roots)
    s.close()


@pytest.mark.parametrize("theta", [0.0, 0.5 * math.pi])
def test_grid_aligned_flow(theta):
    # grid-aligned directions decouple into 1D lines (paper Sec. 3.4)
    _needs_gpu()
    gw, gs = workloads.inflow_values(1, 40)
    p = fv_advection(40, theta, gw, gs, perm_seed=9)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b)
    s = _solver(p)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


MIXED_CASES = {
    "fv128_fp32": (lambda: workloads.fv_random(128, 0.3, True), 1),
    "fv128_bf16": (lambda: workloads.fv_random(128, 0.3, True), 2),
    "dg32_fp32": (lambda: workloads.dg_random(32, math.pi / 5, True), 1),
    "dg32_bf16": (lambda: workloads.dg_random(32, math.pi / 5, True), 2),
}


@pytest.mark.parametrize("case", list(MIXED_CASES))
def test_mixed_precision_reaches_the_fp64_tolerance(case):
    # FP32 / BF16 storage in the V-cycle, FP64 outer FGMRES (iterative
    # refinement): the true FP64 residual reaches 1e-10 and the solution
    # agrees with the FP64 oracle's within the bound the two residuals give.
    # Both satisfy A x = b - r, so x_g - x_o = A^{-1}(r_o - r_g) and
    # |x_g - x_o|_inf <= |A^{-1}|_inf |r_o - r_g|_inf.  |A^{-1}|_inf is one
    # sweep away for the FV system (a triangular M-matrix: A^{-1} >= 0, so it
    # is max(A^{-1} 1)) and comes from the dense inverse for the small DG
    # system.  The perturbation of the V-cycle (FP32 rounding 6e-8, BF16
    # 4e-3 relative) leaves the iteration count of these cases equal to the
    # FP64 oracle's.
    _needs_gpu()
    make, prec = MIXED_CASES[case]
    p = make()
    A = p.scipy()
    xo, its, rel, _, _ = oracle.solve(A, p.b)
    s = _solver(p, precision=prec)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    xg = x.cpu().numpy()
    rg = p.b - A @ xg
    ro = p.b - A @ xo
    if case.startswith("fv"):
        ainv = mmatrix_inverse_inf_norm(A, p.level)
    else:
        ainv = float(np.abs(np.linalg.inv(A.toarray())).sum(axis=1).max())
    bound = ainv * np.abs(ro - rg).max()
    err = np.abs(xg - xo).max()
    print(f"{case}: iterations {info['iterations']} (fp64 oracle {its}), max |x - x_oracle| "
          f"{err:.2e}, bound {bound:.2e} (|A^-1|_inf {ainv:.1f}), relative to max |x| "
          f"{err / np.abs(xo).max():.2e}")
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert np.linalg.norm(rg) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(p.b)
    assert info["iterations"] == its
    # the bound, with room for the rounding of the residuals computed here
    assert err <= 1.01 * bound + 1e-14 * np.abs(xo).max()
    s.close()


def test_locality_order_changes_only_the_summation_order():
    # the F points of every level are re-ordered for the solve; the hierarchy
    # (exported in setup numbering) and the iteration count stay the same
    _needs_gpu()
    p = workloads.fv_random(128, 0.8, True)
    s0 = _solver(p, locality_order=0, keep_setup_data=1)
    s1 = _solver(p, locality_order=1, keep_setup_data=1)
    for l in range(s0.stats()["levels"] - 1):
        a, b = s0.export_level(l), s1.export_level(l)
        assert np.array_equal(a["state"], b["state"])
        for k in ("ff", "fc", "z"):
            for u, v in zip(a[k], b[k]):
                assert np.array_equal(u, v), (l, k)
    bt = torch.from_numpy(p.b).cuda()
    x0, i0 = s0.solve(bt)
    x1, i1 = s1.solve(bt)
    assert i0["iterations"] == i1["iterations"]
    assert float(torch.linalg.norm(x0 - x1) / torch.linalg.norm(x0)) <= 1e-11
    s0.close()
    s1.close()


PAPER_OPTS = dict(poly_order=6, coarse_poly_order=10, trunc_tol=0.1)


@pytest.mark.parametrize("case", ["fd64_paper", "fv64_perm"])
def test_richardson_matches_oracle(case):
    # the paper's outer loop: undamped Richardson from x0 = 1 (Sec. 3)
    _needs_gpu()
    if case == "fd64_paper":
        p = fd_advection(64, math.pi / 4, 0.0)
    else:
        p = workloads.fv_random(64, 0.8, True)
    print(f"case {case} n={p.n}", flush=True)
    prm = oracle.Params(outer="richardson", **PAPER_OPTS)
    x0 = np.ones(p.n)
    xo, its, rel, levels, hist = oracle.solve(p.scipy(), p.b, prm, x0=x0)
    s = _solver(p, outer=1, **PAPER_OPTS)
    x = torch.ones(p.n, dtype=torch.float64, device="cuda")
    x, info = s.solve(torch.from_numpy(p.b).cuda(), x=x, guess=True)
    xg = x.cpu().numpy()
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert abs(info["rel_residual"] - rel) <= 1e-3 * rel + 1e-16
    scale = max(np.linalg.norm(xo), np.linalg.norm(x0))
    assert np.linalg.norm(xg - xo) <= 1e-10 * scale
    # g = 0: the solution is zero, so the error is measured against x0's scale
    assert np.abs(xg - xo).max() <= 1e-10 * max(np.abs(xo).max(), 1.0)
    s.close()


@pytest.mark.parametrize("case", ["fv96_perm", "dg20_perm"])
def test_assembled_smoother_matches_oracle(case):
    # F-point smoothing with the assembled fixed-sparsity Ahat^{-1} (Sec. 2.2)
    _needs_gpu()
    p = workloads.fv_random(96, 0.3, True) if case == "fv96_perm" else \
        workloads.dg_random(20, math.pi / 5, True)
    print(f"case {case} n={p.n}", flush=True)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, oracle.Params(smoother="assembled"))
    s = _solver(p, smoother=1)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


def _permuted_chain(n, seed):
    r = np.random.default_rng(seed)
    B = sp.diags([np.full(n, 2.0), np.full(n - 1, -1.0)], [0, -1]).tocsr()
    q = r.permutation(n)
    P = sp.csr_matrix((np.ones(n), (np.arange(n), q)), shape=(n, n))
    return sp.csr_matrix(P @ B @ P.T), r.uniform(size=n)


DEGENERATE = {
    "1x1": lambda: (sp.csr_matrix(np.array([[2.0]])), np.array([4.0])),
    "2x2_lower": lambda: (sp.csr_matrix(np.array([[2.0, 0.0], [-1.0, 3.0]])), np.array([1.0, 2.0])),
    "diagonal_100": lambda: (sp.diags(np.arange(1.0, 101.0)).tocsr(), np.ones(100)),
    "bidiagonal_300": lambda: (sp.csr_matrix(sp.diags([np.full(300, 2.0), np.full(299, -1.0)],
                                                       [0, -1])), np.ones(300)),
    # permuted chains whose breadth-first distances pass 2^15: the locality
    # key falls back from the Hilbert index to d1 (max d2 + 1) + d2 (40,000:
    # d1 < 40,000, d2 < 20,001) and to d1 alone (70,000, where that product
    # passes 2^31)
    "chain_40000_perm": lambda: _permuted_chain(40000, 5),
    "chain_70000_perm": lambda: _permuted_chain(70000, 6),
}


@pytest.mark.parametrize("case", list(DEGENERATE))
def test_degenerate_systems_match_oracle(case):
    # single-level hierarchies, no off-diagonal entries, a 1D chain (cyclic
    # reduction, Sec. 2): the same iteration count and solution as the oracle
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    A, b = DEGENERATE[case]()
    A = sp.csr_matrix(A)
    A.sort_indices()
    print(f"case {case} n={A.shape[0]}", flush=True)
    xo, its, rel, levels, _ = oracle.solve(A, b)
    s = Solver(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    assert s.stats()["levels"] == len(levels)
    x, info = s.solve(torch.from_numpy(b).cuda())
    assert info["converged"] == 1 and info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * max(np.linalg.norm(xo), 1.0)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


@pytest.mark.parametrize("smoother", [0, 1])
def test_nair_matches_oracle(smoother):
    # nAIR: Neumann polynomials in the smoother and in Ahat^{-1} (Sec. 3.3)
    _needs_gpu()
    p = workloads.fv_random(96, 0.3, True)
    prm = oracle.Params(inverse_type="neumann", smoother="assembled" if smoother else "poly")
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, prm)
    s = _solver(p, inverse_type=1, smoother=smoother, keep_setup_data=1)
    compare_hierarchy(s, levels)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


C_SMOOTH = {
    "fc_poly_fv96": (lambda: workloads.fv_random(96, 0.3, True), "fc", "poly", 0),
    "fcf_poly_fv96": (lambda: workloads.fv_random(96, 0.3, True), "fcf", "poly", 0),
    "fc_assembled_dg20": (lambda: workloads.dg_random(20, math.pi / 5, True), "fc", "assembled", 0),
    "fcf_assembled_fv80x40": (lambda: workloads.fv_random(80, 0.7, True, ny=40), "fcf", "assembled", 0),
    "fcf_poly_fv64_noorder": (lambda: workloads.fv_random(64, 1.1, True), "fcf", "poly", 1),
}


@pytest.mark.parametrize("case", list(C_SMOOTH))
def test_c_point_smoothing_matches_oracle(case):
    # FC / FCF up-smoothing (Sec. 2, Sec. 3.3): the same hierarchy (C-point
    # coefficients bit for bit), the same iterations and solution as the oracle
    _needs_gpu()
    make, st, smoother, noorder = C_SMOOTH[case]
    p = make()
    print(f"case {case} n={p.n}", flush=True)
    prm = oracle.Params(smooth_type=st, smoother=smoother)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, prm)
    s = _solver(p, smooth_type={"fc": 1, "fcf": 2}[st], smoother=int(smoother == "assembled"),
                keep_setup_data=1, locality_order=0 if noorder else 1)
    compare_hierarchy(s, levels)
    for l, L in enumerate(levels[:-1]):
        got = s.export_level(l, what=("alpha",))["alpha_c"]
        assert np.array_equal(got, L.alpha_c), f"level {l}: C-point coefficients differ"
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    # storage in the paper's terms gains A_cf and A_cc on every level
    s_f = _solver(p, smoother=int(smoother == "assembled"))
    extra = sum(L.Acf.nnz + L.Acc.nnz + (L.Ahat_cc.nnz if smoother == "assembled" else 0)
                for L in levels[:-1])
    nnz0 = p.scipy().nnz
    assert s.stats()["storage_complexity"] == pytest.approx(
        s_f.stats()["storage_complexity"] + extra / nnz0, rel=1e-12)
    s_f.close()
    s.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_c_point_smoothing_mixed_precision_and_columns(prec):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(80, 0.4, True)
    B = workloads.rhs_batch(p, 3)
    s = Solver(p.indptr, p.indices, p.data, smooth_type=2, precision=prec)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    X, infos = s.solve(torch.from_numpy(B).cuda())
    A = p.scipy()
    for k in range(3):
        xk = X[k].cpu().numpy()
        assert infos[k]["converged"] == 1
        assert np.linalg.norm(B[k] - A @ xk) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(B[k])
    s.close()


def test_c_point_smoothing_rejections():
    _needs_gpu()
    from paper_2508_17517_amd import AirgError, Solver
    p = workloads.fv_random(32, 0.4, True)
    with pytest.raises(AirgError):
        Solver(p.indptr, p.indices, p.data, smooth_type=1, inverse_type=1)
    with pytest.raises(AirgError):
        Solver(p.indptr, p.indices, p.data, smooth_type=3)


def test_long_arnoldi_cycle_past_the_fused_sweeps():
    # a weak preconditioner (one level, degree-3 Newton polynomial) and
    # restart 40: Arnoldi cycles pass 32 basis vectors, where the fused
    # Gram-Schmidt sweeps give way to the separate ones, and then restart
    _needs_gpu()
    p = workloads.fv_random(64, 0.4, True)
    kw = dict(max_levels=1, coarse_poly_order=3, restart=40)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, oracle.Params(**kw))
    assert its > 40
    s = _solver(p, **kw)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["restarts"] >= 1
    assert info["iterations"] == its
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    assert_elementwise(x.cpu().numpy(), xo)
    assert_elementwise(x.cpu().numpy(), xo)
    s.close()


def test_c_point_smoothing_in_the_adjoint_and_problem_batches():
    # the transpose hierarchy and a block-diagonal batch take the same smooth
    # sequence: both reach the FP64 tolerance, and the adjoint takes the
    # oracle's iterations on A^T
    _needs_gpu()
    from paper_2508_17517_amd import BatchSolver
    p = workloads.fv_random(64, 0.8, True)
    A = p.scipy()
    w = np.random.default_rng(7).standard_normal(p.n)
    lo, its, rel, _, _ = oracle.adjoint_solve(A, w, oracle.Params(smooth_type="fcf"))
    s = _solver(p, smooth_type=2)
    lam, info = s.adjoint_solve(torch.from_numpy(w).cuda())
    assert info["converged"] == 1 and info["iterations"] == its
    assert np.linalg.norm(lam.cpu().numpy() - lo) <= 1e-10 * np.linalg.norm(lo)
    assert_elementwise(lam.cpu().numpy(), lo)
    s.close()
    probs = [workloads.fv_random(40, 0.3, True, seed=201), workloads.fv_random(24, 1.2, True, seed=202)]
    sb = BatchSolver([(q.indptr, q.indices, q.data) for q in probs], smooth_type=1, precision=1)
    xs, infos = sb.solve([torch.from_numpy(q.b).cuda() for q in probs])
    for q, x, i in zip(probs, xs, infos):
        xh = x.cpu().numpy()
        assert i["converged"] == 1
        assert np.linalg.norm(q.b - q.scipy() @ xh) <= 1e-10 * (1 + 1e-6) * np.linalg.norm(q.b)
    sb.close()


def test_decoupled_grid_lines_solve_exactly():
    # theta = 0: every grid line is a separate component (the locality order
    # handles them all at once).  The coarse spectrum is then one repeated
    # block's, so the Newton roots are ill-conditioned and are not compared;
    # the discrete setup decisions and the solve are
    _needs_gpu()
    p = workloads.fv_random(72, 0.0, True)
    A = p.scipy()
    xo, its, rel, levels, _ = oracle.solve(A, p.b)
    s = _solver(p, keep_setup_data=1)
    st = s.stats()
    assert st["levels"] == len(levels)
    for l, L in enumerate(levels[:-1]):
        g = s.export_level(l)
        assert np.array_equal(g["state"], L.state), f"level {l}: CF split differs"
        _csr_equal("Z", g["z"], L.Z, l)
    x, info = s.solve(torch.from_numpy(p.b).cuda())
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert_elementwise(x.cpu().numpy(), xo)
    u = oracle.sweep_solve(A, p.b, p.level)
    assert np.linalg.norm(x.cpu().numpy() - u) <= 1e-9 * np.linalg.norm(u)
    s.close()
