"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks one part of the oracle against something other than itself:
an exact solve, a closed form, a textbook special case, brute force on a tiny
input, or an invariant that a plausible slip (a dropped term, a wrong sign or
index, a transposed operand) would break.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import linalg
from oracle import hierarchy as S
from oracle.params import Params
from airg_inputs import fv_advection, workloads


def _rand_diag_dominant(n, seed, density=0.2, dom=2.0):
    r = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=seed, data_rvs=lambda k: r.uniform(-1, 1, k))
    M = sp.csr_matrix(M)
    M.setdiag(0.0)
    M.eliminate_zeros()
    d = np.abs(M).sum(axis=1).A.ravel() * dom + 1.0
    A = sp.csr_matrix(M + sp.diags(d))
    A.sort_indices()
    return A


# --------------------------------------------------------------------- sweep (P2, P3)

@pytest.mark.parametrize("n,theta,perm", [(16, 0.3, True), (32, 1.2, True), (24, 3 * math.pi / 8, False)])
def test_sweep_is_exact_and_equals_direct_solve(n, theta, perm):
    p = workloads.fv_random(n, theta, perm)
    A = p.scipy()
    u = oracle.sweep_solve(A, p.b, p.level)
    assert np.linalg.norm(p.b - A @ u) <= 1e-14 * np.linalg.norm(p.b) * n
    ud = spla.spsolve(sp.csc_matrix(A), p.b)
    assert np.allclose(u, ud, rtol=1e-13, atol=1e-13)


def test_sweep_rejects_non_triangular_order():
    p = workloads.fv_random(8, 0.5, False)
    with pytest.raises(ValueError):
        oracle.sweep_solve(p.scipy(), p.b, -p.level)


# --------------------------------------------------------------------- vector kernels

def test_spmv_and_tree_sum_agree_with_exact_arithmetic():
    A = _rand_diag_dominant(300, 1)
    x = np.random.default_rng(2).standard_normal(300)
    assert np.allclose(linalg.spmv(A, x), A @ x, rtol=1e-14, atol=1e-14)
    # tree sum of integers-valued doubles is exact
    v = np.arange(1, 1001, dtype=np.float64)
    assert linalg.tree_sum(v) == 500500.0
    # the summation tree: adjacent pairs first, zero padding to a power of two
    g = np.random.default_rng(5).standard_normal(8) * 10.0 ** np.arange(8)
    x0, x1, x2, x3, x4, x5, x6, x7 = g
    assert linalg.tree_sum(g) == ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7))
    assert linalg.tree_sum(g[:5]) == ((x0 + x1) + (x2 + x3)) + x4
    assert linalg.tree_sum(g[:3]) == (x0 + x1) + x2
    assert linalg.dot(x, x) == pytest.approx(math.fsum(x * x), rel=1e-15)


def test_givens_lstsq_matches_lapack_least_squares():
    r = np.random.default_rng(3)
    H = np.triu(r.standard_normal((7, 6)), -1)
    y, res = linalg.givens_lstsq(H, 2.5)
    rhs = np.zeros(7)
    rhs[0] = 2.5
    yl, *_ = np.linalg.lstsq(H, rhs, rcond=None)
    assert np.allclose(y, yl, rtol=1e-12)
    assert res == pytest.approx(np.linalg.norm(rhs - H @ yl), rel=1e-10)


def test_arnoldi_relation_and_orthonormality():
    A = _rand_diag_dominant(200, 4)
    b = np.random.default_rng(5).uniform(size=200)
    V, H, steps, beta = linalg.arnoldi(A, b, 8)
    assert steps == 8
    Vm = np.array(V).T                      # 200 x 8 (last vector not formed)
    assert np.allclose(Vm.T @ Vm, np.eye(8), atol=1e-13)
    # A V_7 = V_8 H_7 (first 7 columns)
    assert np.allclose(A @ Vm[:, :7], Vm @ H[:8, :7], atol=1e-12)


# --------------------------------------------------------------------- GMRES polynomial (P4)

@pytest.mark.parametrize("d", [1, 2, 4, 6])
def test_gmres_poly_minimises_residual_over_krylov_space(d):
    A = _rand_diag_dominant(120, 10 + d, dom=1.5)
    b = np.random.default_rng(d).uniform(size=120)
    alpha = linalg.gmres_poly_coeffs(A, b, d)
    assert len(alpha) == d + 1
    x = linalg.horner_apply(A, alpha, b)
    res = np.linalg.norm(b - A @ x)
    # brute force: min over c of |b - A K c| with K = [b, Ab, ..., A^d b]
    Ad = A.toarray()
    K = np.empty((120, d + 1))
    K[:, 0] = b
    for i in range(1, d + 1):
        K[:, i] = Ad @ K[:, i - 1]
    Q, _ = np.linalg.qr(Ad @ K)
    best = np.linalg.norm(b - Q @ (Q.T @ b))
    # GMRES is the minimiser: never above the projection residual, and equal to
    # it within the conditioning of the monomial Krylov matrix
    assert res <= best * (1 + 1e-9)
    assert res >= best * (1 - 1e-6)
    c, *_ = np.linalg.lstsq(Ad @ K, b, rcond=None)
    assert np.allclose(alpha, c, rtol=1e-4, atol=1e-6 * np.abs(c).max())
    # no perturbation of the coefficients does better
    g = np.random.default_rng(99)
    for _ in range(20):
        a2 = alpha + 1e-3 * g.standard_normal(d + 1) * np.abs(alpha).max()
        assert np.linalg.norm(b - A @ linalg.horner_apply(A, a2, b)) >= res


def test_gmres_poly_exact_for_scaled_identity():
    A = sp.identity(50, format="csr") * 2.5
    b = np.random.default_rng(0).uniform(size=50)
    alpha = linalg.gmres_poly_coeffs(sp.csr_matrix(A), b, 4)
    assert len(alpha) == 1                    # happy breakdown: degree 0
    assert alpha[0] == pytest.approx(0.4, rel=1e-15)


# --------------------------------------------------------------------- Newton form (P5, P6)

def test_harmonic_ritz_values_are_roots_of_gmres_residual_polynomial():
    A = _rand_diag_dominant(150, 21, dom=1.3)
    b = np.random.default_rng(8).uniform(size=150)
    d = 6
    alpha = linalg.gmres_poly_coeffs(A, b, d)
    roots = linalg.newton_roots(A, b, d, use_added_roots=False)
    assert len(roots) == d + 1
    for z in roots:
        q = sum(alpha[i] * z ** i for i in range(d + 1))
        assert abs(1.0 - z * q) < 1e-8 * max(1.0, abs(z) * abs(q))


@pytest.mark.parametrize("d", [2, 5, 8])
def test_newton_form_equals_monomial_form(d):
    A = _rand_diag_dominant(150, 30 + d, dom=1.3)
    b = np.random.default_rng(d).uniform(size=150)
    alpha = linalg.gmres_poly_coeffs(A, b, d)
    roots = linalg.newton_roots(A, b, d, use_added_roots=False)
    r = np.random.default_rng(77).standard_normal(150)
    xm = linalg.horner_apply(A, alpha, r)
    xn = linalg.newton_apply(A, roots, r)
    assert np.allclose(xn, xm, rtol=1e-8, atol=1e-10 * np.abs(xm).max())


def test_rank_reveal_scaled_identity_one_root():
    A = sp.csr_matrix(sp.identity(40) * 3.0)
    roots = linalg.newton_roots(A, np.random.default_rng(1).uniform(size=40), 20)
    assert len(roots) == 1 and roots[0] == pytest.approx(3.0, rel=1e-14)
    r = np.arange(40.0)
    assert np.allclose(linalg.newton_apply(A, roots, r), r / 3.0, rtol=1e-15)


def test_diagonal_with_k_distinct_values_is_solved_exactly():
    vals = np.array([1.0, 2.0, 5.0, 7.5])
    d = np.tile(vals, 10)
    A = sp.csr_matrix(sp.diags(d))
    roots = linalg.newton_roots(A, np.random.default_rng(2).uniform(size=40), 20)
    assert len(roots) <= 4
    r = np.random.default_rng(3).standard_normal(40)
    assert np.allclose(linalg.newton_apply(A, roots, r), r / d, rtol=1e-10)


def test_leja_order_properties():
    roots = [3.0 + 0j, 1 + 2j, 1 - 2j, -0.5 + 0j, 2.0 + 0j]
    out = linalg.leja_order(roots)
    assert sorted(out, key=lambda z: (z.real, z.imag)) == sorted(roots, key=lambda z: (z.real, z.imag))
    assert abs(out[0]) == max(abs(z) for z in roots)
    for i, z in enumerate(out):
        if z.imag > 0:
            assert out[i + 1] == z.conjugate()


def test_added_roots_keep_the_original_roots():
    # widely spread roots trigger extra copies; every original root stays a root
    roots = [complex(x) for x in (0.01, 0.02, 0.05, 1.0, 2.0, 3.0, 50.0, 100.0, 400.0)]
    extra = linalg.added_roots(roots)
    assert len(extra) > 0
    assert all(any(e == r for r in roots) for e in extra)


# --------------------------------------------------------------------- CF splitting (P7, P8)

def _strength_graph(A, theta):
    Smat = S.strength(A, theta)
    return S._csr(Smat + Smat.T)


@pytest.mark.parametrize("theta_s", [0.0, 0.5, 0.99])
def test_pmisr_gives_a_maximal_independent_set_of_f_points(theta_s):
    A = workloads.fv_random(40, 0.9, True).scipy()
    Smat = S.strength(A, theta_s)
    w = oracle.rng.uniform(7, oracle.rng.PMISR, 0, A.shape[0])
    state, rounds = S.pmisr(Smat, w)
    G = _strength_graph(A, theta_s)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(G.indptr))
    isf = state == S.FPT
    assert np.all(state != S.UNDECIDED)
    assert not np.any(isf[rows] & isf[G.indices])           # independent
    has_f_nb = np.zeros(A.shape[0], dtype=bool)
    has_f_nb[rows[isf[G.indices]]] = True
    assert np.all(has_f_nb[state == S.CPT])                  # maximal
    assert rounds >= 1


def test_strength_special_cases():
    A = workloads.fv_random(12, 0.3, False).scipy()
    S0 = S.strength(A, 0.0)
    off = A.copy()
    off.setdiag(0.0)
    off.eliminate_zeros()
    assert (S0 != (off != 0)).nnz == 0                       # theta_s = 0: all off-diagonals
    S1 = S.strength(A, 0.99)
    # theta = 0.3: the west coupling (cos) dominates the south one (sin), so the
    # strong set is every west link plus the south link of first-column rows
    west = [(j * 12 + i, j * 12 + i - 1) for j in range(12) for i in range(1, 12)]
    south = [(j * 12, (j - 1) * 12) for j in range(1, 12)]
    want = sp.csr_matrix((np.ones(len(west) + len(south)), tuple(zip(*(west + south)))), shape=A.shape)
    assert (S1 != want).nnz == 0


def test_ddc_converts_the_closest_bin_boundary_count():
    # F rows with prescribed dominance ratios r_i = i / 400 (a few duplicates)
    n = 800
    rows, cols, vals = [], [], []
    ratios = np.concatenate([np.arange(1, 401) / 400.0, np.zeros(400)])
    for i in range(n):
        rows.append(i); cols.append(i); vals.append(1.0)
        if ratios[i] > 0:
            j = (i + 1) % 400
            rows.append(i); cols.append(j); vals.append(-ratios[i])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    state = np.full(n, S.FPT, dtype=np.int8)
    conv = S.ddc_pass(A, state, A.diagonal(), 0.01)
    # k = ceil(0.01 * 800) = 8; ratios are distinct multiples of r_max / 400, so
    # the 8 largest fall in the top bins exactly: 8 conversions
    assert conv == 8
    assert np.all(state[392:400] == S.CPT) and np.all(state[:392] == S.FPT)
    assert np.all(state[400:] == S.FPT)                      # r = 0 rows never converted


def test_ddc_converts_nothing_when_all_ratios_tie():
    # every F row has the same ratio: the nearest boundary to 1% is "none"
    n = 300
    A = sp.csr_matrix(sp.diags([np.full(n - 1, -0.5), np.ones(n)], [-1, 0]))
    state = np.full(n, S.FPT, dtype=np.int8)
    assert S.ddc_pass(sp.csr_matrix(A), state, np.ones(n), 0.01) == 0


# --------------------------------------------------------------------- operators

def test_fixed_sparsity_is_exact_when_the_pattern_is_closed():
    # block-diagonal A_ff with full blocks: every power keeps the pattern
    blocks = [np.random.default_rng(i).uniform(-0.3, 0.3, (3, 3)) + 2 * np.eye(3) for i in range(20)]
    Aff = sp.csr_matrix(sp.block_diag(blocks))
    Aff.sort_indices()
    alpha = np.array([0.7, -0.2, 0.05, -0.01])
    Ahat = S.fixed_sparsity_inverse(Aff, alpha)
    x = np.random.default_rng(0).standard_normal(60)
    assert np.allclose(Ahat @ x, linalg.horner_apply(Aff, alpha, x), rtol=1e-13, atol=1e-14)


def test_one_point_prolongation_takes_the_largest_c_coupling_with_weight_one():
    A = workloads.fv_random(20, 1.0, True).scipy()
    state = np.where(np.random.default_rng(3).uniform(size=A.shape[0]) < 0.5, S.FPT, S.CPT).astype(np.int8)
    C = np.nonzero(state == S.CPT)[0]
    F = np.nonzero(state == S.FPT)[0]
    cidx = np.full(A.shape[0], -1)
    cidx[C] = np.arange(len(C))
    cmap = S.one_point(A, state, cidx)
    Ad = A.toarray()
    for f, c in zip(F, cmap):
        cand = [(abs(Ad[f, j]), j) for j in C if Ad[f, j] != 0.0]
        if not cand:
            assert c == -1
            continue
        m = max(v for v, _ in cand)
        j = min(j for v, j in cand if v >= m * (1 - 1e-12))
        assert C[c] == j


def test_coarse_operator_equals_schur_form_and_lumping_keeps_row_sums():
    p = workloads.fv_random(24, 0.8, True)
    A = p.scipy()
    prm = Params(a_drop=0.0, r_drop=0.0)
    L, Ac = S.coarsen(A, 0, prm)
    nC = len(L.C)
    W = sp.csr_matrix((np.ones(int((L.cmap >= 0).sum())),
                       (np.nonzero(L.cmap >= 0)[0], L.cmap[L.cmap >= 0])), shape=(len(L.F), nC))
    Acc = A[L.C][:, L.C]
    Acf = A[L.C][:, L.F]
    alt = Acc + Acf @ W + L.Z @ (L.Afc + L.Aff @ W)
    assert abs(Ac - alt).max() <= 1e-13 * abs(alt).max()
    # dropping with lumping preserves every row sum
    Ad = S.relative_drop(Ac, 0.3, True)
    assert Ad.nnz < Ac.nnz
    assert np.allclose(Ad @ np.ones(nC), Ac @ np.ones(nC), rtol=1e-13, atol=1e-14)
    rows = np.repeat(np.arange(nC), np.diff(Ad.indptr))
    off = Ad.indices != rows
    m = S.row_abs_max(Ac, np.repeat(np.arange(nC), np.diff(Ac.indptr)) != Ac.indices)
    assert np.all(np.abs(Ad.data[off]) >= 0.3 * m[rows[off]])


def test_restrictor_is_ideal_when_aff_is_exactly_inverted():
    # theta_s = 0: F is an independent set of A's graph, so A_ff = (vx + vy) I and
    # the degree-0 polynomial is exact; then Z A_ff = -A_cf (Eq. z)
    p = workloads.fv_random(20, 0.6, True)
    A = p.scipy()
    L, _ = S.coarsen(A, 0, Params(strong_threshold=0.0, r_drop=0.0, ddc_its=0))
    assert L.Aff.nnz == len(L.F)
    assert np.allclose(L.Aff.diagonal(), math.cos(0.6) + math.sin(0.6), rtol=1e-15)
    assert len(L.alpha) == 1
    assert abs(L.Z @ L.Aff + L.Acf).max() < 1e-15


# --------------------------------------------------------------------- exactness (P9, P10)

def test_two_level_with_exact_inverses_converges_in_one_iteration():
    p = workloads.fv_random(24, 0.6, True)
    prm = Params(strong_threshold=0.0, r_drop=0.0, a_drop=0.0, ddc_its=0, trunc_tol=0.0,
                 max_levels=2, exact_coarse=True)
    x, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, prm)
    assert len(levels) == 2
    assert its == 1 and rel < 1e-12


def test_one_dimensional_flow_is_cyclic_reduction_exact_on_every_level():
    # theta = 0: uncoupled 1D lines (bidiagonal); with theta_s = 0 every level's
    # A_ff is the identity and the coarse matrix is the exact Schur complement
    p = fv_advection(32, 0.0, np.random.default_rng(1).uniform(size=32), 0.0, perm_seed=4)
    prm = Params(strong_threshold=0.0, r_drop=0.0, a_drop=0.0, ddc_its=0, trunc_tol=0.0,
                 min_coarse_rows=40, exact_coarse=True)
    x, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, prm)
    assert len(levels) >= 3
    for L in levels[:-1]:
        assert L.Aff.nnz == len(L.F)
    assert its == 1 and rel < 1e-12


# --------------------------------------------------------------------- full solve (P1, P2)

def test_constant_inflow_solution_is_constant():
    p = workloads.fv64()
    x, its, rel, levels, _ = oracle.solve(p.scipy(), p.b)
    assert rel <= 1e-10
    assert np.abs(x - 1.0).max() < 1e-8
    assert levels[-1].coarsest and len(levels) >= 2


@pytest.mark.parametrize("n,theta", [(48, 0.3), (64, 1.0)])
def test_airg_solution_matches_sweep(n, theta):
    p = workloads.fv_random(n, theta, True)
    A = p.scipy()
    x, its, rel, levels, _ = oracle.solve(A, p.b)
    u = oracle.sweep_solve(A, p.b, p.level)
    assert rel <= 1e-10
    assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)
    assert its < 30


def test_airg_solution_matches_sweep_on_dg():
    # the block-scaled upwind DG-Q1 system of the mixed-precision workload
    p = workloads.dg_random(32, math.pi / 5, True)
    A = p.scipy()
    x, its, rel, levels, _ = oracle.solve(A, p.b)
    u = oracle.sweep_solve(A, p.b, p.level)
    assert rel <= 1e-10
    assert np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)
    assert its < 30 and len(levels) >= 2


def test_fgmres_matches_brute_force_gmres_residuals():
    A = _rand_diag_dominant(80, 12, dom=1.1)
    b = np.random.default_rng(1).uniform(size=80)
    x, its, rel, hist = oracle.fgmres(A, lambda v: v, b, rtol=1e-10)
    Ad = A.toarray()
    K = [b]
    for k in range(1, 6):
        K.append(Ad @ K[-1])
        Km = np.array(K[1:]).T                 # A K_k
        c, *_ = np.linalg.lstsq(Km, b, rcond=None)
        assert hist[k - 1] == pytest.approx(np.linalg.norm(b - Km @ c) / np.linalg.norm(b), rel=1e-7)
    assert np.allclose(x, np.linalg.solve(Ad, b), rtol=1e-8)


def test_fgmres_absolute_tolerance_stops_at_the_first_small_residual():
    # a residual at or below max(rtol |b|, atol) stops the outer loop (the
    # paper's option set has both, Sec. 3): with rtol negligible, atol = c |b|
    # stops where rtol = c would, at the first brute-force GMRES residual
    # below c |b|; with atol 0 nothing changes
    A = _rand_diag_dominant(80, 12, dom=1.1)
    b = np.random.default_rng(1).uniform(size=80)
    bn = np.linalg.norm(b)
    Ad = A.toarray()
    K, res = [b], []
    for k in range(1, 9):
        K.append(Ad @ K[-1])
        Km = np.array(K[1:]).T
        c, *_ = np.linalg.lstsq(Km, b, rcond=None)
        res.append(np.linalg.norm(b - Km @ c) / bn)
    for c in (1e-1, 1e-2, 1e-3):
        first = next(k + 1 for k, r in enumerate(res) if r <= c)
        x, its, rel, hist = oracle.fgmres(A, lambda v: v, b, rtol=1e-300, atol=c * bn)
        assert its == first, (c, its, first)
        x2, its2, _, _ = oracle.fgmres(A, lambda v: v, b, rtol=c, atol=0.0)
        assert its2 == its and np.array_equal(x, x2)
    # the absolute test is on the residual norm itself, not relative to |b|
    x, its, rel, hist = oracle.fgmres(A, lambda v: v, 1e4 * b, rtol=1e-300, atol=10.0 * bn)
    assert its == next(k + 1 for k, r in enumerate(res) if r <= 1e-3)


def test_richardson_absolute_tolerance():
    p = workloads.fv_random(12, 1.0, True)
    A = p.scipy()
    levels = oracle.setup(A)
    M = lambda v: oracle.vcycle(levels, v)  # noqa: E731
    x, its, rel, hist = oracle.richardson(A, M, p.b, rtol=1e-12)
    bn = np.linalg.norm(p.b)
    for k in range(1, its):
        c = hist[k] / bn * 1.0000001
        x2, its2, _, h2 = oracle.richardson(A, M, p.b, rtol=1e-300, atol=c * bn)
        assert its2 == next(j for j, h in enumerate(hist) if h <= c * bn)


# --------------------------------------------------------------------- adjoint (P11, P12)

def test_adjoint_identity_and_adjoint_solve():
    p = workloads.fv_random(40, 0.3, True)
    A = p.scipy()
    w = np.random.default_rng(2).standard_normal(p.n)
    u = oracle.sweep_solve(A, p.b, p.level)
    lam = oracle.sweep_solve(A, w, p.level, transpose=True)
    assert np.dot(u, w) == pytest.approx(np.dot(p.b, lam), rel=1e-12)
    lam2, its, rel, _, _ = oracle.adjoint_solve(A, w)
    assert rel <= 1e-10
    assert np.linalg.norm(lam2 - lam) <= 1e-8 * np.linalg.norm(lam)


def test_gradients_match_finite_differences():
    n = 32
    theta = 0.3
    gw, gs = workloads.inflow_values(11, n)
    p = fv_advection(n, theta, gw, gs)
    wts = workloads.loss_weights(p)
    wfull = np.zeros(p.n)
    wfull[p.outflow_rows] = wts
    A = p.scipy()
    u = oracle.sweep_solve(A, p.b, p.level)
    lam = oracle.sweep_solve(A, wfull, p.level, transpose=True)
    dgw, dgs, dth = oracle.loss_gradients(p, u, lam)

    def loss(t, gw_, gs_):
        q = fv_advection(n, t, gw_, gs_)
        return float(np.dot(wfull, oracle.sweep_solve(q.scipy(), q.b, q.level)))

    h = 1e-6
    fd = (loss(theta + h, gw, gs) - loss(theta - h, gw, gs)) / (2 * h)
    assert dth == pytest.approx(fd, rel=1e-7)
    for j in (0, 5, 31):
        e = np.zeros(n); e[j] = 1.0
        fdj = (loss(theta, gw + h * e, gs) - loss(theta, gw - h * e, gs)) / (2 * h)
        assert dgw[j] == pytest.approx(fdj, rel=1e-7, abs=1e-9)
        fdj = (loss(theta, gw, gs + h * e) - loss(theta, gw, gs - h * e)) / (2 * h)
        assert dgs[j] == pytest.approx(fdj, rel=1e-7, abs=1e-9)


# --------------------------------------------------------------------- Richardson (Sec. 3)

def test_richardson_residuals_follow_the_error_propagator():
    # r_k = (I - A M)^k r_0 for the V-cycle M, with M formed column by column
    p = workloads.fv_random(10, 0.6, True)
    A = p.scipy()
    levels = oracle.setup(A)
    M = lambda v: oracle.vcycle(levels, v)  # noqa: E731
    n = p.n
    Mm = np.column_stack([M(e) for e in np.eye(n)])
    E = np.eye(n) - A.toarray() @ Mm
    x0 = np.ones(n)
    x, its, rel, hist = oracle.richardson(A, M, p.b, rtol=1e-12, x0=x0)
    r = p.b - A @ x0
    for k in range(1, min(its, 6) + 1):
        r = E @ r
        assert abs(np.linalg.norm(r) - hist[k]) <= 1e-10 * hist[0]


def test_richardson_with_an_exact_inverse_takes_one_step():
    p = workloads.fv_random(12, 1.0, True)
    A = p.scipy()
    lu = sp.linalg.splu(A.tocsc())
    x, its, rel, _ = oracle.richardson(A, lu.solve, p.b, rtol=1e-10)
    assert its == 1 and rel <= 1e-13


def test_richardson_on_the_paper_fd_system_goes_to_zero():
    # g = 0 and x0 = 1 (Sec. 3): the solution is 0 and the test is relative to r_0
    from airg_inputs import fd_advection
    p = fd_advection(40, math.pi / 4, 0.0)
    A = p.scipy()
    prm = oracle.Params(outer="richardson", poly_order=6, coarse_poly_order=10, trunc_tol=0.1)
    x, its, rel, levels, hist = oracle.solve(A, p.b, prm, x0=np.ones(p.n))
    assert rel <= 1e-10 and its < 20
    assert np.abs(x).max() <= 1e-9
    assert hist[-1] <= 1e-10 * hist[0]


# --------------------------------------------------------------------- assembled smoother (Sec. 2.2)

def test_assembled_smoother_equals_the_polynomial_when_the_pattern_is_closed():
    # with theta_s = 0 every upwind neighbour is strong, A_ff is diagonal (P9),
    # its pattern is closed under products, so Ahat^{-1} = q(A_ff) exactly and
    # both smoothers give the same V-cycle
    p = workloads.fv_random(24, 0.6, True)
    A = p.scipy()
    prm = oracle.Params(strong_threshold=0.0, trunc_tol=0.0, min_coarse_rows=64)
    levels = oracle.setup(A, prm)
    L0 = levels[0]
    assert L0.Aff.nnz == L0.Aff.shape[0]
    r = np.random.default_rng(5).standard_normal(p.n)
    e_poly = oracle.vcycle(levels, r)
    e_asm = oracle.vcycle(levels, r, assembled=True)
    assert np.allclose(e_asm, e_poly, rtol=1e-12, atol=1e-12 * np.abs(e_poly).max())


def test_assembled_smoother_solves_to_tolerance():
    p = workloads.fv_random(48, 0.3, True)
    A = p.scipy()
    x, its, rel, levels, _ = oracle.solve(A, p.b, oracle.Params(smoother="assembled"))
    u = oracle.sweep_solve(A, p.b, p.level)
    assert rel <= 1e-10 and np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)
    x2, its2, _, _, _ = oracle.solve(A, p.b, oracle.Params(), levels=levels)
    assert its >= its2 - 1  # the paper: assembled needs as many or more iterations


# --------------------------------------------------------------------- nAIR: Neumann polynomials (Sec. 3.3)

def test_neumann_apply_is_the_jacobi_scaled_series():
    rng_ = np.random.default_rng(11)
    n = 12
    M = np.diag(rng_.uniform(2.0, 3.0, n)) + np.tril(rng_.uniform(-0.4, 0.4, (n, n)), -1)
    A = sp.csr_matrix(M)
    s = rng_.standard_normal(n)
    D = np.diag(M)
    N = np.eye(n) - M / D[:, None]
    for d in (0, 1, 3):
        want = sum(np.linalg.matrix_power(N, k) @ (s / D) for k in range(d + 1))
        assert np.allclose(oracle.linalg.neumann_apply(A, d, s), want, rtol=1e-13, atol=1e-14)
    # N is strictly lower triangular, so N^n = 0: degree n - 1 inverts exactly
    x = oracle.linalg.neumann_apply(A, n - 1, s)
    assert np.allclose(M @ x, s, rtol=0, atol=1e-12)


def test_neumann_fixed_sparsity_on_a_closed_pattern_is_the_series():
    # lower-bidiagonal A_ff: its pattern is not closed, but a dense lower
    # triangle is, so the masked powers are the exact powers there
    rng_ = np.random.default_rng(12)
    n = 8
    M = np.diag(rng_.uniform(1.5, 2.5, n)) + np.tril(rng_.uniform(-0.5, 0.5, (n, n)), -1)
    A = sp.csr_matrix(M)
    D = np.diag(M)
    N = np.eye(n) - M / D[:, None]
    for d in (1, 2, 4):
        want = sum(np.linalg.matrix_power(N, k) for k in range(d + 1)) / D[None, :]
        got = oracle.hierarchy.neumann_fixed_sparsity(A, d).toarray()
        assert np.allclose(got, want, rtol=1e-13, atol=1e-14)


def test_nair_solves_to_tolerance():
    p = workloads.fv_random(48, 0.3, True)
    A = p.scipy()
    for smoother in ("poly", "assembled"):
        prm = oracle.Params(inverse_type="neumann", smoother=smoother)
        x, its, rel, levels, _ = oracle.solve(A, p.b, prm)
        u = oracle.sweep_solve(A, p.b, p.level)
        assert rel <= 1e-10 and np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)


# --------------------------------------------------------------------- C-point smoothing (Sec. 2, Sec. 3.3)

@pytest.mark.parametrize("smooth_type", ["fc", "fcf"])
def test_c_smoothing_keeps_cyclic_reduction_exact(smooth_type):
    # the F smooth already makes the cycle exact here (see the cyclic
    # reduction pin), so a C residual r_c - A_cf e_f - A_cc e_c with every
    # term and sign right is zero and the extra smooths change nothing
    p = fv_advection(32, 0.0, np.random.default_rng(1).uniform(size=32), 0.0, perm_seed=4)
    prm = Params(strong_threshold=0.0, r_drop=0.0, a_drop=0.0, ddc_its=0, trunc_tol=0.0,
                 min_coarse_rows=40, exact_coarse=True, smooth_type=smooth_type)
    x, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, prm)
    assert len(levels) >= 3 and all(L.Acc is not None for L in levels[:-1])
    assert its == 1 and rel < 1e-12


@pytest.mark.parametrize("smooth_type,assembled", [("fc", False), ("fcf", False), ("fcf", True)])
def test_smooths_follow_the_global_relaxation_form(smooth_type, assembled):
    # two levels, exact coarse solve: x = P A_c^{-1} R r, then for each step
    # x_S += M_S (r - A x)_S on the F or C rows, with M_S the dense polynomial
    # sum_i alpha_i A_SS^i (or the assembled matrix): an independent statement
    # of the block formulas the oracle evaluates
    p = workloads.fv_random(12, 0.7, True)
    A = p.scipy()
    prm = Params(max_levels=2, trunc_tol=0.0, smooth_type=smooth_type)
    levels = oracle.setup(A, prm)
    L0, L1 = levels
    assert L1.coarsest
    r = np.random.default_rng(3).standard_normal(p.n)
    got = oracle.vcycle(levels, r, exact_coarse=True, assembled=assembled, smooth_type=smooth_type)
    Ad = A.toarray()
    F, C = L0.F, L0.C
    nF, nC = len(F), len(C)

    def poly(M, alpha):
        out = np.zeros_like(M)
        Pk = np.eye(M.shape[0])
        for a in alpha:
            out += a * Pk
            Pk = Pk @ M
        return out

    if assembled:
        Mf, Mc = L0.Ahat.toarray(), L0.Ahat_cc.toarray()
    else:
        Mf = poly(Ad[np.ix_(F, F)], L0.alpha)
        Mc = poly(Ad[np.ix_(C, C)], L0.alpha_c)
    R = np.zeros((nC, p.n))
    R[:, F] = L0.Z.toarray()
    R[np.arange(nC), C] = 1.0
    P = np.zeros((p.n, nC))
    w = L0.cmap >= 0
    P[F[w], L0.cmap[w]] = 1.0
    P[C, np.arange(nC)] = 1.0
    x = P @ np.linalg.solve(L1.A.toarray(), R @ r)
    for step in smooth_type:
        res = r - Ad @ x
        if step == "f":
            x[F] += Mf @ res[F]
        else:
            x[C] += Mc @ res[C]
    assert np.allclose(got, x, rtol=1e-11, atol=1e-11 * np.abs(x).max())


def test_c_point_polynomial_minimises_the_residual_on_acc():
    # alpha_c: the degree-d minimiser of |b - A_cc q(A_cc) b| for the C stream's
    # b, checked by least squares on the explicit Krylov matrix of the dense A_cc
    p = workloads.fv_random(16, 0.4, True)
    A = p.scipy()
    prm = Params(smooth_type="fc")
    L, _ = S.coarsen(A, 0, prm)
    Acc = A.toarray()[np.ix_(L.C, L.C)]
    b = oracle.rng.uniform(prm.seed, 5, 0, len(L.C))
    K = np.empty((len(b), prm.poly_order + 1))
    v = b.copy()
    for i in range(prm.poly_order + 1):
        v = Acc @ v
        K[:, i] = v
    want, *_ = np.linalg.lstsq(K, b, rcond=None)
    assert len(L.alpha_c) == prm.poly_order + 1
    assert np.allclose(L.alpha_c, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())
    assert abs(L.Acc - sp.csr_matrix(Acc)).max() == 0.0


@pytest.mark.parametrize("smooth_type", ["fc", "fcf"])
@pytest.mark.parametrize("smoother", ["poly", "assembled"])
def test_c_smoothing_solves_to_tolerance(smooth_type, smoother):
    p = workloads.fv_random(48, 0.3, True)
    A = p.scipy()
    prm = oracle.Params(smooth_type=smooth_type, smoother=smoother)
    x, its, rel, levels, _ = oracle.solve(A, p.b, prm)
    u = oracle.sweep_solve(A, p.b, p.level)
    assert rel <= 1e-10 and np.linalg.norm(x - u) <= 1e-8 * np.linalg.norm(u)


def test_c_smoothing_needs_the_gmres_polynomial():
    p = workloads.fv_random(16, 0.4, True)
    with pytest.raises(ValueError):
        oracle.setup(p.scipy(), oracle.Params(smooth_type="fc", inverse_type="neumann"))
