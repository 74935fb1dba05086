"""Hand-worked pins of the oracle parts whose defining step a generic
invariant does not reach.

Every expected number here was worked out by hand (dyadic values, so the
comparisons are exact) or comes from a published table; none is produced by
calling the function under test a second time.  Each test names the slip it
is there to catch.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import linalg, rng
from oracle import hierarchy as H
from oracle.params import Params
from airg_inputs import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _golden_ints(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [int(l) for l in f if l.strip() and not l.startswith("#")]


def _csr(dense):
    M = sp.csr_matrix(np.asarray(dense, dtype=np.float64))
    M.sort_indices()
    return M


# --------------------------------------------------------------------- the solver's random draws

@pytest.mark.parametrize("purpose,level", [(0, 0), (rng.PMISR, 0), (rng.POLY_RHS, 3),
                                           (rng.COARSE_RHS, 7), (rng.TRUNC_RHS, 12),
                                           (rng.CPOLY_RHS, 1)])
def test_oracle_uniform_is_the_published_sequence_at_its_counter(purpose, level):
    # Element i of stream (purpose, level) is SplitMix64 output c + 1 with
    # c = purpose << 56 | level << 40 | i.  Since the generator's state after
    # k steps is seed + k * gamma, choosing seed = 1234567 - c0 * gamma puts
    # element i at output i + 1 of the published seed-1234567 sequence.
    # Catches: a wrong gamma or mixer, an off-by-one in the counter, purpose
    # and level in the wrong bit fields, and a wrong 53-bit conversion.
    want_raw = _golden_ints("splitmix64_seed1234567.txt")
    c0 = (purpose << 56) | (level << 40)
    seed = (1234567 - c0 * GAMMA) & M64
    got = oracle.rng.uniform(seed, purpose, level, len(want_raw))
    want = [(v >> 11) / 2.0 ** 53 for v in want_raw]
    assert list(got) == want


def test_oracle_stream_purposes():
    # the reading's purpose numbers: PMISR weights 1, smoother rhs 2, coarse
    # rhs 3, truncation rhs 4, C-point smoother rhs 5 (all distinct streams)
    assert (rng.PMISR, rng.POLY_RHS, rng.COARSE_RHS, rng.TRUNC_RHS, rng.CPOLY_RHS) == (1, 2, 3, 4, 5)


# --------------------------------------------------------------------- the relative drop on R (Sec. 2)

def test_restrictor_drop_on_hand_worked_rows():
    # tol = 1/4 of the row's largest |z| (all entries count: R has no diagonal)
    #  row 0: [-1, 1/4, 1/5, 1/2]   max 1    -> keep -1, 1/4 (equal: kept), 1/2
    #  row 1: [1/10, -4, 9/10, 3/2]  max 4 (at column 1 = the row index)
    #                                         -> keep -4, 3/2; 9/10 < 1 dropped
    #  row 2: empty stays empty;  row 3: [3, 3] keeps both
    # Catches: a drop relative to the off-"diagonal" entries only (row 1 would
    # keep 9/10), a strict test at the threshold (row 0 would lose 1/4),
    # absolute instead of relative thresholds, and lumping into R.
    Z = sp.csr_matrix((np.array([-1.0, 0.25, 0.2, 0.5, 0.1, -4.0, 0.9, 1.5, 3.0, 3.0]),
                       np.array([0, 2, 3, 5, 0, 1, 3, 4, 1, 2]),
                       np.array([0, 4, 8, 8, 10])), shape=(4, 6))
    D = H.restrictor_drop(Z, 0.25).toarray()
    want = np.zeros((4, 6))
    want[0, [0, 2, 5]] = [-1.0, 0.25, 0.5]
    want[1, [1, 4]] = [-4.0, 1.5]
    want[3, [1, 2]] = [3.0, 3.0]
    assert np.array_equal(D, want)
    # tol = 0 keeps every entry
    assert np.array_equal(H.restrictor_drop(Z, 0.0).toarray(), Z.toarray())


def test_coarse_drop_and_lump_on_hand_worked_rows():
    # a_drop is relative to the largest OFF-diagonal |a| of the row and the
    # dropped values are added to the diagonal:
    #  row 0: diag 10, off [1, 3/10]   tol 1/2 -> threshold 1/2: drop 3/10,
    #         diagonal 10 + 3/10 (not relative to the diagonal's 10, which
    #         would drop 1 as well)
    #  row 1: diag 4, off [-1, 1/5, 1/2] tol 1/4 -> drop 1/5: diagonal 4 + 1/5
    A = sp.csr_matrix((np.array([10.0, 1.0, 0.3, -1.0, 4.0, 0.2, 0.5]),
                       np.array([0, 1, 2, 0, 1, 2, 3]),
                       np.array([0, 3, 7])), shape=(2, 4))
    D0 = H.relative_drop(A[0:1], 0.5, True).toarray()
    assert np.array_equal(D0, np.array([[10.0 + 0.3, 1.0, 0.0, 0.0]]))
    # row 1 placed at index 1 of a square matrix, so that its diagonal is a_11
    A4 = sp.csr_matrix((np.array([1.0, -1.0, 4.0, 0.2, 0.5, 1.0, 1.0]),
                        np.array([0, 0, 1, 2, 3, 2, 3]),
                        np.array([0, 1, 5, 6, 7])), shape=(4, 4))
    D1 = H.relative_drop(A4, 0.25, True).toarray()
    assert np.array_equal(D1[1], np.array([-1.0, 4.0 + 0.2, 0.0, 0.5]))
    D1n = H.relative_drop(A4, 0.25, False).toarray()
    assert np.array_equal(D1n[1], np.array([-1.0, 4.0, 0.0, 0.5]))


# --------------------------------------------------------------------- Eq. fixed_sparsity on a pattern that is not closed

A3 = [[2.0, 1.0, 0.0],
      [3.0, 2.0, 1.0],
      [0.0, 1.0, 2.0]]


def test_fixed_sparsity_inverse_by_hand_on_a_tridiagonal_pattern():
    # A~^1 = A, A~^2 = mask(A A), A~^3 = mask(A~^2 A), by hand:
    #   A A        = [[7,4,1],[12,8,4],[3,4,5]]   -> A~^2 = [[7,4,0],[12,8,4],[0,4,5]]
    #   A~^2 A     = [[26,15,4],[48,32,16],[12,13,14]]
    #                                              -> A~^3 = [[26,15,0],[48,32,16],[0,13,14]]
    # and with alpha = (1/2, 1/4, 1/8, 1/16) the sum below.  Catches: no mask
    # (fill at (0,2) and (2,0)), a mask applied only to the final sum (exact
    # A^3 has 16 at (0,1), not 15), the product in the other order (A A~^2
    # has 16 at (0,1)), and a coefficient on the wrong power.
    alpha = np.array([0.5, 0.25, 0.125, 0.0625])
    got = H.fixed_sparsity_inverse(_csr(A3), alpha).toarray()
    want = np.array([[3.5, 1.6875, 0.0],
                     [5.25, 4.0, 1.75],
                     [0.0, 1.5625, 2.5]])
    assert np.array_equal(got, want)


def test_fixed_sparsity_inverse_on_a_bidiagonal_pattern_has_no_fill():
    # lower bidiagonal A_ff (diagonal d, subdiagonal l): on its own pattern the
    # masked powers are (A^k)_ii = d_i^k and
    # (A^k)_{i,i-1} = l_i sum_{j<k} d_i^j d_{i-1}^{k-1-j}; the exact powers
    # would add entries down to the k-th subdiagonal.
    r = np.random.default_rng(4)
    n, d = 9, 4
    dg = r.uniform(1.0, 2.0, n)
    lo = r.uniform(-1.0, 1.0, n - 1)
    A = _csr(np.diag(dg) + np.diag(lo, -1))
    alpha = r.uniform(-1.0, 1.0, d + 1)
    got = H.fixed_sparsity_inverse(A, alpha).toarray()
    want = np.zeros((n, n))
    for i in range(n):
        want[i, i] = sum(alpha[k] * dg[i] ** k for k in range(d + 1))
        if i > 0:
            want[i, i - 1] = sum(alpha[k] * lo[i - 1] * sum(dg[i] ** j * dg[i - 1] ** (k - 1 - j)
                                                            for j in range(k))
                                 for k in range(1, d + 1))
    assert np.allclose(got, want, rtol=1e-13, atol=1e-15)
    assert np.count_nonzero(np.tril(got, -2)) == 0 and np.count_nonzero(np.triu(got, 1)) == 0


def test_neumann_fixed_sparsity_by_hand_on_a_tridiagonal_pattern():
    # A = [[2,1,0],[3,4,1],[0,1,1]], D = diag(2,4,1), N = I - D^{-1} A on A's
    # pattern: [[0,-1/2,0],[-3/4,0,-1/4],[0,-1,0]].  By hand:
    #   N N     = [[3/8,0,1/8],[0,5/8,0],[3/4,0,1/4]] -> N~^2 = diag(3/8, 5/8, 1/4)
    #   N~^2 N  = [[0,-3/16,0],[-15/32,0,-5/32],[0,-1/4,0]] = N~^3 (inside the pattern)
    #   I + N + N~^2 + N~^3 = [[11/8,-11/16,0],[-39/32,13/8,-13/32],[0,-5/4,5/4]]
    # then column j is scaled by 1/a_jj = (1/2, 1/4, 1).  Catches: no mask
    # (fill at (0,2), (2,0)), row instead of column scaling, D^{-1} on the
    # wrong side, a sign slip in N.
    A = _csr([[2.0, 1.0, 0.0], [3.0, 4.0, 1.0], [0.0, 1.0, 1.0]])
    got = H.neumann_fixed_sparsity(A, 3).toarray()
    want = np.array([[0.6875, -0.171875, 0.0],
                     [-0.609375, 0.40625, -0.40625],
                     [0.0, -0.3125, 1.25]])
    assert np.array_equal(got, want)
    # degree 1: (I + N) D^{-1}
    got1 = H.neumann_fixed_sparsity(A, 1).toarray()
    want1 = np.array([[0.5, -0.125, 0.0], [-0.375, 0.25, -0.25], [0.0, -0.25, 1.0]])
    assert np.array_equal(got1, want1)


# --------------------------------------------------------------------- Loe-Morgan added roots and the Leja order (Sec. 2.3)

def test_added_roots_threshold_and_count_by_hand():
    # pof(k) = prod_{j != k} |1 - theta_k / theta_j|
    # {1, 10001.5}: pof(10001.5) = 10000.5, log10 = 4.0000217 > 4 -> one copy;
    #               pof(1) = |1 - 1/10001.5| < 1 -> none
    assert linalg.added_roots([1.0 + 0j, 10001.5 + 0j]) == [10001.5 + 0j]
    # {1, 9999}: pof = 9998, log10 < 4 -> no copies (threshold is log10 pof > 4)
    assert linalg.added_roots([1.0 + 0j, 9999.0 + 0j]) == []
    # {1, 2, 3, 1e8}: pof(1e8) = (1e8-1)(5e7-1)(1e8/3-1), log10 = 23.22
    # -> ceil((23.22 - 4) / 14) = 2 copies; the small roots have pof <= 1
    lp = math.log10((1e8 - 1) * (5e7 - 1) * (1e8 / 3 - 1))
    assert 23.2 < lp < 23.3
    assert linalg.added_roots([1.0 + 0j, 2.0 + 0j, 3.0 + 0j, 1e8 + 0j]) == [1e8 + 0j, 1e8 + 0j]
    # log10 pof just above 18 -> 2 copies, just below -> 1: {1, 1e18 + 1e15}
    # has pof = 1.001e18 - 1 (log10 18.0004), {1, 9.9e17} log10 17.9956
    assert len(linalg.added_roots([1.0 + 0j, 1.001e18 + 0j])) == 2
    assert len(linalg.added_roots([1.0 + 0j, 9.9e17 + 0j])) == 1


def test_added_roots_for_pairs_and_repeated_roots():
    # {1, +-1e5 i}: pof(1e5 i) = |1 - 1e5 i| * |1 - (1e5 i)/(-1e5 i)|
    #             = sqrt(1 + 1e10) * 2, log10 = 5.301 -> one copy of the PAIR
    got = linalg.added_roots([1.0 + 0j, 1e5j, -1e5j])
    assert sorted(got, key=lambda z: z.imag) == [-1e5j, 1e5j]
    # a repeated outlier: the product skips one copy of itself only, and
    # |1 - theta/theta| = 0 for the other copy, so no copies are added
    assert linalg.added_roots([1.0 + 0j, 1e8 + 0j, 1e8 + 0j]) == []


def test_leja_order_by_hand():
    # {4, -1, 2, 1+i, 1-i}: start at the largest modulus, 4; then the largest
    # product of distances to the roots taken:
    #   -1: 5,  2: 2,  1+i: sqrt(10)              -> -1
    #   2: 2*3 = 6,  1+i: sqrt(10)*sqrt(5) = 7.07 -> 1+i, then its conjugate
    #   2 last.
    # Catches: the smallest product, distances to the last root only (that
    # picks -1 and then 2: |2-(-1)| = 3 > |1+i-(-1)| = 2.24), and a pair split.
    got = linalg.leja_order([2.0 + 0j, 1 - 1j, -1.0 + 0j, 4.0 + 0j, 1 + 1j])
    assert got == [4.0 + 0j, -1.0 + 0j, 1 + 1j, 1 - 1j, 2.0 + 0j]


def test_leja_order_counts_both_members_of_a_pair():
    # {3, 2i, -2i, -2.5}: 3 first; then |2i - 3| = 3.606 vs |-2.5 - 3| = 5.5
    # -> -2.5; then the pair (2i: 3.606 * 3.202 = 11.5, the only candidate),
    # done.  With {3, 2i, -2i, -1.2, 0.1}: after 3, -1.2 (4.2 vs 3.606 and
    # 2.9), then 2i (3.606 * 2.332 = 8.41) over 0.1 (2.9 * 1.3 = 3.77), then
    # its conjugate; 0.1 is scored against all four taken roots, both members
    # of the pair included.
    assert linalg.leja_order([2j, 3.0 + 0j, -2.5 + 0j, -2j]) == [3.0 + 0j, -2.5 + 0j, 2j, -2j]
    assert linalg.leja_order([0.1 + 0j, -1.2 + 0j, 2j, -2j, 3.0 + 0j]) == \
        [3.0 + 0j, -1.2 + 0j, 2j, -2j, 0.1 + 0j]


def test_leja_order_is_greedy_by_brute_force():
    # every position holds the remaining root (a pair counts once) whose
    # product of distances to the roots before it is largest, checked with
    # plain products over random root sets
    r = np.random.default_rng(21)
    for trial in range(20):
        reals = list(r.uniform(0.2, 5.0, 4))
        pairs = [complex(a, b) for a, b in zip(r.uniform(0.2, 5.0, 2), r.uniform(0.1, 2.0, 2))]
        roots = [complex(x) for x in reals] + pairs + [z.conjugate() for z in pairs]
        out = linalg.leja_order(roots)
        assert abs(out[0]) == max(abs(z) for z in roots)
        i = 2 if out[0].imag != 0.0 else 1
        while i < len(out):
            before = out[:i]
            rest = [z for z in out[i:] if z.imag >= 0.0]
            score = lambda z: math.prod(abs(z - t) for t in before)  # noqa: E731
            assert score(out[i]) >= max(score(z) for z in rest) * (1 - 1e-12)
            i += 2 if out[i].imag != 0.0 else 1


# --------------------------------------------------------------------- the truncation decision (Sec. 2.4)

def _residual_by_product_form(A, roots, b):
    """b - A q(A) b = prod_i (I - A / theta_i) b for the Newton polynomial with
    these roots (a pair a +- ib as I - 2a/|theta|^2 A + A^2/|theta|^2), with
    dense matrices: an independent statement of what the Newton recurrence
    computes."""
    Ad = A.toarray()
    v = b.copy()
    i = 0
    while i < len(roots):
        z = roots[i]
        if z.imag == 0.0:
            v = v - Ad @ v / z.real
            i += 1
        else:
            m2 = z.real ** 2 + z.imag ** 2
            Av = Ad @ v
            v = v - (2.0 * z.real / m2) * Av + (Ad @ Av) / m2
            i += 2
    return v


def test_truncation_makes_the_first_passing_level_the_coarsest():
    p = workloads.fv_random(48, 0.3, True)
    A = p.scipy()
    base = Params()
    full = oracle.setup(A, Params(trunc_tol=0.0))
    assert full[-1].A.shape[0] <= base.min_coarse_rows < full[-2].A.shape[0]
    # the test residual of every level below the top, from the truncation
    # stream (purpose 4), for the roots built on the coarse stream (purpose 3)
    rels = {}
    for lvl in range(base.trunc_start_level, len(full) - 1):
        Al = full[lvl].A
        n = Al.shape[0]
        roots = linalg.newton_roots(Al, rng.uniform(base.seed, rng.COARSE_RHS, lvl, n),
                                    base.coarse_poly_order, base.added_roots)
        bt = rng.uniform(base.seed, rng.TRUNC_RHS, lvl, n)
        rel = np.linalg.norm(_residual_by_product_form(Al, roots, bt)) / np.linalg.norm(bt)
        if rel < 1e-12:
            # a polynomial that is exact on this level: both forms only show
            # rounding, which they reach in different ways
            continue
        rels[lvl] = rel
        # the stream matters: the coarse stream's own vector gives another residual
        bc = rng.uniform(base.seed, rng.COARSE_RHS, lvl, n)
        other = np.linalg.norm(_residual_by_product_form(Al, roots, bc)) / np.linalg.norm(bc)
        assert abs(other - rels[lvl]) > 1e-6 * rels[lvl]
    assert len(rels) >= 2
    checked = 0
    for stop in sorted(rels):
        tol = rels[stop] * (1 + 1e-7)
        if any(rels[l] <= tol for l in rels if l < stop):
            continue
        lv = oracle.setup(A, Params(trunc_tol=tol))
        # levels 0..stop, the last one coarsest, with the untruncated A_stop
        assert len(lv) == stop + 1 and lv[-1].coarsest
        assert abs(lv[-1].A - full[stop].A).max() == 0.0
        assert lv[0].trunc_rel is None                 # the test starts at level 1
        for l in range(1, stop + 1):
            assert lv[l].trunc_rel == pytest.approx(rels[l], rel=1e-8)
        checked += 1
    assert checked >= 2
    # a tolerance below rounding truncates nothing
    lv = oracle.setup(A, Params(trunc_tol=1e-30))
    assert len(lv) == len(full)
