"""AIRG hierarchy setup, level by level, following Sec. 2 of the paper.

On each level l with matrix A_l:
  1. automatic truncation test (Sec. 2.4): build the tentative coarse Newton
     polynomial and apply it to a different random b; stop if it reaches the
     tolerance;
  2. CF splitting (Sec. 2.1): strength matrix S, PMISR (a Luby-type independent
     set of F points in S + S^T), then DDC passes;
  3. extraction of A_ff, A_fc, A_cf (Eq. air_two);
  4. smoother coefficients (Eq. gmres_poly) by Arnoldi on a random b;
  5. the fixed-sparsity assembled inverse (Eq. fixed_sparsity);
  6. the approximate ideal restrictor Z = -A_cf Ahat^{-1}, relatively dropped;
  7. the classical one-point prolongator W;
  8. A_{l+1} = R A_l P (Eqs. prolong, z), relatively dropped and lumped to the
     diagonal.

Readings of points the paper leaves open are stated at each function.  Every
row-wise sum runs left to right in ascending column order; sparse products are
scipy's CSR product, which accumulates c_ij over k in ascending order from 0 and
keeps no exact zeros.
"""
from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

from . import linalg, rng
from .params import Params

UNDECIDED, FPT, CPT = 0, 1, 2
DDC_BINS = 1000
ONE_POINT_TIE = 1.0 - 1e-12


class ZeroDiagonal(ArithmeticError):
    pass


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M


def diagonal_of(A):
    """Diagonal values; raises ZeroDiagonal if any row lacks a nonzero one."""
    d = A.diagonal()
    if np.any(d == 0.0) or not np.all(np.isfinite(d)):
        raise ZeroDiagonal("zero or missing diagonal")
    return d


def _rows(A):
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def seq_row_sums(A, vals, mask, init=None):
    """Per row: init + sum of vals[p] over the entries p with mask[p], added left
    to right in ascending column order (init defaults to 0.0)."""
    n = A.shape[0]
    out = np.zeros(n) if init is None else np.array(init, dtype=np.float64, copy=True)
    lens = np.diff(A.indptr)
    if n == 0 or A.nnz == 0:
        return out
    start = A.indptr[:-1].astype(np.int64)
    order = np.argsort(-lens, kind="stable")
    slens = lens[order]
    for k in range(int(slens[0])):
        cnt = int(np.searchsorted(-slens, -k, side="left"))
        rows = order[:cnt]
        p = start[rows] + k
        upd = mask[p]
        out[rows[upd]] = out[rows[upd]] + vals[p][upd]
    return out


def row_abs_max(A, mask):
    """max |a_ij| over the masked entries of each row (0 for none)."""
    n = A.shape[0]
    out = np.zeros(n)
    if A.nnz:
        rows = _rows(A)
        np.maximum.at(out, rows[mask], np.abs(A.data[mask]))
    return out


# ---------------------------------------------------------------------------
# CF splitting (Sec. 2.1)
# ---------------------------------------------------------------------------

def strength(A, theta_s):
    """S_ij = 1 iff j != i, a_ij != 0 and |a_ij| >= theta_s * max_{k != i} |a_ik|.

    Reading: absolute values (the level matrices are asymmetric with mixed
    signs); with theta_s = 0 every off-diagonal connection is strong, so the F
    points become a maximal independent set of A's graph (Sec. 2).
    """
    rows = _rows(A)
    off = A.indices != rows
    m = row_abs_max(A, off)
    thr = theta_s * m
    strong = off & (A.data != 0.0) & (np.abs(A.data) >= thr[rows])
    S = sp.csr_matrix((np.ones(int(strong.sum())), (rows[strong], A.indices[strong])),
                      shape=A.shape)
    return _csr(S)


def pmisr(S, weights):
    """Luby-type independent set of F points in G = S + S^T (Sec. 2.1), run
    until every point is decided.

    Each round, an undecided point whose (weight, index) beats that of every
    undecided G-neighbour becomes F; then every undecided G-neighbour of a new
    F point becomes C.  Points isolated in G become F.  Returns (state, rounds).
    Reading: plain seeded random weights (the measure is not given).
    """
    n = S.shape[0]
    G = _csr(S + S.T)
    gr = _rows(G)
    gc = G.indices.astype(np.int64)
    state = np.zeros(n, dtype=np.int8)
    rounds = 0
    while np.any(state == UNDECIDED):
        rounds += 1
        und = state == UNDECIDED
        both = und[gr] & und[gc]
        nb_wins = (weights[gc] > weights[gr]) | ((weights[gc] == weights[gr]) & (gc > gr))
        lose = np.zeros(n, dtype=bool)
        lose[gr[both & nb_wins]] = True
        new_f = und & ~lose
        state[new_f] = FPT
        touch = np.zeros(n, dtype=bool)
        touch[gr[new_f[gc]]] = True
        state[(state == UNDECIDED) & touch] = CPT
    return state, rounds


def ddc_ratios(A, state, diag):
    """r_i = sum_{j in F, j != i} |a_ij| / |a_ii| for F rows (0 elsewhere)."""
    rows = _rows(A)
    isf = state == FPT
    mask = isf[A.indices] & (A.indices != rows) & isf[rows]
    s = seq_row_sums(A, np.abs(A.data), mask)
    r = np.zeros(A.shape[0])
    r[isf] = s[isf] / np.abs(diag[isf])
    return r


def ddc_pass(A, state, diag, fraction):
    """One diagonal dominance cleanup pass (Sec. 2.1): convert about `fraction`
    of the F points, the least diagonally dominant, to C.

    Readings: k = ceil(fraction * n_F); the ratios r > 0 of the F rows go into
    1000 equal bins on [0, r_max] with bin = min(999, floor(r / r_max * 1000));
    scanning down from the top bin, b* is the first bin where the running count
    reaches k; the cut is placed on the bin boundary (b* or b*+1) whose count is
    closer to k, a tie converting more.  Rows with r = 0 are never converted.
    Returns the number converted.
    """
    isf = state == FPT
    nf = int(isf.sum())
    if nf == 0:
        return 0
    r = ddc_ratios(A, state, diag)
    rmax = float(r[isf].max())
    if rmax == 0.0:
        return 0
    k = int(math.ceil(fraction * nf))
    elig = isf & (r > 0.0)
    bins = np.minimum(DDC_BINS - 1, np.floor((r / rmax) * 1000.0)).astype(np.int64)
    counts = np.bincount(bins[elig], minlength=DDC_BINS)
    cum = 0
    bstar = 0
    for b in range(DDC_BINS - 1, -1, -1):
        cum += int(counts[b])
        if cum >= k:
            bstar = b
            break
    above = cum - int(counts[bstar])
    edge = bstar if (cum - k) <= (k - above) else bstar + 1
    conv = elig & (bins >= edge)
    state[conv] = CPT
    return int(conv.sum())


def cf_split(A, level, p):
    diag = diagonal_of(A)
    S = strength(A, p.strong_threshold)
    w = rng.uniform(p.seed, rng.PMISR, level, A.shape[0])
    state, rounds = pmisr(S, w)
    n_f_pmisr = int((state == FPT).sum())
    converted = []
    for _ in range(p.ddc_its):
        converted.append(ddc_pass(A, state, diag, p.ddc_fraction))
    return state, dict(pmisr_rounds=rounds, n_f_pmisr=n_f_pmisr, ddc_converted=converted)


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------

def neumann_fixed_sparsity(Aff, d):
    """The assembled Neumann approximation of nAIR with fixed sparsity:
    Ahat^{-1} = (I + N~ + N~^2 + ... + N~^d) D^{-1}, N = I - D^{-1} A_ff kept on
    A_ff's pattern (a zero diagonal), N~^1 = N and N~^k = (N~^{k-1} N)
    restricted to A_ff's pattern, as for the GMRES polynomial (Eq.
    fixed_sparsity); the sum runs left to right, then column j is scaled by
    1 / a_jj."""
    n = Aff.shape[0]
    pattern = Aff.copy()
    pattern.data = np.ones_like(pattern.data)
    diag = Aff.diagonal()
    rows = np.repeat(np.arange(n), np.diff(Aff.indptr))
    N = Aff.copy()
    N.data = np.where(Aff.indices == rows, 0.0, -Aff.data / diag[rows])
    S = _csr(sp.identity(n, format="csr"))
    if d >= 1:
        S = _csr(S + N)
    Pk = N
    for _ in range(2, d + 1):
        Pk = _csr((Pk @ N).multiply(pattern))
        S = _csr(S + Pk)
    S = S.copy()
    S.data = S.data * (1.0 / diag)[S.indices]
    return S


def fixed_sparsity_inverse(Aff, alpha):
    """Ahat^{-1} = alpha_0 I + alpha_1 A_ff + alpha_2 A~^2 + ... (Eq. fixed_sparsity)
    with A~^1 = A_ff and A~^k = (A~^{k-1} A_ff) restricted to the sparsity of A_ff
    (reading: the mask is applied to every power in turn)."""
    n = Aff.shape[0]
    pattern = Aff.copy()
    pattern.data = np.ones_like(pattern.data)
    Ahat = _csr(alpha[0] * sp.identity(n, format="csr"))
    if len(alpha) > 1:
        Ahat = _csr(Ahat + alpha[1] * Aff)
    Pk = Aff
    for k in range(2, len(alpha)):
        Pk = _csr((Pk @ Aff).multiply(pattern))
        Ahat = _csr(Ahat + alpha[k] * Pk)
    return Ahat


def relative_drop(M, tol, lump):
    """Drop off-diagonal entries with |m_ij| < tol * max_{k != i} |m_ik|; with
    `lump` the dropped values are added to the diagonal: d + l_1 + l_2 + ...
    left to right in ascending column order (Sec. 2)."""
    n = M.shape[0]
    rows = _rows(M)
    off = M.indices != rows
    m = row_abs_max(M, off)
    drop = off & (np.abs(M.data) < (tol * m)[rows])
    data = M.data.copy()
    if lump and drop.any():
        diag_pos = np.full(n, -1, dtype=np.int64)
        dpos = np.nonzero(~off)[0]
        diag_pos[rows[dpos]] = dpos
        if np.any(diag_pos[np.unique(rows[drop])] < 0):
            raise ZeroDiagonal("lumping into a missing diagonal")
        has = diag_pos >= 0
        init = np.zeros(n)
        init[has] = M.data[diag_pos[has]]
        lumped = seq_row_sums(M, M.data, drop, init)
        data[diag_pos[has]] = lumped[has]
    keep = ~drop
    ptr = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=n))])
    return sp.csr_matrix((data[keep], M.indices[keep], ptr), shape=M.shape)


def restrictor_drop(Z, tol):
    """Drop |z_ij| < tol * max_j |z_ij| in each row of Z (no lumping)."""
    rows = _rows(Z)
    m = row_abs_max(Z, np.ones(Z.nnz, dtype=bool))
    keep = np.abs(Z.data) >= (tol * m)[rows]
    return sp.csr_matrix((Z.data[keep], Z.indices[keep],
                          np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=Z.shape[0]))])),
                         shape=Z.shape)


def one_point(A, state, cidx):
    """Classical one-point prolongation (Sec. 2): each F point takes the value of
    the C point it is most strongly connected to, |a_ij| largest over C columns
    j of its row, with weight 1.  Reading of ties: magnitudes within a relative
    1e-12 of the largest count as equal and the lowest column wins.  An F point
    with no C neighbour gets no interpolation (W row empty).
    Returns cmap: coarse index per F point, or -1."""
    rows = _rows(A)
    isc = state[A.indices] == CPT
    isf_row = state[rows] == FPT
    sel = isc & isf_row
    m = row_abs_max(A, sel)
    thr = m * ONE_POINT_TIE
    cand = sel & (np.abs(A.data) >= thr[rows])
    n = A.shape[0]
    best = np.full(n, np.iinfo(np.int64).max)
    np.minimum.at(best, rows[cand], A.indices[cand].astype(np.int64))
    fidx = np.nonzero(state == FPT)[0]
    cm = best[fidx]
    cmap = np.full(len(fidx), -1, dtype=np.int64)
    ok = cm != np.iinfo(np.int64).max
    cmap[ok] = cidx[cm[ok]]
    return cmap


@dataclass
class Level:
    A: sp.csr_matrix
    coarsest: bool = False
    state: np.ndarray = None
    F: np.ndarray = None
    C: np.ndarray = None
    Aff: sp.csr_matrix = None
    Afc: sp.csr_matrix = None
    Acf: sp.csr_matrix = None
    Z: sp.csr_matrix = None          # n_C x n_F after the relative drop
    cmap: np.ndarray = None          # W: F point -> coarse index (or -1)
    alpha: np.ndarray = None         # smoother coefficients alpha_0..alpha_d
    Ahat: sp.csr_matrix = None       # the assembled fixed-sparsity Ahat^{-1} (Eq. fixed_sparsity)
    Acc: sp.csr_matrix = None        # C-point smoothing only: A_cc,
    alpha_c: np.ndarray = None       # its GMRES polynomial coefficients
    Ahat_cc: sp.csr_matrix = None    # and its fixed-sparsity assembly
    roots: list = None               # Newton roots (coarsest level)
    trunc_rel: float = None          # truncation test result on this level
    info: dict = field(default_factory=dict)


def newton_for_level(A, level, p):
    b = rng.uniform(p.seed, rng.COARSE_RHS, level, A.shape[0])
    return linalg.newton_roots(A, b, p.coarse_poly_order, p.added_roots)


def truncation_test(A, roots, level, p):
    """Relative residual of the tentative coarse solve on a second random b."""
    b = rng.uniform(p.seed, rng.TRUNC_RHS, level, A.shape[0])
    x = linalg.newton_apply(A, roots, b)
    return linalg.norm(b - linalg.spmv(A, x)) / linalg.norm(b)


def coarsen(A, level, p):
    """Steps 2-8 on one level; returns (Level, A_next)."""
    n = A.shape[0]
    state, info = cf_split(A, level, p)
    F = np.nonzero(state == FPT)[0]
    C = np.nonzero(state == CPT)[0]
    L = Level(A=A, state=state, F=F, C=C, info=info)
    if len(C) == 0 or len(F) == 0:
        return L, None
    Ar = A[F]
    Aff = _csr(Ar[:, F])
    Afc = _csr(Ar[:, C])
    Acf = _csr(A[C][:, F])
    if p.inverse_type == "neumann":
        alpha = np.zeros(p.poly_order + 1)   # unused: the Neumann polynomial has no coefficients
        Ahat = neumann_fixed_sparsity(Aff, p.poly_order)
    else:
        bpoly = rng.uniform(p.seed, rng.POLY_RHS, level, len(F))
        alpha = linalg.gmres_poly_coeffs(Aff, bpoly, p.poly_order)
        Ahat = fixed_sparsity_inverse(Aff, alpha)
    Z = _csr(-(Acf @ Ahat))
    Z = _csr(restrictor_drop(Z, p.r_drop))
    cidx = np.full(n, -1, dtype=np.int64)
    cidx[C] = np.arange(len(C))
    cmap = one_point(A, state, cidx)
    nC = len(C)
    # R = [Z I] and P = [W; I] in level numbering
    zr = _rows(Z)
    R = _csr(sp.csr_matrix((np.concatenate([Z.data, np.ones(nC)]),
                            (np.concatenate([zr, np.arange(nC)]),
                             np.concatenate([F[Z.indices], C]))), shape=(nC, n)))
    fw = cmap >= 0
    P = _csr(sp.csr_matrix((np.ones(int(fw.sum()) + nC),
                            (np.concatenate([F[fw], C]), np.concatenate([cmap[fw], np.arange(nC)]))),
                           shape=(n, nC)))
    AP = _csr(A @ P)
    Ac = _csr(R @ AP)
    Ac = _csr(relative_drop(Ac, p.a_drop, p.lump))
    diagonal_of(Ac)
    L.Aff, L.Afc, L.Acf, L.Z, L.cmap, L.alpha = Aff, Afc, Acf, Z, cmap, alpha
    L.Ahat = Ahat
    if "c" in p.smooth_type:
        c_point_smoother(A, L, level, p)
    return L, Ac


def c_point_smoother(A, L, level, p):
    """C-point smoothing (FC / FCF, Sec. 2 and Sec. 3.3): the paper names it and
    its storage (A_cc and A_cf kept on every level) but not its inverse.
    Reading: the same construction as the F-point smoother, on A_cc: the
    GMRES polynomial of degree d from (d+1)-step Arnoldi with its own random
    right-hand side, applied matrix-free or assembled on A_cc's pattern."""
    if p.inverse_type != "arnoldi":
        raise ValueError("C-point smoothing uses the GMRES polynomial")
    Acc = _csr(A[L.C][:, L.C])
    b = rng.uniform(p.seed, rng.CPOLY_RHS, level, len(L.C))
    L.Acc = Acc
    L.alpha_c = linalg.gmres_poly_coeffs(Acc, b, p.poly_order)
    L.Ahat_cc = fixed_sparsity_inverse(Acc, L.alpha_c)


def setup(A, p=None):
    """Build the hierarchy for the CSR matrix A (scipy)."""
    p = p or Params()
    A = _csr(A)
    diagonal_of(A)
    levels = []
    for lvl in range(p.max_levels):
        n = A.shape[0]
        last = n <= p.min_coarse_rows or lvl == p.max_levels - 1
        roots = None
        trunc_rel = None
        if not last and p.trunc_tol > 0 and lvl >= p.trunc_start_level:
            roots = newton_for_level(A, lvl, p)
            trunc_rel = truncation_test(A, roots, lvl, p)
            last = trunc_rel <= p.trunc_tol
        if not last:
            L, Anext = coarsen(A, lvl, p)
            L.trunc_rel = trunc_rel
            if Anext is not None:
                levels.append(L)
                A = Anext
                continue
        if roots is None:
            roots = newton_for_level(A, lvl, p)
        levels.append(Level(A=A, coarsest=True, roots=roots, trunc_rel=trunc_rel))
        break
    return levels
