"""V-cycle, FGMRES outer loop, adjoint solve and gradients, in FP64.

V-cycle (Sec. 2): no down smoothing; restrict r_c' = Z r_f + r_c (R = [Z I]),
recurse, prolong e_f = W e_c (P = [W; I]), then one up F-point smooth
(Eq. f_point) with the smoother polynomial applied matrix-free by Horner:
e_f += q(A_ff) (r_f - A_fc e_c - A_ff e_f).  The coarsest level applies its
Newton polynomial.  The FC and FCF variants add a C-point smooth
e_c += q_c(A_cc) (r_c - A_cf e_f - A_cc e_c) after it (and then a second F
smooth), with a GMRES polynomial of A_cc built the same way.

Outer loop: the paper uses undamped Richardson from an initial guess of one
(Sec. 3), available as `richardson`; the default workloads use
right-preconditioned FGMRES(restart) from x0 = 0 with classical Gram-Schmidt
applied twice, stopping when the Arnoldi residual estimate reaches rtol |b|
and the true residual |b - A x| confirms it.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import linalg
from .params import Params
from .hierarchy import setup


def vcycle(levels, r, lvl=0, exact_coarse=False, assembled=False, neumann=False,
           smooth_type="f"):
    """One V-cycle applied to r.  assembled: the F-point smoother applies the
    assembled fixed-sparsity Ahat^{-1} (one product, Sec. 2.2) instead of the
    polynomial matrix-free.  neumann: the matrix-free polynomial is nAIR's
    Jacobi-scaled Neumann polynomial of the same degree.  smooth_type: the
    up-smooths after the coarse-grid correction, in order ("f", "fc", "fcf"):
    an F smooth is e_f += Abar_ff^{-1} (r_f - A_ff e_f - A_fc e_c) (Eq. f_point),
    a C smooth is e_c += Abar_cc^{-1} (r_c - A_cf e_f - A_cc e_c) with the
    level's C-point polynomial (Sec. 2)."""
    L = levels[lvl]
    if L.coarsest:
        if exact_coarse:
            return spla.spsolve(sp.csc_matrix(L.A), r)
        return linalg.newton_apply(L.A, L.roots, r)
    rf = r[L.F]
    rc = r[L.C]
    rc2 = linalg.spmv(L.Z, rf) + rc
    ec = vcycle(levels, rc2, lvl + 1, exact_coarse, assembled, neumann, smooth_type)
    ef = np.where(L.cmap >= 0, ec[np.maximum(L.cmap, 0)], 0.0)
    for step in smooth_type:
        if step == "f":
            s = rf - linalg.spmv(L.Afc, ec) - linalg.spmv(L.Aff, ef)
            if assembled:
                ef = ef + linalg.spmv(L.Ahat, s)
            elif neumann:
                ef = ef + linalg.neumann_apply(L.Aff, len(L.alpha) - 1, s)
            else:
                ef = ef + linalg.horner_apply(L.Aff, L.alpha, s)
        elif step == "c":
            t = rc - linalg.spmv(L.Acf, ef) - linalg.spmv(L.Acc, ec)
            if assembled:
                ec = ec + linalg.spmv(L.Ahat_cc, t)
            else:
                ec = ec + linalg.horner_apply(L.Acc, L.alpha_c, t)
        else:
            raise ValueError(f"unknown smooth step {step!r}")
    e = np.zeros(len(r))
    e[L.F] = ef
    e[L.C] = ec
    return e


def fgmres(A, precond, b, rtol=1e-10, max_it=500, restart=30, x0=None, atol=0.0):
    """Returns (x, iterations, true relative residual, estimate history).  A
    residual norm at or below max(rtol |b|, atol) stops the iteration (the
    paper's option set has both tolerances, Sec. 3)."""
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0, hist
    tol = max(rtol * bnorm, atol)
    its = 0
    while True:
        r = b - linalg.spmv(A, x)
        beta = linalg.norm(r)
        if beta <= tol or its >= max_it:
            return x, its, beta / bnorm, hist
        V = [r / beta]
        Zs = []
        H = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        k = 0
        for j in range(restart):
            z = precond(V[j])
            Zs.append(z)
            w = linalg.spmv(A, z)
            its += 1
            for _ in range(2):
                h = np.array([linalg.dot(V[i], w) for i in range(j + 1)])
                for i in range(j + 1):
                    w = w - h[i] * V[i]
                H[:j + 1, j] += h
            H[j + 1, j] = linalg.norm(w)
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            a, c = H[j, j], H[j + 1, j]
            rr = math.hypot(a, c)
            cs[j], sn[j] = (a / rr, c / rr) if rr > 0 else (1.0, 0.0)
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            est = abs(g[j + 1])
            hist.append(est / bnorm)
            if est <= tol or its >= max_it:
                break
            hn = linalg.norm(w)
            V.append(w / hn)
        y = np.zeros(k)
        for i in reversed(range(k)):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * Zs[i]


def richardson(A, precond, b, rtol=1e-10, max_it=500, x0=None, atol=0.0):
    """Undamped Richardson, x <- x + M (b - A x), the paper's outer loop (Sec. 3),
    stopped on the unpreconditioned residual: |b - A x| <= rtol |b|, or
    rtol |b - A x0| when b = 0 (the paper's runs have g = 0 and x0 = 1).
    Returns (x, iterations, relative residual, residual-norm history)."""
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - linalg.spmv(A, x)
    rn = linalg.norm(r)
    bnorm = linalg.norm(b)
    ref = bnorm if bnorm > 0.0 else rn
    hist = [rn]
    if ref == 0.0:
        return x, 0, 0.0, hist
    its = 0
    while rn > max(rtol * ref, atol) and its < max_it:
        x = x + precond(r)
        r = b - linalg.spmv(A, x)
        rn = linalg.norm(r)
        hist.append(rn)
        its += 1
    return x, its, rn / ref, hist


def solve(A, b, p=None, levels=None, x0=None):
    """Set up (unless `levels` is given) and solve A x = b with the outer loop
    p.outer (FGMRES, or the paper's Richardson).  x0: the initial guess (zero
    if None).  Returns (x, iterations, relative residual, levels, history)."""
    p = p or Params()
    A = sp.csr_matrix(A)
    if levels is None:
        levels = setup(A, p)
    if p.smoother not in ("poly", "assembled"):
        raise ValueError(f"unknown smoother {p.smoother!r}")
    if p.inverse_type not in ("arnoldi", "neumann"):
        raise ValueError(f"unknown inverse type {p.inverse_type!r}")
    if p.smooth_type not in ("f", "fc", "fcf"):
        raise ValueError(f"unknown smooth type {p.smooth_type!r}")
    M = lambda v: vcycle(levels, v, 0, p.exact_coarse, p.smoother == "assembled",  # noqa: E731
                         p.inverse_type == "neumann", p.smooth_type)
    if p.outer == "richardson":
        x, its, rel, hist = richardson(A, M, b, p.rtol, p.max_it, x0, p.atol)
    elif p.outer == "fgmres":
        x, its, rel, hist = fgmres(A, M, b, p.rtol, p.max_it, p.restart, x0, p.atol)
    else:
        raise ValueError(f"unknown outer loop {p.outer!r}")
    return x, its, rel, levels, hist


def adjoint_solve(A, w, p=None, levels_t=None):
    """Solve A^T lam = w with a hierarchy built on the explicit transpose (same
    parameters and seed)."""
    At = sp.csr_matrix(A.T)
    At.sort_indices()
    return solve(At, w, p, levels_t)


def loss_gradients(problem, u, lam):
    """Gradients of loss = sum_i w_i u_i (u = A^-1 b) given the adjoint solution
    lam = A^-T w_full:
      d loss / d g_W(j) = vx lam at the west inflow cell of row j,
      d loss / d g_S(i) = vy lam at the south inflow cell of column i,
      d loss / d theta  = lam^T (db/dtheta - dA/dtheta u)."""
    vx, vy = math.cos(problem.theta), math.sin(problem.theta)
    dgw = vx * lam[problem.west_rows]
    dgs = vy * lam[problem.south_rows]
    n = problem.n
    dA = sp.csr_matrix((problem.ddata_dtheta, problem.indices, problem.indptr), shape=(n, n))
    dtheta = float(np.dot(lam, problem.db_dtheta - dA @ u))
    return dgw, dgs, dtheta
