"""Exact solves of upwind systems by a sweep (Sec. 1.1).

An upwind discretisation is lower triangular in flow order, so one Gauss-Seidel
pass in that order gives the exact discrete solution.  `level` assigns every
unknown a flow-order level (for the FV grid, i + j); every off-diagonal
dependency must point to a strictly lower level, which is checked.  Unknowns of
one level are independent and are solved together.  The adjoint system A^T is
swept with the levels reversed.
"""
import numpy as np
import scipy.sparse as sp


def sweep_solve(A, b, level, transpose=False):
    A = sp.csr_matrix(A)
    lev = np.asarray(level, dtype=np.int64)
    if transpose:
        A = sp.csr_matrix(A.T)
        lev = -lev
    A.sort_indices()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    off = A.indices != rows
    if np.any(lev[A.indices[off]] >= lev[rows[off]]):
        raise ValueError("matrix is not triangular in the given flow order")
    diag = A.diagonal()
    O = sp.csr_matrix((np.where(off, A.data, 0.0), A.indices, A.indptr), shape=A.shape)
    order = np.argsort(lev, kind="stable")
    slev = lev[order]
    cuts = np.nonzero(np.diff(slev))[0] + 1
    x = np.zeros(n)
    for grp in np.split(order, cuts):
        x[grp] = (b[grp] - O[grp] @ x) / diag[grp]
    return x
