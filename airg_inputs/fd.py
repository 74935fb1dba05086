"""The paper's own discretisation (Sec. 3): first-order upwind finite
differences for v.grad(u) = 0 on an N x N grid of nodes covering the unit
square, non-dimensionalised by the mesh spacing so the stencil does not change
with refinement, with the inflow boundary nodes kept as unknowns.

With v = (cos t, sin t), t in [0, pi/2], node (i, j) with i > 0 and j > 0 gives

    (vx + vy) u_ij - vx u_{i-1,j} - vy u_{i,j-1} = 0,

and every node on the left (i = 0) or bottom (j = 0) boundary is an inflow
node whose row states u = g.  The paper does not say how those rows are
scaled; they are read as identity rows (diagonal 1, right-hand side g).
Unknown k = j N + i, so the matrix is lower triangular in natural order; the
flow-order level of a node is i + j.
"""
from dataclasses import dataclass
import math

import numpy as np

from . import rng


@dataclass
class FDProblem:
    nx: int
    ny: int
    theta: float
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    b: np.ndarray
    g: float
    order: np.ndarray = None
    level: np.ndarray = None

    @property
    def n(self):
        return self.nx * self.ny

    @property
    def nnz(self):
        return int(self.indptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def fd_advection(nx, theta=math.pi / 4.0, g=0.0, perm_seed=None, ny=None):
    """Assemble the FD system above (g: the constant inflow value)."""
    ny = nx if ny is None else ny
    if not (0.0 <= theta <= 0.5 * math.pi):
        raise ValueError("theta must lie in [0, pi/2] so that inflow is left/bottom")
    vx, vy = math.cos(theta), math.sin(theta)
    n = nx * ny
    k = np.arange(n, dtype=np.int64)
    i, j = k % nx, k // nx
    bnd = (i == 0) | (j == 0)
    # three slots per row (south, west, diagonal), ascending columns
    cols = np.stack([k - nx, k - 1, k], axis=1)
    vals = np.empty((n, 3))
    vals[:, 0], vals[:, 1], vals[:, 2] = -vy, -vx, vx + vy
    mask = np.stack([~bnd & (vy != 0.0), ~bnd & (vx != 0.0), np.ones(n, dtype=bool)], axis=1)
    vals[bnd, 2] = 1.0
    b = np.where(bnd, float(g), 0.0)
    level = (i + j).astype(np.int64)
    order = None
    if perm_seed is not None:
        keys = rng.uniform(perm_seed, rng.PERM, 0, n)
        order = np.argsort(keys, kind="stable").astype(np.int64)
        inv = np.empty(n, dtype=np.int64)
        inv[order] = np.arange(n, dtype=np.int64)
        big = np.iinfo(np.int64).max
        cols, vals, mask = cols[order], vals[order], mask[order]
        cols = np.where(mask, inv[np.where(mask, cols, 0)], big)
        srt = np.argsort(cols, axis=1, kind="stable")
        cols = np.take_along_axis(cols, srt, axis=1)
        vals = np.take_along_axis(vals, srt, axis=1)
        mask = np.take_along_axis(mask, srt, axis=1)
        b, level = b[order], level[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=indptr[1:])
    return FDProblem(nx=nx, ny=ny, theta=float(theta), indptr=indptr.astype(np.int32),
                     indices=cols[mask].astype(np.int32), data=vals[mask].copy(), b=b,
                     g=float(g), order=order, level=level)
