"""Upwind discontinuous Galerkin discretisation of v.grad(u) = 0 with bilinear
(Q1) elements on a structured Nx x Ny grid of square cells.

The paper gives no DG details, so this is a reading of the standard upwind DG
method: on each cell, for every test function phi,

    - int_K u v.grad(phi) + int_{dK} (v.n) u_up phi = 0,

where u_up is the cell's own trace on outflow faces and the upwind neighbour's
trace (or the inflow value g) on inflow faces.  With v = (cos t, sin t),
t in [0, pi/2], the west and south faces of a cell are its inflow faces.

Basis: nodal bilinear functions at the cell vertices, local node (a, b) with
a, b in {0, 1} (a along x, b along y), phi_ab(xi, eta) = psi_a(xi) psi_b(eta),
psi_0 = 1 - t, psi_1 = t on the reference cell [0, 1]^2.  All integrals are
exact; everything is divided by h (as in the FV discretisation), which leaves
the 1D matrices

    M = [[1/3, 1/6], [1/6, 1/3]]          M_ac = int psi_a psi_c
    D = [[-1/2, -1/2], [1/2, 1/2]]        D_ac = int psi_c psi_a'

and, for test node (a, b) and trial node (c, d),

    own cell:   -vx D_ac M_bd - vy M_ac D_bd + vx [a=1][c=1] M_bd + vy [b=1][d=1] M_ac
    west cell:  -vx [a=0] M_bd        (trial node (1, d) of the west neighbour)
    south cell: -vy [b=0] M_ac        (trial node (c, 1) of the south neighbour)
    inflow:     b_ab += vx g_W / 2 on a = 0 nodes, vy g_S / 2 on b = 0 nodes.

Element-block scaling (the default) multiplies each cell's four rows by the
inverse of the own-cell block, so the own block becomes the identity and each
row keeps 1 + 2 + 2 nonzeros.  The scaled system is then lower triangular in
the cell order i + j (the four unknowns of a cell do not couple), which the
sweep of the oracle uses.

Unknown 4 (j Nx + i) + 2 b + a; an optional seeded symmetric permutation hides
that ordering from the solver.
"""
from dataclasses import dataclass
import math

import numpy as np

from . import rng

M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
D1 = np.array([[-0.5, -0.5], [0.5, 0.5]])


@dataclass
class DGProblem:
    nx: int
    ny: int
    theta: float
    indptr: np.ndarray      # int32 [n+1]
    indices: np.ndarray     # int32 [nnz], ascending within each row
    data: np.ndarray        # float64 [nnz]
    b: np.ndarray           # float64 [n]
    g_west: np.ndarray      # float64 [ny]
    g_south: np.ndarray     # float64 [nx]
    scaled: bool = True
    order: np.ndarray = None   # unknown p of the (permuted) system is natural unknown order[p]
    level: np.ndarray = None   # i + j of the unknown's cell (flow order, for sweeps)

    @property
    def n(self):
        return 4 * self.nx * self.ny

    @property
    def nnz(self):
        return int(self.indptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def element_blocks(theta):
    """The 4x4 own, west and south coupling blocks (rows: test node 2b + a,
    columns: trial node 2d + c of the cell named), unscaled."""
    vx, vy = math.cos(theta), math.sin(theta)
    own = np.zeros((4, 4))
    west = np.zeros((4, 4))
    south = np.zeros((4, 4))
    for a in range(2):
        for b in range(2):
            r = 2 * b + a
            for c in range(2):
                for d in range(2):
                    q = 2 * d + c
                    v = -vx * D1[a, c] * M1[b, d] - vy * M1[a, c] * D1[b, d]
                    if a == 1 and c == 1:
                        v += vx * M1[b, d]
                    if b == 1 and d == 1:
                        v += vy * M1[a, c]
                    own[r, q] = v
                    if a == 0 and c == 1:
                        west[r, q] = -vx * M1[b, d]
                    if b == 0 and d == 1:
                        south[r, q] = -vy * M1[a, c]
    return own, west, south


def dg_advection(nx, theta, g_west, g_south, perm_seed=None, ny=None, scaled=True):
    """Assemble the upwind DG-Q1 system (see the module docstring)."""
    ny = nx if ny is None else ny
    if not (0.0 <= theta <= 0.5 * math.pi):
        raise ValueError("theta must lie in [0, pi/2] so that inflow is west/south")
    vx, vy = math.cos(theta), math.sin(theta)
    g_west = np.broadcast_to(np.asarray(g_west, dtype=np.float64), (ny,)).copy()
    g_south = np.broadcast_to(np.asarray(g_south, dtype=np.float64), (nx,)).copy()
    own, west, south = element_blocks(theta)
    # inflow load of one cell per unit g: west face on a = 0 nodes, south on b = 0
    lw = np.array([vx * 0.5 if (r % 2) == 0 else 0.0 for r in range(4)])
    ls = np.array([vy * 0.5 if (r // 2) == 0 else 0.0 for r in range(4)])
    if scaled:
        inv = np.linalg.inv(own)
        west, south = inv @ west, inv @ south
        lw, ls = inv @ lw, inv @ ls
        own = np.eye(4)
    ncell = nx * ny
    n = 4 * ncell
    cell = np.arange(ncell, dtype=np.int64)
    ci, cj = cell % nx, cell // nx
    # per cell, a dense 4 x 12 row block over [south cell | west cell | own cell]
    # (ascending column order), with structurally absent entries masked out
    blk = np.concatenate([south, west, own], axis=1)              # [4, 12]
    present = blk != 0.0
    has_s = (cj > 0) & (vy != 0.0)
    has_w = (ci > 0) & (vx != 0.0)
    cols = np.empty((ncell, 4, 12), dtype=np.int64)
    base_s = 4 * (cell - nx)
    base_w = 4 * (cell - 1)
    base_o = 4 * cell
    for q in range(4):
        cols[:, :, q] = (base_s + q)[:, None]
        cols[:, :, 4 + q] = (base_w + q)[:, None]
        cols[:, :, 8 + q] = (base_o + q)[:, None]
    mask = np.broadcast_to(present, (ncell, 4, 12)).copy()
    mask[:, :, 0:4] &= has_s[:, None, None]
    mask[:, :, 4:8] &= has_w[:, None, None]
    vals = np.broadcast_to(blk, (ncell, 4, 12))
    cols = cols.reshape(n, 12)
    mask = mask.reshape(n, 12)
    vals = vals.reshape(n, 12)
    b = np.zeros((ncell, 4))
    wc = ci == 0
    sc = cj == 0
    if vx != 0.0:
        b[wc] += g_west[cj[wc]][:, None] * lw[None, :]
    if vy != 0.0:
        b[sc] += g_south[ci[sc]][:, None] * ls[None, :]
    b = b.reshape(n)
    level = np.repeat(ci + cj, 4)

    order = None
    if perm_seed is not None:
        keys = rng.uniform(perm_seed, rng.PERM, 0, n)
        order = np.argsort(keys, kind="stable").astype(np.int64)
        inv_p = np.empty(n, dtype=np.int64)
        inv_p[order] = np.arange(n, dtype=np.int64)
        cols, vals, mask = cols[order], vals[order], mask[order]
        big = np.iinfo(np.int64).max
        cols = np.where(mask, inv_p[np.where(mask, cols, 0)], big)
        srt = np.argsort(cols, axis=1, kind="stable")
        cols = np.take_along_axis(cols, srt, axis=1)
        vals = np.take_along_axis(vals, srt, axis=1)
        mask = np.take_along_axis(mask, srt, axis=1)
        b = b[order]
        level = level[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=indptr[1:])
    return DGProblem(nx=nx, ny=ny, theta=float(theta), indptr=indptr.astype(np.int32),
                     indices=cols[mask].astype(np.int32), data=vals[mask].copy(), b=b,
                     g_west=g_west, g_south=g_south, scaled=scaled, order=order, level=level)
