"""First-order upwind finite-volume discretisation of v.grad(u) = 0 (Eqs. advection,
advection_bc of the paper) on a structured Nx x Ny grid of square cells.

The flux balance of each cell is divided by the cell size h, so the stencil does
not change under refinement (the paper non-dimensionalises by the mesh
resolution, Sec. 3).  With v = (cos t, sin t), t in (0, pi/2), cell (i, j) gives

    (vx + vy) u_ij - vx u_{i-1,j} - vy u_{i,j-1} = 0,

and a west face at i = 0 or a south face at j = 0 is an inflow face whose value
g moves to the right-hand side: b_ij += vx g_W(j), b_ij += vy g_S(i).

Unknown k = j * Nx + i, so the matrix is lower triangular in this order (the
upwind structure of Sec. 1.1).  An optional seeded symmetric permutation hides
that ordering from the solver.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import rng


@dataclass
class FVProblem:
    nx: int
    ny: int
    theta: float
    indptr: np.ndarray      # int32 [n+1]
    indices: np.ndarray     # int32 [nnz], ascending within each row
    data: np.ndarray        # float64 [nnz]
    b: np.ndarray           # float64 [n]
    g_west: np.ndarray      # float64 [ny]
    g_south: np.ndarray     # float64 [nx]
    order: np.ndarray = None   # unknown p of the (permuted) system is grid cell order[p]
    level: np.ndarray = None   # flow-order level i + j of every unknown (for sweeps)
    # d(data)/d(theta) on the same pattern, and d(b)/d(theta)
    ddata_dtheta: np.ndarray = None
    db_dtheta: np.ndarray = None
    # inflow faces: the unknown each face feeds and the coefficient of g in b there
    west_rows: np.ndarray = None
    south_rows: np.ndarray = None
    outflow_rows: np.ndarray = None   # right column then top row (corner once)
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.nx * self.ny

    @property
    def nnz(self):
        return int(self.indptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _grid_slots(nx, ny, vx, vy, dvx, dvy):
    """Natural-order stencil in three slots per row (south, west, diagonal):
    columns, values, d/dtheta values and a mask of the entries that exist."""
    n = nx * ny
    k = np.arange(n, dtype=np.int64)
    i = k % nx
    j = k // nx
    cols = np.stack([k - nx, k - 1, k], axis=1)
    mask = np.stack([(j > 0) & (vy != 0.0), (i > 0) & (vx != 0.0), np.ones(n, dtype=bool)], axis=1)
    vals = np.empty((n, 3))
    vals[:, 0], vals[:, 1], vals[:, 2] = -vy, -vx, vx + vy
    dvals = np.empty((n, 3))
    dvals[:, 0], dvals[:, 1], dvals[:, 2] = -dvy, -dvx, dvx + dvy
    return cols, vals, dvals, mask, i, j


def _compress(cols, vals, dvals, mask):
    """CSR arrays from the slot layout (slots already ascending in each row)."""
    indptr = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=indptr[1:])
    return indptr, cols[mask], vals[mask], dvals[mask]


def fv_advection(nx, theta, g_west, g_south, perm_seed=None, ny=None):
    """Assemble the upwind FV system.

    g_west: inflow values on the ny west faces (scalar broadcast allowed);
    g_south: inflow values on the nx south faces.  perm_seed: if not None, the
    unknowns are permuted by the argsort of a seeded U[0,1) key per unknown.
    """
    ny = nx if ny is None else ny
    if not (0.0 <= theta <= 0.5 * math.pi):
        raise ValueError("theta must lie in [0, pi/2] so that inflow is west/south")
    vx, vy = math.cos(theta), math.sin(theta)
    dvx, dvy = -math.sin(theta), math.cos(theta)
    g_west = np.broadcast_to(np.asarray(g_west, dtype=np.float64), (ny,)).copy()
    g_south = np.broadcast_to(np.asarray(g_south, dtype=np.float64), (nx,)).copy()
    n = nx * ny
    cols, vals, dvals, mask, ci, cj = _grid_slots(nx, ny, vx, vy, dvx, dvy)

    west_rows = np.arange(ny, dtype=np.int64) * nx
    south_rows = np.arange(nx, dtype=np.int64)
    b = np.zeros(n)
    db = np.zeros(n)
    if vx != 0.0:
        b[west_rows] += vx * g_west
        db[west_rows] += dvx * g_west
    if vy != 0.0:
        b[south_rows] += vy * g_south
        db[south_rows] += dvy * g_south
    level = (ci + cj).astype(np.int64)
    outflow = np.concatenate([np.arange(ny, dtype=np.int64) * nx + (nx - 1),
                              (ny - 1) * nx + np.arange(nx - 1, dtype=np.int64)])

    order = None
    if perm_seed is not None:
        keys = rng.uniform(perm_seed, rng.PERM, 0, n)
        order = np.argsort(keys, kind="stable").astype(np.int64)
        inv = np.empty(n, dtype=np.int64)
        inv[order] = np.arange(n, dtype=np.int64)
        # row p of the permuted system is grid cell order[p]: its (at most three)
        # columns are relabelled, then put in ascending order by a three-element
        # sorting network that carries each entry's slot (absent slots last)
        big = np.iinfo(np.int64).max
        msk = mask[order]
        c = [np.full(n, big, dtype=np.int64) for _ in range(3)]
        for t, off in ((0, nx), (1, 1)):
            sel = msk[:, t]
            c[t][sel] = inv[order[sel] - off]
        c[2] = np.arange(n, dtype=np.int64)
        slot = [np.full(n, t, dtype=np.int8) for t in range(3)]
        for a_, b_ in ((0, 1), (1, 2), (0, 1)):
            sw = c[a_] > c[b_]
            c[a_], c[b_] = np.where(sw, c[b_], c[a_]), np.where(sw, c[a_], c[b_])
            slot[a_], slot[b_] = np.where(sw, slot[b_], slot[a_]), np.where(sw, slot[a_], slot[b_])
        cols = np.stack(c, axis=1)
        slot = np.stack(slot, axis=1)
        mask = cols != big
        vals = vals[0][slot]
        dvals = dvals[0][slot]
        b = b[order]
        db = db[order]
        level = level[order]
        west_rows = inv[west_rows]
        south_rows = inv[south_rows]
        outflow = inv[outflow]
    indptr, indices, data, ddata = _compress(cols, vals, dvals, mask)

    return FVProblem(nx=nx, ny=ny, theta=float(theta),
                     indptr=indptr.astype(np.int32), indices=indices.astype(np.int32),
                     data=data, b=b, g_west=g_west, g_south=g_south, order=order,
                     level=level, ddata_dtheta=ddata, db_dtheta=db,
                     west_rows=west_rows, south_rows=south_rows, outflow_rows=outflow)


def inflow_values(seed, nx, ny=None, sub=0):
    """Seeded U(0,1) values on the west (ny) and south (nx) inflow faces."""
    ny = nx if ny is None else ny
    return rng.uniform(seed, rng.G_WEST, sub, ny), rng.uniform(seed, rng.G_SOUTH, sub, nx)
