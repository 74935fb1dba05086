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


def _grid_csr(nx, ny, vx, vy, dvx, dvy):
    """Natural-order CSR (cols south, west, diag) plus the d/dtheta values."""
    n = nx * ny
    k = np.arange(n, dtype=np.int64)
    i = k % nx
    j = k // nx
    has_s = (j > 0) & (vy != 0.0)
    has_w = (i > 0) & (vx != 0.0)
    cnt = 1 + has_s.astype(np.int64) + has_w.astype(np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=indptr[1:])
    nnz = int(indptr[-1])
    indices = np.empty(nnz, dtype=np.int64)
    data = np.empty(nnz, dtype=np.float64)
    ddata = np.empty(nnz, dtype=np.float64)
    pos = indptr[:-1].copy()
    s = pos[has_s]
    indices[s] = k[has_s] - nx
    data[s] = -vy
    ddata[s] = -dvy
    pos[has_s] += 1
    w = pos[has_w]
    indices[w] = k[has_w] - 1
    data[w] = -vx
    ddata[w] = -dvx
    pos[has_w] += 1
    indices[pos] = k
    data[pos] = vx + vy
    ddata[pos] = dvx + dvy
    return indptr, indices, data, ddata, i, j


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
    indptr, indices, data, ddata, ci, cj = _grid_csr(nx, ny, vx, vy, dvx, dvy)

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
        lens = np.diff(indptr)[order]
        new_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(lens, out=new_ptr[1:])
        src = np.repeat(indptr[order], lens) + (np.arange(new_ptr[-1]) - np.repeat(new_ptr[:-1], lens))
        rows = np.repeat(np.arange(n, dtype=np.int64), lens)
        cols = inv[indices[src]]
        perm_sort = np.lexsort((cols, rows))
        indices = cols[perm_sort]
        data = data[src][perm_sort]
        ddata = ddata[src][perm_sort]
        indptr = new_ptr
        b = b[order]
        db = db[order]
        level = level[order]
        west_rows = inv[west_rows]
        south_rows = inv[south_rows]
        outflow = inv[outflow]

    return FVProblem(nx=nx, ny=ny, theta=float(theta),
                     indptr=indptr.astype(np.int32), indices=indices.astype(np.int32),
                     data=data, b=b, g_west=g_west, g_south=g_south, order=order,
                     level=level, ddata_dtheta=ddata, db_dtheta=db,
                     west_rows=west_rows, south_rows=south_rows, outflow_rows=outflow)


def inflow_values(seed, nx, ny=None, sub=0):
    """Seeded U(0,1) values on the west (ny) and south (nx) inflow faces."""
    ny = nx if ny is None else ny
    return rng.uniform(seed, rng.G_WEST, sub, ny), rng.uniform(seed, rng.G_SOUTH, sub, nx)
