"""Named synthetic workloads: every input is drawn from base seed 17517.

* ``fv64``:    FV 64 x 64, theta = 3 pi / 8, g = 1 on every inflow face, natural order.
* ``fv2048``:  FV 2048 x 2048, theta = 0.3, g ~ U(0,1) per inflow face, unknowns
               randomly permuted.
* ``fv1024``:  FV 1024 x 1024, theta = 0.3, g ~ U(0,1) (the differentiation workload),
               with N(0,1) loss weights on the outflow cells.
* ``fv8192``:  FV 8192 x 8192 with fv2048's settings (a working set far above the
               on-die caches, for HBM roofline measurements).
* ``dg1024``:  upwind DG-Q1 on 1024 x 1024 cells (4 unknowns per cell), theta = pi / 5,
               g ~ U(0,1) per inflow face, element-block scaled, unknowns permuted
               (the mixed-precision workload).
* ``fd_paper(N)``: the paper's own FD system (boundary nodes kept, theta = pi/4,
               g = 0, natural order); N = 3606 is its 13M-unknown single-GPU case.
* ``fv_random(N, theta, permute)`` / ``dg_random(N, theta, permute)``: the same
  recipes at any size (parity cases).
"""
import math

import numpy as np

from . import rng
from .fv import fv_advection, inflow_values
from .dg import dg_advection
from .fd import fd_advection

SEED = rng.DEFAULT_SEED


def fv64():
    return fv_advection(64, 3.0 * math.pi / 8.0, 1.0, 1.0)


def fv_random(n, theta=0.3, permute=True, seed=SEED, ny=None):
    gw, gs = inflow_values(seed, n, ny)
    return fv_advection(n, theta, gw, gs, perm_seed=seed if permute else None, ny=ny)


def dg_random(n, theta=math.pi / 5.0, permute=True, seed=SEED, ny=None):
    gw, gs = inflow_values(seed, n, ny)
    return dg_advection(n, theta, gw, gs, perm_seed=seed if permute else None, ny=ny)


def dg1024():
    return dg_random(1024, math.pi / 5.0, True)


def fd_paper(n=3606):
    """The paper's single-GPU setting (Sec. 3.1): FD with the inflow boundary
    nodes kept, theta = pi/4, g = 0; n = 3606 gives 13.0M unknowns."""
    return fd_advection(n, math.pi / 4.0, 0.0)


def fv2048():
    return fv_random(2048, 0.3, True)


def fv8192():
    return fv_random(8192, 0.3, True)


def fv1024():
    return fv_random(1024, 0.3, False)


def loss_weights(problem, seed=SEED):
    """N(0,1) weights on the outflow cells of ``problem``."""
    return rng.normal(seed, rng.LOSS_W, 0, len(problem.outflow_rows))


def rhs_batch(problem, k, seed=SEED):
    """``k`` right-hand sides for the matrix of ``problem``: g ~ U(0,1) per face, seeded
    by the column index.  Returns an [k, n] array."""
    import numpy as np
    out = np.zeros((k, problem.n))
    vx, vy = math.cos(problem.theta), math.sin(problem.theta)
    for c in range(k):
        gw, gs = inflow_values(seed, problem.nx, problem.ny, sub=1 + c)
        b = np.zeros(problem.n)
        if vx != 0.0:
            b[problem.west_rows] += vx * gw
        if vy != 0.0:
            b[problem.south_rows] += vy * gs
        out[c] = b
    return out


BATCH_SIDES = (128, 256, 512, 1024)


def batch_shapes(count, seed=SEED):
    """Grid sides ~ U{128,256,512,1024} and angles ~ U(0, pi/2) for a batch of problems."""
    u = rng.uniform(seed, rng.BATCH_SIDE, 0, count)
    sides = np.array(BATCH_SIDES)[np.minimum((u * 4).astype(np.int64), 3)]
    theta = rng.uniform(seed, rng.BATCH_THETA, 0, count) * (0.5 * math.pi)
    return sides, theta


def batch_problems(count, seed=SEED, sides=None):
    """``count`` independent FV problems with the shapes of ``batch_shapes``; problem q
    draws its inflow values and permutation from seed + 1 + q.  ``sides`` (optional)
    overrides the drawn grid sides, e.g. to shrink a batch for tests."""
    s, theta = batch_shapes(count, seed)
    if sides is not None:
        s = np.asarray(sides)
    return [fv_random(int(s[q]), float(theta[q]), True, seed=seed + 1 + q) for q in range(count)]
