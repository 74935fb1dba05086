"""Seeded input generators: the published SplitMix64 sequence and the upwind FV
assembly (Eqs. advection, advection_bc; Sec. 1.1 lower-triangular structure)."""
import math
import os

import numpy as np
import scipy.sparse as sp

from airg_inputs import rng, fv_advection, workloads
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_ints(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [int(l) for l in f if l.strip() and not l.startswith("#")]


def test_splitmix64_published_sequence():
    want = _golden_ints("splitmix64_seed1234567.txt")
    got = [int(v) for v in rng.splitmix64_sequence(1234567, 5)]
    assert got == want


def test_counter_stream_is_sequence_position():
    # element i of stream (p, s) is output c+1 of the sequential generator
    seed = 99
    c0 = (3 << 56) | (5 << 40)
    seq_at = rng.splitmix64_sequence((seed + c0 * rng.GAMMA) & rng.MASK64, 4)
    assert np.array_equal(rng.raw(seed, 3, 5, 4), seq_at)


def test_uniform_range_and_moments():
    u = rng.uniform(17517, rng.G_WEST, 0, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3
    z = rng.normal(17517, rng.LOSS_W, 0, 200000)
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1.0) < 1e-2


def test_fv_stencil_and_triangularity():
    p = fv_advection(7, 0.4, 0.0, 0.0, ny=5)
    A = p.scipy().toarray()
    vx, vy = math.cos(0.4), math.sin(0.4)
    assert np.allclose(np.diag(A), vx + vy)
    assert np.allclose(np.triu(A, 1), 0.0)               # lower triangular in k = j*nx + i
    k = 3 * 7 + 4
    assert A[k, k - 1] == -vx and A[k, k - 7] == -vy
    # interior rows annihilate constants (v.grad(1) = 0)
    interior = [(j * 7 + i) for j in range(1, 5) for i in range(1, 7)]
    assert np.allclose((A @ np.ones(35))[interior], 0.0, atol=1e-15)
    assert p.nnz == 35 * 3 - 7 - 5


def test_constant_inflow_gives_constant_solution_exactly():
    # u = g for constant g; with g = 1 the sweep reproduces it bit for bit
    p = workloads.fv64()
    u = oracle.sweep_solve(p.scipy(), p.b, p.level)
    assert np.array_equal(u, np.ones(p.n))


def test_permutation_is_a_symmetric_relabelling():
    gw, gs = workloads.inflow_values(5, 9, 6)
    p0 = fv_advection(9, 1.1, gw, gs, ny=6)
    p1 = fv_advection(9, 1.1, gw, gs, perm_seed=5, ny=6)
    o = p1.order
    A0 = p0.scipy()
    A1 = p1.scipy()
    assert (A1 - A0[o][:, o]).nnz == 0
    assert np.array_equal(p1.b, p0.b[o])
    assert np.array_equal(p1.level, p0.level[o])
    assert np.all(np.diff(p1.indices.reshape(-1)[0:0]) >= 0)
    for r in range(p1.n):
        cols = p1.indices[p1.indptr[r]:p1.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_theta_derivatives_match_finite_differences():
    gw, gs = workloads.inflow_values(3, 6)
    t, h = 0.7, 1e-6
    p = fv_advection(6, t, gw, gs)
    pp = fv_advection(6, t + h, gw, gs)
    pm = fv_advection(6, t - h, gw, gs)
    assert np.allclose((pp.data - pm.data) / (2 * h), p.ddata_dtheta, atol=1e-9)
    assert np.allclose((pp.b - pm.b) / (2 * h), p.db_dtheta, atol=1e-9)


def test_batch_shapes_are_seeded_and_in_range():
    s, t = workloads.batch_shapes(48)
    s2, t2 = workloads.batch_shapes(48)
    assert np.array_equal(s, s2) and np.array_equal(t, t2)
    assert set(np.unique(s)) <= set(workloads.BATCH_SIDES)
    assert np.all((t > 0) & (t < math.pi / 2))
