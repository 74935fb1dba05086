"""Seeded input generators: the published SplitMix64 sequence and the upwind FV
assembly (Eqs. advection, advection_bc; Sec. 1.1 lower-triangular structure)."""
import math
import os

import numpy as np
import pytest
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


# --------------------------------------------------------------------- DG-Q1 (reading of the paper's DG remark)

def test_dg_element_blocks_by_hand():
    # own-block diagonal (vx + vy)/6 on every node; west/south couple only the
    # inflow-face nodes to the neighbour's facing nodes with -v M entries
    from airg_inputs.dg import element_blocks
    t = math.pi / 5
    vx, vy = math.cos(t), math.sin(t)
    own, west, south = element_blocks(t)
    assert np.allclose(np.diag(own), (vx + vy) / 6.0, rtol=0, atol=1e-15)
    # test node (0,0) = row 0: west trial nodes (1,0), (1,1) = columns 1, 3
    assert west[0, 1] == -vx / 3.0 and west[0, 3] == -vx / 6.0
    assert np.count_nonzero(west) == 4 and np.count_nonzero(south) == 4
    # test node (0,0): south trial nodes (0,1), (1,1) = columns 2, 3
    assert south[0, 2] == -vy / 3.0 and south[0, 3] == -vy / 6.0
    # v.grad(1) = 0: the three blocks together annihilate constants
    assert np.allclose((own + west + south).sum(axis=1), 0.0, atol=1e-15)


@pytest.mark.parametrize("scaled", [True, False])
def test_dg_constant_inflow_gives_constant_solution(scaled):
    from airg_inputs import dg_advection
    p = dg_advection(6, math.pi / 5, 0.7, 0.7, scaled=scaled, ny=5)
    u = sp.linalg.spsolve(p.scipy().tocsc(), p.b)
    assert np.abs(u - 0.7).max() < 1e-14
    if scaled:
        # own blocks are the identity and rows keep at most 1 + 2 + 2 entries
        assert np.array_equal(p.scipy().diagonal(), np.ones(p.n))
        assert np.diff(p.indptr).max() == 5


def test_dg_scaled_system_is_triangular_in_cell_order_and_sweeps_exactly():
    p = workloads.dg_random(12, 0.9, True)
    A = p.scipy()
    u = oracle.sweep_solve(A, p.b, p.level)
    assert np.allclose(u, sp.linalg.spsolve(A.tocsc(), p.b), rtol=0, atol=1e-13)


def test_dg_permutation_is_a_relabelling():
    from airg_inputs import dg_advection
    gw, gs = np.linspace(0.1, 0.9, 5), np.linspace(0.2, 0.8, 7)
    p0 = dg_advection(7, 0.6, gw, gs, ny=5)
    p1 = dg_advection(7, 0.6, gw, gs, perm_seed=3, ny=5)
    A0, A1 = p0.scipy(), p1.scipy()
    o = p1.order
    assert np.array_equal(A1.toarray(), A0.toarray()[np.ix_(o, o)])
    assert np.array_equal(p1.b, p0.b[o])
    assert all(np.all(np.diff(p1.indices[p1.indptr[i]:p1.indptr[i + 1]]) > 0) for i in range(p1.n))
