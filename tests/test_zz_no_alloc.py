"""The allocation-free gradient entry point against the allocating one.

airg_fv_gradients_noalloc runs the launches of airg_fv_gradients with its
scratch (the theta terms and the partial sums of the theta contraction) in a
static device array instead of stream-ordered allocations, so both must give
the same bits.  Two calls in a row, the second on a smaller grid, check that
the contents the first call leaves in the shared array do not leak into the
second; a grid beyond the array's limit is refused before anything is
enqueued."""
import ctypes

import numpy as np
import pytest

from airg_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NOALLOC_MAX_N = 1 << 22


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(nx, ny, theta, seed):
    from paper_2508_17517_amd.advection import FVSystem
    gw, gs = workloads.inflow_values(seed, nx, ny)
    sysm = FVSystem(nx, ny, theta, torch.from_numpy(gw), torch.from_numpy(gs))
    rng = np.random.default_rng(seed)
    u = torch.from_numpy(rng.uniform(0.0, 1.0, nx * ny)).cuda()
    lam = torch.from_numpy(rng.standard_normal(nx * ny)).cuda()
    return sysm, u, lam


def _grads(fn, sysm, u, lam):
    from paper_2508_17517_amd import binding, _ptr, _stream_ptr
    lib = binding.load()
    dgw = torch.full((sysm.ny,), np.nan, dtype=torch.float64, device="cuda")
    dgs = torch.full((sysm.nx,), np.nan, dtype=torch.float64, device="cuda")
    dth = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    code = getattr(lib, fn)(sysm.nx, sysm.ny, sysm.theta, _ptr(sysm.rowptr), _ptr(sysm.col),
                            _ptr(sysm.dval), _ptr(sysm.db), _ptr(u), _ptr(lam), _ptr(dgw),
                            _ptr(dgs), _ptr(dth), _stream_ptr(None))
    binding.check(code, lib)
    torch.cuda.synchronize()
    return dgw.cpu().numpy(), dgs.cpu().numpy(), dth.cpu().numpy()


def test_noalloc_gradients_equal_the_allocating_entry_point_twice():
    _needs_gpu()
    # a larger grid first, then a smaller one: the second call must not see
    # the first call's leftovers in the shared scratch array
    for nx, ny, theta, seed in ((517, 389, 0.7, 11), (96, 61, 0.3, 12)):
        print(f"noalloc gradients: {nx} x {ny}, theta {theta}, seed {seed}", flush=True)
        sysm, u, lam = _case(nx, ny, theta, seed)
        ref = _grads("airg_fv_gradients", sysm, u, lam)
        got = _grads("airg_fv_gradients_noalloc", sysm, u, lam)
        for r, g in zip(ref, got):
            assert np.all(np.isfinite(g))
            assert np.array_equal(r, g)


def test_noalloc_gradients_refuse_a_grid_beyond_the_scratch():
    _needs_gpu()
    from paper_2508_17517_amd import binding, _ptr, _stream_ptr
    lib = binding.load()
    sysm, u, lam = _case(8, 8, 0.5, 13)
    dgw = torch.zeros(8, dtype=torch.float64, device="cuda")
    dgs = torch.zeros(8, dtype=torch.float64, device="cuda")
    dth = torch.zeros(1, dtype=torch.float64, device="cuda")
    # the size check comes before any launch, so these small buffers are never read
    code = lib.airg_fv_gradients_noalloc(2049, 2048, 0.5, _ptr(sysm.rowptr), _ptr(sysm.col),
                                         _ptr(sysm.dval), _ptr(sysm.db), _ptr(u), _ptr(lam),
                                         _ptr(dgw), _ptr(dgs), _ptr(dth), _stream_ptr(None))
    assert 2049 * 2048 > NOALLOC_MAX_N
    assert code == -1  # AIRG_ERR_INVALID
    assert b"no-allocation limit" in lib.airg_last_error()
    torch.cuda.synchronize()
    assert float(dth[0]) == 0.0
