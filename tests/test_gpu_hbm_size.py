"""The HBM-sized run's grid, FV 8192 x 8192 (67M unknowns), checked through
properties that hold at any size, since the oracle cannot set up a hierarchy
this large in a test's time.

With constant inflow g = 1 every cell's exact value is 1: the upwind balance
(vx + vy) u_ij = vx u_{i-1,j} + vy u_{i,j-1} (inflow faces in the right-hand
side) holds with u = 1 everywhere.  The system is assembled on the device by
the library's own upwind assembly (the one the differentiable solve uses and
that tests/test_gpu_adjoint.py compares with the generator entry by entry),
unpermuted.  The solve must reach the 1e-10 relative residual, stay within
1e-7 of 1 in every cell, and sampled rows of the residual, recomputed one by
one on the host from the CSR, must agree."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_fv8192_constant_inflow_gives_the_constant_solution():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_17517_amd import Solver
    from paper_2508_17517_amd.advection import FVSystem
    side = 8192
    print(f"FV {side}^2 constant inflow: assembling on the device", flush=True)
    ones = torch.ones(side, dtype=torch.float64)
    sysm = FVSystem(side, side, 0.3, ones, ones)
    print(f"n {sysm.n} nnz {sysm.nnz}: setup", flush=True)
    s = Solver(sysm.rowptr, sysm.col, sysm.val)
    print("solve", flush=True)
    x, info = s.solve(sysm.b)
    print(f"iterations {info['iterations']}, relative residual {info['rel_residual']:.2e}",
          flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    err = float((x - 1.0).abs().max())
    print(f"max |x - 1| = {err:.2e}", flush=True)
    assert err <= 1e-7
    # sampled rows of b - A x, one by one on the host
    rng = np.random.default_rng(8192)
    rows = rng.choice(sysm.n, 64, replace=False)
    rp = sysm.rowptr.cpu().numpy()
    xh = x.cpu().numpy()
    bh = sysm.b.cpu().numpy()
    for i in rows:
        lo, hi = int(rp[i]), int(rp[i + 1])
        cols = sysm.col[lo:hi].cpu().numpy()
        vals = sysm.val[lo:hi].cpu().numpy()
        ri = bh[i] - sum(v * xh[c] for v, c in zip(vals, cols))
        assert abs(ri) <= 1e-8 * np.abs(bh).max() + 1e-12, i
    s.close()
