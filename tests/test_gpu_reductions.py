"""The FGMRES Gram-Schmidt sweeps fuse the basis update with the dot
products after it: a block takes 1024 elements (four per thread), and one
more launch sums the block partials of each vector in block order.  At sizes
with a ragged last block, fewer and more blocks than the final launch has
threads, and up to 32 basis vectors, solves must match the oracle (same
iteration count, elementwise 1e-10) and repeat bit for bit."""
import numpy as np
import pytest

import oracle
from airg_inputs import workloads
from parity import assert_elementwise

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# side: blocks of 1024 elements
SIDES = {
    129: "17 blocks, the last of 257 elements",
    181: "32 blocks, the last of 1017 elements",
    300: "88 blocks, the last of 912 elements",
    512: "256 blocks, one per thread of the final sum",
    580: "329 blocks: the final sum's first 73 threads add two",
}


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("side", list(SIDES))
def test_solves_across_block_counts_match_the_oracle_and_repeat(side):
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(side, 0.3, True)
    print(f"fv{side}: {SIDES[side]}", flush=True)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b)
    s = Solver(p.indptr, p.indices, p.data)
    b = torch.from_numpy(p.b).cuda()
    x, info = s.solve(b)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert_elementwise(x.cpu().numpy(), xo)
    for _ in range(4):
        x2, info2 = s.solve(b)
        assert info2["iterations"] == info["iterations"]
        assert info2["rel_residual"] == info["rel_residual"]
        assert torch.equal(x2, x)
    s.close()


def test_long_arnoldi_cycle_with_32_basis_vectors():
    # one level and a degree-8 Newton polynomial with restart 40: the first
    # cycle passes 32 basis vectors (the widest fused sweep) over 25 blocks
    _needs_gpu()
    from paper_2508_17517_amd import Solver
    p = workloads.fv_random(160, 0.4, True)
    kw = dict(max_levels=1, coarse_poly_order=8, restart=40)
    xo, its, rel, levels, _ = oracle.solve(p.scipy(), p.b, oracle.Params(**kw))
    assert its > 40
    s = Solver(p.indptr, p.indices, p.data, **kw)
    b = torch.from_numpy(p.b).cuda()
    x, info = s.solve(b)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == its
    assert_elementwise(x.cpu().numpy(), xo)
    x2, _ = s.solve(b)
    assert torch.equal(x2, x)
    s.close()
