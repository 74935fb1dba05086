"""Full-size checks at the benchmark workload (FV 2048 x 2048, theta 0.3,
permuted, g ~ U(0,1)) in the launch configuration bench.py times.

* Level 0 of the hierarchy at full size (the oracle computes it in seconds):
  the CF split, A_ff, A_fc, the smoother coefficients, Z, the prolongator and
  A_1 bit for bit.
* The whole oracle solve, stored by tests/golden/make_fv2048_golden.py (a few
  minutes on one core): with the launch shapes the benchmark pins
  (paper_2508_17517_amd/shapes/fv2048_fp64.json), the GPU solve takes the
  oracle's iteration count, every level has the oracle's size and smoother
  coefficients, and the solution at 2048 sampled unknowns agrees element by
  element to 1e-10 of max |x|.
* Properties that hold at any size: the true residual and the distance to the
  exact sweep solution."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import hierarchy as OH
from airg_inputs import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fv2048_oracle.json")


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("building fv2048", flush=True)
    return workloads.fv2048()


def _eq(name, got, want):
    want = sp.csr_matrix(want)
    want.sort_indices()
    rp, col, val = got
    assert np.array_equal(rp, want.indptr), name
    assert np.array_equal(col, want.indices), name
    assert np.array_equal(val, want.data), name


def test_full_size_level0_is_bitwise_the_oracles(big):
    from paper_2508_17517_amd import Solver
    A = big.scipy()
    L, Ac = OH.coarsen(A, 0, oracle.Params())
    s = Solver(big.indptr, big.indices, big.data, keep_setup_data=1)
    g0 = s.export_level(0)
    assert np.array_equal(g0["state"], L.state)
    _eq("A_ff", g0["ff"], L.Aff)
    _eq("A_fc", g0["fc"], L.Afc)
    assert np.array_equal(g0["alpha"], L.alpha)
    _eq("Z", g0["z"], L.Z)
    assert np.array_equal(g0["cmap"], L.cmap)
    g1 = s.export_level(1)
    _eq("A_1", g1["a"], Ac)
    s.close()


def test_full_size_solve_properties(big):
    from paper_2508_17517_amd import Solver
    s = Solver(big.indptr, big.indices, big.data)
    b = torch.from_numpy(big.b).cuda()
    x, info = s.solve(b)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    xg = x.cpu().numpy()
    A = big.scipy()
    r = big.b - A @ xg
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(big.b)
    u = oracle.sweep_solve(A, big.b, big.level)
    # the error is bounded by the condition number times the residual
    assert np.linalg.norm(xg - u) <= 1e-7 * np.linalg.norm(u)
    # sampled rows of the true residual, recomputed one by one
    rows = np.random.default_rng(0).choice(big.n, 64, replace=False)
    for i in rows:
        lo, hi = big.indptr[i], big.indptr[i + 1]
        ri = big.b[i] - sum(big.data[k] * xg[big.indices[k]] for k in range(lo, hi))
        assert abs(ri) <= 1e-8 * np.abs(big.b).max() + 1e-12
    # solving again from the solution takes no iteration; a second solve is identical
    x2, info2 = s.solve(b)
    assert info2["iterations"] == info["iterations"]
    assert torch.equal(x, x2)
    s.close()


def test_full_size_solve_is_the_oracles_in_the_timed_launch_shapes(big):
    from paper_2508_17517_amd import Solver, load_shapes
    with open(GOLDEN) as f:
        g = json.load(f)
    assert g["n"] == big.n and g["nnz"] == big.nnz
    s = Solver(big.indptr, big.indices, big.data)
    s.pin_shapes(load_shapes("fv2048_fp64"))
    st = s.stats()
    lv = g["levels"]
    assert st["levels"] == len(lv)
    for l, L in enumerate(lv):
        assert st["n"][l] == L["n"] and st["nnz"][l] == L["nnz"], l
        if L["trunc_rel"] is not None:
            assert st["trunc_rel"][l] == pytest.approx(float.fromhex(L["trunc_rel"]), rel=1e-8), l
        e = s.export_level(l, what=("alpha", "roots"))
        if L["coarsest"]:
            want = np.array([complex(float.fromhex(a), float.fromhex(b)) for a, b in L["roots"]])
            assert len(e["roots"]) == len(want)
            assert np.allclose(np.sort_complex(e["roots"]), np.sort_complex(want), rtol=1e-9,
                               atol=1e-12)
        else:
            assert st["n_f"][l] == L["n_f"], l
            assert np.array_equal(e["alpha"], np.array([float.fromhex(a) for a in L["alpha"]])), l
    b = torch.from_numpy(big.b).cuda()
    x, info = s.solve(b)
    print(f"fv2048 pinned shapes: gpu {info['iterations']} iterations, rel {info['rel_residual']:.3e}; "
          f"oracle {g['iterations']}, rel {float.fromhex(g['rel_residual']):.3e}", flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-10
    assert info["iterations"] == g["iterations"]
    idx = np.array(g["sample_index"])
    xo = np.array([float.fromhex(v) for v in g["sample_x"]])
    xg = x.cpu().numpy()[idx]
    xmax = float.fromhex(g["x_max_abs"])
    err = np.abs(xg - xo).max()
    print(f"max |x_gpu - x_oracle| over {len(idx)} samples: {err:.3e} (max |x| {xmax:.3e})", flush=True)
    assert err <= 1e-10 * xmax
    s.close()
