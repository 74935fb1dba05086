"""CPU oracle for the AIRG reduction-multigrid solve (FP64, NumPy/SciPy).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow reference of what the
GPU library computes, written from the paper (Dargaville et al., "Solving
advection equations with reduction multigrids on GPUs", Sec. 2 and 3).  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never does, and it never imports the library.

Modules:
  params  -- the solver's options (Sec. 3 option set, workload overrides)
  rng     -- counter-based SplitMix64 for the solver's random draws
  linalg  -- SpMV, dot products, Arnoldi, GMRES polynomials (Eq. gmres_poly),
             harmonic Ritz roots, Newton application (Sec. 2.2, 2.3)
  hierarchy -- PMISR DDC CF splitting (Sec. 2.1), Eq. fixed_sparsity, Eq. z,
             one-point prolongation, R A P with drop and lump, truncation (Sec. 2.4)
  solve   -- V-cycle with up F-point smoothing (Eq. f_point), FGMRES, adjoint
  sweep   -- exact flow-order sweeps (Sec. 1.1), the ground truth

Every function is pinned by a test in tests/test_oracle_pins.py against what
the paper and the mathematics fix (closed forms, invariants, exactness
cases, brute force); what nothing outside the method fixes -- the exact CF
split, level counts and iteration counts of the workloads -- is parity
unpinned and is compared between the library and this oracle only.
"""
from .params import Params  # noqa: F401
from .hierarchy import setup, ZeroDiagonal  # noqa: F401
from .solve import solve, adjoint_solve, vcycle, fgmres, richardson, loss_gradients  # noqa: F401
from .sweep import sweep_solve  # noqa: F401
from . import linalg, rng  # noqa: F401
