"""Solver parameters of the oracle (one field per option of the paper's solver).

Defaults are the paper's option set (Sec. 3) except where the workload fixes a
different value: smoother degree 4, coarse degree 20 and truncation tolerance
1e-2, and an FGMRES outer loop in place of Richardson.
"""
from dataclasses import dataclass


@dataclass
class Params:
    strong_threshold: float = 0.99   # theta_s of the strength test (Sec. 2.1)
    ddc_fraction: float = 0.01       # fraction of local F points converted per DDC pass (Sec. 2.1)
    ddc_its: int = 2                 # DDC passes (Sec. 3 option set)
    a_drop: float = 1e-6             # relative drop on the coarse matrix, lumped (Sec. 2)
    lump: bool = True
    r_drop: float = 0.01             # relative drop on R (value not given in the paper)
    poly_order: int = 4              # degree of the F-point smoother polynomial
    coarse_poly_order: int = 20      # degree of the Newton coarse polynomial
    trunc_tol: float = 1e-2          # automatic truncation tolerance (<= 0 disables)
    trunc_start_level: int = 1
    max_levels: int = 64
    min_coarse_rows: int = 64
    added_roots: bool = True         # extra copies of outlying roots (Loe & Morgan 2022)
    seed: int = 17517
    rtol: float = 1e-10
    atol: float = 1e-50              # absolute residual tolerance of the outer loop (Sec. 3 option set)
    max_it: int = 500
    restart: int = 30
    outer: str = "fgmres"            # or "richardson": the paper's undamped Richardson (Sec. 3)
    smoother: str = "poly"           # or "assembled": F-smoothing with the assembled Ahat^{-1} (Sec. 2.2)
    inverse_type: str = "arnoldi"    # or "neumann": nAIR's Neumann polynomials (Sec. 3.3)
    smooth_type: str = "f"           # up-smooths in order: "f", "fc" or "fcf" (Sec. 2, Sec. 3.3)
    # oracle-only knob for the exactness pins: solve the coarsest level by LU
    exact_coarse: bool = False
