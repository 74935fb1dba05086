"""Writes fv2048_oracle.json: the oracle's solve of the benchmark workload.

The workload is the upwind FV system on a 2048 x 2048 grid (theta 0.3,
unknowns permuted, g ~ U(0,1) per inflow face; airg_inputs.workloads.fv2048)
with the solver's default options (AIRG smoother degree 4, Newton coarse
degree 20, truncation at a 1e-2 contraction, FGMRES(30) to rtol 1e-10 from
x0 = 0).  The file keeps what the full-size GPU parity test compares:

* the oracle's iteration count, true relative residual and the Arnoldi
  residual estimate after every iteration;
* every level's size, nonzeros, F-point count, smoother coefficients and
  truncation-test residual, and the coarsest level's Newton roots;
* the solution at 2048 sampled unknowns (indices drawn from a fixed NumPy
  seed), and max |x|, as hexadecimal floats.

It calls only oracle/ and the input generators; about 2-4 minutes on one core.

    python tests/golden/make_fv2048_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from airg_inputs import workloads  # noqa: E402

OUT = os.path.join(HERE, "fv2048_oracle.json")
SAMPLES = 2048
SAMPLE_SEED = 20480


def main():
    p = workloads.fv2048()
    A = p.scipy()
    t0 = time.perf_counter()
    levels = oracle.setup(A)
    t1 = time.perf_counter()
    print(f"oracle setup {t1 - t0:.1f} s, {len(levels)} levels", flush=True)
    x, its, rel, _, hist = oracle.solve(A, p.b, levels=levels)
    t2 = time.perf_counter()
    print(f"oracle solve {t2 - t1:.1f} s, {its} iterations, rel {rel:.3e}", flush=True)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(p.n, SAMPLES, replace=False))
    lv = []
    for L in levels:
        e = {"n": int(L.A.shape[0]), "nnz": int(L.A.nnz), "coarsest": bool(L.coarsest),
             "trunc_rel": None if L.trunc_rel is None else float(L.trunc_rel).hex()}
        if L.coarsest:
            e["roots"] = [[float(r.real).hex(), float(r.imag).hex()] for r in L.roots]
        else:
            e["n_f"] = int(len(L.F))
            e["alpha"] = [float(a).hex() for a in L.alpha]
        lv.append(e)
    out = {
        "workload": "upwind FV 2048x2048, theta 0.3, permuted, g~U(0,1) (airg_inputs.workloads.fv2048); "
                    "AIRG d=4, m_c=20, trunc 1e-2, FGMRES(30) rtol 1e-10, x0 = 0",
        "n": int(p.n), "nnz": int(p.nnz),
        "iterations": int(its), "rel_residual": float(rel).hex(),
        "estimate_history": [float(h).hex() for h in hist],
        "levels": lv,
        "x_max_abs": float(np.abs(x).max()).hex(),
        "sample_seed": SAMPLE_SEED,
        "sample_index": [int(i) for i in idx],
        "sample_x": [float(v).hex() for v in x[idx]],
        "oracle_seconds": {"setup": round(t1 - t0, 1), "solve": round(t2 - t1, 1)},
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
