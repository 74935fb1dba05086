"""Benchmark: AIRG solve DOF/s to a relative residual of 1e-10 on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload fv2048]

A step is one complete solve of A x = b (FGMRES preconditioned by AIRG
V-cycles, to |b - A x| <= 1e-10 |b|) with the hierarchy already set up and all
inputs resident in HBM; the setup is timed once beforehand and reported.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published peak
METRIC = "AIRG solve DOF/s to rel-res 1e-10 + poly-SpMV HBM GB/s, FP64 vs mixed"

WORKLOADS = {
    # name: (grid side, theta, permuted)
    "fv2048": (2048, 0.3, True),
    "fv1024": (1024, 0.3, False),
    "fv8192": (8192, 0.3, True),
    "fv512": (512, 0.3, True),
    "fv1024p": (1024, 0.3, True),
}


def cpu_baseline(sample_side=1024):
    """The oracle (NumPy/SciPy FP64) timed on the host on a bounded sample: the
    same recipe (theta 0.3, permuted, U(0,1) inflow) on a smaller grid."""
    import oracle
    from airg_inputs import workloads
    p = workloads.fv_random(sample_side, 0.3, True)
    A = p.scipy()
    t0 = time.perf_counter()
    levels = oracle.setup(A)
    t1 = time.perf_counter()
    x, its, rel, _, _ = oracle.solve(A, p.b, levels=levels)
    t2 = time.perf_counter()
    return {"value": p.n / (t2 - t1), "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"FV {sample_side}x{sample_side}, theta 0.3, permuted: oracle solve "
                      f"{t2 - t1:.2f} s ({its} iterations), setup {t1 - t0:.2f} s; host has "
                      f"{os.cpu_count()} cores, the oracle's sparse kernels run on one thread"}


def stream_bandwidth(kind, nbytes, blocks=8192, reps=20):
    """GB/s of the library's hand-written streaming kernels (airg_stream_probe):
    kind "read" reads nbytes, "copy" reads and writes nbytes each (16-byte
    accesses, `blocks` workgroups of 256 threads).  Far above the on-die caches
    this is the practical HBM ceiling the sparse products are compared with."""
    import ctypes
    import torch
    from paper_2508_17517_amd import binding, _ptr, _stream_ptr
    lib = binding.load()
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src) if kind == "copy" else torch.zeros(8, dtype=torch.float64, device="cuda")
    ms = ctypes.c_double()
    binding.check(lib.airg_stream_probe(0 if kind == "read" else 1, _ptr(src), _ptr(dst), nbytes, reps,
                                        blocks, ctypes.byref(ms), _stream_ptr(None)), lib)
    moved = (2 if kind == "copy" else 1) * nbytes
    del src, dst
    return moved / (ms.value * 1e-3) / 1e9


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fv2048_poly_hbm_traffic.md")
# sources that decide the poly-SpMV launches and their operators
TRAFFIC_SOURCES = ["spmv.hip", "hierarchy.cpp", "solve.cpp", "order.hip", "spgemm.hip",
                   "common.hpp"]


def kernel_source_digest():
    """Digest of the sources that decide the poly-SpMV launches, and of the
    launch shapes the counter runs pin."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2508_17517_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2508_17517_amd", "shapes", "fv2048_fp64.json"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per poly-SpMV launch from the committed counter summary, if it
    was taken on this workload with the current kernel sources (else None)."""
    if workload != "fv2048" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and line.split(":")[0].strip() in ("kernel_source_sha256",
                                                              "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return float(vals["traffic_bytes_per_launch"])


TUNE = {"on": True, "file": None}
# solver options every leg uses (set from the command line)
SOLVER_OPTS = {}


def _tune(solver, main=False):
    """Pick the lanes per row of every solve operator by timing (airg_autotune)
    unless --no-autotune; returns a summary.  With --tune-file the main
    solver's shapes are read from that file when it exists (and pinned, so a
    profiled run launches the kernels an unprofiled run chose), else tuned
    and written there."""
    if not TUNE["on"]:
        return None
    path = TUNE["file"] if main else None
    if path and os.path.exists(path):
        with open(path) as f:
            t = json.load(f)
        solver.pin_shapes(t)
        print(f"bench: launch shapes pinned from {path}", file=sys.stderr, flush=True)
        return {"operators": len(t), "pinned_from": os.path.relpath(path, ROOT)}
    t = solver.autotune(reps=10)
    if path:
        with open(path, "w") as f:
            json.dump(t, f)
    for e in t:
        print(f"bench: tune level {e['level']:2d} {e['op']:3s} lanes {e['lanes']:2d} xcd {e['xcd_map']} "
              f"lds {e['lds']} {e['best_us']:8.2f} us (default {e['default_lanes']:2d}/"
              f"{e['default_xcd_map']}/{e['default_lds']} {e['default_us']:8.2f} us)", file=sys.stderr)
    return {"operators": len(t), "changed": sum(e["lanes"] != e["default_lanes"] for e in t),
            "default_us_sum": round(sum(e["default_us"] for e in t), 1),
            "tuned_us_sum": round(sum(e["best_us"] for e in t), 1)}


def _timed(fn, warmup, steps):
    import torch
    for _ in range(warmup):
        r = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, r


def batched_legs(a, p, s64, value64, ip, ix, dv):
    """Batching with FP32 storage in the V-cycle (FP64 FGMRES): many right-hand
    sides of the big matrix as interleaved columns, and many independent
    problems of uneven sizes in one block-diagonal hierarchy (FP32, then BF16
    storage).  Every column and problem must reach the FP64 1e-10 true
    relative residual."""
    import torch
    from airg_inputs import workloads
    from paper_2508_17517_amd import BatchSolver, Solver, binding
    res = {}
    k = a.batch_cols
    print(f"bench: batch: {k} right-hand sides, FP32 V-cycle", file=sys.stderr, flush=True)
    B = torch.from_numpy(workloads.rhs_batch(p, k)).cuda()
    sm = Solver(ip, ix, dv, precision=binding.FP32, **SOLVER_OPTS)
    _tune(sm)
    X = torch.zeros_like(B)
    dt, (X, infos) = _timed(lambda: sm.solve(B, X), 1, max(1, min(a.steps, 3)))
    assert all(i["converged"] == 1 and i["rel_residual"] <= 1e-10 for i in infos), infos
    # the same columns one at a time in FP64, for the error of each column
    xs = torch.zeros_like(B[0])
    err = 0.0
    for c in (0, k - 1):
        xs, _ = s64.solve(B[c], xs)
        err = max(err, float(torch.linalg.norm(X[c] - xs) / torch.linalg.norm(xs)))
    v = p.n * k / dt
    res["columns"] = {"rhs": k, "value": v, "unit": "DOF/s", "ms_per_step": 1e3 * dt,
                      "iterations": max(i["iterations"] for i in infos),
                      "iterations_min": min(i["iterations"] for i in infos),
                      "max_rel_residual": max(i["rel_residual"] for i in infos),
                      "rel_diff_vs_fp64_single": err, "speedup_vs_fp64": v / value64}
    print(f"bench: columns {res['columns']}", file=sys.stderr, flush=True)
    sm.close()
    del B, X
    q = a.batch_problems
    print(f"bench: batch: {q} problems (generating)", file=sys.stderr, flush=True)
    probs = workloads.batch_problems(q)
    ntot = sum(pr.n for pr in probs)
    mats = [(torch.from_numpy(pr.indptr).cuda(), torch.from_numpy(pr.indices).cuda(),
             torch.from_numpy(pr.data).cuda()) for pr in probs]
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    # the last leg also swaps the matrix-free smoother for the assembled
    # fixed-sparsity one (another preconditioner: reported beside, not as,
    # the plain batches)
    for key, prec, extra in (("problems", binding.FP32, {}), ("problems_bf16", binding.BF16, {}),
                             ("problems_bf16_assembled", binding.BF16,
                              {"smoother": binding.SMOOTH_ASSEMBLED})):
        print(f"bench: batch: {q} problems, {key}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sb = BatchSolver(mats, precision=prec, **extra, **SOLVER_OPTS)
        torch.cuda.synchronize()
        setup_b = time.perf_counter() - t0
        _tune(sb)
        xs = [torch.zeros_like(b_) for b_ in bs]
        dt, (xs, infos) = _timed(lambda: sb.solve(bs, xs), 1, max(1, min(a.steps, 3)))
        assert all(i["converged"] == 1 and i["rel_residual"] <= 1e-10 for i in infos), infos
        st = sb.stats()
        v = ntot / dt
        res[key] = {"problems": q, "dofs": ntot,
                    "precision": "fp32" if prec == binding.FP32 else "bf16",
                    "smoother": "assembled" if extra else "polynomial",
                    "value": v, "unit": "DOF/s", "ms_per_step": 1e3 * dt,
                    "iterations": max(i["iterations"] for i in infos),
                    "iterations_min": min(i["iterations"] for i in infos),
                    "max_rel_residual": max(i["rel_residual"] for i in infos),
                    "levels": st["levels"], "setup_s": round(setup_b, 3),
                    "setup_component_ms": {k: round(v, 1) for k, v in
                                           st["setup_component_ms"].items()},
                    "speedup_vs_fp64": v / value64}
        print(f"bench: {key} {res[key]}", file=sys.stderr, flush=True)
        sb.close()
    return res


def dg_legs(a, side=1024):
    """The upwind DG-Q1 system (theta = pi/5, element-block scaled, permuted):
    FP64, then FP32 and BF16 storage in the V-cycle inside FP64 FGMRES, each to
    the FP64 1e-10 true relative residual, with the error against the FP64
    solution."""
    import torch
    from airg_inputs import workloads
    from paper_2508_17517_amd import Solver, binding
    print(f"bench: dg: generating DG-Q1 {side}x{side}", file=sys.stderr, flush=True)
    p = workloads.dg_random(side, math.pi / 5.0, True)
    ip = torch.from_numpy(p.indptr).cuda()
    ix = torch.from_numpy(p.indices).cuda()
    dv = torch.from_numpy(p.data).cuda()
    b = torch.from_numpy(p.b).cuda()
    res = {"workload": f"upwind DG-Q1 {side}x{side} cells, theta pi/5, block-scaled, permuted, "
                       "g~U(0,1)", "n": p.n, "nnz": p.nnz}
    xref = None
    for name, prec in (("fp64", binding.FP64), ("fp32", binding.FP32), ("bf16", binding.BF16)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sm = Solver(ip, ix, dv, precision=prec, **SOLVER_OPTS)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        _tune(sm)
        xm = torch.zeros_like(b)
        dt, (xm, im) = _timed(lambda: sm.solve(b, xm), a.warmup, a.steps)
        assert im["converged"] == 1 and im["rel_residual"] <= 1e-10, im
        kt = sm.time_kernels("poly", reps=a.kernel_reps)
        leg = {"value": p.n / dt, "unit": "DOF/s", "ms_per_step": 1e3 * dt,
               "iterations": im["iterations"], "rel_residual": im["rel_residual"],
               "setup_s": round(setup_s, 3),
               "poly_gbps": kt["bytes_per_launch"] / (kt["avg_launch_ms"] * 1e-3) / 1e9}
        if xref is None:
            xref = xm.clone()
            st = sm.stats()
            leg.update(levels=st["levels"], cycle_complexity=round(st["cycle_complexity"], 2))
        else:
            leg["rel_diff_vs_fp64_solution"] = float(torch.linalg.norm(xm - xref) /
                                                     torch.linalg.norm(xref))
            leg["speedup_vs_fp64"] = leg["value"] / res["fp64"]["value"]
        res[name] = leg
        print(f"bench: dg {name}: {leg}", file=sys.stderr, flush=True)
        sm.close()
    return res


PAPER_SINGLE_GCD = {  # Sec. 3.1, one MI250X GCD, 13M unknowns, pi/4, d = 6
    "truncated_mc10": {"iterations": 7, "levels": 13, "cycle_complexity": 28.0,
                       "storage_complexity": 10.22},
    "untruncated": {"iterations": 7, "levels": 22, "cycle_complexity": 27.2,
                    "storage_complexity": 10.21},
    # Sec. 3.3: nAIR with the same options, 7 iterations on 2 nodes (15 on 2048)
    "nair_truncated_mc10": {"iterations": 7},
    # Sec. 3.4: 500 x N rectangles weak-scaled in y, m_c = 10 (constant over the runs)
    "rectangular_mc10": {"iterations": 6, "levels": 10, "cycle_complexity": 28.2,
                         "storage_complexity": 9.5},
    # Sec. 3.3 (2 nodes): storage 10.5 with F smoothing, 17.2 with matrix-free
    # C smoothing added, 20.2 with assembled F and C smoothing
    "fc_truncated_mc10": {"storage_ratio_vs_f": round(17.2 / 10.5, 3)},
    "fc_assembled_truncated_mc10": {"storage_ratio_vs_f": round(20.2 / 10.5, 3)},
}


def paper_legs(a, side=3606):
    """The paper's own setting (Sec. 3): FD with the inflow boundary nodes kept,
    theta = pi/4, g = 0, x0 = 1, undamped Richardson to 1e-10 of the initial
    residual, smoother degree 6, truncation 1e-1 with coarse degree 10 (and
    100), and without truncation; the paper's single-GCD figures alongside."""
    import torch
    from airg_inputs import workloads
    from paper_2508_17517_amd import Solver, binding
    print(f"bench: paper: generating FD {side}x{side}", file=sys.stderr, flush=True)
    p = workloads.fd_paper(side)
    ip = torch.from_numpy(p.indptr).cuda()
    ix = torch.from_numpy(p.indices).cuda()
    dv = torch.from_numpy(p.data).cuda()
    b = torch.from_numpy(p.b).cuda()
    res = {"workload": f"FD {side}x{side} (inflow boundary nodes kept), theta pi/4, g = 0, x0 = 1, "
                       "Richardson rtol 1e-10, d = 6", "n": p.n, "nnz": p.nnz, "paper": PAPER_SINGLE_GCD}
    legs = (("truncated_mc10", dict(coarse_poly_order=10, trunc_tol=0.1)),
            ("truncated_mc100", dict(coarse_poly_order=100, trunc_tol=0.1)),
            ("untruncated", dict(coarse_poly_order=10, trunc_tol=0.0)),
            ("nair_truncated_mc10", dict(coarse_poly_order=10, trunc_tol=0.1,
                                         inverse_type=binding.INVERSE_NEUMANN)),
            ("fc_truncated_mc10", dict(coarse_poly_order=10, trunc_tol=0.1,
                                       smooth_type=binding.SMOOTH_TYPE_FC)),
            ("fcf_truncated_mc10", dict(coarse_poly_order=10, trunc_tol=0.1,
                                        smooth_type=binding.SMOOTH_TYPE_FCF)),
            ("fc_assembled_truncated_mc10", dict(coarse_poly_order=10, trunc_tol=0.1,
                                                 smooth_type=binding.SMOOTH_TYPE_FC,
                                                 smoother=binding.SMOOTH_ASSEMBLED)),
            ("rectangular_mc10", dict(coarse_poly_order=10, trunc_tol=0.1)))
    for name, over in legs:
        if name == "rectangular_mc10":
            # one GPU's share of the rectangular study: 500 x 26000 nodes (13.0M)
            from airg_inputs import fd_advection
            del ip, ix, dv, b
            q = fd_advection(500, math.pi / 4.0, 0.0, ny=26000)
            ip = torch.from_numpy(q.indptr).cuda()
            ix = torch.from_numpy(q.indices).cuda()
            dv = torch.from_numpy(q.data).cuda()
            b = torch.from_numpy(q.b).cuda()
            p = q
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sm = Solver(ip, ix, dv, poly_order=6, outer=binding.OUTER_RICHARDSON, **over, **SOLVER_OPTS)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        _tune(sm)
        x = torch.ones_like(b)

        def run():
            x.fill_(1.0)
            return sm.solve(b, x=x, guess=True)
        dt, (x, info) = _timed(run, 1, max(1, min(a.steps, 3)))
        assert info["converged"] == 1, info
        st = sm.stats()
        leg = {"iterations": info["iterations"], "rel_residual": info["rel_residual"],
               "levels": st["levels"], "cycle_complexity": round(st["cycle_complexity"], 2),
               "storage_complexity": round(st["storage_complexity"], 2),
               "grid_complexity": round(st["grid_complexity"], 3), "setup_s": round(setup_s, 3),
               "solve_ms": round(1e3 * dt, 3), "value": p.n / dt, "unit": "DOF/s",
               "dof_per_s_per_vcycle": p.n * info["iterations"] / dt}
        if name == "rectangular_mc10":
            leg["grid"] = "500 x 26000"
        if "smooth_type" in over and "truncated_mc10" in res:
            leg["storage_ratio_vs_f"] = round(
                st["storage_complexity"] / res["truncated_mc10"]["storage_complexity"], 3)
        res[name] = leg
        print(f"bench: paper {name}: {leg}", file=sys.stderr, flush=True)
        sm.close()
    return res


def mixed_legs(a, p, x64, value64, ip, ix, dv, b):
    """FP32 and BF16 storage in the V-cycle inside FP64 FGMRES on the bench
    workload, to the same 1e-10 true FP64 residual."""
    import torch
    from paper_2508_17517_amd import Solver, binding
    res = {}
    xref = x64.clone()
    for name, prec in (("fp32", binding.FP32), ("bf16", binding.BF16)):
        sm = Solver(ip, ix, dv, precision=prec, **SOLVER_OPTS)
        _tune(sm)
        xm = torch.zeros_like(b)
        dtm, (xm, im) = _timed(lambda: sm.solve(b, xm), a.warmup, a.steps)
        assert im["converged"] == 1 and im["rel_residual"] <= 1e-10, im
        err = float(torch.linalg.norm(xm - xref) / torch.linalg.norm(xref))
        ktm = sm.time_kernels("poly", reps=a.kernel_reps)
        res[name] = {"value": p.n / dtm, "ms_per_step": 1000.0 * dtm,
                     "iterations": im["iterations"], "rel_residual": im["rel_residual"],
                     "rel_diff_vs_fp64_solution": err, "speedup_vs_fp64": (p.n / dtm) / value64,
                     "poly_gbps": ktm["bytes_per_launch"] / (ktm["avg_launch_ms"] * 1e-3) / 1e9}
        print(f"bench: {name}: {res[name]}", file=sys.stderr, flush=True)
        sm.close()
    return res


def assembled_leg(a, p, value64, ip, ix, dv, b):
    """F-point smoothing with the assembled fixed-sparsity Ahat^{-1} (one
    product per level instead of d matrix-free ones), FP64, same tolerance."""
    import torch
    from paper_2508_17517_amd import Solver, binding
    sm = Solver(ip, ix, dv, smoother=binding.SMOOTH_ASSEMBLED, **SOLVER_OPTS)
    _tune(sm)
    xm = torch.zeros_like(b)
    dt, (xm, im) = _timed(lambda: sm.solve(b, xm), a.warmup, a.steps)
    assert im["converged"] == 1 and im["rel_residual"] <= 1e-10, im
    st = sm.stats()
    res = {"value": p.n / dt, "unit": "DOF/s", "ms_per_step": 1e3 * dt,
           "iterations": im["iterations"], "rel_residual": im["rel_residual"],
           "cycle_complexity": round(st["cycle_complexity"], 2),
           "storage_complexity": round(st["storage_complexity"], 2),
           "ms_per_vcycle": 1e3 * dt / max(im["iterations"], 1),
           "speedup_vs_fp64_poly": (p.n / dt) / value64}
    print(f"bench: assembled smoother: {res}", file=sys.stderr, flush=True)
    sm.close()
    return res


def persistent_coarse_leg(a, p, value64, ip, ix, dv, b, newton_us):
    """The coarsest level's Newton steps in one persistent launch
    (coarse_persistent = 1) against the per-step launches of the main solve:
    same hierarchy and launch shapes, FP64, same tolerance."""
    import torch
    from paper_2508_17517_amd import Solver
    sm = Solver(ip, ix, dv, coarse_persistent=1, **SOLVER_OPTS)
    kept = os.path.join(ROOT, "paper_2508_17517_amd", "shapes", f"{a.workload}_fp64.json")
    if TUNE["on"] and os.path.exists(kept):
        with open(kept) as f:
            sm.pin_shapes(json.load(f))
    else:
        _tune(sm)
    xm = torch.zeros_like(b)
    dt, (xm, im) = _timed(lambda: sm.solve(b, xm), a.warmup, a.steps)
    assert im["converged"] == 1 and im["rel_residual"] <= 1e-10, im
    kt = sm.time_kernels("newton", reps=a.kernel_reps)
    res = {"value": p.n / dt, "unit": "DOF/s", "ms_per_step": 1e3 * dt,
           "iterations": im["iterations"], "rel_residual": im["rel_residual"],
           # one launch per Newton apply where the coarsest level fits, else
           # the per-step launches ran
           "persistent_launch": kt["launches"] == 1,
           "newton_apply_us": 1e3 * kt["avg_launch_ms"] * kt["launches"],
           "per_step_newton_apply_us": newton_us,
           "speedup_vs_fp64": (p.n / dt) / value64}
    print(f"bench: persistent coarse solve: {res}", file=sys.stderr, flush=True)
    sm.close()
    return res


def optional(name, fn, *args):
    """Run one extra bench leg; a failure is reported and does not lose the
    main result."""
    try:
        return fn(*args)
    except Exception as e:  # noqa: BLE001
        print(f"bench: {name} leg failed: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
        return {"error": f"{type(e).__name__}: {e}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fv2048", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-dg", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-file", default=None,
                    help="read the main solver's launch shapes from this JSON file if it "
                         "exists, else tune and write them there (default: the shapes kept "
                         "for the workload in paper_2508_17517_amd/shapes/, which the "
                         "full-size parity test pins too; none kept: tune)")
    ap.add_argument("--retune", action="store_true",
                    help="tune the main solver's shapes instead of pinning the kept ones")
    ap.add_argument("--graph", type=int, default=None, choices=(0, 1),
                    help="replay V-cycles from captured HIP graphs (1) or launch them kernel by "
                         "kernel (0); default: the library's default")
    ap.add_argument("--batch-cols", type=int, default=64)
    ap.add_argument("--batch-problems", type=int, default=48)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the solver has no multi-GPU "
              "path", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from airg_inputs import workloads
    from paper_2508_17517_amd import Solver, binding

    if a.graph is not None:
        SOLVER_OPTS["graph"] = a.graph
    side, theta, perm = WORKLOADS[a.workload]
    print(f"bench: generating {a.workload}", file=sys.stderr, flush=True)
    p = workloads.fv_random(side, theta, perm)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ip = torch.from_numpy(p.indptr).cuda()
    ix = torch.from_numpy(p.indices).cuda()
    dv = torch.from_numpy(p.data).cuda()
    b = torch.from_numpy(p.b).cuda()
    torch.cuda.synchronize()
    print("bench: setup", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = Solver(ip, ix, dv, **SOLVER_OPTS)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    TUNE["on"] = not a.no_autotune
    kept = os.path.join(ROOT, "paper_2508_17517_amd", "shapes", f"{a.workload}_fp64.json")
    TUNE["file"] = a.tune_file or (kept if os.path.exists(kept) and not a.retune else None)
    tune = _tune(s, main=True)
    print(f"bench: autotune {tune}", file=sys.stderr, flush=True)
    st = s.stats()
    for l in range(st["levels"]):
        print(f"bench: level {l}: n {st['n'][l]} nnz {st['nnz'][l]} nF {st['n_f'][l]} "
              f"nnz_ff {st['nnz_ff'][l]} nnz_fc {st['nnz_fc'][l]} nnz_z {st['nnz_z'][l]} "
              f"d {st['poly_degree'][l]}", file=sys.stderr)
    print(f"bench: setup {setup_s:.3f} s {st['setup_component_ms']}", file=sys.stderr, flush=True)
    x = torch.zeros_like(b)
    for w in range(a.warmup):
        x, info = s.solve(b, x)
        print(f"bench: warmup {w} its={info['iterations']} rel={info['rel_residual']:.2e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(a.steps):
        x, info = s.solve(b, x)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for info in infos:
        assert info["converged"] == 1 and info["rel_residual"] <= 1e-10, info
    its = infos[-1]["iterations"]
    value = p.n * a.steps / dt
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"upwind FV {side}x{side}, theta {theta}, "
                               f"{'permuted, ' if perm else ''}g~U(0,1); AIRG d=4, m_c=20, "
                               f"trunc 1e-2, FGMRES(30) rtol 1e-10",
                   "n": p.n, "nnz": p.nnz, "iterations": its,
                   "levels": st["levels"], "cycle_complexity": round(st["cycle_complexity"], 2),
                   "storage_complexity": round(st["storage_complexity"], 2),
                   "grid_complexity": round(st["grid_complexity"], 3),
                   "setup_s": round(setup_s, 3), "autotune": tune,
                   "dof_per_s_per_vcycle": p.n * its * a.steps / dt},
        "roofline": None,
        "cpu_baseline": None,
    }
    # per-class kernel timing (HIP events on the library's stream), right after
    # the timed region on the same hierarchy
    classes = {}
    for cls in ("poly", "horner", "newton", "residual", "restrict", "top_spmv"):
        kt = s.time_kernels(cls, reps=a.kernel_reps)
        kt["gbps"] = kt["bytes_per_launch"] / (kt["avg_launch_ms"] * 1e-3) / 1e9
        classes[cls] = kt
        print(f"bench: {cls:9s} launches/V-cycle {kt['launches']:4d}  avg {1e3 * kt['avg_launch_ms']:8.2f} us"
              f"  {kt['bytes_per_launch'] / 1e6:8.3f} MB/launch  {kt['gbps']:8.1f} GB/s",
              file=sys.stderr, flush=True)
    dom = classes["poly"]
    out["roofline"] = {"bound": "hbm", "kernel": "poly-SpMV (Horner smoother steps + Newton "
                                                 "coarse steps, one V-cycle's launches)",
                       "achieved": dom["gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": dom["gbps"] / HBM_PEAK_GBPS,
                       "traffic": measured_traffic(a.workload),
                       "avg_launch_us": 1e3 * dom["avg_launch_ms"],
                       "bytes_per_launch": dom["bytes_per_launch"],
                       "stored_bytes_per_launch": dom["stored_bytes_per_launch"],
                       "stored_gbps": dom["stored_bytes_per_launch"] /
                                      (dom["avg_launch_ms"] * 1e-3) / 1e9,
                       "launches_per_vcycle": dom["launches"]}
    out["kernel_classes_gbps"] = {k: round(v["gbps"], 1) for k, v in classes.items()}
    # mixed precision: FP32 / BF16 storage in the V-cycle inside FP64 FGMRES,
    # the same 1e-10 true FP64 residual
    if not a.no_mixed:
        out["mixed"] = optional("mixed", mixed_legs, a, p, x, value, ip, ix, dv, b)
    if not a.no_mixed:
        out["assembled_smoother"] = optional("assembled", assembled_leg, a, p, value, ip, ix, dv, b)
        nw = classes["newton"]
        out["persistent_coarse"] = optional("persistent", persistent_coarse_leg, a, p, value, ip, ix,
                                            dv, b, 1e3 * nw["avg_launch_ms"] * nw["launches"])
    if not a.no_batch:
        out["batched"] = optional("batched", batched_legs, a, p, s, value, ip, ix, dv)
    if not a.no_dg:
        out["dg_q1"] = optional("dg", dg_legs, a)
    if not a.no_paper:
        out["paper_fd"] = optional("paper", paper_legs, a)
    # the practical ceilings, from the library's own streaming kernels
    out["hbm_read_gbps"] = stream_bandwidth("read", 1 << 31)
    out["hbm_copy_gbps"] = stream_bandwidth("copy", 1 << 30, blocks=16384)
    out["roofline"]["frac_of_read_ceiling"] = dom["gbps"] / out["hbm_read_gbps"]
    print(f"bench: streaming read {out['hbm_read_gbps']:.1f} GB/s, copy {out['hbm_copy_gbps']:.1f} GB/s "
          f"(library probes)", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_sample)
    s.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
