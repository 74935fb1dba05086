"""ctypes declarations of the C ABI in include/airg.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libairg.so")
HOST_LIB_PATH = os.path.join(HERE, "libairg_dense_host.so")
MAX_LEVELS = 64

c_i32, c_i64, c_u64, c_dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
P = ctypes.POINTER

STATUS = {0: "AIRG_OK", 1: "AIRG_NOT_CONVERGED", -1: "AIRG_ERR_INVALID", -2: "AIRG_ERR_ZERO_DIAG",
          -3: "AIRG_ERR_NONFINITE", -4: "AIRG_ERR_HIP", -5: "AIRG_ERR_NOMEM",
          -6: "AIRG_ERR_BREAKDOWN", -7: "AIRG_ERR_INTERNAL"}
FP64, FP32, BF16 = 0, 1, 2
OUTER_FGMRES, OUTER_RICHARDSON = 0, 1
SMOOTH_POLY, SMOOTH_ASSEMBLED = 0, 1
INVERSE_ARNOLDI, INVERSE_NEUMANN = 0, 1
SMOOTH_TYPE_F, SMOOTH_TYPE_FC, SMOOTH_TYPE_FCF = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [("strong_threshold", c_dbl), ("ddc_fraction", c_dbl), ("a_drop", c_dbl),
                ("r_drop", c_dbl), ("trunc_tol", c_dbl), ("rtol", c_dbl), ("seed", c_u64),
                ("min_coarse_rows", c_i64), ("ddc_its", c_i32), ("lump", c_i32),
                ("poly_order", c_i32), ("coarse_poly_order", c_i32), ("trunc_start_level", c_i32),
                ("max_levels", c_i32), ("added_roots", c_i32), ("precision", c_i32),
                ("max_it", c_i32), ("restart", c_i32), ("keep_setup_data", c_i32),
                ("locality_order", c_i32), ("outer", c_i32), ("smoother", c_i32),
                ("inverse_type", c_i32), ("smooth_type", c_i32), ("atol", c_dbl), ("graph", c_i32),
                ("stagnation_check", c_i32), ("coarse_persistent", c_i32), ("lookahead", c_i32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("converged", c_i32), ("restarts", c_i32),
                ("stagnated", c_i32), ("rel_residual", c_dbl), ("rel_residual_estimate", c_dbl),
                ("solve_ms", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("levels", c_i32), ("coarse_roots", c_i32),
                ("n", c_i64 * MAX_LEVELS), ("nnz", c_i64 * MAX_LEVELS),
                ("n_f", c_i64 * MAX_LEVELS), ("nnz_ff", c_i64 * MAX_LEVELS),
                ("nnz_fc", c_i64 * MAX_LEVELS), ("nnz_z", c_i64 * MAX_LEVELS),
                ("poly_degree", c_i32 * MAX_LEVELS), ("pmisr_rounds", c_i32 * MAX_LEVELS),
                ("trunc_rel", c_dbl * MAX_LEVELS), ("grid_complexity", c_dbl),
                ("cycle_complexity", c_dbl), ("storage_complexity", c_dbl),
                ("vcycle_bytes", c_dbl), ("setup_ms", c_dbl), ("setup_component_ms", c_dbl * 8)]

    def as_dict(self):
        L = self.levels
        out = {"levels": L, "coarse_roots": self.coarse_roots}
        for k in ("n", "nnz", "n_f", "nnz_ff", "nnz_fc", "nnz_z", "poly_degree", "pmisr_rounds",
                  "trunc_rel"):
            out[k] = list(getattr(self, k))[:L]
        for k in ("grid_complexity", "cycle_complexity", "storage_complexity", "vcycle_bytes",
                  "setup_ms"):
            out[k] = getattr(self, k)
        names = ["cf_split", "prolongator", "gmres_poly", "restrictor_spgemm", "coarse_spgemm",
                 "extract", "drop", "truncation"]
        out["setup_component_ms"] = dict(zip(names, list(self.setup_component_ms)))
        return out


class LevelInfo(ctypes.Structure):
    _fields_ = [("n", c_i64), ("n_f", c_i64), ("n_c", c_i64), ("nnz_a", c_i64),
                ("nnz_ff", c_i64), ("nnz_fc", c_i64), ("nnz_z", c_i64), ("is_coarsest", c_i32),
                ("poly_len", c_i32), ("n_roots", c_i32), ("c_poly_len", c_i32)]


class LevelArrays(ctypes.Structure):
    _fields_ = [("state", P(ctypes.c_int8)),
                ("a_rowptr", P(c_i32)), ("a_col", P(c_i32)), ("a_val", P(c_dbl)),
                ("ff_rowptr", P(c_i32)), ("ff_col", P(c_i32)), ("ff_val", P(c_dbl)),
                ("fc_rowptr", P(c_i32)), ("fc_col", P(c_i32)), ("fc_val", P(c_dbl)),
                ("z_rowptr", P(c_i32)), ("z_col", P(c_i32)), ("z_val", P(c_dbl)),
                ("cmap", P(c_i32)), ("alpha", P(c_dbl)), ("roots_re", P(c_dbl)),
                ("roots_im", P(c_dbl)), ("alpha_c", P(c_dbl))]


class KernelTiming(ctypes.Structure):
    _fields_ = [("launches", c_i32), ("reserved", c_i32), ("avg_launch_ms", c_dbl),
                ("bytes_per_launch", c_dbl), ("flops_per_launch", c_dbl),
                ("stored_bytes_per_launch", c_dbl)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class TuneEntry(ctypes.Structure):
    _fields_ = [("level", c_i32), ("op", c_i32), ("lanes", c_i32), ("xcd_map", c_i32),
                ("lds", c_i32), ("default_lanes", c_i32), ("default_xcd_map", c_i32),
                ("default_lds", c_i32), ("best_us", c_dbl), ("default_us", c_dbl)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["op"] = OPERATORS_BY_CODE[d["op"]]
        return d


OPERATORS = {"ff": 0, "b": 1, "z": 2, "a": 3, "top": 4, "hat": 5}
OPERATORS_BY_CODE = {v: k for k, v in OPERATORS.items()}

KERNEL_CLASSES = {"poly": 0, "horner": 1, "newton": 2, "residual": 3, "restrict": 4, "top_spmv": 5}

SYMBOLS = {
    "airg_params_default": (c_i32, [P(Params)]),
    "airg_setup": (c_i32, [P(ctypes.c_void_p), c_i64, c_i64, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_int, P(Params), ctypes.c_void_p]),
    "airg_solve": (c_i32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, c_i64, ctypes.c_void_p,
                           c_i64, ctypes.c_int, P(SolveInfo)]),
    "airg_setup_batch": (c_i32, [P(ctypes.c_void_p), ctypes.c_int, P(c_i64), P(c_i64),
                                 P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_void_p),
                                 ctypes.c_int, P(Params), ctypes.c_void_p]),
    "airg_solve_batch": (c_i32, [ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_void_p),
                                 ctypes.c_int, P(SolveInfo)]),
    "airg_adjoint_solve": (c_i32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, c_i64,
                                   ctypes.c_void_p, c_i64, ctypes.c_int, P(SolveInfo)]),
    "airg_get_stats": (c_i32, [ctypes.c_void_p, P(Stats)]),
    "airg_trim": (c_i32, [ctypes.c_void_p]),
    "airg_level_info_get": (c_i32, [ctypes.c_void_p, ctypes.c_int, P(LevelInfo)]),
    "airg_export_level": (c_i32, [ctypes.c_void_p, ctypes.c_int, P(LevelArrays)]),
    "airg_import_hierarchy": (c_i32, [P(ctypes.c_void_p), ctypes.c_int, P(LevelInfo),
                                      P(LevelArrays), P(Params), ctypes.c_void_p]),
    "airg_time_kernels": (c_i32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, P(KernelTiming)]),
    "airg_autotune": (c_i32, [ctypes.c_void_p, ctypes.c_int, P(TuneEntry), ctypes.c_int, P(ctypes.c_int)]),
    "airg_set_lanes": (c_i32, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int]),
    "airg_fv_nnz": (c_i32, [c_i64, c_i64, c_dbl, P(c_i64)]),
    "airg_fv_assemble": (c_i32, [c_i64, c_i64, c_dbl] + [ctypes.c_void_p] * 9),
    "airg_fv_gradients": (c_i32, [c_i64, c_i64, c_dbl] + [ctypes.c_void_p] * 10),
    "airg_fv_gradients_noalloc": (c_i32, [c_i64, c_i64, c_dbl] + [ctypes.c_void_p] * 10),
    "airg_stream_probe": (c_i32, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, c_i64, ctypes.c_int,
                                  ctypes.c_int, P(c_dbl), ctypes.c_void_p]),
    "airg_set_alloc_budget": (c_i32, [c_i64, P(c_i64)]),
    "airg_set_spin_limit": (c_i32, [c_i64]),
    "airg_destroy": (None, [ctypes.c_void_p]),
    "airg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "airg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path=None):
    """Load libairg.so, or the build at `path`, which then serves every later
    call (Solver, BatchSolver, ...); raises if it has not been built (no
    fallback exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2508_17517_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AirgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code, lib=None):
    lib = lib or load()
    if code < 0:
        raise AirgError(code, lib.airg_last_error().decode())
    return code


def default_params(**overrides):
    p = Params()
    check(load().airg_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def load_host_dense():
    """Host-only build of the library's dense routines (CPU tests); the
    environment variable AIRG_HOST_LIB selects another build of them (the
    sanitizer build)."""
    path = os.environ.get("AIRG_HOST_LIB", HOST_LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run the build")
    lib = ctypes.CDLL(path)
    dp, ip = P(c_dbl), ctypes.c_int
    lib.airg_host_gmres_poly.argtypes = [dp, ip, ip, c_dbl, dp]
    lib.airg_host_gmres_poly.restype = ip
    lib.airg_host_hessenberg_eig.argtypes = [dp, ip, dp, dp]
    lib.airg_host_hessenberg_eig.restype = ip
    lib.airg_host_newton_roots.argtypes = [dp, ip, ip, ip, dp, dp, ip]
    lib.airg_host_newton_roots.restype = ip
    lib.airg_host_numerical_rank.argtypes = [dp, ip, ip, c_dbl]
    lib.airg_host_numerical_rank.restype = ip
    return lib
