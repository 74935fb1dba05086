"""MI355X AIRG reduction-multigrid solver for upwind advection systems.

Thin Python layer over the C ABI of libairg.so (include/airg.h): it only
marshals arguments.  Device memory comes from PyTorch tensors and every step of
the setup and solve runs in the library's HIP kernels.

    from paper_2508_17517_amd import Solver
    s = Solver(indptr, indices, data)          # AIRG setup on the GPU
    x, info = s.solve(b)                       # FGMRES + V-cycles, b a CUDA float64 tensor
    lam, info = s.adjoint_solve(w)             # A^T lam = w on a transpose hierarchy
"""
import ctypes
import json
import os

import numpy as np

from . import binding
from .binding import AirgError, FP64, FP32, BF16, default_params  # noqa: F401

__all__ = ["Solver", "BatchSolver", "AirgError", "default_params", "FP64", "FP32", "BF16"]


SHAPES_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shapes")


def load_shapes(name):
    """Launch shapes kept for a named workload (shapes/<name>.json, e.g.
    "fv2048_fp64"): one entry per solve operator with its level, operator,
    lanes per row, XCD mapping and LDS staging, as airg_autotune chose them on
    an MI355X.  Pinning them with Solver.pin_shapes makes a solve launch
    exactly those kernels, so its rounding (and its results) are reproducible."""
    with open(os.path.join(SHAPES_DIR, name + ".json")) as f:
        return json.load(f)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _as_device(a, dtype):
    """A contiguous CUDA tensor of dtype holding `a` (numpy or torch)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _np_ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Solver:
    """AIRG-preconditioned FGMRES for the CSR matrix (indptr, indices, data).

    indptr/indices are int32, data float64, columns ascending per row with a
    nonzero diagonal; numpy arrays are copied to the device first.  Keyword
    overrides set fields of the parameter struct (e.g. poly_order=6).
    """

    def __init__(self, indptr=None, indices=None, data=None, params=None, stream=None,
                 _handle=None, **overrides):
        self.lib = binding.load()
        self.params = params if params is not None else default_params(**overrides)
        if params is not None:
            for k, v in overrides.items():
                setattr(self.params, k, v)
        self.stream = stream
        self.h = ctypes.c_void_p()
        if _handle is not None:
            self.h = _handle
        else:
            torch = _torch()
            ip = _as_device(indptr, torch.int32)
            ix = _as_device(indices, torch.int32)
            dv = _as_device(data, torch.float64)
            n = ip.numel() - 1
            code = self.lib.airg_setup(ctypes.byref(self.h), n, ix.numel(), _ptr(ip), _ptr(ix),
                                       _ptr(dv), 1, ctypes.byref(self.params),
                                       _stream_ptr(stream))
            binding.check(code, self.lib)
        st = self.stats()
        self.n = st["n"][0]

    # ------------------------------------------------------------------ solve
    def _solve(self, fn, b, x, guess):
        torch = _torch()
        b = _as_device(b, torch.float64)
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if x is None:
            x = torch.zeros_like(b)
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.shape != b.shape:
            raise ValueError("x must be a contiguous CUDA float64 tensor shaped like b")
        infos = (binding.SolveInfo * nrhs)()
        code = fn(self.h, nrhs, _ptr(b), self.n, _ptr(x), self.n, 1 if guess else 0, infos)
        binding.check(code, self.lib)
        res = [i.as_dict() for i in infos]
        return x, (res[0] if b.dim() == 1 else res)

    def solve(self, b, x=None, guess=False):
        """Solve A x = b; b is [n] or [nrhs, n].  Returns (x, info)."""
        return self._solve(self.lib.airg_solve, b, x, guess)

    def adjoint_solve(self, w, lam=None, guess=False):
        """Solve A^T lam = w (the transpose hierarchy is built on first use)."""
        return self._solve(self.lib.airg_adjoint_solve, w, lam, guess)

    def trim(self):
        """Free the workspaces kept for multi-column solves (airg_trim)."""
        binding.check(self.lib.airg_trim(self.h), self.lib)

    # ------------------------------------------------------------------ introspection
    def stats(self):
        s = binding.Stats()
        binding.check(self.lib.airg_get_stats(self.h, ctypes.byref(s)), self.lib)
        return s.as_dict()

    def time_kernels(self, cls="poly", reps=20):
        """Average launch time and algorithmic bytes of one kernel class of the
        V-cycle (see airg_time_kernels)."""
        kt = binding.KernelTiming()
        code = self.lib.airg_time_kernels(self.h, binding.KERNEL_CLASSES[cls], reps, ctypes.byref(kt))
        binding.check(code, self.lib)
        return kt.as_dict()

    def autotune(self, reps=10):
        """Time every solve operator's product with 1..64 lanes per row and keep
        the fastest (see airg_autotune); returns one dict per operator."""
        n = ctypes.c_int()
        cap = 3 * 64 + 2  # three operators per level plus the coarsest and the top matrix
        buf = (binding.TuneEntry * cap)()
        binding.check(self.lib.airg_autotune(self.h, reps, buf, cap, ctypes.byref(n)), self.lib)
        return [buf[i].as_dict() for i in range(min(n.value, cap))]

    def set_lanes(self, level, op, lanes, xcd_map=0, lds=0):
        """Pin the launch shape of one solve operator ("ff", "b", "z", "a", "top"):
        lanes per row (0 = row-block kernel), the XCD mapping and LDS staging."""
        binding.check(self.lib.airg_set_lanes(self.h, level, binding.OPERATORS[op], lanes, xcd_map,
                                              lds), self.lib)

    def pin_shapes(self, shapes):
        """Pin every operator's launch shape from a list of entries (as
        load_shapes or autotune return them)."""
        for e in shapes:
            self.set_lanes(e["level"], e["op"], e["lanes"], e["xcd_map"], e["lds"])

    def level_info(self, level):
        li = binding.LevelInfo()
        binding.check(self.lib.airg_level_info_get(self.h, level, ctypes.byref(li)), self.lib)
        return li

    def export_level(self, level, what=("state", "a", "ff", "fc", "z", "cmap", "alpha", "roots")):
        """Host copies of one level in setup numbering (needs keep_setup_data=1 for
        everything but the coarsest matrix, the coefficients and the roots)."""
        li = self.level_info(level)
        arr = binding.LevelArrays()
        out = {"n": li.n, "n_f": li.n_f, "n_c": li.n_c, "is_coarsest": bool(li.is_coarsest)}
        keep = []

        def csr(name, rows, nnz):
            rp = np.zeros(rows + 1, np.int32)
            col = np.zeros(max(nnz, 1), np.int32)
            val = np.zeros(max(nnz, 1), np.float64)
            keep.extend([rp, col, val])
            setattr(arr, name + "_rowptr", _np_ptr(rp, ctypes.c_int32))
            setattr(arr, name + "_col", _np_ptr(col, ctypes.c_int32))
            setattr(arr, name + "_val", _np_ptr(val, ctypes.c_double))
            out[name] = (rp, col[:nnz], val[:nnz])

        if "a" in what and (level == 0 or li.is_coarsest or self.params.keep_setup_data):
            csr("a", li.n, li.nnz_a)
        if not li.is_coarsest:
            if "state" in what:
                st = np.zeros(li.n, np.int8)
                keep.append(st)
                arr.state = _np_ptr(st, ctypes.c_int8)
                out["state"] = st
            if "ff" in what:
                csr("ff", li.n_f, li.nnz_ff)
            if "fc" in what:
                csr("fc", li.n_f, li.nnz_fc)
            if "z" in what:
                csr("z", li.n_c, li.nnz_z)
            if "cmap" in what:
                cm = np.zeros(max(li.n_f, 1), np.int32)
                keep.append(cm)
                arr.cmap = _np_ptr(cm, ctypes.c_int32)
                out["cmap"] = cm[:li.n_f]
        al = np.zeros(max(li.poly_len, 1))
        ac = np.zeros(max(li.c_poly_len, 1))
        re = np.zeros(max(li.n_roots, 1))
        im = np.zeros(max(li.n_roots, 1))
        keep.extend([al, ac, re, im])
        arr.alpha = _np_ptr(al, ctypes.c_double)
        arr.alpha_c = _np_ptr(ac, ctypes.c_double)
        arr.roots_re = _np_ptr(re, ctypes.c_double)
        arr.roots_im = _np_ptr(im, ctypes.c_double)
        binding.check(self.lib.airg_export_level(self.h, level, ctypes.byref(arr)), self.lib)
        out["alpha"] = al[:li.poly_len]
        out["alpha_c"] = ac[:li.c_poly_len]
        out["roots"] = re[:li.n_roots] + 1j * im[:li.n_roots]
        return out

    @classmethod
    def from_hierarchy(cls, levels, params=None, stream=None, **overrides):
        """Build a solver from given levels (setup numbering).  `levels` is a list
        of dicts: every level but the last has state, ff, fc, z (CSR triples),
        cmap and alpha; level 0 has the top matrix as a; the last level has a
        and roots (complex, applied order)."""
        lib = binding.load()
        prm = params if params is not None else default_params(**overrides)
        nl = len(levels)
        infos = (binding.LevelInfo * nl)()
        arrs = (binding.LevelArrays * nl)()
        keep = []

        def put(arr, name, trip):
            rp, col, val = (np.ascontiguousarray(trip[0], np.int32),
                            np.ascontiguousarray(trip[1], np.int32),
                            np.ascontiguousarray(trip[2], np.float64))
            if len(col) == 0:
                col, val = np.zeros(1, np.int32), np.zeros(1)
            keep.extend([rp, col, val])
            setattr(arr, name + "_rowptr", _np_ptr(rp, ctypes.c_int32))
            setattr(arr, name + "_col", _np_ptr(col, ctypes.c_int32))
            setattr(arr, name + "_val", _np_ptr(val, ctypes.c_double))

        for l, lv in enumerate(levels):
            li, ar = infos[l], arrs[l]
            last = l == nl - 1
            if "a" in lv:
                put(ar, "a", lv["a"])
                li.nnz_a = int(lv["a"][0][-1])
                li.n = len(lv["a"][0]) - 1
            if last:
                li.is_coarsest = 1
                r = np.asarray(lv["roots"], dtype=np.complex128)
                re, im = np.ascontiguousarray(r.real), np.ascontiguousarray(r.imag)
                keep.extend([re, im])
                ar.roots_re, ar.roots_im = _np_ptr(re, ctypes.c_double), _np_ptr(im, ctypes.c_double)
                li.n_roots = len(r)
                continue
            st = np.ascontiguousarray(lv["state"], np.int8)
            cm = np.ascontiguousarray(lv["cmap"], np.int32)
            al = np.ascontiguousarray(lv["alpha"], np.float64)
            keep.extend([st, cm, al])
            ar.state, ar.cmap = _np_ptr(st, ctypes.c_int8), _np_ptr(cm, ctypes.c_int32)
            ar.alpha = _np_ptr(al, ctypes.c_double)
            li.n = len(st)
            li.n_f = int((st == 1).sum())
            li.n_c = int((st == 2).sum())
            li.poly_len = len(al)
            put(ar, "ff", lv["ff"])
            put(ar, "fc", lv["fc"])
            put(ar, "z", lv["z"])
            li.nnz_ff = int(lv["ff"][0][-1])
            li.nnz_fc = int(lv["fc"][0][-1])
            li.nnz_z = int(lv["z"][0][-1])
        h = ctypes.c_void_p()
        code = lib.airg_import_hierarchy(ctypes.byref(h), nl, infos, arrs, ctypes.byref(prm),
                                         _stream_ptr(stream))
        binding.check(code, lib)
        return cls(params=prm, stream=stream, _handle=h)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if self.h and self.h.value:
            self.lib.airg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class BatchSolver(Solver):
    """Many independent problems in one AIRG hierarchy (block-diagonal setup):
    `problems` is a list of (indptr, indices, data) triples.  solve() takes a
    list of right-hand sides, one per problem, and returns (xs, infos)."""

    def __init__(self, problems, params=None, stream=None, **overrides):
        self.lib = binding.load()
        self.params = params if params is not None else default_params(**overrides)
        if params is not None:
            for k, v in overrides.items():
                setattr(self.params, k, v)
        self.stream = stream
        self.h = ctypes.c_void_p()
        torch = _torch()
        np_ = len(problems)
        if np_ < 1:
            raise ValueError("empty batch")
        mats = [(_as_device(a, torch.int32), _as_device(b, torch.int32),
                 _as_device(c, torch.float64)) for a, b, c in problems]
        self._sizes = [m[0].numel() - 1 for m in mats]
        n = (ctypes.c_int64 * np_)(*self._sizes)
        nnz = (ctypes.c_int64 * np_)(*[m[1].numel() for m in mats])
        vp = ctypes.c_void_p * np_
        rp = vp(*[m[0].data_ptr() for m in mats])
        cp = vp(*[m[1].data_ptr() for m in mats])
        dp = vp(*[m[2].data_ptr() for m in mats])
        code = self.lib.airg_setup_batch(ctypes.byref(self.h), np_, n, nnz, rp, cp, dp, 1,
                                         ctypes.byref(self.params), _stream_ptr(stream))
        binding.check(code, self.lib)
        st = self.stats()
        self.n = st["n"][0]

    def solve(self, bs, xs=None, guess=False):
        torch = _torch()
        np_ = len(self._sizes)
        if len(bs) != np_:
            raise ValueError(f"expected {np_} right-hand sides")
        bs = [_as_device(b, torch.float64) for b in bs]
        for b, m in zip(bs, self._sizes):
            if b.numel() != m:
                raise ValueError("right-hand side size does not match its problem")
        if xs is None:
            xs = [torch.zeros_like(b) for b in bs]
        vp = ctypes.c_void_p * np_
        infos = (binding.SolveInfo * np_)()
        code = self.lib.airg_solve_batch(self.h, vp(*[b.data_ptr() for b in bs]),
                                         vp(*[x.data_ptr() for x in xs]), 1 if guess else 0, infos)
        binding.check(code, self.lib)
        return xs, [i.as_dict() for i in infos]

    def adjoint_solve(self, w, lam=None, guess=False):
        raise NotImplementedError("adjoint solves take a single-problem Solver")
