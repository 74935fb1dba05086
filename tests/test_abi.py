"""The C-ABI library loads and exports every symbol include/airg.h declares,
and its host-side dense routines agree with the oracle (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import linalg
from paper_2508_17517_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "airg.h")).read()
    return sorted(set(re.findall(r"\b(airg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = binding.load()
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SYMBOLS)


def test_status_strings_and_defaults_without_gpu():
    lib = binding.load()
    assert lib.airg_status_string(0) == b"ok"
    assert lib.airg_status_string(-2) == b"zero or missing diagonal"
    p = binding.default_params()
    assert p.strong_threshold == 0.99 and p.ddc_its == 2 and p.poly_order == 4
    assert p.coarse_poly_order == 20 and p.trunc_tol == 1e-2 and p.rtol == 1e-10
    assert p.seed == 17517 and p.restart == 30 and p.locality_order == 1 and p.outer == 0
    assert p.smoother == 0 and p.inverse_type == 0 and p.smooth_type == 0
    assert p.atol == 1e-50 and p.graph == 0 and p.stagnation_check == 0
    assert p.coarse_persistent == 0 and p.lookahead == 1


def test_struct_sizes_match_the_header():
    # the ctypes mirrors must have the C layout (fields are naturally aligned)
    assert ctypes.sizeof(binding.Params) == 6 * 8 + 8 + 8 + 16 * 4 + 8 + 4 * 4
    assert ctypes.sizeof(binding.SolveInfo) == 4 * 4 + 3 * 8
    assert ctypes.sizeof(binding.LevelInfo) == 7 * 8 + 4 * 4
    assert ctypes.sizeof(binding.LevelArrays) == 18 * 8


def _arnoldi_case(n, d, seed):
    r = np.random.default_rng(seed)
    M = sp.random(n, n, density=0.05, random_state=seed, data_rvs=lambda k: r.uniform(-1, 1, k))
    A = sp.csr_matrix(M + sp.diags(np.abs(M).sum(axis=1).A.ravel() * 1.5 + 1.0))
    A.sort_indices()
    b = r.uniform(size=n)
    return A, b


@pytest.mark.parametrize("d", [1, 3, 4, 6])
def test_library_poly_coefficients_are_bitwise_the_oracles(d):
    # same Arnoldi relation in, same operation order: identical bits out
    host = binding.load_host_dense()
    A, b = _arnoldi_case(300, d, d)
    m = d + 1
    V, H, steps, beta = linalg.arnoldi(A, b, m)
    want = linalg.gmres_poly_coeffs(A, b, d)
    Hc = np.ascontiguousarray(H)
    got = np.zeros(steps)
    assert host.airg_host_gmres_poly(Hc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m, steps,
                                     beta, got.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (21, 3), (60, 4), (150, 5)])
def test_library_hessenberg_eigenvalues_match_lapack(n, seed):
    host = binding.load_host_dense()
    a = np.triu(np.random.default_rng(seed).standard_normal((n, n)), -1)
    re, im = np.zeros(n), np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    assert host.airg_host_hessenberg_eig(np.ascontiguousarray(a).ctypes.data_as(dp), n,
                                         re.ctypes.data_as(dp), im.ctypes.data_as(dp)) == 0
    got = np.sort_complex(re + 1j * im)
    want = np.sort_complex(np.linalg.eigvals(a))
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    # conjugate pairs are exact
    for z in got[np.abs(got.imag) > 0]:
        assert np.conj(z) in got


@pytest.mark.parametrize("n,seed", [(150, 6), (300, 7)])
def test_library_hessenberg_eigenvalues_are_backward_stable(n, seed):
    # large random Hessenberg matrices have ill-conditioned eigenvalues, so
    # compare backward errors: every computed lambda makes A - lambda I
    # singular to within a few units of rounding of |A|
    host = binding.load_host_dense()
    a = np.triu(np.random.default_rng(seed).standard_normal((n, n)), -1)
    re, im = np.zeros(n), np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    assert host.airg_host_hessenberg_eig(np.ascontiguousarray(a).ctypes.data_as(dp), n,
                                         re.ctypes.data_as(dp), im.ctypes.data_as(dp)) == 0
    nrm = np.linalg.norm(a, 2)
    for lam in re + 1j * im:
        smin = np.linalg.svd(a - lam * np.eye(n), compute_uv=False)[-1]
        assert smin <= 1e-14 * nrm


@pytest.mark.parametrize("n", [4, 9, 32])
def test_library_hessenberg_eigenvalues_of_a_cyclic_shift(n):
    # the cyclic shift's eigenvalues are the n-th roots of unity; the standard
    # double shift stalls on it, so this exercises the exceptional shifts
    host = binding.load_host_dense()
    a = np.zeros((n, n))
    a[1:, :-1] = np.eye(n - 1)
    a[0, -1] = 1.0
    re, im = np.zeros(n), np.zeros(n)
    dp = ctypes.POINTER(ctypes.c_double)
    assert host.airg_host_hessenberg_eig(np.ascontiguousarray(a).ctypes.data_as(dp), n,
                                         re.ctypes.data_as(dp), im.ctypes.data_as(dp)) == 0
    z = re + 1j * im
    assert np.allclose(np.abs(z), 1.0, atol=1e-12)
    assert np.allclose(z ** n, 1.0, atol=1e-11)
    angles = np.sort(np.mod(np.angle(z), 2 * np.pi))
    assert np.allclose(angles, 2 * np.pi * np.arange(n) / n, atol=1e-12)


def test_library_newton_roots_match_oracle():
    host = binding.load_host_dense()
    A, b = _arnoldi_case(200, 20, 7)
    for deg, add in ((8, 0), (20, 1)):
        V, H, steps, beta = linalg.arnoldi(A, b, deg + 1)
        want = linalg.newton_roots(A, b, deg, use_added_roots=bool(add))
        re, im = np.zeros(200), np.zeros(200)
        dp = ctypes.POINTER(ctypes.c_double)
        cnt = host.airg_host_newton_roots(np.ascontiguousarray(H).ctypes.data_as(dp), deg + 1, steps,
                                          add, re.ctypes.data_as(dp), im.ctypes.data_as(dp), 200)
        assert cnt == len(want)
        got = re[:cnt] + 1j * im[:cnt]
        assert np.allclose(np.sort_complex(got), np.sort_complex(np.array(want)), rtol=1e-8)


def test_library_rank_of_singular_block():
    host = binding.load_host_dense()
    H = np.zeros((4, 3))
    H[0, 0], H[1, 0] = 2.0, 1e-20
    H[0, 1], H[1, 1], H[2, 1] = 1.0, 1e-18, 1.0
    H[:, 2] = [1, 2, 3, 4]
    dp = ctypes.POINTER(ctypes.c_double)
    r = host.airg_host_numerical_rank(np.ascontiguousarray(H[:3]).ctypes.data_as(dp), 3, 3, 1e-12)
    assert r == 3
    S = np.ones((3, 3))
    r = host.airg_host_numerical_rank(np.ascontiguousarray(S).ctypes.data_as(dp), 3, 3, 1e-12)
    assert r == 1


def test_loading_a_build_by_path_serves_later_calls():
    # a build loaded by path is the one every later load() returns (and so
    # the one Solver and BatchSolver call)
    lib = binding.load(binding.LIB_PATH)
    assert binding.load() is lib
