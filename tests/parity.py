"""Assertions shared by the GPU-vs-oracle parity tests."""
import numpy as np


def assert_elementwise(got, want, rtol=1e-10, what="solution"):
    """Every element of `got` within rtol * max|want| of `want`: a local error
    in a few cells fails here even where a global 2-norm would hide it."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    scale = float(np.abs(want).max()) if want.size else 0.0
    err = float(np.abs(got - want).max()) if want.size else 0.0
    assert err <= rtol * scale, (f"{what}: max |got - want| = {err:.3e} exceeds "
                                 f"{rtol:g} * max |want| = {rtol * scale:.3e}")
    return err / scale if scale > 0 else 0.0


def mmatrix_inverse_inf_norm(A, level):
    """|A^{-1}|_inf of a triangular M-matrix in flow order (positive diagonal,
    non-positive off-diagonals, as the upwind FV and FD systems are): A^{-1} is
    then entrywise non-negative, so its largest row sum is max(A^{-1} 1),
    computed exactly by one flow-order sweep."""
    import oracle
    d = A.diagonal()
    off = A.copy()
    off.setdiag(0.0)
    off.eliminate_zeros()
    assert (d > 0).all() and (off.data <= 0).all(), "not an M-matrix with positive diagonal"
    return float(oracle.sweep_solve(A, np.ones(A.shape[0]), level).max())
