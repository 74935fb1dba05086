// Small dense FP64 routines of the setup, run on the host: the GMRES
// least-squares problem, monomial coefficients of the smoother polynomial
// (Eq. gmres_poly) and the harmonic Ritz roots of the Newton coarse
// polynomial (Sec. 2.3).  Matrices are row-major std::vector<double>.
#pragma once

#include <complex>
#include <vector>

namespace airg {

using cplx = std::complex<double>;

// y = argmin |beta e_1 - H y| for an (m+1) x m upper Hessenberg H (row-major,
// leading dimension m) by Givens rotations; the operation order is fixed.
std::vector<double> givens_lstsq(const std::vector<double>& H, int m, double beta,
                                 double* resid = nullptr);

// Monomial coefficients alpha_0..alpha_{steps-1} of the GMRES polynomial from
// an Arnoldi run of `steps` steps (H is (m+1) x m with m >= steps).
std::vector<double> gmres_poly_coeffs(const std::vector<double>& H, int m, int steps, double beta);

// Numerical rank of the k x k leading block of H (leading dimension ld) by
// Householder QR with column pivoting, relative tolerance tol.
int numerical_rank(const std::vector<double>& H, int ld, int k, double tol);

// Eigenvalues of an upper Hessenberg matrix (row-major n x n) by the
// Francis double-shift QR iteration.  Complex eigenvalues come in exact
// conjugate pairs; real ones have an exactly zero imaginary part.
std::vector<cplx> hessenberg_eigenvalues(std::vector<double> a, int n);

// Harmonic Ritz values of a k-step Arnoldi relation (H is (m+1) x m, k <= m).
std::vector<cplx> harmonic_ritz(const std::vector<double>& H, int m, int k);

// Loe & Morgan's extra copies of outlying roots, and the modified Leja order.
std::vector<cplx> added_roots(const std::vector<cplx>& roots);
std::vector<cplx> leja_order(const std::vector<cplx>& roots);

// Newton roots from an Arnoldi run: rank cut, harmonic Ritz values, optional
// added roots, Leja order.
std::vector<cplx> newton_roots(const std::vector<double>& H, int m, int steps, bool add_roots);

}  // namespace airg
