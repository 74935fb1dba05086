// Host-only C entry points over the dense routines, for CPU tests of the
// library's least-squares and eigenvalue code (not part of the public ABI).
#include <cstring>
#include <vector>

#include "dense.hpp"
#include "error.hpp"

using namespace airg;

extern "C" {

// alpha (steps entries) from an (m+1) x m Hessenberg matrix; returns 0 or -1.
int airg_host_gmres_poly(const double* H, int m, int steps, double beta, double* alpha) {
  try {
    std::vector<double> h(H, H + (size_t)(m + 1) * m);
    std::vector<double> a = gmres_poly_coeffs(h, m, steps, beta);
    std::memcpy(alpha, a.data(), a.size() * sizeof(double));
    return 0;
  } catch (...) {
    return -1;
  }
}

// Eigenvalues of an upper Hessenberg n x n matrix; returns 0 or -1.
int airg_host_hessenberg_eig(const double* A, int n, double* re, double* im) {
  try {
    std::vector<cplx> ev = hessenberg_eigenvalues(std::vector<double>(A, A + (size_t)n * n), n);
    for (int i = 0; i < n; ++i) {
      re[i] = ev[i].real();
      im[i] = ev[i].imag();
    }
    return 0;
  } catch (...) {
    return -1;
  }
}

// Newton roots from an Arnoldi relation; writes up to cap roots, returns the count or -1.
int airg_host_newton_roots(const double* H, int m, int steps, int add_roots, double* re,
                           double* im, int cap) {
  try {
    std::vector<double> h(H, H + (size_t)(m + 1) * m);
    std::vector<cplx> r = newton_roots(h, m, steps, add_roots != 0);
    if ((int)r.size() > cap) return -1;
    for (size_t i = 0; i < r.size(); ++i) {
      re[i] = r[i].real();
      im[i] = r[i].imag();
    }
    return (int)r.size();
  } catch (...) {
    return -1;
  }
}

int airg_host_numerical_rank(const double* H, int ld, int k, double tol) {
  try {
    std::vector<double> h(H, H + (size_t)k * ld);
    return numerical_rank(h, ld, k, tol);
  } catch (...) {
    return -1;
  }
}

}  // extern "C"
