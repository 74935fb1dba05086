// Small dense FP64 routines of the setup (host).  givens_lstsq and
// gmres_poly_coeffs use a fixed operation order (compiled without FMA
// contraction) so that, given the same Arnoldi relation, they reproduce a
// sequential reference bit for bit.
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>

#include "error.hpp"

namespace airg {

std::vector<double> givens_lstsq(const std::vector<double>& H, int m, double beta, double* resid) {
  std::vector<double> R(H.begin(), H.begin() + (size_t)(m + 1) * m);
  auto r_ = [&](int i, int j) -> double& { return R[(size_t)i * m + j]; };
  std::vector<double> g(m + 1, 0.0), cs(m), sn(m);
  g[0] = beta;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < j; ++i) {
      double a = r_(i, j), b = r_(i + 1, j);
      r_(i, j) = cs[i] * a + sn[i] * b;
      r_(i + 1, j) = -sn[i] * a + cs[i] * b;
    }
    double a = r_(j, j), b = r_(j + 1, j);
    double r = std::sqrt(a * a + b * b);
    double c, s;
    if (r == 0.0) {
      c = 1.0;
      s = 0.0;
    } else {
      c = a / r;
      s = b / r;
    }
    cs[j] = c;
    sn[j] = s;
    r_(j, j) = r;
    r_(j + 1, j) = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
  }
  std::vector<double> y(m, 0.0);
  for (int i = m - 1; i >= 0; --i) {
    double t = g[i];
    for (int k = i + 1; k < m; ++k) t = t - r_(i, k) * y[k];
    y[i] = t / r_(i, i);
  }
  if (resid) *resid = std::fabs(g[m]);
  return y;
}

std::vector<double> gmres_poly_coeffs(const std::vector<double>& H, int m, int steps, double beta) {
  // C(i, k): coefficient of A^i b in the Arnoldi vector v_k
  auto h = [&](int i, int j) { return H[(size_t)i * m + j]; };
  std::vector<double> C((size_t)steps * steps, 0.0);
  auto c_ = [&](int i, int k) -> double& { return C[(size_t)i * steps + k]; };
  c_(0, 0) = 1.0 / beta;
  std::vector<double> c(steps);
  for (int j = 0; j + 1 < steps; ++j) {
    std::fill(c.begin(), c.end(), 0.0);
    for (int i = 0; i <= j; ++i) c[i + 1] = c_(i, j);
    for (int k = 0; k <= j; ++k) {
      const double hk = h(k, j);
      for (int i = 0; i < steps; ++i) c[i] = c[i] - hk * c_(i, k);
    }
    const double d = h(j + 1, j);
    for (int i = 0; i < steps; ++i) c_(i, j + 1) = c[i] / d;
  }
  // least squares on the leading (steps+1) x steps block
  std::vector<double> Hs((size_t)(steps + 1) * steps);
  for (int i = 0; i <= steps; ++i)
    for (int j = 0; j < steps; ++j) Hs[(size_t)i * steps + j] = h(i, j);
  std::vector<double> y = givens_lstsq(Hs, steps, beta);
  std::vector<double> alpha(steps);
  for (int i = 0; i < steps; ++i) {
    double s = 0.0;
    for (int k = 0; k < steps; ++k) s = s + y[k] * c_(i, k);
    alpha[i] = s;
  }
  return alpha;
}

int numerical_rank(const std::vector<double>& H, int ld, int k, double tol) {
  if (k <= 0) return 0;
  std::vector<double> a((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) a[(size_t)i * k + j] = H[(size_t)i * ld + j];
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * k + j]; };
  std::vector<double> rdiag(k, 0.0);
  for (int j = 0; j < k; ++j) {
    // pivot: remaining column of largest norm
    int piv = j;
    double best = -1.0;
    for (int c = j; c < k; ++c) {
      double s = 0.0;
      for (int i = j; i < k; ++i) s += A(i, c) * A(i, c);
      if (s > best) {
        best = s;
        piv = c;
      }
    }
    if (piv != j)
      for (int i = 0; i < k; ++i) std::swap(A(i, j), A(i, piv));
    double nrm = std::sqrt(std::max(best, 0.0));
    if (nrm == 0.0) break;
    double alpha = A(j, j) > 0 ? -nrm : nrm;
    rdiag[j] = alpha;
    // Householder vector v = x - alpha e_1
    std::vector<double> v(k - j);
    for (int i = j; i < k; ++i) v[i - j] = A(i, j);
    v[0] -= alpha;
    double vv = 0.0;
    for (double x : v) vv += x * x;
    if (vv == 0.0) continue;
    for (int c = j; c < k; ++c) {
      double d = 0.0;
      for (int i = j; i < k; ++i) d += v[i - j] * A(i, c);
      double f = 2.0 * d / vv;
      for (int i = j; i < k; ++i) A(i, c) -= f * v[i - j];
    }
  }
  double r0 = std::fabs(rdiag[0]);
  if (r0 == 0.0) return 0;
  int r = 0;
  for (int j = 0; j < k; ++j)
    if (std::fabs(rdiag[j]) > tol * r0) ++r;
  return r;
}

// Eigenvalues of an upper Hessenberg matrix by the implicit double-shift
// QR iteration as Golub & Van Loan present it (Matrix Computations, 4th ed.,
// Sec. 7.5: the Francis step of Algorithm 7.5.1 inside the deflating loop of
// Algorithm 7.5.2; Householder vectors as in Algorithm 5.1.1).  Only the
// active diagonal window is updated, since the eigenvalues alone are wanted.
namespace {

struct HessWork {
  std::vector<double>& h;
  int n;
  double& at(int i, int j) { return h[(size_t)i * n + j]; }
};

// Householder vector of x (len 2 or 3): (I - beta v v^T) x = -+|x| e_1, with
// v[0] = 1.  x is scaled by its largest magnitude first; beta = 0 when x is
// already a multiple of e_1.
struct Reflector {
  double v[3];
  double beta;
};

Reflector householder(const double* x, int len) {
  Reflector r{{1.0, 0.0, 0.0}, 0.0};
  double scale = 0.0;
  for (int i = 0; i < len; ++i) scale = std::max(scale, std::fabs(x[i]));
  if (scale == 0.0) return r;
  double y[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < len; ++i) y[i] = x[i] / scale;
  double tail = 0.0;
  for (int i = 1; i < len; ++i) tail += y[i] * y[i];
  if (tail == 0.0) return r;
  const double mu = std::sqrt(y[0] * y[0] + tail);
  const double v0 = y[0] <= 0.0 ? y[0] - mu : -tail / (y[0] + mu);
  r.beta = 2.0 * v0 * v0 / (tail + v0 * v0);
  for (int i = 1; i < len; ++i) r.v[i] = y[i] / v0;
  return r;
}

// rows q..q+len-1, columns c0..c1 of H  <-  P * (those rows)
void reflect_rows(HessWork& H, const Reflector& P, int len, int q, int c0, int c1) {
  if (P.beta == 0.0) return;
  for (int c = c0; c <= c1; ++c) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += P.v[i] * H.at(q + i, c);
    s *= P.beta;
    for (int i = 0; i < len; ++i) H.at(q + i, c) -= s * P.v[i];
  }
}

// columns q..q+len-1, rows r0..r1 of H  <-  (those columns) * P
void reflect_cols(HessWork& H, const Reflector& P, int len, int q, int r0, int r1) {
  if (P.beta == 0.0) return;
  for (int r = r0; r <= r1; ++r) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += H.at(r, q + i) * P.v[i];
    s *= P.beta;
    for (int i = 0; i < len; ++i) H.at(r, q + i) -= s * P.v[i];
  }
}

// One implicit double-shift sweep over the unreduced window lo..hi (at least
// 3 x 3).  The shifts enter only through their sum and product: the first
// column of (H - s1 I)(H - s2 I) starts a bulge that the reflectors chase
// down the subdiagonal until the matrix is Hessenberg again.
void francis_sweep(HessWork& H, int lo, int hi, double shift_sum, double shift_prod) {
  const double h00 = H.at(lo, lo), h10 = H.at(lo + 1, lo);
  double col[3] = {h00 * h00 + H.at(lo, lo + 1) * h10 - shift_sum * h00 + shift_prod,
                   h10 * (h00 + H.at(lo + 1, lo + 1) - shift_sum), h10 * H.at(lo + 2, lo + 1)};
  for (int q = lo; q + 2 <= hi; ++q) {
    if (q > lo) {
      col[0] = H.at(q, q - 1);
      col[1] = H.at(q + 1, q - 1);
      col[2] = H.at(q + 2, q - 1);
    }
    const Reflector P = householder(col, 3);
    reflect_rows(H, P, 3, q, q > lo ? q - 1 : lo, hi);
    reflect_cols(H, P, 3, q, lo, std::min(q + 3, hi));
    if (q > lo) H.at(q + 1, q - 1) = H.at(q + 2, q - 1) = 0.0;
  }
  const double tail[2] = {H.at(hi - 1, hi - 2), H.at(hi, hi - 2)};
  const Reflector P = householder(tail, 2);
  reflect_rows(H, P, 2, hi - 1, hi - 2, hi);
  reflect_cols(H, P, 2, hi - 1, lo, hi);
  H.at(hi, hi - 2) = 0.0;
}

// Eigenvalues of [[a, b], [c, d]]: real ones by the cancellation-free form of
// the quadratic formula, complex ones as an exact conjugate pair.
void eig2(double a, double b, double c, double d, cplx& first, cplx& second) {
  const double half = 0.5 * (a - d);
  const double disc = half * half + b * c;
  if (disc >= 0.0) {
    const double big = half + std::copysign(std::sqrt(disc), half);
    first = cplx(d + big, 0.0);
    second = cplx(big != 0.0 ? d - (b * c) / big : d, 0.0);
  } else {
    const double im = std::sqrt(-disc);
    first = cplx(d + half, im);
    second = cplx(d + half, -im);
  }
}

}  // namespace

std::vector<cplx> hessenberg_eigenvalues(std::vector<double> a, int n) {
  std::vector<cplx> eig(n);
  HessWork H{a, n};
  double fro = 0.0;
  for (double v : a) fro += v * v;
  fro = std::sqrt(fro);
  const double eps = std::numeric_limits<double>::epsilon();
  const int max_sweeps = 40 * std::max(n, 1);
  int sweeps = 0;
  int since_split = 0;  // sweeps since the window last shrank
  int hi = n - 1;
  while (hi >= 0) {
    // largest unreduced window ending at hi: walk up the subdiagonal until an
    // entry is negligible next to its two diagonal neighbours
    int lo = hi;
    while (lo > 0) {
      double nb = std::fabs(H.at(lo, lo)) + std::fabs(H.at(lo - 1, lo - 1));
      if (nb == 0.0) nb = fro;
      if (std::fabs(H.at(lo, lo - 1)) <= eps * nb) {
        H.at(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    const int size = hi - lo + 1;
    if (size <= 2) {
      if (size == 1)
        eig[hi] = cplx(H.at(hi, hi), 0.0);
      else
        eig2(H.at(lo, lo), H.at(lo, hi), H.at(hi, lo), H.at(hi, hi), eig[lo], eig[hi]);
      hi -= size;
      since_split = 0;
      continue;
    }
    if (++sweeps > max_sweeps) fail(AIRG_ERR_BREAKDOWN, "Hessenberg QR did not converge");
    ++since_split;
    double shift_sum, shift_prod;
    if (since_split % 12 == 0) {
      // a window that will not split: move both shifts off the trailing
      // block's eigenvalues by the size of the last two subdiagonals
      const double w = std::fabs(H.at(hi, hi - 1)) + std::fabs(H.at(hi - 1, hi - 2));
      const double c = H.at(hi, hi) + 0.5 * w;
      shift_sum = 2.0 * c;
      shift_prod = c * c + w * w;
    } else {
      // the trailing 2 x 2 block's eigenvalues (Wilkinson-style double shift)
      const double p = H.at(hi - 1, hi - 1), q = H.at(hi - 1, hi), r = H.at(hi, hi - 1),
                   s = H.at(hi, hi);
      shift_sum = p + s;
      shift_prod = p * s - q * r;
    }
    francis_sweep(H, lo, hi, shift_sum, shift_prod);
  }
  return eig;
}

std::vector<cplx> harmonic_ritz(const std::vector<double>& H, int m, int k) {
  // H_k^T f = e_k by Gaussian elimination with partial pivoting
  std::vector<double> T((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) T[(size_t)i * k + j] = H[(size_t)j * m + i];
  std::vector<double> f(k, 0.0);
  f[k - 1] = 1.0;
  std::vector<int> perm(k);
  for (int i = 0; i < k; ++i) perm[i] = i;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(T[(size_t)r * k + c]) > std::fabs(T[(size_t)piv * k + c])) piv = r;
    if (T[(size_t)piv * k + c] == 0.0) fail(AIRG_ERR_BREAKDOWN, "singular Hessenberg block");
    if (piv != c) {
      for (int j = 0; j < k; ++j) std::swap(T[(size_t)c * k + j], T[(size_t)piv * k + j]);
      std::swap(f[c], f[piv]);
    }
    for (int r = c + 1; r < k; ++r) {
      double l = T[(size_t)r * k + c] / T[(size_t)c * k + c];
      if (l == 0.0) continue;
      for (int j = c; j < k; ++j) T[(size_t)r * k + j] -= l * T[(size_t)c * k + j];
      f[r] -= l * f[c];
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = f[i];
    for (int j = i + 1; j < k; ++j) s -= T[(size_t)i * k + j] * f[j];
    f[i] = s / T[(size_t)i * k + i];
  }
  const double h = H[(size_t)k * m + (k - 1)];
  std::vector<double> M((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) M[(size_t)i * k + j] = H[(size_t)i * m + j];
  for (int i = 0; i < k; ++i) M[(size_t)i * k + (k - 1)] += h * h * f[i];
  return hessenberg_eigenvalues(M, k);
}

static std::vector<cplx> representatives(const std::vector<cplx>& roots) {
  std::vector<cplx> reps;
  for (const cplx& z : roots)
    if (z.imag() >= 0.0) reps.push_back(z);
  std::stable_sort(reps.begin(), reps.end(), [](const cplx& a, const cplx& b) {
    return a.real() < b.real() || (a.real() == b.real() && a.imag() < b.imag());
  });
  return reps;
}

std::vector<cplx> leja_order(const std::vector<cplx>& roots) {
  std::vector<cplx> remaining = representatives(roots);
  std::vector<cplx> taken, out;
  while (!remaining.empty()) {
    size_t best = 0;
    double bscore = -std::numeric_limits<double>::infinity();
    for (size_t c = 0; c < remaining.size(); ++c) {
      double sc;
      if (taken.empty()) {
        sc = std::abs(remaining[c]);
      } else {
        sc = 0.0;
        for (const cplx& t : taken) {
          double d = std::abs(remaining[c] - t);
          sc += d > 0.0 ? std::log(d) : -std::numeric_limits<double>::infinity();
        }
      }
      if (c == 0 || sc > bscore) {
        bscore = sc;
        best = c;
      }
    }
    cplx z = remaining[best];
    remaining.erase(remaining.begin() + best);
    out.push_back(z);
    taken.push_back(z);
    if (z.imag() != 0.0) {
      out.push_back(std::conj(z));
      taken.push_back(std::conj(z));
    }
  }
  return out;
}

std::vector<cplx> added_roots(const std::vector<cplx>& roots) {
  std::vector<cplx> extra;
  for (const cplx& z : representatives(roots)) {
    double lp = 0.0;
    bool skipped = false;
    for (const cplx& t : roots) {
      if (t == z && !skipped) {
        skipped = true;
        continue;
      }
      double d = std::abs(1.0 - z / t);
      lp += d > 0.0 ? std::log10(d) : -std::numeric_limits<double>::infinity();
    }
    if (lp > 4.0) {
      int cnt = (int)std::ceil((lp - 4.0) / 14.0);
      for (int c = 0; c < cnt; ++c) {
        extra.push_back(z);
        if (z.imag() != 0.0) extra.push_back(std::conj(z));
      }
    }
  }
  return extra;
}

std::vector<cplx> newton_roots(const std::vector<double>& H, int m, int steps, bool add_roots) {
  int k = steps;
  int r = numerical_rank(H, m, k, 1e-12);
  k = std::max(1, std::min(k, r));
  std::vector<cplx> roots = harmonic_ritz(H, m, k);
  if (add_roots) {
    std::vector<cplx> e = added_roots(roots);
    roots.insert(roots.end(), e.begin(), e.end());
  }
  return leja_order(roots);
}

}  // namespace airg
