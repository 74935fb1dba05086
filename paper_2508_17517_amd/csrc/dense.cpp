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

std::vector<cplx> hessenberg_eigenvalues(std::vector<double> a, int n) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  std::vector<cplx> ev(n);
  double anorm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(i - 1, 0); j < n; ++j) anorm += std::fabs(A(i, j));
  int nn = n - 1;
  double t = 0.0;
  while (nn >= 0) {
    int its = 0;
    for (;;) {
      int l;
      // a negligible subdiagonal entry splits the active block
      for (l = nn; l >= 1; --l) {
        double s = std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l));
        if (s == 0.0) s = anorm;
        if (std::fabs(A(l, l - 1)) + s == s) {
          A(l, l - 1) = 0.0;
          break;
        }
      }
      double x = A(nn, nn);
      if (l == nn) {  // a 1 x 1 block
        ev[nn] = cplx(x + t, 0.0);
        --nn;
        break;
      }
      double y = A(nn - 1, nn - 1);
      double w = A(nn, nn - 1) * A(nn - 1, nn);
      if (l == nn - 1) {  // a 2 x 2 block
        double p = 0.5 * (y - x);
        double q = p * p + w;
        double z = std::sqrt(std::fabs(q));
        x += t;
        if (q >= 0.0) {
          z = p + std::copysign(z, p);
          double r1 = x + z;
          double r2 = (z != 0.0) ? x - w / z : r1;
          ev[nn - 1] = cplx(r1, 0.0);
          ev[nn] = cplx(r2, 0.0);
        } else {
          ev[nn - 1] = cplx(x + p, z);
          ev[nn] = cplx(x + p, -z);
        }
        nn -= 2;
        break;
      }
      if (its == 60) fail(AIRG_ERR_BREAKDOWN, "Hessenberg QR did not converge");
      if (its == 10 || its == 20) {  // exceptional shift
        t += x;
        for (int i = 0; i <= nn; ++i) A(i, i) -= x;
        double s = std::fabs(A(nn, nn - 1)) + std::fabs(A(nn - 1, nn - 2));
        x = y = 0.75 * s;
        w = -0.4375 * s * s;
      }
      ++its;
      // double-shift start: look for two consecutive small subdiagonals
      int m;
      double p = 0, q = 0, r = 0, z;
      for (m = nn - 2; m >= l; --m) {
        z = A(m, m);
        r = x - z;
        double s = y - z;
        p = (r * s - w) / A(m + 1, m) + A(m, m + 1);
        q = A(m + 1, m + 1) - z - r - s;
        r = A(m + 2, m + 1);
        s = std::fabs(p) + std::fabs(q) + std::fabs(r);
        p /= s;
        q /= s;
        r /= s;
        if (m == l) break;
        double u = std::fabs(A(m, m - 1)) * (std::fabs(q) + std::fabs(r));
        double v = std::fabs(p) * (std::fabs(A(m - 1, m - 1)) + std::fabs(z) + std::fabs(A(m + 1, m + 1)));
        if (u + v == v) break;
      }
      for (int i = m + 2; i <= nn; ++i) {
        A(i, i - 2) = 0.0;
        if (i != m + 2) A(i, i - 3) = 0.0;
      }
      // chase the bulge with 3 x 3 Householder reflections
      for (int k = m; k <= nn - 1; ++k) {
        if (k != m) {
          p = A(k, k - 1);
          q = A(k + 1, k - 1);
          r = 0.0;
          if (k != nn - 1) r = A(k + 2, k - 1);
          x = std::fabs(p) + std::fabs(q) + std::fabs(r);
          if (x != 0.0) {
            p /= x;
            q /= x;
            r /= x;
          }
        }
        double s = std::copysign(std::sqrt(p * p + q * q + r * r), p);
        if (s != 0.0) {
          if (k == m) {
            if (l != m) A(k, k - 1) = -A(k, k - 1);
          } else {
            A(k, k - 1) = -s * x;
          }
          p += s;
          x = p / s;
          y = q / s;
          z = r / s;
          q /= p;
          r /= p;
          for (int j = k; j <= nn; ++j) {
            p = A(k, j) + q * A(k + 1, j);
            if (k != nn - 1) {
              p += r * A(k + 2, j);
              A(k + 2, j) -= p * z;
            }
            A(k + 1, j) -= p * y;
            A(k, j) -= p * x;
          }
          int mmin = nn < k + 3 ? nn : k + 3;
          for (int i = l; i <= mmin; ++i) {
            p = x * A(i, k) + y * A(i, k + 1);
            if (k != nn - 1) {
              p += z * A(i, k + 2);
              A(i, k + 2) -= p * r;
            }
            A(i, k + 1) -= p * q;
            A(i, k) -= p;
          }
        }
      }
    }
  }
  return ev;
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
