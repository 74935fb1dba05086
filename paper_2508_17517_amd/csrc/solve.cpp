// Solve phase (paper Sec. 2, Eq. f_point): V-cycles with no down smoothing,
// restriction by R = [Z I], one-point prolongation by P = [W; I] and one up
// F-point smooth with the GMRES polynomial applied matrix-free by Horner;
// the coarsest level applies its Newton polynomial.  The outer loop is
// right-preconditioned FGMRES(restart) with classical Gram-Schmidt applied
// twice; the Hessenberg column comes to the host once per iteration.
#include "solve.hpp"

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace airg {

Workspace::~Workspace() {
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
}

void workspace_init(const Hierarchy& H, Workspace& W) {
  hipStream_t s = H.s;
  const int64_t n = H.n0;
  W.ld = (n + 63) / 64 * 64;
  W.restart = H.p.restart;
  W.V.alloc((size_t)(W.restart + 1) * W.ld, s);
  W.Zb.alloc((size_t)W.restart * W.ld, s);
  W.w.alloc(n, s);
  W.rr.alloc(n, s);
  int64_t maxf = 1;
  for (const Level& L : H.levels) maxf = std::max(maxf, L.nF);
  W.sv.alloc(maxf, s);
  W.y0.alloc(maxf, s);
  W.y1.alloc(maxf, s);
  const int64_t nc = std::max<int64_t>(1, H.levels.back().n);
  W.cw0.alloc(nc, s);
  W.cw1.alloc(nc, s);
  W.ct.alloc(nc, s);
  W.bperm.alloc(n, s);
  W.xperm.alloc(n, s);
  W.hbuf.alloc(2 * (W.restart + 1) + 2, s);
  W.ybuf.alloc(W.restart + 1, s);
  W.dot_work.alloc(dot_work_size(n, 64), s);
  AIRG_HIP(hipEventCreate(&W.ev0));
  AIRG_HIP(hipEventCreate(&W.ev1));
}

namespace {

void horner(const Level& L, const double* sv, double* ef, Workspace& W, hipStream_t s) {
  const std::vector<double>& a = L.alpha;
  const int d = (int)a.size() - 1;
  if (d == 0) {
    axpy_first(ef, sv, a[0], false, L.nF, s);
    return;
  }
  if (d == 1) {
    spmv_horner(L.Aff, L.tpr_ff, sv, sv, ef, a[1], a[0], true, s);
    return;
  }
  double* y[2] = {W.y0.get(), W.y1.get()};
  int c = 0;
  spmv_horner(L.Aff, L.tpr_ff, sv, sv, y[0], a[d], a[d - 1], false, s);
  for (int k = d - 2; k >= 1; --k) {
    spmv_horner(L.Aff, L.tpr_ff, y[c], sv, y[c ^ 1], 1.0, a[k], false, s);
    c ^= 1;
  }
  spmv_horner(L.Aff, L.tpr_ff, y[c], sv, ef, 1.0, a[0], true, s);
}

void dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* out,
          Workspace& W, hipStream_t s) {
  for (int k0 = 0; k0 < nv; k0 += 64) {
    int cnt = std::min(64, nv - k0);
    launch_tree_dots(V + (int64_t)k0 * ld, ld, cnt, w, n, out + k0, W.dot_work.get(), s);
  }
}

double norm_host(const double* x, int64_t n, Workspace& W, hipStream_t s) {
  double* out = W.hbuf.get() + 2 * (W.restart + 1) + 1;
  launch_tree_dots(x, 0, 1, x, n, out, W.dot_work.get(), s);
  return std::sqrt(fetch(out, s));
}

}  // namespace

void vcycle(const Hierarchy& H, Workspace& W, const double* in, double* e) {
  hipStream_t s = H.s;
  const int L = (int)H.levels.size() - 1;
  double* rr = W.rr.get();
  for (int l = 0; l < L; ++l) {
    const Level& lv = H.levels[l];
    const double* src = (l == 0 ? in : rr) + lv.off;
    double* dst = rr + H.levels[l + 1].off;
    spmv_restrict(lv.Z, lv.tpr_z, src, src + lv.nF, dst, s);
  }
  const Level& lc = H.levels[L];
  const double* rc = (L == 0 ? in : rr) + lc.off;
  newton_apply_dev(lc.A, lc.tpr_a, lc.roots, rc, e + lc.off, W.cw0.get(), W.cw1.get(),
                   W.ct.get(), s);
  for (int l = L - 1; l >= 0; --l) {
    const Level& lv = H.levels[l];
    const double* rf = (l == 0 ? in : rr) + lv.off;
    double* ef = e + lv.off;
    const double* ec = e + H.levels[l + 1].off;
    residual_fpoint(lv.Aff, lv.Afc, lv.cmap.get(), lv.tpr_fc, rf, ec, ef, W.sv.get(), s);
    horner(lv, W.sv.get(), ef, W, s);
  }
}

int fgmres_solve(const Hierarchy& H, Workspace& W, const double* b, double* x, bool guess,
                 airg_solve_info* info) {
  hipStream_t s = H.s;
  const int64_t n = H.n0;
  const int R = W.restart;
  const int64_t ld = W.ld;
  const int32_t* pos = H.levels[0].pos.get();
  const double rtol = H.p.rtol;
  const int max_it = H.p.max_it;
  AIRG_HIP(hipEventRecord(W.ev0, s));

  launch_scatter(W.bperm.get(), b, pos, n, s);
  if (guess) launch_scatter(W.xperm.get(), x, pos, n, s);
  else launch_fill(W.xperm.get(), n, 0.0, s);
  const double bnorm = norm_host(W.bperm.get(), n, W, s);

  airg_solve_info out{};
  int status = AIRG_OK;
  if (bnorm == 0.0) {
    launch_fill(x, n, 0.0, s);
    out.converged = 1;
  } else if (!std::isfinite(bnorm)) {
    fail(AIRG_ERR_NONFINITE, "right-hand side is not finite");
  } else {
    int its = 0;
    std::vector<double> Hm((size_t)(R + 1) * R), g(R + 1), cs(R), sn(R), hh(2 * (R + 1) + 2), y(R);
    double* V = W.V.get();
    double* Zb = W.Zb.get();
    double* hd = W.hbuf.get();
    for (;;) {
      spmv(H.Aperm, H.tpr_top, W.xperm.get(), W.w.get(), s);
      launch_sub(V, W.bperm.get(), W.w.get(), n, s);
      const double beta = norm_host(V, n, W, s);
      out.rel_residual = beta / bnorm;
      if (beta <= rtol * bnorm) {
        out.converged = 1;
        break;
      }
      if (its >= max_it) break;
      if (its > 0) out.restarts++;
      launch_divide(V, V, beta, n, s);
      std::fill(Hm.begin(), Hm.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;
      for (int j = 0; j < R; ++j) {
        double* vj = V + (int64_t)j * ld;
        double* zj = Zb + (int64_t)j * ld;
        vcycle(H, W, vj, zj);
        spmv(H.Aperm, H.tpr_top, zj, W.w.get(), s);
        ++its;
        dots(V, ld, j + 1, W.w.get(), n, hd, W, s);
        launch_cgs_update(W.w.get(), V, ld, hd, j + 1, n, s);
        dots(V, ld, j + 1, W.w.get(), n, hd + (R + 1), W, s);
        launch_cgs_update(W.w.get(), V, ld, hd + (R + 1), j + 1, n, s);
        launch_tree_dots(W.w.get(), 0, 1, W.w.get(), n, hd + 2 * (R + 1), W.dot_work.get(), s);
        W.hbuf.to_host(hh.data(), 2 * (R + 1) + 1);
        AIRG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i <= j; ++i) Hm[(size_t)i * R + j] = hh[i] + hh[(R + 1) + i];
        const double hn = std::sqrt(hh[2 * (R + 1)]);
        Hm[(size_t)(j + 1) * R + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double a = Hm[(size_t)i * R + j], c = Hm[(size_t)(i + 1) * R + j];
          Hm[(size_t)i * R + j] = cs[i] * a + sn[i] * c;
          Hm[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * c;
        }
        const double a = Hm[(size_t)j * R + j], c = Hm[(size_t)(j + 1) * R + j];
        const double rr = std::hypot(a, c);
        if (rr > 0) {
          cs[j] = a / rr;
          sn[j] = c / rr;
        } else {
          cs[j] = 1.0;
          sn[j] = 0.0;
        }
        Hm[(size_t)j * R + j] = rr;
        Hm[(size_t)(j + 1) * R + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        const double est = std::fabs(g[j + 1]);
        out.rel_residual_estimate = est / bnorm;
        if (!std::isfinite(est)) fail(AIRG_ERR_BREAKDOWN, "FGMRES breakdown (non-finite residual)");
        if (est <= rtol * bnorm || its >= max_it) break;
        if (hn == 0.0) break;
        launch_divide(V + (int64_t)(j + 1) * ld, W.w.get(), hn, n, s);
      }
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= Hm[(size_t)i * R + q] * y[q];
        y[i] = t / Hm[(size_t)i * R + i];
      }
      W.ybuf.from_host(y.data(), k);
      launch_basis_combine(W.xperm.get(), Zb, ld, W.ybuf.get(), k, n, s);
      out.iterations = its;
    }
    out.iterations = its;
    launch_gather(x, W.xperm.get(), pos, n, s);
    if (!out.converged) status = AIRG_NOT_CONVERGED;
  }
  AIRG_HIP(hipEventRecord(W.ev1, s));
  AIRG_HIP(hipEventSynchronize(W.ev1));
  float ms = 0.f;
  AIRG_HIP(hipEventElapsedTime(&ms, W.ev0, W.ev1));
  out.solve_ms = ms;
  if (info) *info = out;
  return status;
}

}  // namespace airg
