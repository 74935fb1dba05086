// Solve phase (paper Sec. 2, Eq. f_point): V-cycles with no down smoothing,
// restriction by R = [Z I], one-point prolongation by P = [W; I] and one up
// F-point smooth with the GMRES polynomial applied matrix-free by Horner;
// the coarsest level applies its Newton polynomial.  The outer loop is
// right-preconditioned FGMRES(restart) with classical Gram-Schmidt applied
// twice; the Hessenberg column comes to the host once per iteration.
//
// Mixed precision: with FP32 or BF16 storage the V-cycle runs on FP32 vectors
// (matrices in the storage type, rows accumulated in FP32) between a
// conversion of its FP64 input and of its output back to FP64; the outer
// FGMRES, its orthogonalisation and the true residual stay in FP64, so the
// outer loop acts as iterative refinement.
#include "solve.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

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
  int64_t maxf = 1;
  for (const Level& L : H.levels) maxf = std::max(maxf, L.nF);
  const int64_t nc = std::max<int64_t>(1, H.levels.back().n);
  if (H.p.precision == AIRG_FP64) {
    W.rr.alloc(n, s);
    W.sv.alloc(maxf, s);
    W.y0.alloc(maxf, s);
    W.y1.alloc(maxf, s);
    W.cw0.alloc(nc, s);
    W.cw1.alloc(nc, s);
    W.ct.alloc(nc, s);
  } else {
    W.in32.alloc(n, s);
    W.e32.alloc(n, s);
    W.rr32.alloc(n, s);
    W.sv32.alloc(maxf, s);
    W.y032.alloc(maxf, s);
    W.y132.alloc(maxf, s);
    W.cw032.alloc(nc, s);
    W.cw132.alloc(nc, s);
    W.ct32.alloc(nc, s);
  }
  W.bperm.alloc(n, s);
  W.xperm.alloc(n, s);
  W.hbuf.alloc(2 * (W.restart + 1) + 2, s);
  W.ybuf.alloc(W.restart + 1, s);
  W.dot_work.alloc(dot_work_size(n, 64), s);
  AIRG_HIP(hipEventCreate(&W.ev0));
  AIRG_HIP(hipEventCreate(&W.ev1));
}

namespace {

// Vectors of one V-cycle in vector type X (nested numbering).
template <class X>
struct VecSet {
  const X* in;  // top-level residual
  X* e;         // correction, all levels
  X* rr;        // restricted residuals, levels >= 1
  X* sv;        // F-point residual of the current level
  X* y0;
  X* y1;        // Horner ping-pong
  X* cw0;
  X* cw1;
  X* ct;        // Newton scratch
};

VecSet<double> vecs64(Workspace& W, const double* in, double* e) {
  return {in, e, W.rr.get(), W.sv.get(), W.y0.get(), W.y1.get(), W.cw0.get(), W.cw1.get(), W.ct.get()};
}
VecSet<float> vecs32(Workspace& W) {
  return {W.in32.get(), W.e32.get(), W.rr32.get(), W.sv32.get(), W.y032.get(), W.y132.get(),
          W.cw032.get(), W.cw132.get(), W.ct32.get()};
}

struct LevelOps {
  OpView ff, fc, z, a;
};
LevelOps ops_of(const Level& L, int prec) {
  return {op_view(L.Aff, L.ff32, L.ff16, prec), op_view(L.Afc, L.fc32, L.fc16, prec),
          op_view(L.Z, L.z32, L.z16, prec), op_view(L.A, L.a32, L.a16, prec)};
}

double vt_bytes(ValType vt) { return vt == VT_F64 ? 8.0 : vt == VT_F32 ? 4.0 : 2.0; }

template <class X>
void horner(const Level& L, const OpView& Aff, const X* sv, X* ef, X* y0, X* y1, hipStream_t s,
            LaunchTally* tally = nullptr) {
  const std::vector<double>& a = L.alpha;
  const int d = (int)a.size() - 1;
  const int64_t n = L.nF;
  const double xb = (double)sizeof(X);
  const double mb = csr_bytes(n, Aff.nnz, vt_bytes(Aff.vt)), mf = 2.0 * (double)Aff.nnz;
  // per step: y gathered, s read, out written (and read when accumulating)
  auto count = [&](bool acc) {
    if (tally) tally->add(mb + xb * n * (acc ? 4 : 3), mf + 3.0 * n);
  };
  if (d == 0) {
    axpy_first_t<X>(ef, sv, a[0], false, n, s);
    if (tally) tally->add(3.0 * xb * n, 2.0 * n);
    return;
  }
  if (d == 1) {
    spmv_horner_t<X>(Aff, L.tpr_ff, sv, sv, ef, a[1], a[0], true, s);
    count(true);
    return;
  }
  X* y[2] = {y0, y1};
  int c = 0;
  spmv_horner_t<X>(Aff, L.tpr_ff, sv, sv, y[0], a[d], a[d - 1], false, s);
  count(false);
  for (int k = d - 2; k >= 1; --k) {
    spmv_horner_t<X>(Aff, L.tpr_ff, y[c], sv, y[c ^ 1], 1.0, a[k], false, s);
    count(false);
    c ^= 1;
  }
  spmv_horner_t<X>(Aff, L.tpr_ff, y[c], sv, ef, 1.0, a[0], true, s);
  count(true);
}

template <class X>
void vcycle_t(const Hierarchy& H, const VecSet<X>& v) {
  hipStream_t s = H.s;
  const int prec = H.p.precision;
  const int L = (int)H.levels.size() - 1;
  for (int l = 0; l < L; ++l) {
    const Level& lv = H.levels[l];
    const X* src = (l == 0 ? v.in : v.rr) + lv.off;
    X* dst = v.rr + H.levels[l + 1].off;
    spmv_restrict_t<X>(ops_of(lv, prec).z, lv.tpr_z, src, src + lv.nF, dst, s);
  }
  const Level& lc = H.levels[L];
  const X* rc = (L == 0 ? v.in : v.rr) + lc.off;
  newton_apply_t<X>(ops_of(lc, prec).a, lc.tpr_a, lc.roots, rc, v.e + lc.off, v.cw0, v.cw1, v.ct, s);
  for (int l = L - 1; l >= 0; --l) {
    const Level& lv = H.levels[l];
    const LevelOps o = ops_of(lv, prec);
    const X* rf = (l == 0 ? v.in : v.rr) + lv.off;
    X* ef = v.e + lv.off;
    const X* ec = v.e + H.levels[l + 1].off;
    residual_fpoint_t<X>(o.ff, o.fc, lv.cmap.get(), lv.tpr_fc, rf, ec, ef, v.sv, s);
    horner<X>(lv, o.ff, v.sv, ef, v.y0, v.y1, s);
  }
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
  if (H.p.precision == AIRG_FP64) {
    vcycle_t<double>(H, vecs64(W, in, e));
    return;
  }
  convert_d2f(W.in32.get(), in, H.n0, H.s);
  vcycle_t<float>(H, vecs32(W));
  convert_f2d(e, W.e32.get(), H.n0, H.s);
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

namespace {

template <class X>
void time_pass(const Hierarchy& H, const VecSet<X>& v, int cls, LaunchTally* t) {
  hipStream_t s = H.s;
  const int prec = H.p.precision;
  const int L = (int)H.levels.size() - 1;
  const double xb = (double)sizeof(X);
  const double vb = value_bytes(prec);
  const bool poly = cls == AIRG_K_POLY;
  if (poly || cls == AIRG_K_HORNER)
    for (int l = 0; l < L; ++l) {
      const Level& lv = H.levels[l];
      horner<X>(lv, ops_of(lv, prec).ff, v.sv, v.e + lv.off, v.y0, v.y1, s, t);
    }
  if (poly || cls == AIRG_K_NEWTON) {
    const Level& lc = H.levels[L];
    newton_apply_t<X>(ops_of(lc, prec).a, lc.tpr_a, lc.roots, v.rr + lc.off, v.e + lc.off, v.cw0,
                      v.cw1, v.ct, s, t);
  }
  if (cls == AIRG_K_RESIDUAL)
    for (int l = 0; l < L; ++l) {
      const Level& lv = H.levels[l];
      const LevelOps o = ops_of(lv, prec);
      residual_fpoint_t<X>(o.ff, o.fc, lv.cmap.get(), lv.tpr_fc, v.rr + lv.off,
                           v.e + H.levels[l + 1].off, v.e + lv.off, v.sv, s);
      if (t)
        t->add(csr_bytes(lv.nF, lv.Aff.nnz, vb) + csr_bytes(lv.nF, lv.Afc.nnz, vb) + 4.0 * lv.nF +
                   xb * (lv.nC + 3 * lv.nF),
               2.0 * (lv.Aff.nnz + lv.Afc.nnz) + lv.nF);
    }
  if (cls == AIRG_K_RESTRICT)
    for (int l = 0; l < L; ++l) {
      const Level& lv = H.levels[l];
      spmv_restrict_t<X>(ops_of(lv, prec).z, lv.tpr_z, v.rr + lv.off, v.rr + lv.off + lv.nF,
                         v.rr + H.levels[l + 1].off, s);
      if (t) t->add(csr_bytes(lv.nC, lv.Z.nnz, vb) + xb * (lv.nF + 2 * lv.nC), 2.0 * lv.Z.nnz + lv.nC);
    }
}

}  // namespace

int time_kernels(const Hierarchy& H, Workspace& W, int cls, int reps, airg_kernel_timing* out) {
  hipStream_t s = H.s;
  if (reps < 1) fail(AIRG_ERR_INVALID, "reps must be >= 1");
  if (cls < AIRG_K_POLY || cls > AIRG_K_TOP_SPMV) fail(AIRG_ERR_INVALID, "unknown kernel class");
  const bool f64 = H.p.precision == AIRG_FP64;
  double* in = W.V.get();
  launch_fill(in, H.n0, 1.0, s);
  if (f64) {
    launch_fill(W.Zb.get(), H.n0, 0.5, s);
    launch_fill(W.rr.get(), H.n0, 0.25, s);
    launch_fill(W.sv.get(), (int64_t)W.sv.size(), 0.125, s);
  } else {
    convert_d2f(W.e32.get(), in, H.n0, s);
    convert_d2f(W.rr32.get(), in, H.n0, s);
    convert_d2f(W.sv32.get(), in, (int64_t)W.sv32.size(), s);
  }
  auto pass = [&](LaunchTally* t) {
    if (cls == AIRG_K_TOP_SPMV) {
      spmv(H.Aperm, H.tpr_top, in, W.w.get(), s);
      if (t) t->add(csr_bytes(H.n0, H.Aperm.nnz) + 16.0 * H.n0, 2.0 * H.Aperm.nnz);
      return;
    }
    if (f64) time_pass<double>(H, vecs64(W, in, W.Zb.get()), cls, t);
    else time_pass<float>(H, vecs32(W), cls, t);
  };
  LaunchTally tally;
  pass(&tally);  // warm-up pass, also counts the launches and bytes
  AIRG_HIP(hipEventRecord(W.ev0, s));
  for (int r = 0; r < reps; ++r) pass(nullptr);
  AIRG_HIP(hipEventRecord(W.ev1, s));
  AIRG_HIP(hipEventSynchronize(W.ev1));
  float ms = 0.f;
  AIRG_HIP(hipEventElapsedTime(&ms, W.ev0, W.ev1));
  std::memset(out, 0, sizeof(*out));
  out->launches = tally.launches;
  if (tally.launches > 0) {
    out->avg_launch_ms = (double)ms / ((double)reps * tally.launches);
    out->bytes_per_launch = tally.bytes / tally.launches;
    out->flops_per_launch = tally.flops / tally.launches;
  }
  return AIRG_OK;
}

}  // namespace airg
