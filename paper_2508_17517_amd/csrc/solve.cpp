// Solve phase (paper Sec. 2, Eq. f_point): V-cycles with no down smoothing,
// restriction by R = [Z I], one-point prolongation by P = [W; I] and one up
// F-point smooth with the GMRES polynomial applied matrix-free by Horner;
// the coarsest level applies its Newton polynomial.  The outer loop is
// right-preconditioned FGMRES(restart) with classical Gram-Schmidt applied
// twice; the Hessenberg column comes to the host once per iteration.
//
// Many right-hand sides are solved together as K interleaved columns: every
// V-cycle kernel is then an SpMM that reads each matrix entry once for all
// columns, and the top-level product and the Gram-Schmidt, normalisation and
// update kernels likewise cover all columns per launch, while each column
// keeps its own FGMRES process (Hessenberg matrix, rotations, stopping test,
// restarts) on the host.  A block-diagonal batch of problems ordered
// problem-major runs one process per problem in the same way, its
// reductions and updates working on each problem's ranges of the nested
// numbering; without that order, one Krylov process runs over the whole
// system, each problem being a convergence group (its stopping test is
// tightened so that every problem reaches the tolerance on its own).
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

// With params.stagnation_check, a restart cycle (Richardson: `restart` steps)
// must bring the true residual norm below this fraction of its value at the
// cycle's start, or the process stops as not converged.
constexpr double kStagnation = 0.99;

Workspace::~Workspace() {
  for (const VcycleGraph& g : graphs) (void)hipGraphExecDestroy(g.exec);
  if (cap) (void)hipStreamDestroy(cap);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  for (hipEvent_t e : evh)
    if (e) (void)hipEventDestroy(e);
  if (pin) (void)hipHostFree(pin);
}

// The outer loop reads a few coefficients back every iteration and waits for
// them; from pinned memory the copy needs no staging through pageable memory.
static void read_small(Workspace& W, const double* dev, double* host, size_t n, hipStream_t s) {
  if (n > W.pin_n) fail(AIRG_ERR_INTERNAL, "pinned staging buffer too small");
  if (n == 0) return;
  AIRG_HIP(hipMemcpyAsync(W.pin, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipStreamSynchronize(s));
  std::memcpy(host, W.pin, n * sizeof(double));
}

void workspace_init(const Hierarchy& H, Workspace& W, int K) {
  hipStream_t s = H.s;
  // captured V-cycles hold the old buffers' addresses
  for (const VcycleGraph& g : W.graphs) (void)hipGraphExecDestroy(g.exec);
  W.graphs.clear();
  const int64_t n = H.n0 * K;
  W.K = K;
  // the bases' stride: a multiple of 4 KiB plus 4.5 KiB, so that successive
  // vectors do not start at the same offset of a power-of-two interleave
  // (n is often a power of two; a Gram-Schmidt sweep reads up to 32 basis
  // vectors at the same index)
  W.ld = (n + 511) / 512 * 512 + 576;
  W.restart = H.p.restart;
  W.V.alloc((size_t)(W.restart + 1) * W.ld, s);
  // the FGMRES Z basis: FP64, or FP32 with lower-precision storage (the
  // V-cycle's output is FP32 there, so an FP32 copy holds it exactly);
  // Richardson keeps its one correction in FP64
  W.z32 = H.p.precision != AIRG_FP64 && H.p.outer == AIRG_OUTER_FGMRES;
  if (W.z32) W.Zb32.alloc((size_t)W.restart * W.ld, s);
  else W.Zb.alloc((size_t)(H.p.outer == AIRG_OUTER_RICHARDSON ? 1 : W.restart) * W.ld, s);
  W.w.alloc(n, s);
  // smoother scratch: F rows, and C rows too with C-point smoothing
  const bool csm = H.p.smooth_type != AIRG_SMOOTH_TYPE_F;
  int64_t maxf = 1;
  for (const Level& L : H.levels) maxf = std::max(maxf, csm ? std::max(L.nF, L.nC) : L.nF);
  maxf *= K;
  const int64_t nc = std::max<int64_t>(1, H.levels.back().n) * K;
  if (H.p.precision == AIRG_FP64) {
    W.rr.alloc(n, s);
    W.sv.alloc(maxf, s);
    W.y0.alloc(maxf, s);
    W.y1.alloc(maxf, s);
    W.cw0.alloc(nc, s);
    W.cw1.alloc(nc, s);
    W.ct.alloc(nc, s);
    if (csm) W.rin.alloc(std::max<int64_t>(1, H.stacked_len) * K, s);
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
    if (csm) W.rin32.alloc(std::max<int64_t>(1, H.stacked_len) * K, s);
  }
  W.bperm.alloc(n, s);
  W.xperm.alloc(n, s);
  if (!H.seg.empty()) W.nat.alloc(H.n0, s);
  const size_t G = std::max<size_t>((size_t)K, H.seg.empty() ? 1 : H.seg.size());
  W.hbuf.alloc((2 * (W.restart + 1) + 2) * G, s);
  W.ybuf.alloc((W.restart + 1) * G, s);
  if (K > 1) {
    W.cdiv.alloc(K, s);
    W.cdot_work.alloc(col_dots_work_size(H.n0, K), s);
    W.cfused_work.alloc(col_fused_work_size(H.n0, K), s);
  } else {
    W.fused_work.alloc(cgs_fused_work_size(n), s);
  }
  // a batch ordered problem-major: one outer process per problem
  const int np = H.seg.empty() ? 0 : (int)H.seg.size() - 1;
  if (K == 1 && np > 0 && !H.granges.empty()) {
    build_group_items(H.granges, np, W.gitems, s);
    W.gdot_work.alloc(group_dots_work_size(W.gitems), s);
    build_group_items(H.granges, np, W.gitems_f, s, 256);
    W.gfused_work.alloc(group_fused_work_size(W.gitems_f), s);
    if (H.mgroups > 0) {
      W.active.alloc(np, s);
      W.gmask.alloc(H.mgroups, s);
    }
    W.cdiv.alloc(np, s);
  }
  const size_t ng = std::max<size_t>((size_t)K, H.seg.empty() ? 1 : H.seg.size());
  W.gbuf.alloc(ng + 1, s);
  W.pin_slot = (2 * (size_t)(W.restart + 1) + 2) * G;
  W.pin_n = std::max(2 * W.pin_slot, ng + 1);
  if (W.pin) (void)hipHostFree(W.pin);
  W.pin = nullptr;
  AIRG_HIP(hipHostMalloc((void**)&W.pin, W.pin_n * sizeof(double), hipHostMallocDefault));
  W.dot_work.alloc(dot_work_size(n, 64), s);
  W.col_work.alloc(col_sumsq_work_size(H.n0, K), s);
  if (!W.ev0) AIRG_HIP(hipEventCreate(&W.ev0));
  if (!W.ev1) AIRG_HIP(hipEventCreate(&W.ev1));
  for (hipEvent_t& e : W.evh)
    if (!e) AIRG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  W.pc.ok = false;
  if (K == 1 && H.seg.empty() && H.p.coarse_persistent)
    coarse_plan_build(W.pc, H.levels.back().A, H.levels.back().roots, H.p.precision, s);
}

namespace {

// Vectors of one V-cycle in vector type X (nested numbering, K columns).
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
  X* rin;       // stacked level residuals (C-point smoothing), or null
  const uint8_t* gmask;  // activity masks of a problem batch, or null
  const CoarsePlan* pc;  // the persistent coarse solve, or null (per-step launches)
};

VecSet<double> vecs64(Workspace& W, const double* in, double* e) {
  return {in,        e,         W.rr.get(), W.sv.get(), W.y0.get(), W.y1.get(),
          W.cw0.get(), W.cw1.get(), W.ct.get(), W.rin.get(), W.mask_on ? W.gmask.get() : nullptr,
          W.pc.ok ? &W.pc : nullptr};
}
VecSet<float> vecs32(Workspace& W, float* e) {
  return {W.in32.get(), e, W.rr32.get(), W.sv32.get(), W.y032.get(), W.y132.get(),
          W.cw032.get(), W.cw132.get(), W.ct32.get(), W.rin32.get(),
          W.mask_on ? W.gmask.get() : nullptr, W.pc.ok ? &W.pc : nullptr};
}

struct LevelOps {
  OpView ff, b, z, a, hat;
};
LevelOps ops_of(const Level& L, int prec) {
  return {op_view(L.Aff, L.ff32, L.ff16, prec), op_view(L.B, L.b32, L.b16, prec),
          op_view(L.Z, L.z32, L.z16, prec), op_view(L.A, L.a32, L.a16, prec),
          op_view(L.Ahat, L.hat32, L.hat16, prec)};
}
// the view of A with the activity masks gm (null: unmasked)
OpView masked(OpView v, const CSR& A, const uint8_t* gm) {
  if (gm && A.mask_off >= 0) v.gmask = gm + A.mask_off;
  return v;
}
// The operators of a V-cycle over a problem batch's per-problem processes:
// A_ff, B, Z and the coarsest matrix skip the row groups whose problems are
// inactive.  Their input there is exactly zero, so the skipped sums (0) are
// the ones the products would give.
LevelOps ops_of(const Level& L, int prec, const uint8_t* gm) {
  LevelOps o = ops_of(L, prec);
  o.ff = masked(o.ff, L.Aff, gm);
  o.b = masked(o.b, L.B, gm);
  o.z = masked(o.z, L.Z, gm);
  o.a = masked(o.a, L.A, gm);
  return o;
}

double vt_bytes(ValType vt) { return vt == VT_F64 ? 8.0 : vt == VT_F32 ? 4.0 : 2.0; }

template <class X>
void horner(const Level& L, const OpView& Aff, int K, const X* sv, const X* ec, X* ef, X* y0,
            X* y1, hipStream_t s, LaunchTally* tally = nullptr) {
  const std::vector<double>& a = L.alpha;
  const int d = (int)a.size() - 1;
  const int64_t n = L.nF * K;
  const double xb = (double)sizeof(X);
  const double mb = csr_bytes(L.nF, Aff.nnz, vt_bytes(Aff.vt)), mf = 2.0 * (double)Aff.nnz * K;
  // per step: y gathered, s read, out written; the last step also reads cmap
  // and gathers W e_c
  auto count = [&](bool last) {
    if (tally)
      tally->add(mb + xb * n * (last ? 4 : 3) + (last ? 4.0 * L.nF : 0.0), mf + 3.0 * n,
                 col_saving(Aff));
  };
  const int32_t* cmap = L.cmap.get();
  if (d == 0) {
    prolong_axpy_t<X>(ef, sv, cmap, ec, a[0], L.nF, K, s);
    if (tally) tally->add(4.0 * xb * n + 4.0 * L.nF, 2.0 * n);
    return;
  }
  if (d == 1) {
    spmv_horner_prolong_t<X>(Aff, L.tpr_ff, K, sv, sv, ef, a[1], a[0], cmap, ec, s);
    count(true);
    return;
  }
  X* y[2] = {y0, y1};
  int c = 0;
  spmv_horner_t<X>(Aff, L.tpr_ff, K, sv, sv, y[0], a[d], a[d - 1], false, s);
  count(false);
  for (int k = d - 2; k >= 1; --k) {
    spmv_horner_t<X>(Aff, L.tpr_ff, K, y[c], sv, y[c ^ 1], 1.0, a[k], false, s);
    count(false);
    c ^= 1;
  }
  spmv_horner_prolong_t<X>(Aff, L.tpr_ff, K, y[c], sv, ef, 1.0, a[0], cmap, ec, s);
  count(true);
}

// The F-point smoother: the polynomial matrix-free (Horner), or one product
// with the assembled Ahat^{-1} fused with the prolongation.
template <class X>
const X* dinv_of(const Level& L);
template <>
const double* dinv_of<double>(const Level& L) { return L.dinv.get(); }
template <>
const float* dinv_of<float>(const Level& L) { return L.dinv32.get(); }

// nAIR's Neumann smoother: y = D^{-1} s, then d steps y += D^{-1} (s - A_ff y),
// the last one fused with the prolongation
template <class X>
void neumann(const Level& L, const OpView& Aff, int K, const X* sv, const X* ec, X* ef, X* y0,
             X* y1, hipStream_t s, LaunchTally* tally) {
  const int d = (int)L.alpha.size() - 1;
  const int64_t n = L.nF * K;
  const double xb = (double)sizeof(X);
  const X* dinv = dinv_of<X>(L);
  const int32_t* cmap = L.cmap.get();
  const double mb = csr_bytes(L.nF, Aff.nnz, vt_bytes(Aff.vt)), mf = 2.0 * (double)Aff.nnz * K;
  if (d == 0) {
    dinv_apply_t<X>(ef, sv, dinv, cmap, ec, L.nF, K, s);
    if (tally) tally->add(3.0 * xb * n + xb * L.nF + 4.0 * L.nF, 2.0 * n);
    return;
  }
  X* y[2] = {y0, y1};
  dinv_apply_t<X>(y[0], sv, dinv, nullptr, nullptr, L.nF, K, s);
  if (tally) tally->add(2.0 * xb * n + xb * L.nF, (double)n);
  int c = 0;
  for (int k = 1; k < d; ++k) {
    spmv_neumann_t<X>(Aff, L.tpr_ff, K, y[c], sv, dinv, y[c ^ 1], s);
    if (tally) tally->add(mb + xb * n * 3 + xb * L.nF, mf + 3.0 * n, col_saving(Aff));
    c ^= 1;
  }
  spmv_neumann_prolong_t<X>(Aff, L.tpr_ff, K, y[c], sv, dinv, ef, cmap, ec, s);
  if (tally) tally->add(mb + xb * n * 4 + xb * L.nF + 4.0 * L.nF, mf + 4.0 * n, col_saving(Aff));
}

template <class X>
void smooth(const Level& L, const LevelOps& o, int K, const X* sv, const X* ec, X* ef, X* y0,
            X* y1, hipStream_t s, LaunchTally* tally = nullptr) {
  if (L.Ahat.rows == 0) {
    if (L.dinv.get()) neumann<X>(L, o.ff, K, sv, ec, ef, y0, y1, s, tally);
    else horner<X>(L, o.ff, K, sv, ec, ef, y0, y1, s, tally);
    return;
  }
  spmv_horner_prolong_t<X>(o.hat, L.tpr_hat, K, sv, sv, ef, 1.0, 0.0, L.cmap.get(), ec, s);
  if (tally) {
    const double xb = (double)sizeof(X);
    const int64_t n = L.nF * K;
    tally->add(csr_bytes(L.nF, o.hat.nnz, vt_bytes(o.hat.vt)) + xb * n * 4 + 4.0 * L.nF,
               2.0 * (double)o.hat.nnz * K + 3.0 * n, col_saving(o.hat));
  }
}

// out += q(A) s by Horner with the last product accumulating into out (the
// C smooth, and the second F smooth of FCF): d products with A.
template <class X>
void horner_acc(const OpView& A, int tpr, const std::vector<double>& a, int64_t rows, int K,
                const X* sv, X* out, X* y0, X* y1, hipStream_t s) {
  const int d = (int)a.size() - 1;
  if (d < 0) return;
  if (d == 0) {
    axpy_first_t<X>(out, sv, a[0], false, rows * K, s);
    return;
  }
  if (d == 1) {
    spmv_horner_t<X>(A, tpr, K, sv, sv, out, a[1], a[0], true, s);
    return;
  }
  X* y[2] = {y0, y1};
  int c = 0;
  spmv_horner_t<X>(A, tpr, K, sv, sv, y[0], a[d], a[d - 1], false, s);
  for (int k = d - 2; k >= 1; --k) {
    spmv_horner_t<X>(A, tpr, K, y[c], sv, y[c ^ 1], 1.0, a[k], false, s);
    c ^= 1;
  }
  spmv_horner_t<X>(A, tpr, K, y[c], sv, out, 1.0, a[0], true, s);
}

// After the first F smooth of level L: the C smooth
//   t = r_c - A_cf e_f - A_cc e_c,  e_c += q_c(A_cc) t,
// and for FCF a second F smooth with the updated e_c
//   s = r_f - A_fc e_c - A_ff e_f,  e_f += q(A_ff) s
// (the assembled inverses with AIRG_SMOOTH_ASSEMBLED).  rf is the level's
// residual, its C part following its nF F rows.
template <class X>
void smooth_c(const Hierarchy& H, const Level& L, const LevelOps& o, int K, const X* rf, X* ec,
              X* ef, const VecSet<X>& v, hipStream_t s) {
  const int prec = H.p.precision;
  const bool asm_smoother = H.p.smoother == AIRG_SMOOTH_ASSEMBLED;
  const X* rc = rf + L.nF * K;
  spmv_residual_t<X>(L.cf.view(prec), L.cf.tpr, K, ef, rc, v.y1, s);
  spmv_residual_t<X>(L.cc.view(prec), L.cc.tpr, K, ec, v.y1, v.sv, s);
  if (asm_smoother)
    spmv_horner_t<X>(L.hat_cc.view(prec), L.hat_cc.tpr, K, v.sv, v.sv, ec, 1.0, 0.0, true, s);
  else
    horner_acc<X>(L.cc.view(prec), L.cc.tpr, L.alpha_c, L.nC, K, v.sv, ec, v.y0, v.y1, s);
  if (H.p.smooth_type != AIRG_SMOOTH_TYPE_FCF) return;
  spmv_residual_t<X>(L.fc.view(prec), L.fc.tpr, K, ec, rf, v.y1, s);
  spmv_residual_t<X>(o.ff, L.tpr_ff, K, ef, v.y1, v.sv, s);
  if (asm_smoother)
    spmv_horner_t<X>(o.hat, L.tpr_hat, K, v.sv, v.sv, ef, 1.0, 0.0, true, s);
  else
    horner_acc<X>(o.ff, L.tpr_ff, L.alpha, L.nF, K, v.sv, ef, v.y0, v.y1, s);
}

template <class X>
void vcycle_t(const Hierarchy& H, const VecSet<X>& v, int K, hipStream_t s) {
  const int prec = H.p.precision;
  const int L = (int)H.levels.size() - 1;
  // level l's residual (l >= 1): the suffix at off_l of rr, each restriction
  // overwriting the C part of the level above in place; with C-point
  // smoothing, which reads r_c again on the way up, its own segment of rin
  const bool csm = H.p.smooth_type != AIRG_SMOOTH_TYPE_F;
  auto input = [&](int l) -> X* {
    return csm ? v.rin + H.levels[l].in_off * K : v.rr + H.levels[l].off * K;
  };
  for (int l = 0; l < L; ++l) {
    const Level& lv = H.levels[l];
    const X* src = l == 0 ? v.in : input(l);
    spmv_restrict_t<X>(ops_of(lv, prec, v.gmask).z, lv.tpr_z, K, src, src + lv.nF * K,
                       input(l + 1), s);
  }
  const Level& lc = H.levels[L];
  const X* rc = L == 0 ? v.in : input(L);
  if (v.pc && K == 1)
    coarse_persistent_t<X>(*v.pc, ops_of(lc, prec, v.gmask).a, rc, v.e + lc.off, s);
  else
    newton_apply_t<X>(ops_of(lc, prec, v.gmask).a, lc.tpr_a, K, lc.roots, rc, v.e + lc.off * K,
                      v.cw0, v.cw1, v.ct, s);
  for (int l = L - 1; l >= 0; --l) {
    const Level& lv = H.levels[l];
    const LevelOps o = ops_of(lv, prec, v.gmask);
    const X* rf = l == 0 ? v.in : input(l);
    X* ef = v.e + lv.off * K;
    X* ec = v.e + H.levels[l + 1].off * K;
    spmv_residual_t<X>(o.b, lv.tpr_b, K, ec, rf, v.sv, s);
    smooth<X>(lv, o, K, v.sv, ec, ef, v.y0, v.y1, s);
    if (csm) smooth_c<X>(H, lv, o, K, rf, ec, ef, v, s);
  }
}

void dots(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* out,
          Workspace& W, hipStream_t s) {
  for (int k0 = 0; k0 < nv; k0 += 64) {
    int cnt = std::min(64, nv - k0);
    launch_tree_dots(V + (int64_t)k0 * ld, ld, cnt, w, n, out + k0, W.dot_work.get(), s);
  }
}

// Norms of the convergence groups of a stacked vector in nested numbering:
// its K columns, or (K = 1, a batch of problems) each problem's rows.
std::vector<double> group_norms(const Hierarchy& H, Workspace& W, const double* v) {
  hipStream_t s = H.s;
  const int K = W.K;
  double* g = W.gbuf.get();
  size_t ng;
  if (K > 1) {
    ng = (size_t)K;
    launch_col_sumsq(v, H.n0, K, g, W.col_work.get(), s);
  } else if (!H.seg.empty()) {
    ng = H.seg.size() - 1;
    launch_gather(W.nat.get(), v, H.levels[0].pos.get(), H.n0, s);
    for (size_t p = 0; p < ng; ++p) {
      const double* a = W.nat.get() + H.seg[p];
      launch_tree_dots(a, 0, 1, a, H.seg[p + 1] - H.seg[p], g + p, W.dot_work.get(), s);
    }
  } else {
    ng = 1;
    launch_tree_dots(v, 0, 1, v, H.n0, g, W.dot_work.get(), s);
  }
  std::vector<double> out(ng);
  read_small(W, W.gbuf.get(), out.data(), ng, s);
  for (double& x : out) x = std::sqrt(x);
  return out;
}

// Givens-rotated Arnoldi state of one column's FGMRES cycle.
struct ColumnCycle {
  std::vector<double> Hm, g, cs, sn, y;
  int k = 0;  // Arnoldi steps taken in this cycle
  void reset(int R, double beta) {
    Hm.assign((size_t)(R + 1) * R, 0.0);
    g.assign(R + 1, 0.0);
    cs.assign(R, 0.0);
    sn.assign(R, 0.0);
    y.assign(R, 0.0);
    g[0] = beta;
    k = 0;
  }
  // Append Hessenberg column j (h[i], i <= j, and h_{j+1,j} = hn), rotate it
  // and return the residual estimate |g_{j+1}|.
  double push(int R, int j, const double* h, double hn) {
    for (int i = 0; i <= j; ++i) Hm[(size_t)i * R + j] = h[i];
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
    return std::fabs(g[j + 1]);
  }
  // Back substitution for the k coefficients of the solution update.
  void solve_upper(int R) {
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= Hm[(size_t)i * R + q] * y[q];
      y[i] = t / Hm[(size_t)i * R + i];
    }
  }
};

// The kernels of G independent outer processes run together: the K
// interleaved columns of a multi-column solve (G = K), or the problems of a
// batch ordered problem-major (G problems, ranges of one column).
struct Procs {
  const Hierarchy& H;
  Workspace& W;
  int G;
  bool cols;
  // the problems' activity on the device while the Arnoldi step's w is zero
  // on the stopped problems (null: every item is computed)
  const uint8_t* act = nullptr;
  void dots(const double* V, int64_t ld, int nv, const double* w, double* out) {
    if (cols) launch_col_dots(V, ld, nv, w, H.n0, W.K, out, W.cdot_work.get(), H.s);
    else launch_group_dots(V, ld, nv, w, W.gitems, out, W.gdot_work.get(), H.s, act);
  }
  // the first sweep of an Arnoldi step: V^T w (fused per problem where a
  // fused kernel exists)
  void first_dots(const double* V, int64_t ld, int nv, const double* w, double* out) {
    if (!cols && nv <= kFusedVecs)
      launch_group_fused_dots(V, ld, nv, w, W.gitems_f, out, W.gfused_work.get(), H.s, act);
    else
      dots(V, ld, nv, w, out);
  }
  void update(double* w, const double* V, int64_t ld, const double* h, int nv) {
    if (cols) launch_cgs_update_cols(w, V, ld, h, nv, H.n0, W.K, H.s);
    else launch_group_update(w, V, ld, h, nv, W.gitems, H.s);
  }
  // w = w - V h, then the next sweep's coefficients (one pass over the basis
  // where a fused kernel exists)
  void update_dots(double* w, const double* V, int64_t ld, const double* h, int nv, double* out) {
    if (nv <= kFusedVecs) {
      if (cols)
        launch_cols_update_dots(w, V, ld, h, nv, H.n0, W.K, out, W.cfused_work.get(), H.s);
      else
        launch_group_update_dots(w, V, ld, h, nv, W.gitems_f, out, W.gfused_work.get(), H.s, act);
      return;
    }
    update(w, V, ld, h, nv);
    dots(V, ld, nv, w, out);
  }
  // w = w - V h, then w . w
  void update_sumsq(double* w, const double* V, int64_t ld, const double* h, int nv, double* out) {
    if (nv <= kFusedVecs) {
      if (cols)
        launch_cols_update_norm2(w, V, ld, h, nv, H.n0, W.K, out, W.cfused_work.get(), H.s);
      else
        launch_group_update_norm2(w, V, ld, h, nv, W.gitems_f, out, W.gfused_work.get(), H.s, act);
      return;
    }
    update(w, V, ld, h, nv);
    sumsq(w, out);
  }
  void sumsq(const double* v, double* out) {
    if (cols) launch_col_sumsq(v, H.n0, W.K, out, W.col_work.get(), H.s);
    else launch_group_dots(v, 0, 1, v, W.gitems, out, W.gdot_work.get(), H.s);
  }
  // y = x / d per process (and y32 = (float) y when given)
  void divide(double* y, const double* x, const double* d, float* y32 = nullptr) {
    if (cols) launch_divide_cols(y, x, d, H.n0, W.K, H.s, y32);
    else launch_group_divide(y, x, d, W.gitems, H.s, y32);
  }
  template <class ZT>
  void combine(double* x, const ZT* Z, int64_t ld, const double* y, int nv) {
    if (cols) launch_basis_combine_cols(x, Z, ld, y, nv, H.n0, W.K, H.s);
    else launch_group_combine(x, Z, ld, y, nv, W.gitems, H.s);
  }
  std::vector<double> norms(const double* v) {
    sumsq(v, W.gbuf.get());
    std::vector<double> out(G);
    read_small(W, W.gbuf.get(), out.data(), G, H.s);
    for (double& x : out) x = std::sqrt(x);
    return out;
  }
};

// G outer processes at once (see fgmres_solve).  A process that has stopped
// (converged, out of iterations, or at the end of its Arnoldi process in
// this cycle) is carried through the shared launches as zeros: its divisor
// is 0, so its next basis vector, V-cycle input and products vanish, and it
// gets a zero weight in every solution update.
void solve_processes(const Hierarchy& H, Workspace& W, Procs& P, std::vector<airg_solve_info>& out,
                     bool& all_converged) {
  hipStream_t s = H.s;
  const int K = W.K;
  const int G = P.G;
  const int64_t n0 = H.n0;
  const int64_t n = n0 * K;
  const int R = W.restart;
  const int64_t ld = W.ld;
  const double rtol = H.p.rtol, atol = H.p.atol;
  // a residual is small enough at rtol times its reference norm or at atol
  auto tol = [&](double ref) { return std::max(rtol * ref, atol); };
  const int max_it = H.p.max_it;
  const OpView A = opview(H.Aperm);
  double* V = W.V.get();
  double* Zb = W.Zb.get();
  // with an FP32 Z basis: the V-cycle reads (float) V_j, which every
  // normalisation also writes to W.in32, and leaves z_j in FP32
  float* Zb32 = W.z32 ? W.Zb32.get() : nullptr;
  float* in32 = W.z32 ? W.in32.get() : nullptr;
  double* dv = W.cdiv.get();

  std::vector<double> bn = P.norms(W.bperm.get());
  for (double v : bn)
    if (!std::isfinite(v)) fail(AIRG_ERR_NONFINITE, "right-hand side is not finite");
  std::vector<int> its(G, 0), rst(G, 0), done(G, 0), stag(G, 0);
  std::vector<double> rn(G, 0.0), est(G, 0.0), ref = bn, dh(G), yh((size_t)R * G);
  // stagnation check: a process whose true residual falls by less than
  // kStagnation over a restart cycle (Richardson: over `restart` steps) stops
  const bool stag_check = H.p.stagnation_check != 0;
  std::vector<double> rwin(G, 0.0);
  auto upload_div = [&]() { W.cdiv.from_host(dh.data(), G); };
  auto residual = [&](double* r) {
    spmv_t<double>(A, H.tpr_top, K, W.xperm.get(), W.w.get(), s);
    launch_sub(r, W.bperm.get(), W.w.get(), n, s);
    rn = P.norms(r);
  };
  if (H.p.outer == AIRG_OUTER_RICHARDSON) {
    // x <- x + M (b - A x) for the columns still running; a column with b = 0
    // is measured against its initial residual
    double* r = V;
    double* e = Zb;
    residual(r);
    for (int c = 0; c < G; ++c) {
      if (ref[c] == 0.0) ref[c] = rn[c];
      done[c] = rn[c] <= tol(ref[c]) || max_it <= 0;
      rwin[c] = rn[c];
    }
    for (;;) {
      bool any = false;
      for (int c = 0; c < G; ++c) {
        dh[c] = done[c] ? 0.0 : 1.0;
        any = any || !done[c];
      }
      if (!any) break;
      vcycle(H, W, r, e);
      W.ybuf.from_host(dh.data(), G);
      P.combine(W.xperm.get(), e, ld, W.ybuf.get(), 1);
      residual(r);
      for (int c = 0; c < G; ++c) {
        if (done[c]) continue;
        ++its[c];
        if (!std::isfinite(rn[c])) fail(AIRG_ERR_BREAKDOWN, "Richardson diverged (non-finite residual)");
        if (rn[c] <= tol(ref[c]) || its[c] >= max_it) {
          done[c] = 1;
        } else if (stag_check && its[c] % R == 0) {
          if (rn[c] > kStagnation * rwin[c]) done[c] = stag[c] = 1;
          rwin[c] = rn[c];
        }
      }
    }
  } else {
    // b = 0: the solution of A x = 0, whatever the guess
    bool zero = false;
    for (int c = 0; c < G; ++c) {
      dh[c] = bn[c] == 0.0 ? 0.0 : 1.0;
      zero = zero || bn[c] == 0.0;
      done[c] = bn[c] == 0.0;
    }
    if (zero) {
      upload_div();
      P.divide(W.xperm.get(), W.xperm.get(), dv);
    }
    std::vector<ColumnCycle> cyc(G);
    std::vector<int> act(G, 0);
    double* hd = W.hbuf.get();
    std::vector<double> hh((size_t)(2 * (R + 1) + 1) * G), hc(R + 1);
    for (;;) {
      residual(V);
      bool any = false;
      for (int c = 0; c < G; ++c) {
        act[c] = 0;
        if (done[c]) continue;
        if (rn[c] <= tol(bn[c]) || its[c] >= max_it) {
          done[c] = 1;
          continue;
        }
        if (!std::isfinite(rn[c])) fail(AIRG_ERR_BREAKDOWN, "FGMRES breakdown (non-finite residual)");
        if (stag_check && its[c] > 0 && rn[c] > kStagnation * rwin[c]) {
          done[c] = stag[c] = 1;
          continue;
        }
        rwin[c] = rn[c];
        if (its[c] > 0) ++rst[c];
        act[c] = 1;
        any = true;
      }
      if (!any) break;
      for (int c = 0; c < G; ++c) {
        dh[c] = act[c] ? rn[c] : 0.0;
        cyc[c].reset(R, act[c] ? rn[c] : 0.0);
      }
      upload_div();
      P.divide(V, V, dv, in32);
      // problems of a batch whose processes are not running have a zero
      // basis vector: the V-cycle and the top product skip their rows
      const bool mask = !P.cols && W.gmask.size() > 0;
      std::vector<uint8_t> amask(mask ? G : 0, 2);  // last uploaded activity (2: none yet)
      OpView Am = A;
      if (mask) Am = masked(A, H.Aperm, W.gmask.get());
      for (int j = 0; j < R; ++j) {
        double* vj = V + (int64_t)j * ld;
        double* zj = Zb + (int64_t)j * ld;
        if (mask) {
          bool changed = false;
          for (int c = 0; c < G; ++c) {
            const uint8_t a = act[c] ? 1 : 0;
            changed = changed || amask[c] != a;
            amask[c] = a;
          }
          if (changed) {
            W.active.from_host(amask.data(), G);
            launch_group_mask(H.mgp0.get(), H.mgp1.get(), W.active.get(), H.mgroups,
                              W.gmask.get(), s);
          }
          W.mask_on = true;
        }
        if (Zb32) {
          float* zj32 = Zb32 + (int64_t)j * ld;
          vcycle(H, W, vj, nullptr, zj32, true);
          W.mask_on = false;
          spmv_x32(mask ? Am : A, H.tpr_top, K, zj32, W.w.get(), s);
        } else {
          vcycle(H, W, vj, zj);
          W.mask_on = false;
          spmv_t<double>(mask ? Am : A, H.tpr_top, K, zj, W.w.get(), s);
        }
        double* h1 = hd;
        double* h2 = hd + (size_t)(R + 1) * G;
        double* hn2 = hd + (size_t)2 * (R + 1) * G;
        // a stopped problem's basis vector was zero, so its V-cycle output,
        // product and every Gram-Schmidt term are zero: the sweeps skip it
        if (mask) P.act = W.active.get();
        P.first_dots(V, ld, j + 1, W.w.get(), h1);
        P.update_dots(W.w.get(), V, ld, h1, j + 1, h2);
        P.update_sumsq(W.w.get(), V, ld, h2, j + 1, hn2);
        P.act = nullptr;
        read_small(W, W.hbuf.get(), hh.data(), (size_t)(2 * (R + 1) + 1) * G, s);
        bool more = false;
        for (int c = 0; c < G; ++c) {
          dh[c] = 0.0;
          if (!act[c]) continue;
          for (int i = 0; i <= j; ++i)
            hc[i] = hh[(size_t)i * G + c] + hh[(size_t)(R + 1) * G + (size_t)i * G + c];
          const double hn = std::sqrt(hh[(size_t)2 * (R + 1) * G + c]);
          ++its[c];
          est[c] = cyc[c].push(R, j, hc.data(), hn);
          if (!std::isfinite(est[c])) fail(AIRG_ERR_BREAKDOWN, "FGMRES breakdown (non-finite residual)");
          if (est[c] <= tol(bn[c]) || its[c] >= max_it || hn == 0.0) {
            act[c] = 0;
            continue;
          }
          dh[c] = hn;
          more = true;
        }
        if (!more || j + 1 == R) break;
        upload_div();
        P.divide(V + (int64_t)(j + 1) * ld, W.w.get(), dv, in32);
      }
      int kmax = 0;
      std::fill(yh.begin(), yh.end(), 0.0);
      for (int c = 0; c < G; ++c) {
        ColumnCycle& cc = cyc[c];
        if (cc.k == 0) continue;
        cc.solve_upper(R);
        for (int i = 0; i < cc.k; ++i) yh[(size_t)i * G + c] = cc.y[i];
        kmax = std::max(kmax, cc.k);
      }
      W.ybuf.from_host(yh.data(), (size_t)kmax * G);
      if (Zb32) P.combine(W.xperm.get(), Zb32, ld, W.ybuf.get(), kmax);
      else P.combine(W.xperm.get(), Zb, ld, W.ybuf.get(), kmax);
    }
  }
  all_converged = true;
  out.assign(G, airg_solve_info{});
  for (int c = 0; c < G; ++c) {
    airg_solve_info& o = out[c];
    o.iterations = its[c];
    o.restarts = rst[c];
    o.stagnated = stag[c];
    o.converged = rn[c] <= tol(ref[c]) ? 1 : 0;
    o.rel_residual = ref[c] > 0.0 ? rn[c] / ref[c] : 0.0;
    o.rel_residual_estimate = H.p.outer == AIRG_OUTER_RICHARDSON
                                  ? o.rel_residual
                                  : (bn[c] > 0.0 ? est[c] / bn[c] : 0.0);
    if (!o.converged) all_converged = false;
  }
}

}  // namespace

// The launches of one V-cycle, enqueued on s: e64 = M in, or with
// lower-precision storage e32 = M in when e32 is given (the V-cycle's FP32
// output kept as it is); in32_ready: the caller already wrote (float) in to
// W.in32.
void vcycle_launches(const Hierarchy& H, Workspace& W, const double* in, double* e64, float* e32,
                     bool in32_ready, hipStream_t s) {
  const int64_t n = H.n0 * W.K;
  if (H.p.precision == AIRG_FP64) {
    vcycle_t<double>(H, vecs64(W, in, e64), W.K, s);
    return;
  }
  if (!in32_ready) convert_d2f(W.in32.get(), in, n, s);
  vcycle_t<float>(H, vecs32(W, e32 ? e32 : W.e32.get()), W.K, s);
  if (!e32) convert_f2d(e64, W.e32.get(), n, s);
}

// The V-cycle as an instantiated HIP graph: captured once per set of vectors
// (in, e64, e32, whether in32 is ready, activity masks on or off) and
// launch-shape epoch on the workspace's own capture stream (capture needs a
// stream other than the null stream; capturing executes nothing), then
// replayed on the hierarchy's stream.  The V-cycle's kernels take every
// coefficient and pointer as a launch argument and no memset or copy is among
// them, so a replay repeats exactly the launches of the direct path.
hipGraphExec_t vcycle_graph(const Hierarchy& H, Workspace& W, const double* in, double* e64,
                            float* e32, bool in32_ready) {
  const bool mask = W.mask_on;
  for (const VcycleGraph& g : W.graphs)
    if (g.in == in && g.e64 == e64 && g.e32 == e32 && g.in32_ready == in32_ready &&
        g.mask == mask && g.epoch == H.shape_epoch)
      return g.exec;
  if (!W.cap) AIRG_HIP(hipStreamCreateWithFlags(&W.cap, hipStreamNonBlocking));
  AIRG_HIP(hipStreamBeginCapture(W.cap, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    vcycle_launches(H, W, in, e64, e32, in32_ready, W.cap);
  } catch (...) {
    (void)hipStreamEndCapture(W.cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  AIRG_HIP(hipStreamEndCapture(W.cap, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  AIRG_HIP(err);
  // graphs of an older launch-shape epoch are stale: drop them
  std::vector<VcycleGraph> keep;
  for (const VcycleGraph& g : W.graphs) {
    if (g.epoch == H.shape_epoch) keep.push_back(g);
    else (void)hipGraphExecDestroy(g.exec);
  }
  keep.push_back({in, e64, e32, in32_ready, mask, H.shape_epoch, exec});
  W.graphs.swap(keep);
  return exec;
}

void vcycle(const Hierarchy& H, Workspace& W, const double* in, double* e64, float* e32,
            bool in32_ready) {
  if (H.p.graph) {
    AIRG_HIP(hipGraphLaunch(vcycle_graph(H, W, in, e64, e32, in32_ready), H.s));
    return;
  }
  vcycle_launches(H, W, in, e64, e32, in32_ready, H.s);
}

int fgmres_solve(const Hierarchy& H, Workspace& W, const double* b, int64_t ldb, double* x,
                 int64_t ldx, int kvalid, bool guess, airg_solve_info* info) {
  hipStream_t s = H.s;
  const int K = W.K;
  const int64_t n = H.n0 * K;  // stacked length
  const int R = W.restart;
  const int64_t ld = W.ld;
  const int32_t* pos = H.levels[0].pos.get();
  const double rtol = H.p.rtol, atol = H.p.atol;
  auto tol = [&](double ref) { return std::max(rtol * ref, atol); };
  const int max_it = H.p.max_it;
  AIRG_HIP(hipEventRecord(W.ev0, s));

  const bool groups = K == 1 && W.gitems.n > 0;
  if (K > 1 || groups) {
    if (K > 1) {
      launch_scatter_cols(W.bperm.get(), b, ldb, pos, H.n0, K, kvalid, s);
      if (guess) launch_scatter_cols(W.xperm.get(), x, ldx, pos, H.n0, K, kvalid, s);
      else launch_fill(W.xperm.get(), n, 0.0, s);
    } else {
      launch_scatter(W.bperm.get(), b, pos, H.n0, s);
      if (guess) launch_scatter(W.xperm.get(), x, pos, H.n0, s);
      else launch_fill(W.xperm.get(), n, 0.0, s);
    }
    Procs P{H, W, groups ? W.gitems.G : K, !groups};
    std::vector<airg_solve_info> res;
    bool ok = false;
    solve_processes(H, W, P, res, ok);
    if (K > 1) launch_gather_cols(x, ldx, W.xperm.get(), pos, H.n0, K, kvalid, s);
    else launch_gather(x, W.xperm.get(), pos, H.n0, s);
    AIRG_HIP(hipEventRecord(W.ev1, s));
    AIRG_HIP(hipEventSynchronize(W.ev1));
    float ms = 0.f;
    AIRG_HIP(hipEventElapsedTime(&ms, W.ev0, W.ev1));
    if (info) {
      const int nout = groups ? P.G : kvalid;
      for (int c = 0; c < nout; ++c) {
        info[c] = res[c];
        info[c].solve_ms = ms;
      }
    }
    return ok ? AIRG_OK : AIRG_NOT_CONVERGED;
  }
  launch_scatter(W.bperm.get(), b, pos, H.n0, s);
  if (guess) launch_scatter(W.xperm.get(), x, pos, H.n0, s);
  else launch_fill(W.xperm.get(), n, 0.0, s);
  const std::vector<double> bn = group_norms(H, W, W.bperm.get());
  const size_t ng = bn.size();
  double bmin = 0.0, btot2 = 0.0;
  for (double v : bn) {
    if (!std::isfinite(v)) fail(AIRG_ERR_NONFINITE, "right-hand side is not finite");
    btot2 += v * v;
    if (v > 0.0 && (bmin == 0.0 || v < bmin)) bmin = v;
  }
  const double bnorm = std::sqrt(btot2);
  // stopping test of the stacked Krylov process: |r| <= rtol min_g |b_g| (or
  // atol) makes every group's residual small enough (it equals rtol |b| for
  // one group)
  const double thr = tol(bmin);

  std::vector<airg_solve_info> out(ng);
  for (auto& o : out) std::memset(&o, 0, sizeof(o));
  int status = AIRG_OK;
  int its = 0, restarts = 0;
  int stagnated = 0;
  const bool stag_check = H.p.stagnation_check != 0;
  double rwin = 0.0;  // the residual norm the stagnation check compares with
  double est_rel = 0.0;
  std::vector<double> rn(ng, 0.0);
  std::vector<double> ref = bn;  // the norms the relative residuals refer to
  bool converged = false;
  if (H.p.outer == AIRG_OUTER_RICHARDSON) {
    // undamped Richardson x <- x + M (b - A x) (Sec. 3); a group with b = 0
    // is measured against its initial residual
    double* r = W.V.get();
    double* e = W.Zb.get();
    const double one = 1.0;
    W.ybuf.from_host(&one, 1);
    auto residual = [&]() {
      spmv_t<double>(opview(H.Aperm), H.tpr_top, K, W.xperm.get(), W.w.get(), s);
      launch_sub(r, W.bperm.get(), W.w.get(), n, s);
      rn = group_norms(H, W, r);
      for (size_t q = 0; q < ng; ++q)
        if (!std::isfinite(rn[q])) fail(AIRG_ERR_BREAKDOWN, "Richardson diverged (non-finite residual)");
    };
    auto done = [&]() {
      for (size_t q = 0; q < ng; ++q)
        if (!(rn[q] <= tol(ref[q]))) return false;
      return true;
    };
    residual();
    for (size_t q = 0; q < ng; ++q)
      if (ref[q] == 0.0) ref[q] = rn[q];
    converged = done();
    auto total = [&]() {
      double t = 0.0;
      for (double v : rn) t += v * v;
      return std::sqrt(t);
    };
    rwin = total();
    while (!converged && its < max_it) {
      vcycle(H, W, r, e);
      launch_basis_combine(W.xperm.get(), e, W.ld, W.ybuf.get(), 1, n, s);
      ++its;
      residual();
      converged = done();
      if (!converged && stag_check && its % R == 0) {
        if (total() > kStagnation * rwin) {
          stagnated = 1;
          break;
        }
        rwin = total();
      }
    }
    est_rel = 0.0;
    for (size_t q = 0; q < ng; ++q) est_rel = std::max(est_rel, ref[q] > 0 ? rn[q] / ref[q] : 0.0);
  } else if (bnorm == 0.0) {
    launch_fill(W.xperm.get(), n, 0.0, s);  // the solution of A x = 0
    converged = true;
  } else {
    std::vector<double> Hm((size_t)(R + 1) * R), g(R + 1), cs(R), sn(R), hh(2 * (R + 1) + 2), y(R);
    double* V = W.V.get();
    double* Zb = W.Zb.get();
    float* Zb32 = W.z32 ? W.Zb32.get() : nullptr;  // FP32 Z basis (see solve_processes)
    float* in32 = W.z32 ? W.in32.get() : nullptr;
    double* hd = W.hbuf.get();
    for (;;) {
      spmv_t<double>(opview(H.Aperm), H.tpr_top, K, W.xperm.get(), W.w.get(), s);
      launch_sub(V, W.bperm.get(), W.w.get(), n, s);
      rn = group_norms(H, W, V);
      converged = true;
      double beta2 = 0.0;
      for (size_t q = 0; q < ng; ++q) {
        beta2 += rn[q] * rn[q];
        if (!(rn[q] <= tol(bn[q]))) converged = false;
      }
      const double beta = std::sqrt(beta2);
      if (converged || its >= max_it) break;
      if (!std::isfinite(beta)) fail(AIRG_ERR_BREAKDOWN, "FGMRES breakdown (non-finite residual)");
      if (stag_check && its > 0 && beta > kStagnation * rwin) {
        stagnated = 1;
        break;
      }
      rwin = beta;
      if (its > 0) ++restarts;
      launch_divide(V, V, beta, n, s, in32);
      std::fill(Hm.begin(), Hm.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;
      // Arnoldi step j on the device: V-cycle, product, CGS2 (h1 = V^T w;
      // w -= V h1; h2 = V^T w; w -= V h2; |w|^2, each sweep fused with the
      // reduction after it), and the copy of its coefficients to pinned
      // slot `slot`, marked by that slot's event
      const size_t nh = 2 * (size_t)(R + 1) + 1;
      auto enqueue_step = [&](int j, int slot) {
        double* vj = V + (int64_t)j * ld;
        if (Zb32) {
          float* zj32 = Zb32 + (int64_t)j * ld;
          vcycle(H, W, vj, nullptr, zj32, true);
          spmv_x32(opview(H.Aperm), H.tpr_top, K, zj32, W.w.get(), s);
        } else {
          double* zj = Zb + (int64_t)j * ld;
          vcycle(H, W, vj, zj);
          spmv_t<double>(opview(H.Aperm), H.tpr_top, K, zj, W.w.get(), s);
        }
        if (j + 1 <= kFusedVecs) {
          launch_cgs_dots(V, ld, j + 1, W.w.get(), n, hd, W.fused_work.get(), s);
          launch_cgs_update_dots(W.w.get(), V, ld, hd, j + 1, n, hd + (R + 1), W.fused_work.get(), s);
          launch_cgs_update_norm2(W.w.get(), V, ld, hd + (R + 1), j + 1, n, hd + 2 * (R + 1),
                                  W.fused_work.get(), s);
        } else {
          dots(V, ld, j + 1, W.w.get(), n, hd, W, s);
          launch_cgs_update(W.w.get(), V, ld, hd, j + 1, n, s);
          dots(V, ld, j + 1, W.w.get(), n, hd + (R + 1), W, s);
          launch_cgs_update(W.w.get(), V, ld, hd + (R + 1), j + 1, n, s);
          launch_tree_dots(W.w.get(), 0, 1, W.w.get(), n, hd + 2 * (R + 1), W.dot_work.get(), s);
        }
        AIRG_HIP(hipMemcpyAsync(W.pin + slot * W.pin_slot, hd, nh * sizeof(double),
                                hipMemcpyDeviceToHost, s));
        AIRG_HIP(hipEventRecord(W.evh[slot], s));
      };
      // Look-ahead: step j + 1 (its basis vector divided by the device's own
      // square root of |w|^2, the same value the host would pass) is queued
      // before the host reads step j's coefficients, when the residual
      // estimates predict that step j does not converge: the estimate has
      // fallen by r per step lately, and est_{j-1} r must stay above four
      // times the threshold.  A wrong prediction costs one step's work,
      // never the results, which are the same bits either way.
      const bool look = H.p.lookahead != 0;
      double est_m1 = beta, est_m2 = 0.0;  // the estimates of steps j-1 and j-2
      bool ahead = false;
      int slot = 0;
      for (int j = 0; j < R; ++j) {
        if (!ahead) enqueue_step(j, slot);
        ++its;
        ahead = false;
        if (look && j + 1 < R && its < max_it) {
          const double r = est_m2 > 0.0 ? std::min(1.0, est_m1 / est_m2) : 0.5;
          if (est_m1 * r > 4.0 * thr) {
            launch_divide_norm2(V + (int64_t)(j + 1) * ld, W.w.get(), hd + 2 * (R + 1), n, s,
                                in32);
            enqueue_step(j + 1, slot ^ 1);
            ahead = true;
          }
        }
        AIRG_HIP(hipEventSynchronize(W.evh[slot]));
        std::memcpy(hh.data(), W.pin + slot * W.pin_slot, nh * sizeof(double));
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
        est_rel = est / bnorm;
        if (!std::isfinite(est)) fail(AIRG_ERR_BREAKDOWN, "FGMRES breakdown (non-finite residual)");
        if (est <= thr || its >= max_it) break;
        if (hn == 0.0) break;
        est_m2 = est_m1;
        est_m1 = est;
        if (!ahead) launch_divide(V + (int64_t)(j + 1) * ld, W.w.get(), hn, n, s, in32);
        slot ^= 1;
      }
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= Hm[(size_t)i * R + q] * y[q];
        y[i] = t / Hm[(size_t)i * R + i];
      }
      W.ybuf.from_host(y.data(), k);
      if (Zb32) launch_basis_combine(W.xperm.get(), Zb32, ld, W.ybuf.get(), k, n, s);
      else launch_basis_combine(W.xperm.get(), Zb, ld, W.ybuf.get(), k, n, s);
    }
  }
  launch_gather(x, W.xperm.get(), pos, H.n0, s);
  if (!converged) status = AIRG_NOT_CONVERGED;
  AIRG_HIP(hipEventRecord(W.ev1, s));
  AIRG_HIP(hipEventSynchronize(W.ev1));
  float ms = 0.f;
  AIRG_HIP(hipEventElapsedTime(&ms, W.ev0, W.ev1));
  for (size_t q = 0; q < ng; ++q) {
    out[q].iterations = its;
    out[q].restarts = restarts;
    out[q].stagnated = stagnated;
    out[q].converged = rn[q] <= tol(ref[q]) ? 1 : 0;
    out[q].rel_residual = ref[q] > 0.0 ? rn[q] / ref[q] : 0.0;
    out[q].rel_residual_estimate = est_rel;
    out[q].solve_ms = ms;
  }
  if (info)
    for (size_t q = 0; q < ng; ++q) info[q] = out[q];
  if (coarse_plan_error(W.pc, s) != 0)
    fail(AIRG_ERR_INTERNAL, "the persistent coarse solve's barrier wait gave up");
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
      smooth<X>(lv, ops_of(lv, prec), 1, v.sv, v.e + H.levels[l + 1].off, v.e + lv.off, v.y0,
                v.y1, s, t);
    }
  if (poly || cls == AIRG_K_NEWTON) {
    const Level& lc = H.levels[L];
    if (v.pc) {
      // one launch: the matrix is read once, each step's vector is written
      // and gathered once; x and r once
      coarse_persistent_t<X>(*v.pc, ops_of(lc, prec).a, v.rr + lc.off, v.e + lc.off, s);
      if (t)
        t->add(csr_bytes(lc.n, lc.A.nnz, vb) + xb * lc.n * (2.0 + 2.0 * v.pc->nsteps),
               2.0 * lc.A.nnz * v.pc->nsteps + 6.0 * lc.n * v.pc->nsteps);
    } else {
      newton_apply_t<X>(ops_of(lc, prec).a, lc.tpr_a, 1, lc.roots, v.rr + lc.off, v.e + lc.off,
                        v.cw0, v.cw1, v.ct, s, t);
    }
  }
  if (cls == AIRG_K_RESIDUAL)
    for (int l = 0; l < L; ++l) {
      const Level& lv = H.levels[l];
      const LevelOps o = ops_of(lv, prec);
      spmv_residual_t<X>(o.b, lv.tpr_b, 1, v.e + H.levels[l + 1].off, v.rr + lv.off, v.sv, s);
      if (t)
        t->add(csr_bytes(lv.nF, lv.B.nnz, vb) + xb * (lv.nC + 2 * lv.nF), 2.0 * lv.B.nnz + lv.nF,
               col_saving(o.b));
    }
  if (cls == AIRG_K_RESTRICT)
    for (int l = 0; l < L; ++l) {
      const Level& lv = H.levels[l];
      spmv_restrict_t<X>(ops_of(lv, prec).z, lv.tpr_z, 1, v.rr + lv.off, v.rr + lv.off + lv.nF,
                         v.rr + H.levels[l + 1].off, s);
      if (t)
        t->add(csr_bytes(lv.nC, lv.Z.nnz, vb) + xb * (lv.nF + 2 * lv.nC), 2.0 * lv.Z.nnz + lv.nC,
               col_saving(ops_of(lv, prec).z));
    }
}

}  // namespace

int time_kernels(const Hierarchy& H, Workspace& W, int cls, int reps, airg_kernel_timing* out) {
  hipStream_t s = H.s;
  if (reps < 1) fail(AIRG_ERR_INVALID, "reps must be >= 1");
  if (cls < AIRG_K_POLY || cls > AIRG_K_TOP_SPMV) fail(AIRG_ERR_INVALID, "unknown kernel class");
  if (W.K != 1) fail(AIRG_ERR_INTERNAL, "kernel timing uses the single-column workspace");
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
      if (t)
        t->add(csr_bytes(H.n0, H.Aperm.nnz) + 16.0 * H.n0, 2.0 * H.Aperm.nnz,
               col_saving(opview(H.Aperm)));
      return;
    }
    if (f64) time_pass<double>(H, vecs64(W, in, W.Zb.get()), cls, t);
    else time_pass<float>(H, vecs32(W, W.e32.get()), cls, t);
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
    out->stored_bytes_per_launch = tally.stored / tally.launches;
    out->flops_per_launch = tally.flops / tally.launches;
  }
  return AIRG_OK;
}

}  // namespace airg

namespace airg {

namespace {

template <class X>
double time_product(const OpView& A, int tpr, const X* x, X* y, int reps, Workspace& W,
                    hipStream_t s) {
  spmv_t<X>(A, tpr, 1, x, y, s);  // warm-up
  AIRG_HIP(hipEventRecord(W.ev0, s));
  for (int r = 0; r < reps; ++r) spmv_t<X>(A, tpr, 1, x, y, s);
  AIRG_HIP(hipEventRecord(W.ev1, s));
  AIRG_HIP(hipEventSynchronize(W.ev1));
  float ms = 0.f;
  AIRG_HIP(hipEventElapsedTime(&ms, W.ev0, W.ev1));
  return 1e3 * (double)ms / reps;
}

struct TuneTarget {
  int level, op;
  OpView A;
  int* tpr;
  bool f64;  // product in FP64 vectors
};

}  // namespace

int autotune(Hierarchy& H, Workspace& W, int reps, std::vector<airg_tune_entry>& out) {
  if (reps < 1) fail(AIRG_ERR_INVALID, "reps must be >= 1");
  if (W.K != 1) fail(AIRG_ERR_INTERNAL, "tuning uses the single-column workspace");
  ++H.shape_epoch;
  hipStream_t s = H.s;
  const int prec = H.p.precision;
  const bool low = prec != AIRG_FP64;
  const int L = (int)H.levels.size() - 1;
  std::vector<TuneTarget> t;
  for (int l = 0; l < L; ++l) {
    Level& lv = H.levels[l];
    const LevelOps o = ops_of(lv, prec);
    t.push_back({l, AIRG_OP_FF, o.ff, &lv.tpr_ff, !low});
    t.push_back({l, AIRG_OP_B, o.b, &lv.tpr_b, !low});
    t.push_back({l, AIRG_OP_Z, o.z, &lv.tpr_z, !low});
    if (lv.Ahat.rows > 0) t.push_back({l, AIRG_OP_HAT, o.hat, &lv.tpr_hat, !low});
  }
  Level& lc = H.levels[L];
  t.push_back({L, AIRG_OP_A, ops_of(lc, prec).a, &lc.tpr_a, !low});
  t.push_back({0, AIRG_OP_TOP, opview(H.Aperm), &H.tpr_top, true});
  double* x64 = W.V.get();
  launch_fill(x64, H.n0, 1.0, s);
  float* x32 = low ? W.in32.get() : nullptr;
  if (low) convert_d2f(x32, x64, H.n0, s);
  out.clear();
  for (const TuneTarget& g : t) {
    if (g.A.rows <= 0) continue;
    airg_tune_entry e{};
    e.level = g.level;
    e.op = g.op;
    e.default_lanes = *g.tpr & 0xff;
    e.default_xcd_map = (*g.tpr >> 8) & 1;
    e.default_lds = (*g.tpr & kShapeEntries) ? 2 : (*g.tpr >> 9) & 1;
    e.best_us = 1e300;
    e.default_us = 1e300;
    int best = *g.tpr;
    std::vector<int> shapes;
    for (int tpr = g.A.rblk ? 0 : 1; tpr <= 64; tpr = tpr ? tpr << 1 : 1) {
      if (g.A.rows * (int64_t)tpr > (int64_t)INT32_MAX) break;
      shapes.push_back(tpr);
    }
    if (g.A.col16)  // LDS-staged kernel: 64-row groups, 2..16 lanes per row
      for (int tpr = 2; tpr <= 16; tpr <<= 1) shapes.push_back(tpr | kShapeLds);
    shapes.push_back(1 | kShapeEntries);  // entry-staged kernel, one lane per row
    for (int base : shapes)
      for (int xcd = 0; xcd < 2; ++xcd) {
        const int shape = base | (xcd << 8);
        const double us = g.f64 ? time_product<double>(g.A, shape, x64, W.w.get(), reps, W, s)
                                : time_product<float>(g.A, shape, x32, W.e32.get(), reps, W, s);
        if (shape == *g.tpr) e.default_us = us;
        if (us < e.best_us) {
          e.best_us = us;
          best = shape;
        }
      }
    e.lanes = best & 0xff;
    e.xcd_map = (best >> 8) & 1;
    e.lds = (best & kShapeEntries) ? 2 : (best >> 9) & 1;
    *g.tpr = best;
    out.push_back(e);
  }
  return AIRG_OK;
}

void set_lanes(Hierarchy& H, int level, int op, int lanes, int xcd_map, int lds) {
  if (lanes < 0 || lanes > 64 || (lanes & (lanes - 1)))
    fail(AIRG_ERR_INVALID, "lanes must be 0 or a power of two in 1..64");
  if (xcd_map != 0 && xcd_map != 1) fail(AIRG_ERR_INVALID, "xcd_map must be 0 or 1");
  if (lds < 0 || lds > 2) fail(AIRG_ERR_INVALID, "lds must be 0, 1 or 2");
  if (lds == 1 && (lanes < 2 || lanes > 16))
    fail(AIRG_ERR_INVALID, "the LDS-staged product takes 2, 4, 8 or 16 lanes per row");
  if (lds == 2 && lanes != 1)
    fail(AIRG_ERR_INVALID, "the entry-staged product takes one lane per row");
  ++H.shape_epoch;
  const int L = (int)H.levels.size() - 1;
  const CSR* A = nullptr;
  int* tpr = nullptr;
  if (op == AIRG_OP_TOP) {
    A = &H.Aperm;
    tpr = &H.tpr_top;
  } else if (op == AIRG_OP_A) {
    A = &H.levels[L].A;
    tpr = &H.levels[L].tpr_a;
  } else {
    if (level < 0 || level >= L) fail(AIRG_ERR_INVALID, "level has no such operator");
    Level& lv = H.levels[level];
    switch (op) {
      case AIRG_OP_FF: A = &lv.Aff; tpr = &lv.tpr_ff; break;
      case AIRG_OP_B: A = &lv.B; tpr = &lv.tpr_b; break;
      case AIRG_OP_Z: A = &lv.Z; tpr = &lv.tpr_z; break;
      case AIRG_OP_HAT:
        if (lv.Ahat.rows == 0) fail(AIRG_ERR_INVALID, "no assembled smoother (smoother = poly)");
        A = &lv.Ahat;
        tpr = &lv.tpr_hat;
        break;
      default: fail(AIRG_ERR_INVALID, "unknown operator");
    }
  }
  if (lanes == 0 && !A->rblk.get())
    fail(AIRG_ERR_INVALID, "this operator has no row blocks (rows shorter than 8 on average)");
  if (lds == 1 && !A->col16.get())
    fail(AIRG_ERR_INVALID, "this operator has no compressed columns for the LDS-staged product");
  *tpr = lanes | (xcd_map << 8) | (lds == 1 ? kShapeLds : lds == 2 ? kShapeEntries : 0);
}

}  // namespace airg
