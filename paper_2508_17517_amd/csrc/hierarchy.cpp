// AIRG setup on the device, level by level (paper Sec. 2):
//   truncation test (Sec. 2.4) -> strength, PMISR, DDC (Sec. 2.1) -> A_ff, A_fc,
//   A_cf (Eq. air_two) -> smoother coefficients by Arnoldi (Eq. gmres_poly) ->
//   Ahat^{-1} (Eq. fixed_sparsity) -> Z = -A_cf Ahat^{-1} with relative drop
//   (Eq. z) -> one-point W -> A_{l+1} = R (A P), dropped and lumped.
// Small dense problems (least squares, harmonic Ritz values) run on the host.
#include "hierarchy.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>

#include "kernels.hpp"

namespace airg {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Wall time of a setup component, measured to the end of its device work.
struct Section {
  double& acc;
  hipStream_t s;
  double t0;
  Section(double& a, hipStream_t st) : acc(a), s(st), t0(now_ms()) {}
  ~Section() {
    (void)hipStreamSynchronize(s);
    acc += now_ms() - t0;
  }
};

enum { C_CF = 0, C_PROLONG, C_POLY, C_RSPGEMM, C_ASPGEMM, C_EXTRACT, C_DROP, C_TRUNC };

// Dot products in tree order, any number of vectors (chunks of 64).
void dots_dev(const double* V, int64_t ld, int nv, const double* w, int64_t n, double* out,
              DBuf<double>& work, hipStream_t s) {
  for (int k0 = 0; k0 < nv; k0 += 64) {
    int cnt = std::min(64, nv - k0);
    launch_tree_dots(V + (int64_t)k0 * ld, ld, cnt, w, n, out + k0, work.get(), s);
  }
}

double dot1(const double* x, const double* y, int64_t n, DBuf<double>& work, DBuf<double>& res,
            hipStream_t s) {
  launch_tree_dots(x, 0, 1, y, n, res.get(), work.get(), s);
  return fetch(res.get(), s);
}

struct ArnoldiOut {
  std::vector<double> H;  // (m+1) x m row-major
  int m = 0, steps = 0;
  double beta = 0.0;
};

// m steps of Arnoldi on K(A, b) with classical Gram-Schmidt applied twice, in
// the operation order of a sequential implementation: the Hessenberg matrix
// comes out bit for bit the same as the CPU reference's.
ArnoldiOut arnoldi_dev(const CSR& A, const double* b, int m, hipStream_t s) {
  const int64_t n = A.rows;
  const int64_t ld = (n + 63) / 64 * 64;
  ArnoldiOut R;
  R.m = m;
  R.steps = m;
  R.H.assign((size_t)(m + 1) * m, 0.0);
  DBuf<double> V((size_t)m * ld, s), w(n, s), hd(m + 1, s), res(1, s);
  DBuf<double> work(dot_work_size(n, 64), s);
  R.beta = std::sqrt(dot1(b, b, n, work, res, s));
  launch_divide(V.get(), b, R.beta, n, s);
  std::vector<double> h(m + 1);
  for (int j = 0; j < m; ++j) {
    spmv_seq(A, V.get() + (int64_t)j * ld, w.get(), s);
    const double w0 = std::sqrt(dot1(w.get(), w.get(), n, work, res, s));
    for (int pass = 0; pass < 2; ++pass) {
      dots_dev(V.get(), ld, j + 1, w.get(), n, hd.get(), work, s);
      hd.to_host(h.data(), j + 1);
      AIRG_HIP(hipStreamSynchronize(s));
      launch_cgs_update(w.get(), V.get(), ld, hd.get(), j + 1, n, s);
      for (int k = 0; k <= j; ++k) R.H[(size_t)k * m + j] = R.H[(size_t)k * m + j] + h[k];
    }
    const double hn = std::sqrt(dot1(w.get(), w.get(), n, work, res, s));
    R.H[(size_t)(j + 1) * m + j] = hn;
    if (hn <= 1e-14 * w0) {
      R.steps = j + 1;
      break;
    }
    if (j + 1 < m) launch_divide(V.get() + (int64_t)(j + 1) * ld, w.get(), hn, n, s);
  }
  AIRG_HIP(hipStreamSynchronize(s));
  return R;
}

std::vector<cplx> coarse_roots(const CSR& A, int level, const airg_params& p, hipStream_t s) {
  const int64_t n = A.rows;
  DBuf<double> b(n, s);
  launch_uniform(b.get(), n, p.seed, RNG_COARSE_RHS, level, s);
  int m = (int)std::min<int64_t>((int64_t)p.coarse_poly_order + 1, n);
  ArnoldiOut ar = arnoldi_dev(A, b.get(), m, s);
  return newton_roots(ar.H, ar.m, ar.steps, p.added_roots != 0);
}

double truncation_test(const CSR& A, const std::vector<cplx>& roots, int level,
                       const airg_params& p, hipStream_t s) {
  const int64_t n = A.rows;
  DBuf<double> b(n, s), x(n, s), w0(n, s), w1(n, s), t(n, s), r(n, s), res(1, s);
  DBuf<double> work(dot_work_size(n, 1), s);
  launch_uniform(b.get(), n, p.seed, RNG_TRUNC_RHS, level, s);
  newton_apply_dev(A, pick_tpr(A.rows, A.nnz), roots, b.get(), x.get(), w0.get(), w1.get(),
                   t.get(), s);
  spmv_seq(A, x.get(), r.get(), s);
  launch_sub(r.get(), b.get(), r.get(), n, s);
  double rn = std::sqrt(dot1(r.get(), r.get(), n, work, res, s));
  double bn = std::sqrt(dot1(b.get(), b.get(), n, work, res, s));
  return rn / bn;
}

// Exclusive scan of 0/1 flags: idx[i] = rank of i among the flagged points,
// returns the count.
int64_t flag_scan(const DBuf<int8_t>& state, int64_t n, int which, DBuf<int64_t>& idx,
                  hipStream_t s) {
  idx.alloc(n + 1, s);
  DBuf<int64_t> work(scan_work_size(n), s);
  launch_flag(state.get(), n, which, idx.get(), s);
  launch_scan_i64(idx.get(), idx.get(), n, work.get(), s);
  return fetch(idx.get() + n, s);
}

void extract(const CSR& A, const DBuf<int8_t>& state, int rs, int cs, const DBuf<int64_t>& fidx,
             const DBuf<int64_t>& cidx, int64_t nrows, int64_t ncols, CSR& out, hipStream_t s) {
  DBuf<int64_t> cnt(nrows, s), off(nrows + 1, s), work(scan_work_size(nrows), s);
  launch_extract_count(A, state.get(), rs, cs, cnt.get(), rs == 1 ? fidx.get() : cidx.get(), s);
  launch_scan_i64(cnt.get(), off.get(), nrows, work.get(), s);
  out.rows = nrows;
  out.cols = ncols;
  out.rowptr.alloc(nrows + 1, s);
  DBuf<int32_t> ovf(1, s);
  launch_fill_i32(ovf.get(), 1, 0, s);
  launch_offsets_to_i32(off.get(), out.rowptr.get(), nrows + 1, ovf.get(), s);
  out.nnz = fetch(off.get() + nrows, s);
  out.col.alloc(out.nnz, s);
  out.val.alloc(out.nnz, s);
  launch_extract_fill(A, state.get(), rs, cs, fidx.get(), cidx.get(), out.rowptr.get(),
                      out.col.get(), out.val.get(), s);
}

// CF splitting of one level: strength, PMISR rounds, DDC passes.
void cf_split(const CSR& A, const DBuf<double>& diag, int level, const airg_params& p,
              DBuf<int8_t>& state, int& rounds, hipStream_t s) {
  const int64_t n = A.rows;
  DBuf<int8_t> mask(A.nnz, s);
  launch_strength(A, p.strong_threshold, mask.get(), nullptr, s);
  DBuf<int64_t> colcount(n, s), st_off(n + 1, s), cursor(n, s), work(scan_work_size(n), s);
  colcount.zero();
  launch_pattern_transpose_count(A, mask.get(), colcount.get(), s);
  launch_scan_i64(colcount.get(), st_off.get(), n, work.get(), s);
  int64_t nst = fetch(st_off.get() + n, s);
  DBuf<int32_t> st_col(nst, s);
  cursor.zero();
  launch_pattern_transpose_fill(A, mask.get(), st_off.get(), cursor.get(), st_col.get(), s);

  state.alloc(n, s);
  state.zero();
  DBuf<int32_t> und(1, s);
  rounds = 0;
  for (;;) {
    ++rounds;
    launch_pmisr_select(A, mask.get(), st_off.get(), st_col.get(), state.get(), p.seed, level, s);
    launch_pmisr_neighbours(A, mask.get(), st_off.get(), st_col.get(), state.get(), s);
    launch_fill_i32(und.get(), 1, 0, s);
    launch_pmisr_finalize(state.get(), n, und.get(), s);
    if (fetch(und.get(), s) == 0) break;
    if (rounds > 100000) fail(AIRG_ERR_INTERNAL, "PMISR did not terminate");
  }

  DBuf<double> r(n, s);
  DBuf<unsigned long long> rmax(1, s);
  DBuf<int32_t> nf(1, s), counts(1000, s);
  std::vector<int32_t> hc(1000);
  for (int it = 0; it < p.ddc_its; ++it) {
    rmax.zero();
    launch_fill_i32(nf.get(), 1, 0, s);
    launch_ddc_ratio(A, state.get(), diag.get(), r.get(), rmax.get(), nf.get(), s);
    int32_t nF = fetch(nf.get(), s);
    unsigned long long bits = fetch(rmax.get(), s);
    double rm;
    std::memcpy(&rm, &bits, sizeof(double));
    if (nF == 0 || rm == 0.0) break;
    const int64_t k = (int64_t)std::ceil(p.ddc_fraction * (double)nF);
    counts.zero();
    launch_ddc_hist(r.get(), state.get(), n, rm, counts.get(), s);
    counts.to_host(hc.data(), 1000);
    AIRG_HIP(hipStreamSynchronize(s));
    // the bin boundary whose conversion count is closest to k (a tie converts more)
    int64_t cum = 0;
    int bstar = 0;
    for (int b = 999; b >= 0; --b) {
      cum += hc[b];
      if (cum >= k) {
        bstar = b;
        break;
      }
    }
    int64_t above = cum - hc[bstar];
    int edge = (cum - k) <= (k - above) ? bstar : bstar + 1;
    launch_ddc_convert(r.get(), state.get(), n, rm, edge, s);
  }
}

std::vector<double> smoother_coeffs(const CSR& Aff, int level, const airg_params& p,
                                    hipStream_t s, int purpose = RNG_POLY_RHS) {
  const int64_t nf = Aff.rows;
  DBuf<double> b(nf, s);
  launch_uniform(b.get(), nf, p.seed, purpose, level, s);
  int m = (int)std::min<int64_t>((int64_t)p.poly_order + 1, nf);
  ArnoldiOut ar = arnoldi_dev(Aff, b.get(), m, s);
  return gmres_poly_coeffs(ar.H, ar.m, ar.steps, ar.beta);
}

// Steps 2-8 on level `lvl`; returns false when the level cannot coarsen (no C
// or no F points).  On success L holds the level operators in setup numbering
// and Anext the coarse matrix.
bool coarsen(Hierarchy& H, int lvl, const CSR& A, Level& L, CSR& Anext) {
  hipStream_t s = H.s;
  const airg_params& p = H.p;
  const int64_t n = A.rows;
  DBuf<double> diag(n, s);
  validate_csr(A, diag, s, false);
  {
    Section t(H.comp_ms[C_CF], s);
    cf_split(A, diag, lvl, p, L.state, L.pmisr_rounds, s);
  }
  L.nF = flag_scan(L.state, n, 1, L.fidx, s);
  L.nC = flag_scan(L.state, n, 2, L.cidx, s);
  if (L.nF == 0 || L.nC == 0) return false;
  CSR Acf;
  const bool csmooth = p.smooth_type != AIRG_SMOOTH_TYPE_F;
  {
    Section t(H.comp_ms[C_EXTRACT], s);
    extract(A, L.state, 1, 1, L.fidx, L.cidx, L.nF, L.nF, L.Aff, s);
    extract(A, L.state, 1, 2, L.fidx, L.cidx, L.nF, L.nC, L.Afc_nat, s);
    extract(A, L.state, 2, 1, L.fidx, L.cidx, L.nC, L.nF, Acf, s);
    if (csmooth) extract(A, L.state, 2, 2, L.fidx, L.cidx, L.nC, L.nC, L.Acc_nat, s);
  }
  const bool neumann = p.inverse_type == AIRG_INVERSE_NEUMANN;
  {
    Section t(H.comp_ms[C_POLY], s);
    // nAIR's Neumann polynomial has no fitted coefficients: only its degree
    if (neumann) L.alpha.assign((size_t)p.poly_order + 1, 0.0);
    else L.alpha = smoother_coeffs(L.Aff, lvl, p, s);
    // the C-point smoother: A_cc's GMRES polynomial from its own stream
    if (csmooth) L.alpha_c = smoother_coeffs(L.Acc_nat, lvl, p, s, RNG_CPOLY_RHS);
  }
  {
    Section t(H.comp_ms[C_RSPGEMM], s);
    CSR Ahat, Zfull;
    if (neumann) neumann_fixed_sparsity(L.Aff, (int)L.alpha.size() - 1, Ahat, s);
    else fixed_sparsity_inverse(L.Aff, L.alpha, Ahat, s);
    spgemm(Acf, Ahat, Zfull, s);
    restrictor_drop(Zfull, p.r_drop, true, L.Z_nat, s);
  }
  if (csmooth) L.Acf_nat = std::move(Acf);
  {
    Section t(H.comp_ms[C_PROLONG], s);
    L.cmap_nat.alloc(L.nF, s);
    launch_one_point(A, L.state.get(), L.fidx.get(), L.cidx.get(), L.cmap_nat.get(), s);
  }
  CSR RAP;
  {
    Section t(H.comp_ms[C_ASPGEMM], s);
    DBuf<int64_t> flist(L.nF, s), clist(L.nC, s);
    launch_inverse_map(L.state.get(), n, 1, L.fidx.get(), flist.get(), s);
    launch_inverse_map(L.state.get(), n, 2, L.cidx.get(), clist.get(), s);
    CSR R, P, AP;
    build_r(L.Z_nat, flist.get(), clist.get(), n, R, s);
    build_p(L.state.get(), L.fidx.get(), L.cidx.get(), L.cmap_nat.get(), n, L.nC, P, s);
    spgemm(A, P, AP, s);
    spgemm(R, AP, RAP, s);
  }
  {
    Section t(H.comp_ms[C_DROP], s);
    DBuf<int32_t> bad(1, s);
    launch_fill_i32(bad.get(), 1, 0, s);
    drop_lump(RAP, p.a_drop, p.lump != 0, Anext, bad.get(), s);
    if (fetch(bad.get(), s))
      fail(AIRG_ERR_ZERO_DIAG, "coarse matrix on level " + std::to_string(lvl + 1) +
                                   " has a zero or missing diagonal");
  }
  return true;
}

}  // namespace

void validate_csr(const CSR& A, DBuf<double>& diag, hipStream_t s, bool top) {
  DBuf<int32_t> flags(1, s);
  launch_fill_i32(flags.get(), 1, 0, s);
  launch_validate(A, diag.get(), flags.get(), s);
  int32_t f = fetch(flags.get(), s);
  const char* where = top ? "input matrix" : "level matrix";
  if (f & 1) fail(AIRG_ERR_INVALID, std::string(where) + ": CSR columns must be ascending and in range");
  if (f & 2) fail(AIRG_ERR_NONFINITE, std::string(where) + ": non-finite value");
  if (f & 4) fail(AIRG_ERR_ZERO_DIAG, std::string(where) + ": zero or missing diagonal");
}

OpView op_view(const CSR& A, const DBuf<float>& v32, const DBuf<bf16>& v16, int prec) {
  OpView v = opview(A);
  if (prec == AIRG_FP32) {
    v.val = v32.get();
    v.vt = VT_F32;
  } else if (prec == AIRG_BF16) {
    v.val = v16.get();
    v.vt = VT_BF16;
  }
  return v;
}

template <class X>
void newton_apply_t(const OpView& A, int tpr, int K, const std::vector<cplx>& roots, const X* r,
                    X* x, X* w0, X* w1, X* t, hipStream_t s, LaunchTally* tally) {
  const int64_t n = A.rows * K;  // vector elements; the matrix is read once per launch
  const double xb = (double)sizeof(X);
  const double vb = A.vt == VT_F64 ? 8.0 : A.vt == VT_F32 ? 4.0 : 2.0;
  const double mb = csr_bytes(A.rows, A.nnz, vb), mf = 2.0 * (double)A.nnz * K;
  auto count = [&](double vecs, double vec_flops) {
    if (tally) tally->add(mb + xb * n * vecs, mf + vec_flops, col_saving(A));
  };
  const int m = (int)roots.size();
  if (m == 0) fail(AIRG_ERR_INTERNAL, "no coarse roots");
  const X* w = r;
  X* bufs[2] = {w0, w1};
  int nb = 0;
  bool first = true;
  int i = 0;
  while (i < m) {
    const cplx z = roots[i];
    if (z.imag() == 0.0) {
      const double inv = 1.0 / z.real();
      if (i == m - 1) {  // last root: no product with A
        axpy_first_t<X>(x, w, inv, first, n, s);
        if (tally) tally->add(xb * n * (first ? 2 : 3), 2.0 * n);
        return;
      }
      double inv_last = 0.0;
      int skip = 0;
      if (i + 1 == m - 1 && roots[i + 1].imag() == 0.0) {
        inv_last = 1.0 / roots[i + 1].real();
        skip = 1;
      }
      X* wn = bufs[nb];
      newton_real_t<X>(A, tpr, K, w, wn, x, inv, first, inv_last, s);
      // w gathered, wn written, x written (and read unless first)
      count(first ? 3 : 4, (inv_last != 0.0 ? 6.0 : 4.0) * n);
      first = false;
      w = wn;
      nb ^= 1;
      i += 1 + skip;
    } else {
      const double a = z.real(), b = z.imag();
      const double mod2 = a * a + b * b;
      const double c1 = 2.0 * a / mod2, c2 = 1.0 / mod2;
      newton_pair1_t<X>(A, tpr, K, w, t, x, c1, c2, first, s);
      // w gathered, t written, x written (and read unless first)
      count(first ? 3 : 4, 4.0 * n);
      first = false;
      if (i + 1 == m - 1) return;  // last pair
      double inv_last = 0.0;
      int skip = 0;
      if (i + 2 == m - 1 && roots[i + 2].imag() == 0.0) {
        inv_last = 1.0 / roots[i + 2].real();
        skip = 1;
      }
      X* wn = bufs[nb];
      newton_pair2_t<X>(A, tpr, K, w, t, wn, x, c1, c2, inv_last, s);
      // t gathered, w read, wn written (x read and written when fused)
      count(inv_last != 0.0 ? 5 : 3, (inv_last != 0.0 ? 6.0 : 4.0) * n);
      w = wn;
      nb ^= 1;
      i += 2 + skip;
    }
  }
}
template void newton_apply_t<double>(const OpView&, int, int, const std::vector<cplx>&, const double*,
                                     double*, double*, double*, double*, hipStream_t, LaunchTally*);
template void newton_apply_t<float>(const OpView&, int, int, const std::vector<cplx>&, const float*,
                                    float*, float*, float*, float*, hipStream_t, LaunchTally*);

void build_hierarchy(Hierarchy& H, CSR&& Ain) {
  const double t0 = now_ms();
  hipStream_t s = H.s;
  const airg_params& p = H.p;
  H.A0 = std::move(Ain);
  H.n0 = H.A0.rows;
  H.nnz0 = H.A0.nnz;
  H.levels.clear();
  H.levels.reserve(p.max_levels);
  CSR cur;  // level matrix for lvl >= 1
  for (int lvl = 0; lvl < p.max_levels; ++lvl) {
    const CSR& A = lvl == 0 ? H.A0 : cur;
    const int64_t n = A.rows;
    H.levels.emplace_back();
    Level& L = H.levels.back();
    L.n = n;
    L.nnz_a = A.nnz;
    bool last = n <= p.min_coarse_rows || lvl == p.max_levels - 1;
    std::vector<cplx> roots;
    if (!last && p.trunc_tol > 0 && lvl >= p.trunc_start_level) {
      Section t(H.comp_ms[C_TRUNC], s);
      roots = coarse_roots(A, lvl, p, s);
      L.trunc_rel = truncation_test(A, roots, lvl, p, s);
      last = L.trunc_rel <= p.trunc_tol;
    }
    if (!last) {
      CSR next;
      if (coarsen(H, lvl, A, L, next)) {
        if (p.keep_setup_data && lvl > 0) L.A = std::move(cur);
        cur = std::move(next);
        continue;
      }
      // cannot coarsen: this level becomes the coarsest
      L.state.release();
      L.fidx.release();
      L.cidx.release();
      L.Aff = CSR();
      L.Afc_nat = CSR();
      L.nF = L.nC = 0;
    }
    if (roots.empty()) {
      Section t(H.comp_ms[C_TRUNC], s);
      roots = coarse_roots(A, lvl, p, s);
    }
    L.coarsest = true;
    L.roots = std::move(roots);
    if (lvl == 0) copy_csr(H.A0, L.A, s);
    else L.A = std::move(cur);
    L.tpr_a = pick_tpr(L.A.rows, L.A.nnz);
    break;
  }
  finalize_hierarchy(H);
  AIRG_HIP(hipStreamSynchronize(s));
  H.setup_ms = now_ms() - t0;
}

void finalize_hierarchy(Hierarchy& H) {
  hipStream_t s = H.s;
  const int nl = (int)H.levels.size();
  const bool order = H.p.locality_order != 0;
  // locality keys, top down: the Hilbert index of two breadth-first
  // distances on A_0 + A_0^T, inherited by the coarse points
  std::vector<DBuf<int32_t>> key(nl);
  // a batch orders every level problem-major (key = problem * mult + key), so
  // that each problem's unknowns form ranges of the nested numbering; mult
  // 0 where that would overflow the 31-bit keys (the batch then runs one
  // outer process over all problems)
  const int np = H.seg.empty() ? 0 : (int)H.seg.size() - 1;
  int64_t mult = 0, mult_c = 0;
  H.granges.clear();
  if (order) {
    key[0].alloc(H.n0, s);
    if (np > 1) {
      // every component of every problem at once
      locality_keys_by_component(H.A0, key[0].get(), s, true);
    } else {
      locality_keys(H.A0, key[0].get(), s, true);
    }
    if (np > 1) {
      const int64_t m = (int64_t)max_key(key[0].get(), H.n0, s) + 1;
      if ((int64_t)np * m <= (int64_t)INT32_MAX) {
        problem_major_keys(key[0].get(), H.n0, H.seg, m, s);
        mult = m;
      }
    }
    for (int l = 0; l + 1 < nl; ++l) {
      Level& L = H.levels[l];
      DBuf<int64_t> clist(L.nC, s);
      launch_inverse_map(L.state.get(), L.n, 2, L.cidx.get(), clist.get(), s);
      key[l + 1].alloc(L.nC, s);
      inherit_keys(key[l].get(), clist.get(), L.nC, key[l + 1].get(), s);
    }
  }
  // the coarsest level: ordered by keys of its own graph (its Newton steps
  // are most of the V-cycle's products, and the couplings of a deep coarse
  // matrix reach far beyond what the top grid's distances keep together),
  // its matrix permuted to match
  Level& Lc = H.levels.back();
  Lc.pos.alloc(Lc.n, s);
  if (order) {
    if (nl > 1) {
      DBuf<int32_t> pid;
      if (mult) {
        pid.alloc(Lc.n, s);
        key_problems(key[nl - 1].get(), Lc.n, mult, pid.get(), s);
      }
      if (mult) locality_keys_by_component(Lc.A, key[nl - 1].get(), s, false);
      else locality_keys(Lc.A, key[nl - 1].get(), s, false);
      if (mult) {
        const int64_t m = (int64_t)max_key(key[nl - 1].get(), Lc.n, s) + 1;
        if ((int64_t)np * m <= (int64_t)INT32_MAX) {
          problem_major_keys(key[nl - 1].get(), pid.get(), Lc.n, m, s);
          mult_c = m;
        }
      }
    } else {
      mult_c = mult;
    }
    rank_points(key[nl - 1].get(), Lc.n, Lc.pos.get(), s);
    CSR Ap;
    permute_rows(Lc.A, Lc.pos.get(), Lc.pos.get(), Lc.n, Ap, s);
    sort_rows(Ap, s);
    Lc.A = std::move(Ap);
    Lc.a_permuted = true;
  } else {
    launch_iota(Lc.pos.get(), Lc.n, s);
  }
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = H.levels[l];
    Level& N = H.levels[l + 1];
    L.pos.alloc(L.n, s);
    L.cmap.alloc(L.nF, s);
    const bool asm_smoother = H.p.smoother == AIRG_SMOOTH_ASSEMBLED;
    const bool neumann = H.p.inverse_type == AIRG_INVERSE_NEUMANN;
    CSR Ahat_setup;  // the assembled smoother in setup numbering, from A_ff and alpha
    if (asm_smoother) {
      if (neumann) neumann_fixed_sparsity(L.Aff, (int)L.alpha.size() - 1, Ahat_setup, s);
      else fixed_sparsity_inverse(L.Aff, L.alpha, Ahat_setup, s);
    }
    DBuf<double> dinv_setup;  // D^{-1} of A_ff for the matrix-free Neumann smoother
    if (neumann && !asm_smoother) diag_inverse(L.Aff, dinv_setup, s);
    DBuf<int32_t> frank;
    if (order) {
      frank.alloc(L.nF, s);
      rank_f_points(L.state.get(), L.fidx.get(), key[l].get(), L.n, L.nF, frank.get(), s);
      if (asm_smoother) {
        permute_rows(Ahat_setup, frank.get(), frank.get(), L.nF, L.Ahat, s);
        sort_rows(L.Ahat, s);
      }
      if (dinv_setup.get()) {
        L.dinv.alloc(L.nF, s);
        launch_scatter(L.dinv.get(), dinv_setup.get(), frank.get(), L.nF, s);
      }
      launch_nested_pos_ranked(L.state.get(), L.fidx.get(), L.cidx.get(), frank.get(), L.nF,
                               N.pos.get(), L.n, L.pos.get(), s);
      CSR Aff;
      permute_rows(L.Aff, frank.get(), frank.get(), L.nF, Aff, s);
      if (H.p.keep_setup_data) L.Aff_nat = std::move(L.Aff);
      L.Aff = std::move(Aff);
      permute_rows(L.Afc_nat, frank.get(), N.pos.get(), L.nC, L.Afc, s);
      permute_rows(L.Z_nat, N.pos.get(), frank.get(), L.nF, L.Z, s);
      // ascending columns in the solve numbering: neighbouring lanes gather
      // neighbouring elements
      sort_rows(L.Aff, s);
      sort_rows(L.Z, s);
      launch_remap_ranked(L.cmap_nat.get(), N.pos.get(), frank.get(), L.nF, L.cmap.get(), s);
    } else {
      if (asm_smoother) L.Ahat = std::move(Ahat_setup);
      if (dinv_setup.get()) L.dinv = std::move(dinv_setup);
      launch_nested_pos(L.state.get(), L.fidx.get(), L.cidx.get(), L.nF, N.pos.get(), L.n,
                        L.pos.get(), s);
      permute_rows(L.Afc_nat, nullptr, N.pos.get(), L.nC, L.Afc, s);
      permute_rows(L.Z_nat, N.pos.get(), nullptr, L.nF, L.Z, s);
      launch_remap(L.cmap_nat.get(), N.pos.get(), L.nF, L.cmap.get(), s);
    }
    // the residual operator on e_c; A_fc itself is needed only by the second
    // F smooth of FCF
    merge_fc_ffw(L.Afc, L.Aff, L.cmap.get(), L.B, s);
    L.nnz_fc = L.Afc.nnz;
    if (H.p.smooth_type == AIRG_SMOOTH_TYPE_FCF) {
      L.fc.m = std::move(L.Afc);
      sort_rows(L.fc.m, s);
      L.fc.tpr = pick_tpr(L.fc.m.rows, L.fc.m.nnz);
    }
    L.Afc = CSR();
    // C-point smoothing: A_cf and A_cc in the solve numbering, and A_cc's
    // assembled polynomial
    if (H.p.smooth_type != AIRG_SMOOTH_TYPE_F) {
      if (L.Acf_nat.rows != L.nC || L.Acc_nat.rows != L.nC || L.alpha_c.empty())
        fail(AIRG_ERR_INVALID, "C-point smoothing data missing on level " + std::to_string(l));
      permute_rows(L.Acf_nat, N.pos.get(), order ? frank.get() : nullptr, L.nF, L.cf.m, s);
      permute_rows(L.Acc_nat, N.pos.get(), N.pos.get(), L.nC, L.cc.m, s);
      sort_rows(L.cf.m, s);
      sort_rows(L.cc.m, s);
      L.cf.tpr = pick_tpr(L.cf.m.rows, L.cf.m.nnz);
      L.cc.tpr = pick_tpr(L.cc.m.rows, L.cc.m.nnz);
      if (asm_smoother) {
        CSR hc;
        fixed_sparsity_inverse(L.Acc_nat, L.alpha_c, hc, s);
        permute_rows(hc, N.pos.get(), N.pos.get(), L.nC, L.hat_cc.m, s);
        sort_rows(L.hat_cc.m, s);
        L.hat_cc.tpr = pick_tpr(L.hat_cc.m.rows, L.hat_cc.m.nnz);
      }
    }
    L.tpr_ff = pick_tpr(L.Aff.rows, L.Aff.nnz);
    L.tpr_b = pick_tpr(L.B.rows, L.B.nnz);
    L.tpr_z = pick_tpr(L.Z.rows, L.Z.nnz);
    if (asm_smoother) L.tpr_hat = pick_tpr(L.Ahat.rows, L.Ahat.nnz);
  }
  int64_t off = 0;
  for (Level& L : H.levels) {
    L.off = off;
    off += L.nF;
  }
  // each problem's ranges of the nested numbering: its F points on every
  // level, then its points of the coarsest level
  if (mult && mult_c) {
    for (int l = 0; l < nl; ++l) {
      const Level& L = H.levels[l];
      const std::vector<int32_t> cnt =
          L.coarsest ? count_problems(nullptr, key[l].get(), L.n, mult_c, np, s)
                     : count_problems(L.state.get(), key[l].get(), L.n, mult, np, s);
      int64_t start = L.off;
      for (int p = 0; p < np; ++p) {
        if (cnt[p] > 0) H.granges.push_back({start, (int64_t)cnt[p], (int32_t)p});
        start += cnt[p];
      }
      if (start != L.off + (L.coarsest ? L.n : L.nF))
        fail(AIRG_ERR_INTERNAL, "problem ranges do not cover level " + std::to_string(l));
    }
  }
  // segments of the stacked residual buffer, one per level below the top
  H.stacked_len = 0;
  for (size_t l = 1; l < H.levels.size(); ++l) {
    H.levels[l].in_off = H.stacked_len;
    H.stacked_len += H.levels[l].n;
  }
  permute_rows(H.A0, H.levels[0].pos.get(), H.levels[0].pos.get(), H.n0, H.Aperm, s);
  if (order) sort_rows(H.Aperm, s);
  H.tpr_top = pick_tpr(H.Aperm.rows, H.Aperm.nnz);
  // The rows of the top matrix and of every Z are points of several blocks
  // of the nested numbering (level l's F points, then level l+1's, ...),
  // each block in locality order; taken in that order, the rows of each
  // block sweep the whole domain again and gather the blocks they couple to
  // once per sweep.  Stored in the order of the points' locality keys
  // instead, the rows of all blocks that lie together are taken together,
  // and each gathered element is fetched about once (the epilogues read and
  // write through the row map, which keeps the blocks' own orders).
  if (order) {
    DBuf<int32_t> rkey(H.n0, s);
    launch_scatter_i32(rkey.get(), key[0].get(), H.levels[0].pos.get(), H.n0, s);
    spatial_row_order(H.Aperm, rkey.get(), s);
    for (int l = 0; l + 1 < nl; ++l) {
      Level& L = H.levels[l];
      const Level& N = H.levels[l + 1];
      launch_scatter_i32(rkey.get(), key[l + 1].get(), N.pos.get(), L.nC, s);
      spatial_row_order(L.Z, rkey.get(), s);
    }
  }
  // value copies in the storage precision of the mixed-precision V-cycle
  if (H.p.precision != AIRG_FP64) {
    const bool bf = H.p.precision == AIRG_BF16;
    auto lower = [&](const CSR& A, DBuf<float>& v32, DBuf<bf16>& v16) {
      if (bf) {
        v16.alloc(A.nnz, s);
        convert_d2bf(v16.get(), A.val.get(), A.nnz, s);
      } else {
        v32.alloc(A.nnz, s);
        convert_d2f(v32.get(), A.val.get(), A.nnz, s);
      }
    };
    for (Level& L : H.levels) {
      if (L.coarsest) {
        lower(L.A, L.a32, L.a16);
        continue;
      }
      lower(L.Aff, L.ff32, L.ff16);
      lower(L.B, L.b32, L.b16);
      lower(L.Z, L.z32, L.z16);
      if (L.Ahat.rows > 0) lower(L.Ahat, L.hat32, L.hat16);
      for (SolveOp* o : {&L.cf, &L.cc, &L.hat_cc, &L.fc})
        if (o->m.rows > 0) lower(o->m, o->v32, o->v16);
      if (L.dinv.get()) {
        L.dinv32.alloc(L.nF, s);
        convert_d2f(L.dinv32.get(), L.dinv.get(), L.nF, s);
      }
    }
  }
  // compressed columns for every solve operator whose row blocks allow them,
  // and row blocks for the operators with long rows
  auto prepare = [&](CSR& A) {
    compress_columns(A, s);
    if (A.rows > 0 && A.nnz >= 8 * A.rows) build_row_blocks(A, s);
  };
  prepare(H.Aperm);
  for (Level& L : H.levels) {
    if (L.coarsest) {
      prepare(L.A);
      continue;
    }
    prepare(L.Aff);
    prepare(L.B);
    prepare(L.Z);
    if (L.Ahat.rows > 0) prepare(L.Ahat);
    for (SolveOp* o : {&L.cf, &L.cc, &L.hat_cc, &L.fc})
      if (o->m.rows > 0) prepare(o->m);
  }
  // every solve-phase operator is checked once, so an inconsistent hierarchy
  // (for example a bad import) fails here instead of in a kernel
  {
    DBuf<int32_t> flags(1, s);
    launch_fill_i32(flags.get(), 1, 0, s);
    launch_check_csr(H.Aperm, flags.get(), s);
    for (int l = 0; l < nl; ++l) {
      const Level& L = H.levels[l];
      if (L.coarsest) {
        launch_check_csr(L.A, flags.get(), s);
        continue;
      }
      launch_check_csr(L.Aff, flags.get(), s);
      launch_check_csr(L.B, flags.get(), s);
      launch_check_csr(L.Z, flags.get(), s);
      if (H.p.smoother == AIRG_SMOOTH_ASSEMBLED) {
        if (L.Ahat.rows != L.nF || L.Ahat.cols != L.nF)
          fail(AIRG_ERR_INVALID, "assembled smoother missing on level " + std::to_string(l));
        launch_check_csr(L.Ahat, flags.get(), s);
      }
      const int st = H.p.smooth_type;
      if (st != AIRG_SMOOTH_TYPE_F) {
        const bool asm_c = H.p.smoother == AIRG_SMOOTH_ASSEMBLED;
        if (L.cf.m.rows != L.nC || L.cf.m.cols != L.nF || L.cc.m.rows != L.nC ||
            L.cc.m.cols != L.nC || (asm_c && (L.hat_cc.m.rows != L.nC || L.hat_cc.m.cols != L.nC)) ||
            (st == AIRG_SMOOTH_TYPE_FCF && (L.fc.m.rows != L.nF || L.fc.m.cols != L.nC)))
          fail(AIRG_ERR_INVALID, "C-point smoothing operators missing on level " + std::to_string(l));
        for (const SolveOp* o : {&L.cf, &L.cc, &L.hat_cc, &L.fc})
          if (o->m.rows > 0) launch_check_csr(o->m, flags.get(), s);
      }
      launch_check_map(L.cmap.get(), L.nF, -1, L.nC, flags.get(), s);
      launch_check_map(L.pos.get(), L.n, 0, L.n, flags.get(), s);
      if (L.Aff.rows != L.nF || L.Aff.cols != L.nF || L.B.rows != L.nF || L.B.cols != L.nC ||
          L.Z.rows != L.nC || L.Z.cols != L.nF || H.levels[l + 1].n != L.nC)
        fail(AIRG_ERR_INVALID, "inconsistent operator shapes on level " + std::to_string(l));
    }
    if (H.levels.back().A.rows != H.levels.back().n)
      fail(AIRG_ERR_INVALID, "coarsest matrix does not match its level size");
    if (fetch(flags.get(), s)) fail(AIRG_ERR_INVALID, "hierarchy operators fail the index check");
  }
  // the problems of every 64-row group of the solve operators, for the
  // activity masks of a batch's per-problem processes: rows of A_ff and B
  // are level l's F block at off_l, rows of Z level l + 1's points at
  // off_{l+1}, the coarsest matrix's at its off, the top matrix's all of them
  H.mgroups = 0;
  if (!H.granges.empty()) {
    std::vector<int32_t> pp((size_t)H.n0, -1);
    for (const GroupRange& r : H.granges)
      std::fill(pp.begin() + r.start, pp.begin() + r.start + r.len, r.group);
    for (int32_t v : pp)
      if (v < 0) fail(AIRG_ERR_INTERNAL, "problem ranges do not cover the nested numbering");
    std::vector<int32_t> g0, g1;
    auto add = [&](CSR& A, int64_t first) {
      A.mask_off = -1;
      if (A.rows <= 0) return;
      if (first < 0 || first + A.rows > H.n0) fail(AIRG_ERR_INTERNAL, "operator rows outside the numbering");
      A.mask_off = (int64_t)g0.size();
      // stored row r is the operator's row rm[r]
      std::vector<int32_t> rm;
      if (A.rmap.get()) rm = A.rmap.host(A.rows);
      auto prob = [&](int64_t r) { return pp[first + (rm.empty() ? r : (int64_t)rm[r])]; };
      for (int64_t r0 = 0; r0 < A.rows; r0 += 64) {
        int32_t lo = prob(r0), hi = lo;
        for (int64_t r = r0 + 1; r < std::min(A.rows, r0 + 64); ++r) {
          lo = std::min(lo, prob(r));
          hi = std::max(hi, prob(r));
        }
        g0.push_back(lo);
        g1.push_back(hi);
      }
    };
    for (int l = 0; l < nl; ++l) {
      Level& L = H.levels[l];
      if (L.coarsest) {
        add(L.A, L.off);
      } else {
        add(L.Aff, L.off);
        add(L.B, L.off);
        add(L.Z, L.off + L.nF);
      }
    }
    add(H.Aperm, 0);
    H.mgroups = (int64_t)g0.size();
    H.mgp0.alloc(g0.size(), s);
    H.mgp1.alloc(g1.size(), s);
    H.mgp0.from_host(g0.data(), g0.size());
    H.mgp1.from_host(g1.data(), g1.size());
    AIRG_HIP(hipStreamSynchronize(s));  // g0 and g1 go out of scope
  }
  if (!H.p.keep_setup_data) {
    for (int l = 0; l < nl; ++l) {
      Level& L = H.levels[l];
      if (!L.coarsest) L.A = CSR();
      L.state.release();
      L.fidx.release();
      L.cidx.release();
      L.Afc_nat = CSR();
      L.Z_nat = CSR();
      L.Acf_nat = CSR();
      L.Acc_nat = CSR();
      L.cmap_nat.release();
    }
  }
  AIRG_HIP(hipStreamSynchronize(s));
}

void upload_csr(CSR& out, int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                const int32_t* col, const double* val, hipStream_t s) {
  if (!rowptr || (nnz > 0 && (!col || !val))) fail(AIRG_ERR_INVALID, "missing CSR array");
  out.alloc(rows, cols, nnz, s);
  out.rowptr.from_host(rowptr, rows + 1);
  out.col.from_host(col, nnz);
  out.val.from_host(val, nnz);
  AIRG_HIP(hipStreamSynchronize(s));
}

void import_hierarchy(Hierarchy& H, int nlevels, const airg_level_info* infos,
                      const airg_level_arrays* arr) {
  hipStream_t s = H.s;
  H.levels.clear();
  H.levels.resize(nlevels);
  const airg_level_info& i0 = infos[0];
  upload_csr(H.A0, i0.n, i0.n, i0.nnz_a, arr[0].a_rowptr, arr[0].a_col, arr[0].a_val, s);
  {
    DBuf<double> diag(i0.n, s);
    validate_csr(H.A0, diag, s, true);
  }
  H.n0 = i0.n;
  H.nnz0 = i0.nnz_a;
  for (int l = 0; l < nlevels; ++l) {
    const airg_level_info& in = infos[l];
    const airg_level_arrays& a = arr[l];
    Level& L = H.levels[l];
    L.n = in.n;
    L.nnz_a = in.nnz_a;
    if (l == nlevels - 1) {
      if (!in.is_coarsest || in.n_roots <= 0 || !a.roots_re || !a.roots_im)
        fail(AIRG_ERR_INVALID, "the last level must be the coarsest, with roots");
      L.coarsest = true;
      if (l == 0) copy_csr(H.A0, L.A, s);
      else upload_csr(L.A, in.n, in.n, in.nnz_a, a.a_rowptr, a.a_col, a.a_val, s);
      for (int k = 0; k < in.n_roots; ++k) L.roots.emplace_back(a.roots_re[k], a.roots_im[k]);
      L.tpr_a = pick_tpr(L.A.rows, L.A.nnz);
      continue;
    }
    if (in.is_coarsest || !a.state || !a.cmap || !a.alpha || in.poly_len <= 0)
      fail(AIRG_ERR_INVALID, "level " + std::to_string(l) + " lacks state, cmap or alpha");
    L.state.alloc(in.n, s);
    L.state.from_host(a.state, in.n);
    L.nF = flag_scan(L.state, in.n, 1, L.fidx, s);
    L.nC = flag_scan(L.state, in.n, 2, L.cidx, s);
    if (L.nF != in.n_f || L.nC != in.n_c || L.nF + L.nC != in.n || L.nC != infos[l + 1].n)
      fail(AIRG_ERR_INVALID, "level " + std::to_string(l) + ": inconsistent F/C sizes");
    upload_csr(L.Aff, in.n_f, in.n_f, in.nnz_ff, a.ff_rowptr, a.ff_col, a.ff_val, s);
    upload_csr(L.Afc_nat, in.n_f, in.n_c, in.nnz_fc, a.fc_rowptr, a.fc_col, a.fc_val, s);
    upload_csr(L.Z_nat, in.n_c, in.n_f, in.nnz_z, a.z_rowptr, a.z_col, a.z_val, s);
    L.cmap_nat.alloc(in.n_f, s);
    L.cmap_nat.from_host(a.cmap, in.n_f);
    L.alpha.assign(a.alpha, a.alpha + in.poly_len);
    // imported indices are checked before finalize indexes through them
    DBuf<int32_t> flags(1, s);
    launch_fill_i32(flags.get(), 1, 0, s);
    launch_check_csr(L.Aff, flags.get(), s);
    launch_check_csr(L.Afc_nat, flags.get(), s);
    launch_check_csr(L.Z_nat, flags.get(), s);
    launch_check_map(L.cmap_nat.get(), L.nF, -1, L.nC, flags.get(), s);
    if (fetch(flags.get(), s))
      fail(AIRG_ERR_INVALID, "level " + std::to_string(l) + ": index out of range");
  }
  {
    Level& Lc = H.levels.back();
    DBuf<int32_t> flags(1, s);
    launch_fill_i32(flags.get(), 1, 0, s);
    launch_check_csr(Lc.A, flags.get(), s);
    if (fetch(flags.get(), s) || Lc.A.rows != Lc.n)
      fail(AIRG_ERR_INVALID, "coarsest matrix: index out of range");
  }
  finalize_hierarchy(H);
}

void hierarchy_stats(const Hierarchy& H, airg_stats* st) {
  std::memset(st, 0, sizeof(*st));
  const int nl = (int)H.levels.size();
  st->levels = nl;
  double grid = 0, cyc = 0, sto = 0, bytes = 0;
  const double nnz0 = (double)H.nnz0;
  auto csr_bytes = [](double rows, double nnz) { return 12.0 * nnz + 4.0 * (rows + 1); };
  for (int l = 0; l < nl && l < AIRG_MAX_LEVELS; ++l) {
    const Level& L = H.levels[l];
    st->n[l] = L.n;
    st->nnz[l] = L.nnz_a;
    st->n_f[l] = L.nF;
    st->nnz_ff[l] = L.Aff.nnz;
    st->nnz_fc[l] = L.nnz_fc;
    st->nnz_z[l] = L.Z.nnz;
    st->poly_degree[l] = L.coarsest ? 0 : (int)L.alpha.size() - 1;
    st->pmisr_rounds[l] = L.pmisr_rounds;
    st->trunc_rel[l] = L.trunc_rel;
    grid += (double)L.n;
    if (L.coarsest) {
      const double spmvs = (double)L.roots.size() - 1.0;
      cyc += spmvs * (double)L.A.nnz;
      sto += (double)L.A.nnz;
      // per product: the matrix, w gathered, wn written, x read and written
      bytes += spmvs * (csr_bytes((double)L.n, (double)L.A.nnz) + 8.0 * 4 * L.n);
      st->coarse_roots = (int)L.roots.size();
    } else {
      const int d = (int)L.alpha.size() - 1;
      // complexities in the paper's terms: Z, A_fc and A_ff (d + 1 times), or
      // Z, A_fc, A_ff and Ahat^{-1} once each with the assembled smoother
      const bool asm_smoother = L.Ahat.rows > 0;
      const double smooth = asm_smoother ? (double)L.Aff.nnz + (double)L.Ahat.nnz
                                         : (double)L.Aff.nnz * (1 + d);
      cyc += (double)L.Z.nnz + (double)L.nnz_fc + smooth;
      sto += (double)L.Z.nnz + (double)L.nnz_fc + (double)L.Aff.nnz +
             (asm_smoother ? (double)L.Ahat.nnz : 0.0);
      // restriction: Z, r_f gathered, r_c read, r_c' written
      bytes += csr_bytes((double)L.nC, (double)L.Z.nnz) + 8.0 * (L.nF + 2 * L.nC);
      // residual: B, e_c gathered, r_f read, s written
      bytes += csr_bytes((double)L.nF, (double)L.B.nnz) + 8.0 * (L.nC + 2 * L.nF);
      // d Horner steps (or one product with Ahat^{-1}): the operator, y
      // gathered, s read, out written; the last one also reads cmap and
      // gathers W e_c
      if (asm_smoother)
        bytes += csr_bytes((double)L.nF, (double)L.Ahat.nnz) + 8.0 * 3 * L.nF + 12.0 * L.nF;
      else
        bytes += d * (csr_bytes((double)L.nF, (double)L.Aff.nnz) + 8.0 * 3 * L.nF) + 12.0 * L.nF;
      if (H.p.smooth_type != AIRG_SMOOTH_TYPE_F) {
        // C smooth: the residual r_c - A_cf e_f - A_cc e_c (two products), then
        // d_c Horner steps with A_cc (or one product with its assembly), the
        // last one updating e_c in place; storage gains A_cf and A_cc (and the
        // assembly), as the paper counts for FC smoothing
        const double ncf = (double)L.cf.m.nnz, ncc = (double)L.cc.m.nnz;
        const int dc = (int)L.alpha_c.size() - 1;
        const double nhc = (double)L.hat_cc.m.nnz;
        cyc += ncf + ncc + (asm_smoother ? nhc : dc * ncc);
        sto += ncf + ncc + (asm_smoother ? nhc : 0.0);
        bytes += csr_bytes((double)L.nC, ncf) + 8.0 * (L.nF + 2 * L.nC);
        bytes += csr_bytes((double)L.nC, ncc) + 8.0 * 3 * L.nC;
        if (asm_smoother) bytes += csr_bytes((double)L.nC, nhc) + 8.0 * 3 * L.nC;
        else bytes += dc * (csr_bytes((double)L.nC, ncc) + 8.0 * 3 * L.nC) + (dc > 0 ? 8.0 * L.nC : 0.0);
        if (H.p.smooth_type == AIRG_SMOOTH_TYPE_FCF) {
          // second F smooth: r_f - A_fc e_c - A_ff e_f, then the smoother
          // accumulating into e_f
          cyc += (double)L.nnz_fc + smooth;  // smooth counts A_ff's residual product
          bytes += csr_bytes((double)L.nF, (double)L.nnz_fc) + 8.0 * (L.nC + 2 * L.nF);
          bytes += csr_bytes((double)L.nF, (double)L.Aff.nnz) + 8.0 * 3 * L.nF;
          if (asm_smoother)
            bytes += csr_bytes((double)L.nF, (double)L.Ahat.nnz) + 8.0 * 3 * L.nF;
          else
            bytes += d * (csr_bytes((double)L.nF, (double)L.Aff.nnz) + 8.0 * 3 * L.nF) +
                     (d > 0 ? 8.0 * L.nF : 0.0);
        }
      }
    }
  }
  st->grid_complexity = grid / (double)H.n0;
  st->cycle_complexity = cyc / nnz0;
  st->storage_complexity = sto / nnz0;
  st->vcycle_bytes = bytes;
  st->setup_ms = H.setup_ms;
  for (int i = 0; i < 8; ++i) st->setup_component_ms[i] = H.comp_ms[i];
}

}  // namespace airg
