// C ABI of the AIRG library (declared in include/airg.h).  Every entry point
// catches the library's exceptions and turns them into status codes.
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>

#include "airg.h"
#include "hierarchy.hpp"
#include "kernels.hpp"
#include "solve.hpp"

using namespace airg;

namespace airg {

namespace {
std::atomic<int64_t> g_device_bytes{0};
std::atomic<int64_t> g_device_budget{0};
}  // namespace

void account_device_bytes(int64_t delta) { g_device_bytes += delta; }
void check_device_budget(size_t bytes) {
  const int64_t budget = g_device_budget.load();
  if (budget > 0 && g_device_bytes.load() + (int64_t)bytes > budget)
    fail(AIRG_ERR_NOMEM, "device allocation of " + std::to_string(bytes) +
                             " bytes would pass the allocation budget of " +
                             std::to_string(budget) + " bytes");
}
void set_device_budget(int64_t bytes) { g_device_budget = bytes > 0 ? bytes : 0; }

}  // namespace airg

struct airg_ctx {
  Hierarchy H;
  Workspace W;
  std::map<int, std::unique_ptr<Workspace>> Wk;   // K-column workspaces, made on first use
  std::unique_ptr<Hierarchy> Ht;  // adjoint hierarchy (built on A^T on first use)
  std::unique_ptr<Workspace> Wt;
  std::map<int, std::unique_ptr<Workspace>> Wtk;
};

namespace {

thread_local std::string g_last_error;

template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return AIRG_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return AIRG_ERR_INTERNAL;
  } catch (...) {
    g_last_error = "unknown error";
    return AIRG_ERR_INTERNAL;
  }
}

void check_params(const airg_params& p) {
  auto bad = [](const char* what) { fail(AIRG_ERR_INVALID, std::string("invalid parameter: ") + what); };
  if (!(p.strong_threshold >= 0.0 && p.strong_threshold <= 1.0)) bad("strong_threshold");
  if (!(p.ddc_fraction >= 0.0 && p.ddc_fraction <= 1.0)) bad("ddc_fraction");
  if (p.ddc_its < 0 || p.ddc_its > 1000) bad("ddc_its");
  if (!(p.a_drop >= 0.0 && p.a_drop < 1.0)) bad("a_drop");
  if (!(p.r_drop >= 0.0 && p.r_drop <= 1.0)) bad("r_drop");
  if (p.poly_order < 0 || p.poly_order > 64) bad("poly_order");
  if (p.coarse_poly_order < 0 || p.coarse_poly_order > 4096) bad("coarse_poly_order");
  if (!std::isfinite(p.trunc_tol)) bad("trunc_tol");
  if (p.trunc_start_level < 0) bad("trunc_start_level");
  if (p.max_levels < 1 || p.max_levels > AIRG_MAX_LEVELS) bad("max_levels");
  if (p.min_coarse_rows < 1) bad("min_coarse_rows");
  if (p.precision != AIRG_FP64 && p.precision != AIRG_FP32 && p.precision != AIRG_BF16) bad("precision");
  if (!(p.rtol > 0.0 && p.rtol < 1.0)) bad("rtol");
  if (!(p.atol >= 0.0 && std::isfinite(p.atol))) bad("atol");
  if (p.graph != 0 && p.graph != 1) bad("graph");
  if (p.stagnation_check != 0 && p.stagnation_check != 1) bad("stagnation_check");
  if (p.coarse_persistent != 0 && p.coarse_persistent != 1) bad("coarse_persistent");
  if (p.lookahead != 0 && p.lookahead != 1) bad("lookahead");
  if (p.max_it < 0) bad("max_it");
  if (p.restart < 1 || p.restart > 512) bad("restart");
  if (p.outer != AIRG_OUTER_FGMRES && p.outer != AIRG_OUTER_RICHARDSON) bad("outer");
  if (p.smoother != AIRG_SMOOTH_POLY && p.smoother != AIRG_SMOOTH_ASSEMBLED) bad("smoother");
  if (p.inverse_type != AIRG_INVERSE_ARNOLDI && p.inverse_type != AIRG_INVERSE_NEUMANN)
    bad("inverse_type");
  if (p.smooth_type < AIRG_SMOOTH_TYPE_F || p.smooth_type > AIRG_SMOOTH_TYPE_FCF) bad("smooth_type");
  if (p.smooth_type != AIRG_SMOOTH_TYPE_F && p.inverse_type != AIRG_INVERSE_ARNOLDI)
    bad("smooth_type (C-point smoothing uses the GMRES polynomial)");
}

// Copy the caller's CSR (host or device) into library memory.
void load_csr(CSR& A, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
              const double* val, int on_device, hipStream_t s) {
  if (n <= 0 || nnz < n || nnz > 2147483647ll) fail(AIRG_ERR_INVALID, "bad matrix size");
  if (!rowptr || !col || !val) fail(AIRG_ERR_INVALID, "null matrix pointer");
  A.alloc(n, n, nnz, s);
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  AIRG_HIP(hipMemcpyAsync(A.rowptr.get(), rowptr, (n + 1) * sizeof(int32_t), k, s));
  AIRG_HIP(hipMemcpyAsync(A.col.get(), col, nnz * sizeof(int32_t), k, s));
  AIRG_HIP(hipMemcpyAsync(A.val.get(), val, nnz * sizeof(double), k, s));
  int32_t ends[2];
  AIRG_HIP(hipMemcpyAsync(&ends[0], A.rowptr.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipMemcpyAsync(&ends[1], A.rowptr.get() + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipStreamSynchronize(s));
  if (ends[0] != 0 || ends[1] != nnz) fail(AIRG_ERR_INVALID, "rowptr must start at 0 and end at nnz");
  DBuf<double> diag(n, s);
  validate_csr(A, diag, s, true);
}

// Up to 64 columns are solved together as K interleaved columns, K the next
// power of two (padding columns are zero), fewer when n K would pass 2^31.
int solve_columns(Hierarchy& H, Workspace& W, std::map<int, std::unique_ptr<Workspace>>& Wk,
                  int nrhs, const double* b, int64_t ldb, double* x, int64_t ldx, int guess,
                  airg_solve_info* info) {
  if (nrhs < 0) fail(AIRG_ERR_INVALID, "nrhs must be >= 0");
  if (nrhs > 0 && (!b || !x)) fail(AIRG_ERR_INVALID, "null vector pointer");
  if (nrhs > 1 && (ldb < H.n0 || ldx < H.n0)) fail(AIRG_ERR_INVALID, "leading dimension < n");
  if (!H.seg.empty())
    fail(AIRG_ERR_INVALID, "a batch handle solves through airg_solve_batch (one entry per problem)");
  int status = AIRG_OK;
  for (int k0 = 0; k0 < nrhs;) {
    // K interleaved columns, with n K elements addressable by one launch
    int kmax = 64;
    while (kmax > 1 && H.n0 * (int64_t)kmax > (int64_t)INT32_MAX) kmax >>= 1;
    const int cnt = std::min(kmax, nrhs - k0);
    int K = 1;
    while (K < cnt) K <<= 1;
    Workspace* ws = &W;
    if (K > 1) {
      auto it = Wk.find(K);
      if (it == Wk.end()) {
        std::unique_ptr<Workspace> w(new Workspace());
        workspace_init(H, *w, K);
        it = Wk.emplace(K, std::move(w)).first;
      }
      ws = it->second.get();
    }
    int st;
    try {
      st = fgmres_solve(H, *ws, b + (int64_t)k0 * ldb, ldb, x + (int64_t)k0 * ldx, ldx, cnt,
                        guess != 0, info ? info + k0 : nullptr);
    } catch (const Error&) {
      // a persistent coarse solve whose barrier gave up leaves garbage that
      // can also break the outer loop down: report the cause
      if (coarse_plan_error(ws->pc, H.s) != 0)
        fail(AIRG_ERR_INTERNAL, "the persistent coarse solve's barrier wait gave up");
      throw;
    }
    if (st != AIRG_OK) status = st;
    k0 += cnt;
  }
  return status;
}

airg_ctx* handle_of(airg_handle h) {
  if (!h) fail(AIRG_ERR_INVALID, "null handle");
  return h;
}

const CSR* level_matrix(const airg_ctx* c, int l) {
  const Level& L = c->H.levels[l];
  if (l == 0) return &c->H.A0;
  if (L.A.rows > 0 || L.coarsest) return &L.A;
  return nullptr;
}

template <class T>
void copy_out(T* dst, const DBuf<T>& src, int64_t n, hipStream_t s, const char* what) {
  if (!dst) return;
  if (n > 0 && !src.get()) fail(AIRG_ERR_INVALID, std::string(what) + " was not kept (keep_setup_data = 0)");
  src.to_host(dst, n);
}

void copy_csr_out(int32_t* rp, int32_t* col, double* val, const CSR* A, hipStream_t s,
                  const char* what) {
  if (!rp && !col && !val) return;
  if (!A || !A->rowptr.get()) fail(AIRG_ERR_INVALID, std::string(what) + " was not kept (keep_setup_data = 0)");
  copy_out(rp, A->rowptr, A->rows + 1, s, what);
  copy_out(col, A->col, A->nnz, s, what);
  copy_out(val, A->val, A->nnz, s, what);
}

}  // namespace

extern "C" {

int airg_params_default(airg_params* p) {
  if (!p) return AIRG_ERR_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->strong_threshold = 0.99;
  p->ddc_fraction = 0.01;
  p->a_drop = 1e-6;
  p->r_drop = 0.01;
  p->trunc_tol = 1e-2;
  p->rtol = 1e-10;
  p->seed = 17517;
  p->min_coarse_rows = 64;
  p->ddc_its = 2;
  p->lump = 1;
  p->poly_order = 4;
  p->coarse_poly_order = 20;
  p->trunc_start_level = 1;
  p->max_levels = AIRG_MAX_LEVELS;
  p->added_roots = 1;
  p->precision = AIRG_FP64;
  p->max_it = 500;
  p->restart = 30;
  p->keep_setup_data = 0;
  p->locality_order = 1;
  p->outer = AIRG_OUTER_FGMRES;
  p->smoother = AIRG_SMOOTH_POLY;
  p->inverse_type = AIRG_INVERSE_ARNOLDI;
  p->smooth_type = AIRG_SMOOTH_TYPE_F;
  p->atol = 1e-50;
  p->graph = 0;
  p->stagnation_check = 0;
  p->coarse_persistent = 0;
  p->lookahead = 1;
  return AIRG_OK;
}

int airg_setup(airg_handle* out, int64_t n, int64_t nnz, const int32_t* rowptr,
               const int32_t* colidx, const double* vals, int on_device, const airg_params* p,
               void* hip_stream) {
  return guard([&]() {
    if (!out) fail(AIRG_ERR_INVALID, "null output handle");
    *out = nullptr;
    airg_params prm;
    if (p) prm = *p;
    else airg_params_default(&prm);
    check_params(prm);
    std::unique_ptr<airg_ctx> c(new airg_ctx());
    c->H.p = prm;
    c->H.s = (hipStream_t)hip_stream;
    CSR A;
    load_csr(A, n, nnz, rowptr, colidx, vals, on_device, c->H.s);
    build_hierarchy(c->H, std::move(A));
    workspace_init(c->H, c->W);
    AIRG_HIP(hipStreamSynchronize(c->H.s));
    *out = c.release();
    return (int)AIRG_OK;
  });
}

int airg_solve(airg_handle h, int nrhs, const double* b, int64_t ldb, double* x, int64_t ldx,
               int use_x_as_guess, airg_solve_info* info) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    return solve_columns(c->H, c->W, c->Wk, nrhs, b, ldb, x, ldx, use_x_as_guess, info);
  });
}

int airg_setup_batch(airg_handle* out, int nprob, const int64_t* n, const int64_t* nnz,
                     const int32_t* const* rowptr, const int32_t* const* colidx,
                     const double* const* vals, int on_device, const airg_params* p,
                     void* hip_stream) {
  return guard([&]() {
    if (!out || nprob < 1 || !n || !nnz || !rowptr || !colidx || !vals)
      fail(AIRG_ERR_INVALID, "bad batch arguments");
    *out = nullptr;
    airg_params prm;
    if (p) prm = *p;
    else airg_params_default(&prm);
    check_params(prm);
    std::unique_ptr<airg_ctx> c(new airg_ctx());
    c->H.p = prm;
    hipStream_t s = (hipStream_t)hip_stream;
    c->H.s = s;
    int64_t N = 0, NZ = 0;
    std::vector<int64_t> seg(1, 0);
    for (int q = 0; q < nprob; ++q) {
      if (n[q] <= 0 || nnz[q] < n[q]) fail(AIRG_ERR_INVALID, "bad problem size in the batch");
      N += n[q];
      NZ += nnz[q];
      seg.push_back(N);
    }
    if (NZ > 2147483647ll || N > 2147483647ll) fail(AIRG_ERR_INVALID, "batch too large");
    // block-diagonal concatenation: problem q's rows and columns shift by seg[q]
    CSR A;
    A.alloc(N, N, NZ, s);
    int64_t zoff = 0;
    for (int q = 0; q < nprob; ++q) {
      CSR Aq;
      load_csr(Aq, n[q], nnz[q], rowptr[q], colidx[q], vals[q], on_device, s);
      launch_offset_copy_i32(A.rowptr.get() + seg[q], Aq.rowptr.get(), n[q] + 1, zoff, s);
      launch_offset_copy_i32(A.col.get() + zoff, Aq.col.get(), nnz[q], seg[q], s);
      AIRG_HIP(hipMemcpyAsync(A.val.get() + zoff, Aq.val.get(), nnz[q] * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      zoff += nnz[q];
      AIRG_HIP(hipStreamSynchronize(s));
    }
    DBuf<double> diag(N, s);
    validate_csr(A, diag, s, true);
    c->H.seg = seg;
    build_hierarchy(c->H, std::move(A));
    workspace_init(c->H, c->W);
    AIRG_HIP(hipStreamSynchronize(s));
    *out = c.release();
    return (int)AIRG_OK;
  });
}

int airg_solve_batch(airg_handle h, const double* const* b, double* const* x,
                     int use_x_as_guess, airg_solve_info* info) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    const std::vector<int64_t>& seg = c->H.seg;
    if (seg.empty()) fail(AIRG_ERR_INVALID, "not a batch handle");
    if (!b || !x) fail(AIRG_ERR_INVALID, "null pointer array");
    hipStream_t s = c->H.s;
    const int np = (int)seg.size() - 1;
    DBuf<double> bc(c->H.n0, s), xc(c->H.n0, s);
    for (int q = 0; q < np; ++q) {
      if (!b[q] || !x[q]) fail(AIRG_ERR_INVALID, "null vector pointer");
      const size_t bytes = (seg[q + 1] - seg[q]) * sizeof(double);
      AIRG_HIP(hipMemcpyAsync(bc.get() + seg[q], b[q], bytes, hipMemcpyDeviceToDevice, s));
      if (use_x_as_guess)
        AIRG_HIP(hipMemcpyAsync(xc.get() + seg[q], x[q], bytes, hipMemcpyDeviceToDevice, s));
    }
    int st = fgmres_solve(c->H, c->W, bc.get(), c->H.n0, xc.get(), c->H.n0, 1,
                          use_x_as_guess != 0, info);
    for (int q = 0; q < np; ++q)
      AIRG_HIP(hipMemcpyAsync(x[q], xc.get() + seg[q], (seg[q + 1] - seg[q]) * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    AIRG_HIP(hipStreamSynchronize(s));
    return st;
  });
}

int airg_adjoint_solve(airg_handle h, int nrhs, const double* w, int64_t ldw, double* lam,
                       int64_t ldl, int use_guess, airg_solve_info* info) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    if (!c->H.seg.empty()) fail(AIRG_ERR_INVALID, "adjoint solves take a single-problem handle");
    if (!c->Ht) {
      std::unique_ptr<Hierarchy> Ht(new Hierarchy());
      Ht->p = c->H.p;
      Ht->s = c->H.s;
      CSR At;
      transpose(c->H.A0, At, c->H.s);
      build_hierarchy(*Ht, std::move(At));
      std::unique_ptr<Workspace> Wt(new Workspace());
      workspace_init(*Ht, *Wt);
      c->Ht = std::move(Ht);
      c->Wt = std::move(Wt);
    }
    return solve_columns(*c->Ht, *c->Wt, c->Wtk, nrhs, w, ldw, lam, ldl, use_guess, info);
  });
}

int airg_get_stats(airg_handle h, airg_stats* s) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    if (!s) fail(AIRG_ERR_INVALID, "null stats");
    hierarchy_stats(c->H, s);
    return (int)AIRG_OK;
  });
}

int airg_level_info_get(airg_handle h, int level, airg_level_info* out) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    if (!out || level < 0 || level >= (int)c->H.levels.size()) fail(AIRG_ERR_INVALID, "bad level");
    const Level& L = c->H.levels[level];
    std::memset(out, 0, sizeof(*out));
    out->n = L.n;
    out->n_f = L.nF;
    out->n_c = L.nC;
    out->nnz_a = L.nnz_a;
    out->nnz_ff = L.Aff.nnz;
    out->nnz_fc = L.coarsest ? 0 : L.nnz_fc;
    out->nnz_z = L.coarsest ? 0 : (L.Z_nat.rowptr.get() ? L.Z_nat.nnz : L.Z.nnz);
    out->is_coarsest = L.coarsest ? 1 : 0;
    out->poly_len = (int32_t)L.alpha.size();
    out->n_roots = (int32_t)L.roots.size();
    out->c_poly_len = (int32_t)L.alpha_c.size();
    return (int)AIRG_OK;
  });
}

int airg_export_level(airg_handle h, int level, airg_level_arrays* o) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    if (!o || level < 0 || level >= (int)c->H.levels.size()) fail(AIRG_ERR_INVALID, "bad level");
    const Level& L = c->H.levels[level];
    hipStream_t s = c->H.s;
    copy_out(o->state, L.state, L.coarsest ? 0 : L.n, s, "state");
    if (L.coarsest && level > 0 && L.a_permuted) {
      // the coarsest matrix is kept in its solve order: undo the permutation
      DBuf<int32_t> inv(L.n, s);
      invert_perm(L.pos.get(), L.n, inv.get(), s);
      CSR A;
      permute_rows(L.A, inv.get(), inv.get(), L.n, A, s);
      sort_rows(A, s);
      copy_csr_out(o->a_rowptr, o->a_col, o->a_val, &A, s, "level matrix");
      AIRG_HIP(hipStreamSynchronize(s));
    } else {
      copy_csr_out(o->a_rowptr, o->a_col, o->a_val, level_matrix(c, level), s, "level matrix");
    }
    if (!L.coarsest) {
      // A_ff in setup numbering: the solve copy unless the solve order differs
      const CSR* ff = L.Aff_nat.rowptr.get() ? &L.Aff_nat
                      : (c->H.p.locality_order ? nullptr : &L.Aff);
      copy_csr_out(o->ff_rowptr, o->ff_col, o->ff_val, ff, s, "A_ff");
      copy_csr_out(o->fc_rowptr, o->fc_col, o->fc_val, &L.Afc_nat, s, "A_fc");
      copy_csr_out(o->z_rowptr, o->z_col, o->z_val, &L.Z_nat, s, "Z");
      copy_out(o->cmap, L.cmap_nat, L.nF, s, "cmap");
    }
    AIRG_HIP(hipStreamSynchronize(s));
    if (o->alpha)
      for (size_t k = 0; k < L.alpha.size(); ++k) o->alpha[k] = L.alpha[k];
    if (o->alpha_c)
      for (size_t k = 0; k < L.alpha_c.size(); ++k) o->alpha_c[k] = L.alpha_c[k];
    for (size_t k = 0; k < L.roots.size(); ++k) {
      if (o->roots_re) o->roots_re[k] = L.roots[k].real();
      if (o->roots_im) o->roots_im[k] = L.roots[k].imag();
    }
    return (int)AIRG_OK;
  });
}

int airg_import_hierarchy(airg_handle* out, int nlevels, const airg_level_info* infos,
                          const airg_level_arrays* levels, const airg_params* p, void* hip_stream) {
  return guard([&]() {
    if (!out || !infos || !levels || nlevels < 1 || nlevels > AIRG_MAX_LEVELS)
      fail(AIRG_ERR_INVALID, "bad import arguments");
    *out = nullptr;
    airg_params prm;
    if (p) prm = *p;
    else airg_params_default(&prm);
    check_params(prm);
    if (prm.smooth_type != AIRG_SMOOTH_TYPE_F)
      fail(AIRG_ERR_INVALID, "C-point smoothing needs a hierarchy built by airg_setup");
    std::unique_ptr<airg_ctx> c(new airg_ctx());
    c->H.p = prm;
    c->H.s = (hipStream_t)hip_stream;
    import_hierarchy(c->H, nlevels, infos, levels);
    workspace_init(c->H, c->W);
    AIRG_HIP(hipStreamSynchronize(c->H.s));
    *out = c.release();
    return (int)AIRG_OK;
  });
}

int airg_time_kernels(airg_handle h, int cls, int reps, airg_kernel_timing* out) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    if (!out) fail(AIRG_ERR_INVALID, "null output");
    return time_kernels(c->H, c->W, cls, reps, out);
  });
}

int airg_trim(airg_handle h) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    AIRG_HIP(hipStreamSynchronize(c->H.s));
    c->Wk.clear();
    c->Wtk.clear();
    return (int)AIRG_OK;
  });
}

int airg_autotune(airg_handle h, int reps, airg_tune_entry* out, int max_out, int* n_out) {
  return guard([&]() {
    airg_ctx* c = handle_of(h);
    std::vector<airg_tune_entry> e;
    autotune(c->H, c->W, reps, e);
    if (out)
      for (int i = 0; i < (int)e.size() && i < max_out; ++i) out[i] = e[i];
    if (n_out) *n_out = (int)e.size();
    return (int)AIRG_OK;
  });
}

int airg_set_lanes(airg_handle h, int level, int op, int lanes, int xcd_map, int lds) {
  return guard([&]() {
    set_lanes(handle_of(h)->H, level, op, lanes, xcd_map, lds);
    return (int)AIRG_OK;
  });
}

int airg_fv_nnz(int64_t nx, int64_t ny, double theta, int64_t* nnz) {
  return guard([&]() {
    if (nx < 1 || ny < 1 || !nnz || !(theta >= 0.0 && theta <= 1.5707963267948966))
      fail(AIRG_ERR_INVALID, "bad grid or angle");
    *nnz = fv_nnz(nx, ny, theta);
    return (int)AIRG_OK;
  });
}

int airg_fv_assemble(int64_t nx, int64_t ny, double theta, const double* g_west,
                     const double* g_south, int32_t* rowptr, int32_t* col, double* val, double* b,
                     double* dval_dtheta, double* db_dtheta, void* hip_stream) {
  return guard([&]() {
    if (nx < 1 || ny < 1 || !(theta >= 0.0 && theta <= 1.5707963267948966))
      fail(AIRG_ERR_INVALID, "bad grid or angle");
    if (!g_west || !g_south || !rowptr || !col || !val || !b) fail(AIRG_ERR_INVALID, "null pointer");
    if (fv_nnz(nx, ny, theta) > 2147483647ll) fail(AIRG_ERR_INVALID, "grid too large");
    hipStream_t s = (hipStream_t)hip_stream;
    fv_assemble(nx, ny, theta, g_west, g_south, rowptr, col, val, b, dval_dtheta, db_dtheta, s);
    AIRG_HIP(hipStreamSynchronize(s));
    return (int)AIRG_OK;
  });
}

int airg_fv_gradients(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                      const int32_t* col, const double* dval_dtheta, const double* db_dtheta,
                      const double* u, const double* lam, double* dg_west, double* dg_south,
                      double* dtheta, void* hip_stream) {
  return guard([&]() {
    if (nx < 1 || ny < 1) fail(AIRG_ERR_INVALID, "bad grid");
    if (!rowptr || !col || !dval_dtheta || !db_dtheta || !u || !lam || !dg_west || !dg_south ||
        !dtheta)
      fail(AIRG_ERR_INVALID, "null pointer");
    fv_gradients(nx, ny, theta, rowptr, col, dval_dtheta, db_dtheta, u, lam, dg_west, dg_south,
                 dtheta, (hipStream_t)hip_stream);
    return (int)AIRG_OK;
  });
}

int airg_stream_probe(int kind, const void* src, void* dst, int64_t bytes, int reps, int blocks,
                      double* avg_ms, void* hip_stream) {
  return guard([&]() {
    if (kind != 0 && kind != 1) fail(AIRG_ERR_INVALID, "kind must be 0 (read) or 1 (copy)");
    if (!src || !dst || !avg_ms) fail(AIRG_ERR_INVALID, "null pointer");
    if (bytes < 16 || bytes % 16 != 0) fail(AIRG_ERR_INVALID, "bytes must be a positive multiple of 16");
    if (reps < 1 || blocks < 1 || blocks > (1 << 20)) fail(AIRG_ERR_INVALID, "bad reps or blocks");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
      fail(AIRG_ERR_INVALID, "buffers must be 16-byte aligned");
    *avg_ms = stream_probe(kind, src, dst, bytes, reps, blocks, (hipStream_t)hip_stream);
    return (int)AIRG_OK;
  });
}

int airg_fv_gradients_noalloc(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                              const int32_t* col, const double* dval_dtheta,
                              const double* db_dtheta, const double* u, const double* lam,
                              double* dg_west, double* dg_south, double* dtheta,
                              void* hip_stream) {
  return guard([&]() {
    if (nx < 1 || ny < 1) fail(AIRG_ERR_INVALID, "bad grid");
    if (!rowptr || !col || !dval_dtheta || !db_dtheta || !u || !lam || !dg_west || !dg_south ||
        !dtheta)
      fail(AIRG_ERR_INVALID, "null pointer");
    fv_gradients_noalloc(nx, ny, theta, rowptr, col, dval_dtheta, db_dtheta, u, lam, dg_west,
                         dg_south, dtheta, (hipStream_t)hip_stream);
    return (int)AIRG_OK;
  });
}

int airg_set_alloc_budget(int64_t bytes, int64_t* in_use) {
  return guard([&]() {
    set_device_budget(bytes);
    if (in_use) *in_use = g_device_bytes.load();
    return (int)AIRG_OK;
  });
}

int airg_set_spin_limit(int64_t polls) {
  return guard([&]() {
    set_grid_spin_limit(polls);
    return (int)AIRG_OK;
  });
}

void airg_destroy(airg_handle h) {
  if (!h) return;
  hipStream_t s = h->H.s;
  (void)hipStreamSynchronize(s);
  delete h;
  (void)hipStreamSynchronize(s);
}

const char* airg_status_string(int code) {
  switch (code) {
    case AIRG_OK: return "ok";
    case AIRG_NOT_CONVERGED: return "not converged";
    case AIRG_ERR_INVALID: return "invalid argument";
    case AIRG_ERR_ZERO_DIAG: return "zero or missing diagonal";
    case AIRG_ERR_NONFINITE: return "non-finite value";
    case AIRG_ERR_HIP: return "HIP runtime error";
    case AIRG_ERR_NOMEM: return "out of device memory";
    case AIRG_ERR_BREAKDOWN: return "Krylov breakdown";
    case AIRG_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* airg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
