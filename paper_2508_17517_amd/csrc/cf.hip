// CF splitting and sub-block extraction kernels (paper Sec. 2.1 and Eq. air_two).
// Every decision is taken in FP64 on the same bits a sequential implementation
// would see: row sums run left to right, maxima are exact, and the Luby
// weights are counter-based draws recomputed wherever they are compared.
#include <cmath>

#include "kernels.hpp"

namespace airg {

constexpr int8_t kU = 0, kF = 1, kC = 2, kFNew = 3;
constexpr double kOnePointTie = 1.0 - 1e-12;

__device__ __forceinline__ uint64_t mix64d(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double pmisr_weight(uint64_t seed, uint64_t base, int64_t i) {
  uint64_t c = base + (uint64_t)i;
  uint64_t z = mix64d(seed + (c + 1ull) * 0x9E3779B97F4A7C15ull);
  return (double)(z >> 11) * 0x1.0p-53;
}

// ------------------------------------------------------------------ validation
__global__ void validate_kernel(CSRView A, int64_t ncols, double* diag, int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int s = A.rowptr[i], e = A.rowptr[i + 1];
  if (e < s) {
    atomicOr(flags, 1);
    diag[i] = 0.0;
    return;
  }
  double d = 0.0;
  bool found = false;
  int prev = -1;
  for (int p = s; p < e; ++p) {
    int j = A.col[p];
    double v = A.val[p];
    if (j <= prev || j < 0 || j >= ncols) atomicOr(flags, 1);
    prev = j;
    if (!isfinite(v)) atomicOr(flags, 2);
    if (j == i) {
      d = v;
      found = true;
    }
  }
  if (!found || d == 0.0) atomicOr(flags, 4);
  diag[i] = d;
}

void launch_validate(const CSR& A, double* diag, int32_t* flags, hipStream_t s) {
  if (A.rows <= 0) return;
  validate_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), A.cols, diag, flags);
  AIRG_CHECK_LAUNCH();
}

// Structural check of a constructed matrix: monotone row pointers inside
// [0, nnz] and every column inside [0, ncols).
__global__ void check_csr_kernel(CSRView A, int64_t nnz, int64_t ncols, int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int s = A.rowptr[i], e = A.rowptr[i + 1];
  if (s < 0 || e < s || (int64_t)e > nnz) {
    atomicOr(flags, 1);
    return;
  }
  for (int p = s; p < e; ++p) {
    int j = A.col[p];
    if (j < 0 || (int64_t)j >= ncols) atomicOr(flags, 1);
  }
}
__global__ void check_map_kernel(const int32_t* m, int64_t n, int64_t lo, int64_t hi,
                                 int32_t* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (m[i] < lo || m[i] >= hi)) atomicOr(flags, 2);
}
void launch_check_csr(const CSR& A, int32_t* flags, hipStream_t s) {
  if (A.rows <= 0) return;
  check_csr_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), A.nnz, A.cols, flags);
  AIRG_CHECK_LAUNCH();
}
void launch_check_map(const int32_t* m, int64_t n, int64_t lo, int64_t hi, int32_t* flags,
                      hipStream_t s) {
  if (n <= 0) return;
  check_map_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(m, n, lo, hi, flags);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ strength
// S_ij = 1 iff j != i, a_ij != 0 and |a_ij| >= theta * max_{k != i} |a_ik|
__global__ void strength_kernel(CSRView A, double theta, int8_t* mask, int64_t* row_count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int s = A.rowptr[i], e = A.rowptr[i + 1];
  double m = 0.0;
  for (int p = s; p < e; ++p)
    if (A.col[p] != i) m = fmax(m, fabs(A.val[p]));
  double thr = theta * m;
  int64_t cnt = 0;
  for (int p = s; p < e; ++p) {
    double v = A.val[p];
    int8_t st = (A.col[p] != i && v != 0.0 && fabs(v) >= thr) ? 1 : 0;
    mask[p] = st;
    cnt += st;
  }
  if (row_count) row_count[i] = cnt;
}

void launch_strength(const CSR& A, double theta, int8_t* mask, int64_t* row_count, hipStream_t s) {
  if (A.rows <= 0) return;
  strength_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), theta, mask, row_count);
  AIRG_CHECK_LAUNCH();
}

__global__ void pt_count_kernel(CSRView A, const int8_t* mask, unsigned long long* colcount) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    if (mask[p]) atomicAdd(&colcount[A.col[p]], 1ull);
}
__global__ void pt_fill_kernel(CSRView A, const int8_t* mask, const int64_t* off,
                               unsigned long long* cursor, int32_t* st_col) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    if (mask[p]) {
      int j = A.col[p];
      unsigned long long k = atomicAdd(&cursor[j], 1ull);
      st_col[off[j] + (int64_t)k] = (int32_t)i;
    }
}
void launch_pattern_transpose_count(const CSR& A, const int8_t* mask, int64_t* colcount,
                                    hipStream_t s) {
  if (A.rows <= 0) return;
  pt_count_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), mask,
                                                               (unsigned long long*)colcount);
  AIRG_CHECK_LAUNCH();
}
void launch_pattern_transpose_fill(const CSR& A, const int8_t* mask, const int64_t* off,
                                   int64_t* cursor, int32_t* st_col, hipStream_t s) {
  if (A.rows <= 0) return;
  pt_fill_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), mask, off,
                                                              (unsigned long long*)cursor, st_col);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ PMISR
// Round, part 1: an undecided point whose (weight, index) beats every
// undecided G-neighbour becomes a new F point.  A neighbour turning new-F in
// this same pass is still counted as undecided, so the outcome does not depend
// on the order threads run in.
__global__ void pmisr_select_kernel(CSRView A, const int8_t* mask, const int64_t* st_off,
                                    const int32_t* st_col, int8_t* state, uint64_t seed,
                                    uint64_t base) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  if (state[i] != kU) return;
  const double wi = pmisr_weight(seed, base, i);
  bool lose = false;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1] && !lose; ++p) {
    if (!mask[p]) continue;
    int j = A.col[p];
    int8_t sj = state[j];
    if (sj == kU || sj == kFNew) {
      double wj = pmisr_weight(seed, base, j);
      if (wj > wi || (wj == wi && j > i)) lose = true;
    }
  }
  for (int64_t q = st_off[i]; q < st_off[i + 1] && !lose; ++q) {
    int j = st_col[q];
    int8_t sj = state[j];
    if (sj == kU || sj == kFNew) {
      double wj = pmisr_weight(seed, base, j);
      if (wj > wi || (wj == wi && j > i)) lose = true;
    }
  }
  if (!lose) state[i] = kFNew;
}

// Round, part 2: an undecided point with a new-F G-neighbour becomes C.
__global__ void pmisr_neighbours_kernel(CSRView A, const int8_t* mask, const int64_t* st_off,
                                        const int32_t* st_col, int8_t* state) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  if (state[i] != kU) return;
  bool hit = false;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1] && !hit; ++p)
    if (mask[p] && state[A.col[p]] == kFNew) hit = true;
  for (int64_t q = st_off[i]; q < st_off[i + 1] && !hit; ++q)
    if (state[st_col[q]] == kFNew) hit = true;
  if (hit) state[i] = kC;
}

__global__ void pmisr_finalize_kernel(int8_t* state, int64_t n, int32_t* undecided) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int8_t s = state[i];
  if (s == kFNew) state[i] = kF;
  else if (s == kU) atomicAdd(undecided, 1);
}

void launch_pmisr_select(const CSR& A, const int8_t* mask, const int64_t* st_off,
                         const int32_t* st_col, int8_t* state, uint64_t seed, int level,
                         hipStream_t s) {
  if (A.rows <= 0) return;
  uint64_t base = ((uint64_t)RNG_PMISR << 56) | ((uint64_t)level << 40);
  pmisr_select_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), mask, st_off, st_col,
                                                                   state, seed, base);
  AIRG_CHECK_LAUNCH();
}
void launch_pmisr_neighbours(const CSR& A, const int8_t* mask, const int64_t* st_off,
                             const int32_t* st_col, int8_t* state, hipStream_t s) {
  if (A.rows <= 0) return;
  pmisr_neighbours_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), mask, st_off,
                                                                       st_col, state);
  AIRG_CHECK_LAUNCH();
}
void launch_pmisr_finalize(int8_t* state, int64_t n, int32_t* undecided, hipStream_t s) {
  if (n <= 0) return;
  pmisr_finalize_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, n, undecided);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ DDC
// r_i = sum_{j in F, j != i} |a_ij| / |a_ii| (left to right) for F rows.
__global__ void ddc_ratio_kernel(CSRView A, const int8_t* state, const double* diag, double* r,
                                 unsigned long long* rmax_bits, int32_t* nf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  if (state[i] != kF) {
    r[i] = 0.0;
    return;
  }
  double sum = 0.0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
    int j = A.col[p];
    if (j != i && state[j] == kF) sum = sum + fabs(A.val[p]);
  }
  double ri = sum / fabs(diag[i]);
  r[i] = ri;
  // non-negative doubles order like their bit patterns
  atomicMax(rmax_bits, (unsigned long long)__double_as_longlong(ri));
  atomicAdd(nf, 1);
}

__device__ __forceinline__ int ddc_bin(double r, double rmax) {
  double q = floor((r / rmax) * 1000.0);
  return q >= 999.0 ? 999 : (int)q;
}

__global__ void ddc_hist_kernel(const double* r, const int8_t* state, int64_t n, double rmax,
                                int32_t* counts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != kF) return;
  double ri = r[i];
  if (ri > 0.0) atomicAdd(&counts[ddc_bin(ri, rmax)], 1);
}

__global__ void ddc_convert_kernel(const double* r, int8_t* state, int64_t n, double rmax,
                                   int edge) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != kF) return;
  double ri = r[i];
  if (ri > 0.0 && ddc_bin(ri, rmax) >= edge) state[i] = kC;
}

void launch_ddc_ratio(const CSR& A, const int8_t* state, const double* diag, double* r,
                      unsigned long long* rmax_bits, int32_t* nf, hipStream_t s) {
  if (A.rows <= 0) return;
  ddc_ratio_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), state, diag, r,
                                                                rmax_bits, nf);
  AIRG_CHECK_LAUNCH();
}
void launch_ddc_hist(const double* r, const int8_t* state, int64_t n, double rmax, int32_t* counts,
                     hipStream_t s) {
  if (n <= 0) return;
  ddc_hist_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(r, state, n, rmax, counts);
  AIRG_CHECK_LAUNCH();
}
void launch_ddc_convert(const double* r, int8_t* state, int64_t n, double rmax, int edge,
                        hipStream_t s) {
  if (n <= 0) return;
  ddc_convert_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(r, state, n, rmax, edge);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ extraction
__global__ void flag_kernel(const int8_t* state, int64_t n, int which, int64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = state[i] == which ? 1 : 0;
}
void launch_flag(const int8_t* state, int64_t n, int which, int64_t* out, hipStream_t s) {
  if (n <= 0) return;
  flag_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, n, which, out);
  AIRG_CHECK_LAUNCH();
}

__global__ void extract_count_kernel(CSRView A, const int8_t* state, int rs, int cs, int64_t* count,
                                     const int64_t* rowidx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows || state[i] != rs) return;
  int64_t c = 0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) c += (state[A.col[p]] == cs);
  count[rowidx[i]] = c;
}
__global__ void extract_fill_kernel(CSRView A, const int8_t* state, int rs, int cs,
                                    const int64_t* rowidx, const int64_t* colidx,
                                    const int32_t* rowptr_out, int32_t* col_out, double* val_out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows || state[i] != rs) return;
  int64_t q = rowptr_out[rowidx[i]];
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
    int j = A.col[p];
    if (state[j] == cs) {
      col_out[q] = (int32_t)colidx[j];
      val_out[q] = A.val[p];
      ++q;
    }
  }
}
void launch_extract_count(const CSR& A, const int8_t* state, int rs, int cs, int64_t* count,
                          const int64_t* rowidx, hipStream_t s) {
  if (A.rows <= 0) return;
  extract_count_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), state, rs, cs, count,
                                                                    rowidx);
  AIRG_CHECK_LAUNCH();
}
void launch_extract_fill(const CSR& A, const int8_t* state, int rs, int cs, const int64_t* fidx,
                         const int64_t* cidx, const int32_t* rowptr_out, int32_t* col_out,
                         double* val_out, hipStream_t s) {
  if (A.rows <= 0) return;
  const int64_t* rowidx = rs == kF ? fidx : cidx;
  const int64_t* colidx = cs == kF ? fidx : cidx;
  extract_fill_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(
      view(A), state, rs, cs, rowidx, colidx, rowptr_out, col_out, val_out);
  AIRG_CHECK_LAUNCH();
}

__global__ void inverse_map_kernel(const int8_t* state, int64_t n, int which, const int64_t* idx,
                                   int64_t* list) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && state[i] == which) list[idx[i]] = i;
}
void launch_inverse_map(const int8_t* state, int64_t n, int which, const int64_t* idx,
                        int64_t* list, hipStream_t s) {
  if (n <= 0) return;
  inverse_map_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, n, which, idx, list);
  AIRG_CHECK_LAUNCH();
}

__global__ void nested_pos_kernel(const int8_t* state, const int64_t* fidx, const int64_t* cidx,
                                  int64_t nF, const int32_t* pos_next, int64_t n, int32_t* pos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pos[i] = state[i] == kF ? (int32_t)fidx[i] : (int32_t)(nF + pos_next[cidx[i]]);
}
void launch_nested_pos(const int8_t* state, const int64_t* fidx, const int64_t* cidx, int64_t nF,
                       const int32_t* pos_next, int64_t n, int32_t* pos, hipStream_t s) {
  if (n <= 0) return;
  nested_pos_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, fidx, cidx, nF, pos_next, n,
                                                            pos);
  AIRG_CHECK_LAUNCH();
}

__global__ void remap_kernel(const int32_t* cmap, const int32_t* pos_next, int64_t nf,
                             int32_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  int32_t c = cmap[i];
  out[i] = c >= 0 ? pos_next[c] : -1;
}
void launch_remap(const int32_t* cmap, const int32_t* pos_next, int64_t nf, int32_t* out,
                  hipStream_t s) {
  if (nf <= 0) return;
  remap_kernel<<<blocks_for(nf, kBlock), kBlock, 0, s>>>(cmap, pos_next, nf, out);
  AIRG_CHECK_LAUNCH();
}

__global__ void iota_kernel(int32_t* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (int32_t)i;
}
void launch_iota(int32_t* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  iota_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, n);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ one-point prolongation
// The F point takes the C point with the largest |a_ij| in its row; magnitudes
// within a relative 1e-12 of the largest tie and the lowest column wins.
__global__ void one_point_kernel(CSRView A, const int8_t* state, const int64_t* fidx,
                                 const int64_t* cidx, int32_t* cmap) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows || state[i] != kF) return;
  const int s = A.rowptr[i], e = A.rowptr[i + 1];
  double m = 0.0;
  bool any = false;
  for (int p = s; p < e; ++p)
    if (state[A.col[p]] == kC) {
      m = fmax(m, fabs(A.val[p]));
      any = true;
    }
  int32_t out = -1;
  if (any) {
    const double thr = m * kOnePointTie;
    for (int p = s; p < e; ++p) {
      int j = A.col[p];
      if (state[j] == kC && fabs(A.val[p]) >= thr) {
        out = (int32_t)cidx[j];
        break;
      }
    }
  }
  cmap[fidx[i]] = out;
}
void launch_one_point(const CSR& A, const int8_t* state, const int64_t* fidx, const int64_t* cidx,
                      int32_t* cmap, hipStream_t s) {
  if (A.rows <= 0) return;
  one_point_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), state, fidx, cidx, cmap);
  AIRG_CHECK_LAUNCH();
}

}  // namespace airg
