// Sparse products and structural kernels of the setup (paper Eqs. z,
// fixed_sparsity, prolong and the coarse product R A P).
//
// C = A B is formed row by row with a k-way merge of the sorted rows of B
// selected by row i of A (one thread per row for short rows of A, one
// wavefront per row for longer ones), so every c_ij is accumulated over A's
// entries in stored (ascending k) order starting from 0.0 and the result does
// not depend on scheduling.  Exact zeros are dropped afterwards.
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace airg {

static void scan_counts(const DBuf<int64_t>& cnt, int64_t n, DBuf<int64_t>& off, hipStream_t s) {
  off.alloc(n + 1, s);
  DBuf<int64_t> work(scan_work_size(n), s);
  launch_scan_i64(cnt.get(), off.get(), n, work.get(), s);
}

// int32 rowptr from int64 offsets, failing on overflow.
static int64_t offsets_to_rowptr(const DBuf<int64_t>& off, int64_t n, DBuf<int32_t>& rowptr,
                                 hipStream_t s) {
  rowptr.alloc(n + 1, s);
  DBuf<int32_t> ovf(1, s);
  launch_fill_i32(ovf.get(), 1, 0, s);
  launch_offsets_to_i32(off.get(), rowptr.get(), n + 1, ovf.get(), s);
  int64_t total = fetch(off.get() + n, s);
  if (fetch(ovf.get(), s) || total > 2147483647ll)
    fail(AIRG_ERR_NOMEM, "sparse matrix exceeds 2^31 nonzeros");
  return total;
}

// ------------------------------------------------------------------ k-way merge product
__global__ void merge_init_kernel(CSRView A, CSRView B, int32_t* cur) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) cur[p] = B.rowptr[A.col[p]];
}

__global__ void merge_count_kernel(CSRView A, CSRView B, int32_t* cur, int64_t* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  const int s = A.rowptr[i], e = A.rowptr[i + 1];
  int64_t c = 0;
  for (;;) {
    int mn = 0x7fffffff;
    for (int p = s; p < e; ++p) {
      int q = cur[p];
      if (q < B.rowptr[A.col[p] + 1]) mn = min(mn, B.col[q]);
    }
    if (mn == 0x7fffffff) break;
    ++c;
    for (int p = s; p < e; ++p) {
      int q = cur[p];
      if (q < B.rowptr[A.col[p] + 1] && B.col[q] == mn) cur[p] = q + 1;
    }
  }
  count[i] = c;
}

__global__ void merge_numeric_kernel(CSRView A, CSRView B, int32_t* cur, const int32_t* rowptr,
                                     int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  const int s = A.rowptr[i], e = A.rowptr[i + 1];
  int64_t o = rowptr[i];
  for (;;) {
    int mn = 0x7fffffff;
    for (int p = s; p < e; ++p) {
      int q = cur[p];
      if (q < B.rowptr[A.col[p] + 1]) mn = min(mn, B.col[q]);
    }
    if (mn == 0x7fffffff) break;
    double acc = 0.0;
    for (int p = s; p < e; ++p) {  // ascending k
      int q = cur[p];
      if (q < B.rowptr[A.col[p] + 1] && B.col[q] == mn) {
        acc = acc + A.val[p] * B.val[q];
        cur[p] = q + 1;
      }
    }
    col[o] = mn;
    val[o] = acc;
    ++o;
  }
}

__global__ void nonzero_count_kernel(CSRView A, int64_t* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int64_t c = 0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) c += (A.val[p] != 0.0);
  count[i] = c;
}
__global__ void nonzero_fill_kernel(CSRView A, const int32_t* rowptr, int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int64_t o = rowptr[i];
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    if (A.val[p] != 0.0) {
      col[o] = A.col[p];
      val[o] = A.val[p];
      ++o;
    }
}

// Drop the explicit zeros of `in` into `out`.
static void drop_zeros(const CSR& in, CSR& out, hipStream_t s) {
  const int64_t n = in.rows;
  DBuf<int64_t> cnt(n, s), off;
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    nonzero_count_kernel<<<nb, kBlock, 0, s>>>(view(in), cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, n, off, s);
  out.rows = n;
  out.cols = in.cols;
  out.nnz = offsets_to_rowptr(off, n, out.rowptr, s);
  out.col.alloc(out.nnz, s);
  out.val.alloc(out.nnz, s);
  if (n > 0) {
    nonzero_fill_kernel<<<nb, kBlock, 0, s>>>(view(in), out.rowptr.get(), out.col.get(),
                                              out.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

// The same merge with one wavefront per row of A: lane l holds the cursors of
// A's entries s + l + 64 t (t < T), the smallest pending column is found with
// a wave-wide min, and the products of the entries that hit it are added in
// ascending entry order (t, then lane) -- the order of the one-thread merge,
// so the results agree bit for bit.  Rows are visited in a wave-stride loop.
__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

template <int T, bool NUMERIC>
__global__ __launch_bounds__(256) void wave_merge_kernel(CSRView A, CSRView B,
                                                         const int32_t* rowptrC, int32_t* colC,
                                                         double* valC, int64_t* count,
                                                         int64_t nwaves) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w0 >= nwaves) return;  // the grid's last block may hold spare waves
  for (int64_t i = w0; i < A.rows; i += nwaves) {
    const int s = A.rowptr[i], e = A.rowptr[i + 1];
    int q[T], qe[T], head[T];
    double a[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int p = s + lane + 64 * t;
      q[t] = qe[t] = 0;
      a[t] = 0.0;
      head[t] = 0x7fffffff;
      if (p < e) {
        const int k = A.col[p];
        q[t] = B.rowptr[k];
        qe[t] = B.rowptr[k + 1];
        a[t] = A.val[p];
        if (q[t] < qe[t]) head[t] = B.col[q[t]];
      }
    }
    int64_t o = NUMERIC ? (int64_t)rowptrC[i] : 0;
    int64_t c = 0;
    for (;;) {
      int m = 0x7fffffff;
#pragma unroll
      for (int t = 0; t < T; ++t) m = min(m, head[t]);
      m = wave_min_i32(m);
      if (m == 0x7fffffff) break;
      if constexpr (NUMERIC) {
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const bool hit = head[t] == m;
          double prod = 0.0;
          if (hit) prod = a[t] * B.val[q[t]];
          unsigned long long mask = __ballot(hit);
          while (mask) {
            const int l = __ffsll(mask) - 1;
            mask &= mask - 1;
            acc = acc + __shfl(prod, l, 64);
          }
        }
        if (lane == 0) {
          colC[o] = m;
          valC[o] = acc;
        }
        ++o;
      } else {
        ++c;
      }
#pragma unroll
      for (int t = 0; t < T; ++t)
        if (head[t] == m) {
          ++q[t];
          head[t] = q[t] < qe[t] ? B.col[q[t]] : 0x7fffffff;
        }
    }
    if (!NUMERIC && lane == 0) count[i] = c;
  }
}

__global__ void max_row_len_kernel(CSRView A, unsigned long long* mx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.rows) atomicMax(mx, (unsigned long long)(A.rowptr[i + 1] - A.rowptr[i]));
}

template <bool NUMERIC>
static void launch_wave_merge(int T, const CSR& A, const CSR& B, const int32_t* rowptrC,
                              int32_t* colC, double* valC, int64_t* count, hipStream_t s) {
  const int64_t nwaves = std::min<int64_t>(A.rows, (int64_t)1 << 22);
  const unsigned nb = blocks_for(nwaves * 64, 256);
  switch (T) {
    case 1: wave_merge_kernel<1, NUMERIC><<<nb, 256, 0, s>>>(view(A), view(B), rowptrC, colC, valC, count, nwaves); break;
    case 2: wave_merge_kernel<2, NUMERIC><<<nb, 256, 0, s>>>(view(A), view(B), rowptrC, colC, valC, count, nwaves); break;
    case 4: wave_merge_kernel<4, NUMERIC><<<nb, 256, 0, s>>>(view(A), view(B), rowptrC, colC, valC, count, nwaves); break;
    case 8: wave_merge_kernel<8, NUMERIC><<<nb, 256, 0, s>>>(view(A), view(B), rowptrC, colC, valC, count, nwaves); break;
    default: fail(AIRG_ERR_INTERNAL, "bad cursor count");
  }
  AIRG_CHECK_LAUNCH();
}

void spgemm(const CSR& A, const CSR& B, CSR& C, hipStream_t s) {
  if (A.cols != B.rows) fail(AIRG_ERR_INTERNAL, "spgemm shape mismatch");
  const int64_t n = A.rows;
  unsigned nb = blocks_for(n, kBlock);
  // rows of A with more than 8 entries: one wavefront per row; else one thread
  int T = 0;
  if (n > 0) {
    DBuf<unsigned long long> mx(1, s);
    launch_zero_bytes(mx.get(), sizeof(unsigned long long), s);
    max_row_len_kernel<<<nb, kBlock, 0, s>>>(view(A), mx.get());
    AIRG_CHECK_LAUNCH();
    const unsigned long long la = fetch(mx.get(), s);
    if (la > 8 && la <= 512) {
      T = 1;
      while (64 * (unsigned long long)T < la) T <<= 1;
    }
  }
  DBuf<int32_t> cur;
  if (T == 0) cur.alloc(A.nnz, s);
  DBuf<int64_t> cnt(n, s), off;
  if (n > 0) {
    if (T) {
      launch_wave_merge<false>(T, A, B, nullptr, nullptr, nullptr, cnt.get(), s);
    } else {
      merge_init_kernel<<<nb, kBlock, 0, s>>>(view(A), view(B), cur.get());
      AIRG_CHECK_LAUNCH();
      merge_count_kernel<<<nb, kBlock, 0, s>>>(view(A), view(B), cur.get(), cnt.get());
      AIRG_CHECK_LAUNCH();
    }
  }
  scan_counts(cnt, n, off, s);
  CSR full;
  full.rows = n;
  full.cols = B.cols;
  full.nnz = offsets_to_rowptr(off, n, full.rowptr, s);
  full.col.alloc(full.nnz, s);
  full.val.alloc(full.nnz, s);
  if (n > 0) {
    if (T) {
      launch_wave_merge<true>(T, A, B, full.rowptr.get(), full.col.get(), full.val.get(), nullptr,
                              s);
    } else {
      merge_init_kernel<<<nb, kBlock, 0, s>>>(view(A), view(B), cur.get());
      AIRG_CHECK_LAUNCH();
      merge_numeric_kernel<<<nb, kBlock, 0, s>>>(view(A), view(B), cur.get(), full.rowptr.get(),
                                                 full.col.get(), full.val.get());
      AIRG_CHECK_LAUNCH();
    }
  }
  drop_zeros(full, C, s);
}

// ------------------------------------------------------------------ fixed sparsity
// T_out[p] = sum over q in row i (ascending) of T_in[q] * Aff[col(q), col(p)],
// i.e. (T_in Aff) restricted to the pattern of Aff.
__device__ __forceinline__ int find_col(const int32_t* col, int lo, int hi, int j) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int c = col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// One thread per output entry p (its row i from the entry's row index): the
// entry sums over the row's entries q in ascending order.
__global__ void masked_power_entry_kernel(CSRView Aff, const int32_t* __restrict__ row_of,
                                          int64_t nnz, const double* tin, double* tout) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int i = row_of[p];
  const int s = Aff.rowptr[i], e = Aff.rowptr[i + 1];
  const int j = Aff.col[p];
  double acc = 0.0;
  for (int q = s; q < e; ++q) {
    const int k = Aff.col[q];
    int r = find_col(Aff.col, Aff.rowptr[k], Aff.rowptr[k + 1], j);
    if (r >= 0) acc = acc + tin[q] * Aff.val[r];
  }
  tout[p] = acc;
}
__global__ void row_of_entry_kernel(CSRView A, int32_t* row_of) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) row_of[p] = (int32_t)i;
}

// v = alpha_0 [i == j]; v = v + alpha_k T_k  (k = 1..d, left to right)
__global__ void poly_init_kernel(CSRView Aff, double a0, double a1, int has_a1, double* v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Aff.rows) return;
  for (int p = Aff.rowptr[i]; p < Aff.rowptr[i + 1]; ++p) {
    double x = (Aff.col[p] == i) ? a0 : 0.0;
    if (has_a1) x = x + a1 * Aff.val[p];
    v[p] = x;
  }
}
__global__ void poly_add_kernel(int64_t nnz, double a, const double* t, double* v) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) v[p] = v[p] + a * t[p];
}

void fixed_sparsity_inverse(const CSR& Aff, const std::vector<double>& alpha, CSR& out,
                            hipStream_t s) {
  const int64_t n = Aff.rows;
  if (alpha.empty()) fail(AIRG_ERR_INTERNAL, "empty polynomial");
  CSR full;
  full.rows = n;
  full.cols = Aff.cols;
  full.nnz = Aff.nnz;
  full.rowptr.alloc(n + 1, s);
  full.col.alloc(Aff.nnz, s);
  full.val.alloc(Aff.nnz, s);
  AIRG_HIP(hipMemcpyAsync(full.rowptr.get(), Aff.rowptr.get(), (n + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
  AIRG_HIP(hipMemcpyAsync(full.col.get(), Aff.col.get(), Aff.nnz * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    poly_init_kernel<<<nb, kBlock, 0, s>>>(view(Aff), alpha[0], alpha.size() > 1 ? alpha[1] : 0.0,
                                           alpha.size() > 1 ? 1 : 0, full.val.get());
    AIRG_CHECK_LAUNCH();
  }
  if (alpha.size() > 2) {
    DBuf<double> ta(Aff.nnz, s), tb(Aff.nnz, s);
    DBuf<int32_t> row_of(Aff.nnz, s);
    row_of_entry_kernel<<<nb, kBlock, 0, s>>>(view(Aff), row_of.get());
    AIRG_CHECK_LAUNCH();
    AIRG_HIP(hipMemcpyAsync(ta.get(), Aff.val.get(), Aff.nnz * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
    for (size_t k = 2; k < alpha.size(); ++k) {
      masked_power_entry_kernel<<<blocks_for(Aff.nnz, kBlock), kBlock, 0, s>>>(
          view(Aff), row_of.get(), Aff.nnz, ta.get(), tb.get());
      AIRG_CHECK_LAUNCH();
      poly_add_kernel<<<blocks_for(Aff.nnz, kBlock), kBlock, 0, s>>>(Aff.nnz, alpha[k], tb.get(),
                                                                     full.val.get());
      AIRG_CHECK_LAUNCH();
      std::swap(ta, tb);
    }
  }
  drop_zeros(full, out, s);
}

// ------------------------------------------------------------------ Neumann (nAIR)
__global__ void row_diag_kernel(CSRView A, double* d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  double v = 0.0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    if (A.col[p] == i) v = A.val[p];
  d[i] = v;
}
// N = I - D^{-1} A on A's pattern: -a_ij / a_ii off the diagonal, 0 on it
__global__ void jacobi_iteration_matrix_kernel(CSRView A, const double* d, double* nval) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    nval[p] = A.col[p] == i ? 0.0 : -A.val[p] / d[i];
}
__global__ void col_scale_kernel(int64_t nnz, const int32_t* col, const double* dinv, double* val) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) val[p] = val[p] * dinv[col[p]];
}
__global__ void reciprocal_kernel(int64_t n, const double* d, double* r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = 1.0 / d[i];
}

void diag_inverse(const CSR& A, DBuf<double>& dinv, hipStream_t s) {
  const int64_t n = A.rows;
  DBuf<double> d(n, s);
  dinv.alloc(n, s);
  if (n <= 0) return;
  row_diag_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(view(A), d.get());
  AIRG_CHECK_LAUNCH();
  reciprocal_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(n, d.get(), dinv.get());
  AIRG_CHECK_LAUNCH();
}

void neumann_fixed_sparsity(const CSR& Aff, int degree, CSR& out, hipStream_t s) {
  const int64_t n = Aff.rows;
  DBuf<double> d(n, s), dinv;
  CSR N;
  copy_csr(Aff, N, s);
  if (n > 0) {
    row_diag_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(view(Aff), d.get());
    AIRG_CHECK_LAUNCH();
    jacobi_iteration_matrix_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(view(Aff), d.get(),
                                                                           N.val.get());
    AIRG_CHECK_LAUNCH();
  }
  // I + N + N~^2 + ... + N~^d through the fixed-sparsity sum with unit coefficients
  std::vector<double> ones((size_t)std::max(degree, 0) + 1, 1.0);
  CSR S;
  fixed_sparsity_inverse(N, ones, S, s);
  diag_inverse(Aff, dinv, s);
  if (S.nnz > 0) {
    col_scale_kernel<<<blocks_for(S.nnz, kBlock), kBlock, 0, s>>>(S.nnz, S.col.get(), dinv.get(),
                                                                 S.val.get());
    AIRG_CHECK_LAUNCH();
  }
  drop_zeros(S, out, s);
}



// ------------------------------------------------------------------ drops
__global__ void rdrop_count_kernel(CSRView Z, double tol, int64_t* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Z.rows) return;
  double m = 0.0;
  for (int p = Z.rowptr[i]; p < Z.rowptr[i + 1]; ++p) m = fmax(m, fabs(Z.val[p]));
  const double thr = tol * m;
  int64_t c = 0;
  for (int p = Z.rowptr[i]; p < Z.rowptr[i + 1]; ++p) c += (fabs(Z.val[p]) >= thr);
  count[i] = c;
}
__global__ void rdrop_fill_kernel(CSRView Z, double tol, double sign, const int32_t* rowptr,
                                  int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Z.rows) return;
  double m = 0.0;
  for (int p = Z.rowptr[i]; p < Z.rowptr[i + 1]; ++p) m = fmax(m, fabs(Z.val[p]));
  const double thr = tol * m;
  int64_t o = rowptr[i];
  for (int p = Z.rowptr[i]; p < Z.rowptr[i + 1]; ++p)
    if (fabs(Z.val[p]) >= thr) {
      col[o] = Z.col[p];
      val[o] = sign * Z.val[p];
      ++o;
    }
}

void restrictor_drop(const CSR& Zin, double tol, bool negate, CSR& Z, hipStream_t s) {
  const int64_t n = Zin.rows;
  DBuf<int64_t> cnt(n, s), off;
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    rdrop_count_kernel<<<nb, kBlock, 0, s>>>(view(Zin), tol, cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, n, off, s);
  Z.rows = n;
  Z.cols = Zin.cols;
  Z.nnz = offsets_to_rowptr(off, n, Z.rowptr, s);
  Z.col.alloc(Z.nnz, s);
  Z.val.alloc(Z.nnz, s);
  if (n > 0) {
    rdrop_fill_kernel<<<nb, kBlock, 0, s>>>(view(Zin), tol, negate ? -1.0 : 1.0, Z.rowptr.get(),
                                            Z.col.get(), Z.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

// Off-diagonal relative drop; dropped values lumped to the diagonal as
// d + l_1 + l_2 + ... in ascending column order.
__global__ void adrop_count_kernel(CSRView A, double tol, int lump, int64_t* count, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  double m = 0.0;
  bool has_diag = false;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
    if (A.col[p] != i) m = fmax(m, fabs(A.val[p]));
    else has_diag = true;
  }
  const double thr = tol * m;
  int64_t c = 0;
  bool dropped = false;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
    bool drop = A.col[p] != i && fabs(A.val[p]) < thr;
    c += !drop;
    dropped |= drop;
  }
  if (!has_diag || (lump && dropped && !has_diag)) atomicOr(bad, 1);
  count[i] = c;
}
__global__ void adrop_fill_kernel(CSRView A, double tol, int lump, const int32_t* rowptr,
                                  int32_t* col, double* val, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  const int s = A.rowptr[i], e = A.rowptr[i + 1];
  double m = 0.0;
  double d = 0.0;
  for (int p = s; p < e; ++p) {
    if (A.col[p] != i) m = fmax(m, fabs(A.val[p]));
    else d = A.val[p];
  }
  const double thr = tol * m;
  if (lump)
    for (int p = s; p < e; ++p)
      if (A.col[p] != i && fabs(A.val[p]) < thr) d = d + A.val[p];
  int64_t o = rowptr[i];
  for (int p = s; p < e; ++p) {
    const int j = A.col[p];
    if (j != i && fabs(A.val[p]) < thr) continue;
    col[o] = j;
    val[o] = (j == i) ? d : A.val[p];
    ++o;
  }
  if (d == 0.0 || !isfinite(d)) atomicOr(bad, 1);
}

void drop_lump(const CSR& Ain, double tol, bool lump, CSR& Aout, int32_t* bad_diag,
               hipStream_t s) {
  const int64_t n = Ain.rows;
  DBuf<int64_t> cnt(n, s), off;
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    adrop_count_kernel<<<nb, kBlock, 0, s>>>(view(Ain), tol, lump ? 1 : 0, cnt.get(), bad_diag);
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, n, off, s);
  Aout.rows = n;
  Aout.cols = Ain.cols;
  Aout.nnz = offsets_to_rowptr(off, n, Aout.rowptr, s);
  Aout.col.alloc(Aout.nnz, s);
  Aout.val.alloc(Aout.nnz, s);
  if (n > 0) {
    adrop_fill_kernel<<<nb, kBlock, 0, s>>>(view(Ain), tol, lump ? 1 : 0, Aout.rowptr.get(),
                                            Aout.col.get(), Aout.val.get(), bad_diag);
    AIRG_CHECK_LAUNCH();
  }
}

// ------------------------------------------------------------------ R and P
// R row c: Z row c with F columns mapped to level indices (fpos, ascending),
// plus 1.0 at level index cpos[c], merged in column order.
__global__ void build_r_kernel(CSRView Z, const int64_t* fpos, const int64_t* cpos,
                               const int32_t* rowptr, int32_t* col, double* val) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Z.rows) return;
  const int32_t me = (int32_t)cpos[c];
  int64_t o = rowptr[c];
  bool placed = false;
  for (int p = Z.rowptr[c]; p < Z.rowptr[c + 1]; ++p) {
    int32_t j = (int32_t)fpos[Z.col[p]];
    if (!placed && me < j) {
      col[o] = me;
      val[o] = 1.0;
      ++o;
      placed = true;
    }
    col[o] = j;
    val[o] = Z.val[p];
    ++o;
  }
  if (!placed) {
    col[o] = me;
    val[o] = 1.0;
  }
}
__global__ void rowlen_plus_one_kernel(CSRView Z, int64_t* cnt) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < Z.rows) cnt[c] = (int64_t)(Z.rowptr[c + 1] - Z.rowptr[c]) + 1;
}

void build_r(const CSR& Z, const int64_t* fpos, const int64_t* cpos, int64_t n, CSR& R,
             hipStream_t s) {
  const int64_t nc = Z.rows;
  DBuf<int64_t> cnt(nc, s), off;
  unsigned nb = blocks_for(nc, kBlock);
  if (nc > 0) {
    rowlen_plus_one_kernel<<<nb, kBlock, 0, s>>>(view(Z), cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, nc, off, s);
  R.rows = nc;
  R.cols = n;
  R.nnz = offsets_to_rowptr(off, nc, R.rowptr, s);
  R.col.alloc(R.nnz, s);
  R.val.alloc(R.nnz, s);
  if (nc > 0) {
    build_r_kernel<<<nb, kBlock, 0, s>>>(view(Z), fpos, cpos, R.rowptr.get(), R.col.get(),
                                         R.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

__global__ void p_count_kernel(const int8_t* state, const int64_t* fidx, const int32_t* cmap,
                               int64_t n, int64_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cnt[i] = (state[i] == 2) ? 1 : (cmap[fidx[i]] >= 0 ? 1 : 0);
}
__global__ void p_fill_kernel(const int8_t* state, const int64_t* fidx, const int64_t* cidx,
                              const int32_t* cmap, int64_t n, const int32_t* rowptr, int32_t* col,
                              double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = rowptr[i];
  if (state[i] == 2) {
    col[o] = (int32_t)cidx[i];
    val[o] = 1.0;
  } else {
    int32_t c = cmap[fidx[i]];
    if (c >= 0) {
      col[o] = c;
      val[o] = 1.0;
    }
  }
}

void build_p(const int8_t* state, const int64_t* fidx, const int64_t* cidx, const int32_t* cmap,
             int64_t n, int64_t nc, CSR& P, hipStream_t s) {
  DBuf<int64_t> cnt(n, s), off;
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    p_count_kernel<<<nb, kBlock, 0, s>>>(state, fidx, cmap, n, cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, n, off, s);
  P.rows = n;
  P.cols = nc;
  P.nnz = offsets_to_rowptr(off, n, P.rowptr, s);
  P.col.alloc(P.nnz, s);
  P.val.alloc(P.nnz, s);
  if (n > 0) {
    p_fill_kernel<<<nb, kBlock, 0, s>>>(state, fidx, cidx, cmap, n, P.rowptr.get(), P.col.get(),
                                        P.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

// ------------------------------------------------------------------ permutation / transpose
__global__ void perm_count_kernel(CSRView A, const int32_t* newrow, int64_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.rows) cnt[newrow ? newrow[i] : i] = A.rowptr[i + 1] - A.rowptr[i];
}
__global__ void perm_fill_kernel(CSRView A, const int32_t* newrow, const int32_t* colmap,
                                 const int32_t* rowptr, int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  int64_t o = rowptr[newrow ? newrow[i] : i];
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p, ++o) {
    int j = A.col[p];
    col[o] = colmap ? colmap[j] : j;
    val[o] = A.val[p];
  }
}

void permute_rows(const CSR& A, const int32_t* newrow, const int32_t* colmap, int64_t out_cols,
                  CSR& out, hipStream_t s) {
  const int64_t n = A.rows;
  DBuf<int64_t> cnt(n, s), off;
  unsigned nb = blocks_for(n, kBlock);
  if (n > 0) {
    perm_count_kernel<<<nb, kBlock, 0, s>>>(view(A), newrow, cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, n, off, s);
  out.rows = n;
  out.cols = out_cols;
  out.nnz = offsets_to_rowptr(off, n, out.rowptr, s);
  out.col.alloc(out.nnz, s);
  out.val.alloc(out.nnz, s);
  if (n > 0) {
    perm_fill_kernel<<<nb, kBlock, 0, s>>>(view(A), newrow, colmap, out.rowptr.get(),
                                           out.col.get(), out.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

__global__ void tcount_kernel(CSRView A, unsigned long long* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) atomicAdd(&cnt[A.col[p]], 1ull);
}
__global__ void tfill_kernel(CSRView A, const int32_t* rowptr, unsigned long long* cursor,
                             int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
    int j = A.col[p];
    unsigned long long k = atomicAdd(&cursor[j], 1ull);
    col[rowptr[j] + (int64_t)k] = (int32_t)i;
    val[rowptr[j] + (int64_t)k] = A.val[p];
  }
}
__global__ void row_sort_kernel(int64_t rows, const int32_t* rowptr, int32_t* col, double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int s = rowptr[i], e = rowptr[i + 1];
  for (int p = s + 1; p < e; ++p) {
    int c = col[p];
    double v = val[p];
    int q = p - 1;
    while (q >= s && col[q] > c) {
      col[q + 1] = col[q];
      val[q + 1] = val[q];
      --q;
    }
    col[q + 1] = c;
    val[q + 1] = v;
  }
}

__global__ void inverse_perm_kernel(const int32_t* perm, int64_t n, int32_t* inv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[perm[i]] = (int32_t)i;
}

void spatial_row_order(CSR& A, const int32_t* rkey, hipStream_t s) {
  if (A.rows <= 0) return;
  if (A.rmap.get()) fail(AIRG_ERR_INTERNAL, "operator rows are already reordered");
  DBuf<int32_t> rank(A.rows, s);
  rank_points(rkey, A.rows, rank.get(), s);
  CSR P;
  permute_rows(A, rank.get(), nullptr, A.cols, P, s);
  P.rmap.alloc(A.rows, s);
  inverse_perm_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(rank.get(), A.rows, P.rmap.get());
  AIRG_CHECK_LAUNCH();
  A = std::move(P);
}

void sort_rows(CSR& A, hipStream_t s) {
  if (A.rows <= 0 || A.nnz <= 0) return;
  row_sort_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(A.rows, A.rowptr.get(), A.col.get(),
                                                                A.val.get());
  AIRG_CHECK_LAUNCH();
}

void transpose(const CSR& A, CSR& At, hipStream_t s) {
  const int64_t m = A.cols;
  DBuf<int64_t> cnt(m, s), off;
  launch_zero_bytes(cnt.get(), m * sizeof(int64_t), s);
  unsigned nb = blocks_for(A.rows, kBlock);
  if (A.rows > 0) {
    tcount_kernel<<<nb, kBlock, 0, s>>>(view(A), (unsigned long long*)cnt.get());
    AIRG_CHECK_LAUNCH();
  }
  scan_counts(cnt, m, off, s);
  At.rows = m;
  At.cols = A.rows;
  At.nnz = offsets_to_rowptr(off, m, At.rowptr, s);
  At.col.alloc(At.nnz, s);
  At.val.alloc(At.nnz, s);
  DBuf<int64_t> cursor(m, s);
  launch_zero_bytes(cursor.get(), m * sizeof(int64_t), s);
  if (A.rows > 0) {
    tfill_kernel<<<nb, kBlock, 0, s>>>(view(A), At.rowptr.get(), (unsigned long long*)cursor.get(),
                                       At.col.get(), At.val.get());
    AIRG_CHECK_LAUNCH();
  }
  if (m > 0) {
    row_sort_kernel<<<blocks_for(m, kBlock), kBlock, 0, s>>>(m, At.rowptr.get(), At.col.get(),
                                                              At.val.get());
    AIRG_CHECK_LAUNCH();
  }
}

void copy_csr(const CSR& A, CSR& out, hipStream_t s) {
  out.alloc(A.rows, A.cols, A.nnz, s);
  AIRG_HIP(hipMemcpyAsync(out.rowptr.get(), A.rowptr.get(), (A.rows + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
  if (A.nnz) {
    AIRG_HIP(hipMemcpyAsync(out.col.get(), A.col.get(), A.nnz * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
    AIRG_HIP(hipMemcpyAsync(out.val.get(), A.val.get(), A.nnz * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace airg

namespace airg {

// ------------------------------------------------------------------ merged F-point residual operator
// B = A_fc + A_ff W with W the one-point prolongation (column j of A_ff moves
// to column cmap[j] of e_c; columns with cmap[j] < 0 drop out).  Each row's
// entries are collected (A_fc first, then A_ff in stored order), sorted by
// column with a stable insertion sort and equal columns summed left to right.
__global__ void fcw_count_kernel(CSRView Afc, CSRView Aff, const int32_t* cmap, int64_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Afc.rows) return;
  int64_t c = Afc.rowptr[i + 1] - Afc.rowptr[i];
  for (int p = Aff.rowptr[i]; p < Aff.rowptr[i + 1]; ++p) c += cmap[Aff.col[p]] >= 0 ? 1 : 0;
  cnt[i] = c;
}
__global__ void fcw_fill_kernel(CSRView Afc, CSRView Aff, const int32_t* cmap, const int32_t* off,
                                int32_t* col, double* val, int64_t* distinct) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Afc.rows) return;
  const int s = off[i];
  int e = s;
  for (int p = Afc.rowptr[i]; p < Afc.rowptr[i + 1]; ++p, ++e) {
    col[e] = Afc.col[p];
    val[e] = Afc.val[p];
  }
  for (int p = Aff.rowptr[i]; p < Aff.rowptr[i + 1]; ++p) {
    const int m = cmap[Aff.col[p]];
    if (m < 0) continue;
    col[e] = m;
    val[e] = Aff.val[p];
    ++e;
  }
  for (int p = s + 1; p < e; ++p) {  // stable: strictly greater moves right
    const int c = col[p];
    const double v = val[p];
    int q = p - 1;
    while (q >= s && col[q] > c) {
      col[q + 1] = col[q];
      val[q + 1] = val[q];
      --q;
    }
    col[q + 1] = c;
    val[q + 1] = v;
  }
  int w = s;
  for (int p = s; p < e; ++p) {
    if (p > s && col[p] == col[w - 1]) {
      val[w - 1] = val[w - 1] + val[p];
    } else {
      col[w] = col[p];
      val[w] = val[p];
      ++w;
    }
  }
  distinct[i] = w - s;
}
__global__ void fcw_compact_kernel(int64_t rows, const int32_t* off, const int32_t* rowptr,
                                   const int32_t* tcol, const double* tval, int32_t* col,
                                   double* val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int s = off[i];
  for (int p = rowptr[i], q = s; p < rowptr[i + 1]; ++p, ++q) {
    col[p] = tcol[q];
    val[p] = tval[q];
  }
}

void merge_fc_ffw(const CSR& Afc, const CSR& Aff, const int32_t* cmap, CSR& B, hipStream_t s) {
  const int64_t n = Afc.rows;
  B.rows = n;
  B.cols = Afc.cols;
  if (n <= 0) {
    B.nnz = 0;
    B.rowptr.alloc(1, s);
    launch_fill_i32(B.rowptr.get(), 1, 0, s);
    return;
  }
  const unsigned nb = blocks_for(n, kBlock);
  DBuf<int64_t> cnt(n, s), off;
  fcw_count_kernel<<<nb, kBlock, 0, s>>>(view(Afc), view(Aff), cmap, cnt.get());
  AIRG_CHECK_LAUNCH();
  scan_counts(cnt, n, off, s);
  DBuf<int32_t> toff;
  const int64_t tot = offsets_to_rowptr(off, n, toff, s);
  DBuf<int32_t> tcol(std::max<int64_t>(tot, 1), s);
  DBuf<double> tval(std::max<int64_t>(tot, 1), s);
  fcw_fill_kernel<<<nb, kBlock, 0, s>>>(view(Afc), view(Aff), cmap, toff.get(), tcol.get(),
                                        tval.get(), cnt.get());
  AIRG_CHECK_LAUNCH();
  DBuf<int64_t> boff;
  scan_counts(cnt, n, boff, s);
  B.nnz = offsets_to_rowptr(boff, n, B.rowptr, s);
  B.col.alloc(B.nnz, s);
  B.val.alloc(B.nnz, s);
  fcw_compact_kernel<<<nb, kBlock, 0, s>>>(n, toff.get(), B.rowptr.get(), tcol.get(), tval.get(),
                                           B.col.get(), B.val.get());
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ compressed columns
// Every block of 2^kColBlockShift consecutive rows whose columns span less
// than 65536 stores them as 16-bit offsets from the block's smallest column
// (true for almost every block of a locality-ordered operator, whose rows see
// nearby columns); a block that spans more keeps its int32 columns, marked by
// a negative base.  Saves 2 of the 12 bytes of an FP64 entry.
__global__ void col_span_kernel(CSRView A, int64_t nblk, int32_t* cbase, int32_t* cspan,
                                unsigned long long* nwide, unsigned long long* maxspan) {
  int64_t blk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= nblk) return;
  const int64_t r0 = blk << kColBlockShift;
  const int64_t r1 = min(r0 + ((int64_t)1 << kColBlockShift), A.rows);
  int mn = 0x7fffffff, mx = -1;
  for (int p = A.rowptr[r0]; p < A.rowptr[r1]; ++p) {
    const int c = A.col[p];
    mn = min(mn, c);
    mx = max(mx, c);
  }
  if (mx < 0) mn = mx = 0;
  if (mx - mn > 65535) {
    cbase[blk] = -1;
    cspan[blk] = 0;
    atomicAdd(nwide, 1ull);
  } else {
    cbase[blk] = mn;
    cspan[blk] = mx - mn + 1;
    atomicMax(maxspan, (unsigned long long)(mx - mn + 1));
  }
}
__global__ void col16_kernel(CSRView A, const int32_t* cbase, uint16_t* col16) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.rows) return;
  const int b = cbase[i >> kColBlockShift];
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    col16[p] = b >= 0 ? (uint16_t)(A.col[p] - b) : (uint16_t)0;
}

bool compress_columns(CSR& A, hipStream_t s) {
  A.col16.release();
  A.cbase.release();
  A.cspan.release();
  A.max_span = 0;
  if (A.rows <= 0 || A.nnz <= 0) return false;
  const int64_t nblk = (A.rows + (1 << kColBlockShift) - 1) >> kColBlockShift;
  DBuf<unsigned long long> stat(2, s);
  launch_zero_bytes(stat.get(), 2 * sizeof(unsigned long long), s);
  A.cbase.alloc(nblk, s);
  A.cspan.alloc(nblk, s);
  col_span_kernel<<<blocks_for(nblk, kBlock), kBlock, 0, s>>>(view(A), nblk, A.cbase.get(),
                                                             A.cspan.get(), stat.get(),
                                                             stat.get() + 1);
  AIRG_CHECK_LAUNCH();
  unsigned long long st[2];
  stat.to_host(st, 2);
  AIRG_HIP(hipStreamSynchronize(s));
  // worth it only if nearly every block compresses
  if (st[0] * 16 > (unsigned long long)nblk) {
    A.cbase.release();
    A.cspan.release();
    return false;
  }
  A.max_span = (int64_t)st[1];
  A.col16.alloc(A.nnz, s);
  col16_kernel<<<blocks_for(A.rows, kBlock), kBlock, 0, s>>>(view(A), A.cbase.get(), A.col16.get());
  AIRG_CHECK_LAUNCH();
  return true;
}

// ------------------------------------------------------------------ row blocks
// Row blocks for the row-block product: greedy over the rows, a block takes
// consecutive rows of one 64-row group while its entries fit in
// kRowBlockEntries; a longer row is a block by itself.
void build_row_blocks(CSR& A, hipStream_t s) {
  constexpr int64_t kRowBlockEntries = 2048;
  A.rblk.release();
  A.nrblk = 0;
  if (A.rows <= 0) return;
  std::vector<int32_t> rp(A.rows + 1);
  A.rowptr.to_host(rp.data(), A.rows + 1);
  AIRG_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> rb;
  rb.reserve(A.rows / 4 + 2);
  int64_t r = 0;
  rb.push_back(0);
  while (r < A.rows) {
    const int64_t start = r;
    const int64_t gend = std::min<int64_t>(((r >> kColBlockShift) + 1) << kColBlockShift, A.rows);
    int64_t nz = 0;
    while (r < gend) {
      const int64_t len = rp[r + 1] - rp[r];
      if (r > start && nz + len > kRowBlockEntries) break;
      nz += len;
      ++r;
    }
    rb.push_back((int32_t)r);
  }
  A.nrblk = (int64_t)rb.size() - 1;
  A.rblk.alloc(rb.size(), s);
  A.rblk.from_host(rb.data(), rb.size());
  AIRG_HIP(hipStreamSynchronize(s));
}

}  // namespace airg
