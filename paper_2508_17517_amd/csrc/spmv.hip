// CSR SpMV / SpMM kernels of the solve and setup.
//
// Vectors hold K interleaved columns: element (row, c) at row * K + c.  With
// K = 1 a group of TPR lanes (a power of two up to 64) handles one row: the
// lanes stride over the row's entries and combine with a shuffle tree inside
// the group.  With K > 1 a group of K lanes handles one row, lane c owning
// column c: every matrix entry is loaded once for all K columns and the x
// gathers are K-wide and contiguous.  The row result goes to a fused epilogue
// (Horner step, restriction, Newton step, ...) indexed by row * K + c, so each
// smoother and coarse-solver step is one pass over its matrix.  With K = 1 and
// TPR = 1 a row is summed left to right from 0, the order the setup relies on.
//
// The kernels are generic over the matrix value storage (FP64, FP32 or BF16)
// and the vector type (FP64 or FP32); rows accumulate in the vector type.
#include "kernels.hpp"

namespace airg {

__device__ __forceinline__ double ldv(double v) { return v; }
__device__ __forceinline__ float ldv(float v) { return v; }
__device__ __forceinline__ float ldv(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }

// Kernel view of a CSR operator with values of type MV; with C16 the columns
// are read in the compressed form (16-bit offsets from a base per 64 rows,
// int32 columns in the blocks whose base is negative).
template <class MV, bool C16>
struct CSRT {
  const int32_t* __restrict__ rowptr;
  const int32_t* __restrict__ col;
  const uint16_t* __restrict__ col16;
  const int32_t* __restrict__ cbase;
  const MV* __restrict__ val;
  int64_t rows;
  const uint8_t* __restrict__ gmask;  // see OpView::gmask
  const int32_t* __restrict__ rmap;   // see OpView::rmap
  // false where the row's 64-row group is masked off: its sum is 0
  __device__ __forceinline__ bool computed(int64_t row) const {
    return gmask == nullptr || gmask[row >> kColBlockShift] != 0;
  }
  // the operator row of stored row `row`: where its epilogue reads and writes
  __device__ __forceinline__ int64_t out_row(int64_t row) const {
    return rmap ? (int64_t)rmap[row] : row;
  }
  __device__ __forceinline__ int base(int64_t row) const {
    if constexpr (C16) return cbase[row >> kColBlockShift];
    return 0;
  }
  // the column of entry p in a row of base b (callers pass b >= 0 only with C16)
  __device__ __forceinline__ int column(int p, int b) const {
    if constexpr (C16) return b + (int)col16[p];
    return col[p];
  }
};

template <class MV, bool C16>
static CSRT<MV, C16> csr_t(const OpView& A) {
  return {A.rowptr, A.col, A.col16, A.cbase, (const MV*)A.val, A.rows, A.gmask, A.rmap};
}

// Entries in flight per lane: every lane first loads the column indices and
// values of its next U entries, then their x values, and only then adds them,
// so a row costs two dependent memory round trips per U entries instead of
// two per entry.  The additions keep the lane's ascending entry order.
template <int TPR>
constexpr int unroll_for() { return 4; }

// Column index transforms for row_dot: the CSR column itself, or the column
// looked up in a map (entries whose mapped index is negative are skipped).
struct IdxPlain {
  __device__ __forceinline__ int operator()(int c) const { return c; }
};
struct IdxMap {
  const int32_t* __restrict__ m;
  __device__ __forceinline__ int operator()(int c) const { return m[c]; }
};

// sum over entries p = s + lane, s + lane + TPR, ... < e of val[p] * x[idx(col[p]) * K + c]
template <int TPR, int U, int K, class MV, bool C16, class X, class XI, class Idx>
__device__ __forceinline__ X row_dot_cols(const CSRT<MV, C16>& A, int s, int e, int b, int lane,
                                          const XI* __restrict__ x, int c, Idx idx, X sum) {
  for (int p0 = s + lane; p0 < e; p0 += TPR * U) {
    int col[U];
    X v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * TPR;
      col[u] = p < e ? idx(A.column(p, b)) : -1;
      v[u] = p < e ? (X)ldv(A.val[p]) : X(0);
    }
    X xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = col[u] >= 0 ? (X)x[(int64_t)col[u] * K + c] : X(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (col[u] >= 0) sum = sum + v[u] * xv[u];
  }
  return sum;
}
// b: the row's column base in the compressed form; a negative base (a block
// that kept int32 columns) takes the int32 path.  Rows of one wavefront lie
// in one 64-row block, so the branch is uniform.
template <int TPR, int U, int K, class MV, bool C16, class X, class XI, class Idx>
__device__ __forceinline__ X row_dot(const CSRT<MV, C16>& A, int s, int e, int b, int lane,
                                     const XI* __restrict__ x, int c, Idx idx, X sum) {
  if constexpr (C16) {
    if (b < 0) {
      const CSRT<MV, false> W{A.rowptr, A.col, nullptr, nullptr, A.val, A.rows, nullptr, nullptr};
      return row_dot_cols<TPR, U, K>(W, s, e, 0, lane, x, c, idx, sum);
    }
  }
  return row_dot_cols<TPR, U, K>(A, s, e, b, lane, x, c, idx, sum);
}

// Pair loads (K = 1, two or more lanes per row): a lane takes the aligned
// entry pairs (2q, 2q+1), q = s/2 + lane, s/2 + lane + TPR, ..., and fetches
// a pair's two values and two column indices with one wide load each, so the
// load instructions per entry halve and more entries are in flight.  An entry
// of a pair outside [s, e) is masked: a pair may straddle a row boundary, and
// every array is padded past its end.  A lane adds its entries in ascending
// order; the lanes of a row then combine by the shuffle tree.
template <class X, class MV>
__device__ __forceinline__ void load_pair(const MV* __restrict__ v, int q, X& a, X& b);
template <>
__device__ __forceinline__ void load_pair<double, double>(const double* __restrict__ v, int q,
                                                          double& a, double& b) {
  const double2 t = reinterpret_cast<const double2*>(v)[q];
  a = t.x;
  b = t.y;
}
template <>
__device__ __forceinline__ void load_pair<float, float>(const float* __restrict__ v, int q, float& a,
                                                        float& b) {
  const float2 t = reinterpret_cast<const float2*>(v)[q];
  a = t.x;
  b = t.y;
}
template <>
__device__ __forceinline__ void load_pair<float, bf16>(const bf16* __restrict__ v, int q, float& a,
                                                       float& b) {
  const uint32_t w = reinterpret_cast<const uint32_t*>(v)[q];
  a = __uint_as_float(w << 16);
  b = __uint_as_float(w & 0xffff0000u);
}
// the two columns of pair q in a row of base b (compressed form), or as stored
template <class MV, bool C16>
__device__ __forceinline__ void column_pair(const CSRT<MV, C16>& A, int q, int b, int& c0, int& c1) {
  if constexpr (C16) {
    const uint32_t w = reinterpret_cast<const uint32_t*>(A.col16)[q];
    c0 = b + (int)(w & 0xffffu);
    c1 = b + (int)(w >> 16);
  } else {
    const int2 w = reinterpret_cast<const int2*>(A.col)[q];
    c0 = w.x;
    c1 = w.y;
  }
}
// The pairs of entries [s, e) that a lane owns, gathered through gx: with
// OFF the gather index is the raw 16-bit offset (x staged in LDS from the
// row's base), else the column.  load_pairs fetches the U pairs of one step
// (q0, q0 + TPR, ...) and add_pairs gathers and adds them in ascending order.
template <int TPR, int U, bool OFF, class MV, bool C16, class X>
__device__ __forceinline__ void load_pairs(const CSRT<MV, C16>& A, int q0, int qe, int s, int e,
                                           int b, int (&c0)[U], int (&c1)[U], X (&v0)[U],
                                           X (&v1)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = q0 + u * TPR;
    c0[u] = -1;
    c1[u] = -1;
    v0[u] = X(0);
    v1[u] = X(0);
    if (q < qe) {
      load_pair<X>(A.val, q, v0[u], v1[u]);
      column_pair(A, q, OFF ? 0 : b, c0[u], c1[u]);
      if (2 * q < s) c0[u] = -1;
      if (2 * q + 1 >= e) c1[u] = -1;
    }
  }
}
template <int U, class X, class XI>
__device__ __forceinline__ X add_pairs(const XI* __restrict__ gx, const int (&c0)[U],
                                       const int (&c1)[U], const X (&v0)[U], const X (&v1)[U],
                                       X sum) {
  X x0[U], x1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x0[u] = c0[u] >= 0 ? (X)gx[c0[u]] : X(0);
    x1[u] = c1[u] >= 0 ? (X)gx[c1[u]] : X(0);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (c0[u] >= 0) sum = sum + v0[u] * x0[u];
    if (c1[u] >= 0) sum = sum + v1[u] * x1[u];
  }
  return sum;
}
template <int TPR, int U, bool OFF, class MV, bool C16, class X, class XI>
__device__ __forceinline__ X row_dot_pairs_cols(const CSRT<MV, C16>& A, int s, int e, int b,
                                                int lane, const XI* __restrict__ gx, X sum) {
  const int qe = (e + 1) >> 1;
  for (int q0 = (s >> 1) + lane; q0 < qe; q0 += TPR * U) {
    int c0[U], c1[U];
    X v0[U], v1[U];
    load_pairs<TPR, U, OFF>(A, q0, qe, s, e, b, c0, c1, v0, v1);
    sum = add_pairs<U>(gx, c0, c1, v0, v1, sum);
  }
  return sum;
}
// global gathers; a negative base (int32 block) takes the int32 columns
template <int TPR, int U, class MV, bool C16, class X, class XI>
__device__ __forceinline__ X row_dot_pairs(const CSRT<MV, C16>& A, int s, int e, int b, int lane,
                                           const XI* __restrict__ x, X sum) {
  if constexpr (C16) {
    if (b < 0) {
      const CSRT<MV, false> W{A.rowptr, A.col, nullptr, nullptr, A.val, A.rows, nullptr, nullptr};
      return row_dot_pairs_cols<TPR, U, false>(W, s, e, 0, lane, x, sum);
    }
  }
  return row_dot_pairs_cols<TPR, U, false>(A, s, e, b, lane, x, sum);
}

// Workgroups go to the 8 XCDs round robin (workgroup i to XCD i mod 8), and
// each XCD has its own L2.  With the XCD mapping (launch shape bit 8) the grid
// is padded to a multiple of 8 and workgroup i takes row block
// (i mod 8) * (grid / 8) + i / 8, so every XCD sweeps one contiguous eighth of
// the rows and the x elements that neighbouring rows share are fetched into
// one L2, not up to eight; without it workgroup i takes block i, which spreads
// uneven rows evenly over the XCDs.  The tuner picks per operator.
__device__ __forceinline__ int64_t row_block_index(int xcd) {
  if (!xcd) return blockIdx.x;
  const int64_t per = gridDim.x >> 3;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}
static unsigned grid_for(int64_t rows, int rows_per_block, int xcd) {
  const int64_t nb = (rows + rows_per_block - 1) / rows_per_block;
  return (unsigned)(xcd ? (nb + 7) & ~(int64_t)7 : (nb < 1 ? 1 : nb));
}

// lanes-per-row kernel (K = 1)
template <int TPR, class MV, bool C16, class X, class Epi, bool MASK, class XI>
__global__ __launch_bounds__(256) void spmv_kernel(CSRT<MV, C16> A, const XI* __restrict__ x,
                                                   Epi epi, int xcd) {
  const int lane = threadIdx.x & (TPR - 1);
  const int64_t row = row_block_index(xcd) * (256 / TPR) + threadIdx.x / TPR;
  const bool live = row < A.rows;
  typename Epi::Pre pre{};
  if (live && lane == 0) pre = epi.pre(A.out_row(row));
  X sum = 0;
  if (live) {
    const int rs = A.rowptr[row];
    const int re = (!MASK || A.computed(row)) ? A.rowptr[row + 1] : rs;
    if constexpr (TPR >= 2)
      sum = row_dot_pairs<TPR, unroll_for<TPR>()>(A, rs, re, A.base(row), lane, x, sum);
    else
      sum = row_dot<1, 4, 1>(A, rs, re, A.base(row), 0, x, 0, IdxPlain{}, sum);
  }
  if constexpr (TPR > 1) {
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) sum = sum + __shfl_down(sum, o, TPR);
  }
  if (lane == 0 && live) epi(A.out_row(row), sum, pre);
}

// column-per-lane kernel (K > 1 interleaved columns): each column's row sum
// runs left to right from 0, as the TPR = 1 kernel does
template <int K, class MV, bool C16, class X, class Epi, class XI>
__global__ __launch_bounds__(256) void spmm_kernel(CSRT<MV, C16> A, const XI* __restrict__ x,
                                                   Epi epi, int xcd) {
  const int c = threadIdx.x & (K - 1);
  const int64_t row = row_block_index(xcd) * (256 / K) + threadIdx.x / K;
  if (row >= A.rows) return;
  const int64_t orow = A.out_row(row);
  const typename Epi::Pre pre = epi.pre(orow * K + c);
  const X sum = row_dot<1, 4, K>(A, A.rowptr[row], A.rowptr[row + 1], A.base(row), 0, x, c,
                                 IdxPlain{}, X(0));
  epi(orow * K + c, sum, pre);
}

// Row-block kernel (K = 1, selected with tpr = 0): a workgroup takes one row
// block -- up to 64 consecutive rows inside one 64-row group, holding at most
// kRowBlockNnz entries, or a single longer row -- and loads all its entries
// at once, 8 per thread, coalesced across the workgroup; their products go to
// LDS and each row's owner thread then adds its products left to right from
// 0.  The sum order is that of the TPR = 1 kernel, so the results are the
// same bit for bit; what changes is that a workgroup needs two dependent
// memory round trips for all of its rows, which suits long rows.
constexpr int kRowBlockNnz = 2048;

template <class MV, bool C16, class X, class Epi, bool MASK, class XI>
__global__ __launch_bounds__(256) void spmv_rowblock_kernel(CSRT<MV, C16> A,
                                                            const int32_t* __restrict__ rblk,
                                                            int64_t nblk, const XI* __restrict__ x,
                                                            Epi epi, int xcd) {
  __shared__ X prod[kRowBlockNnz];
  const int64_t b = row_block_index(xcd);
  if (b >= nblk) return;
  const int t = threadIdx.x;
  const int r0 = rblk[b], r1 = rblk[b + 1];
  const int64_t row = (int64_t)r0 + t;
  const bool mine = row < r1;
  typename Epi::Pre pre{};
  int rs = 0, re = 0;
  if (mine) {
    pre = epi.pre(A.out_row(row));
    rs = A.rowptr[row];
    re = A.rowptr[row + 1];
  }
  const int p0 = A.rowptr[r0], p1 = (!MASK || A.computed(r0)) ? A.rowptr[r1] : p0;
  const int base = A.base(r0);  // one 64-row group per block
  X sum = 0;
  for (int c0 = p0; c0 < p1; c0 += kRowBlockNnz) {  // one pass unless a single long row
    const int c1 = min(c0 + kRowBlockNnz, p1);
    int col[8];
    X v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = c0 + t + 256 * u;
      bool in = p < c1;
      if constexpr (C16) col[u] = in ? (base >= 0 ? A.column(p, base) : A.col[p]) : 0;
      else col[u] = in ? A.col[p] : 0;
      v[u] = in ? (X)ldv(A.val[p]) : X(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int p = c0 + t + 256 * u;
      if (p < c1) prod[p - c0] = v[u] * (X)x[col[u]];
    }
    __syncthreads();
    if (mine) {
      const int e = min(re, c1);
      for (int p = max(rs, c0); p < e; ++p) sum = sum + prod[p - c0];
    }
    __syncthreads();
  }
  if (mine) epi(A.out_row(row), sum, pre);
}

// Entry-staged kernel (K = 1, shape bit 10): a workgroup takes 256
// consecutive rows, one thread per row.  Short rows make the one-lane kernel's
// loads scattered (each lane walks its own few entries); here the workgroup
// loads the entries of its rows in chunks of 1024, thread t taking entries
// t, t + 256, ... so that every load instruction reads consecutive addresses,
// gathers x for each, and leaves the products in LDS; each row's thread then
// adds its products left to right from 0.  The products and the order of the
// sum are those of the one-lane kernel, so the results are the same bit for
// bit.  The rows span four 64-row groups, each with its own column base (and
// activity mask) in the compressed form; an entry's group comes from the
// groups' first entries.
constexpr int kEntryChunk = 1024;

template <class MV, bool C16, class X, class Epi, bool MASK, class XI>
__global__ __launch_bounds__(256) void spmv_entries_kernel(CSRT<MV, C16> A, const XI* __restrict__ x,
                                                           Epi epi, int xcd) {
  __shared__ X prod[kEntryChunk];
  const int64_t r0 = row_block_index(xcd) * 256;
  if (r0 >= A.rows) return;  // the same for the whole workgroup
  const int t = threadIdx.x;
  const int64_t row = r0 + t;
  const bool live = row < A.rows;
  const int64_t rend = r0 + 256 < A.rows ? r0 + 256 : A.rows;
  typename Epi::Pre pre{};
  int rs = 0, re = 0;
  if (live) {
    pre = epi.pre(A.out_row(row));
    rs = A.rowptr[row];
    re = (!MASK || A.computed(row)) ? A.rowptr[row + 1] : rs;
  }
  // first entry of each 64-row group of the block (gstart[4]: the block's end),
  // the group's column base and whether it is computed
  int gstart[5], gbase[4];
  bool gon[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t gr = r0 + 64 * g;
    gstart[g] = A.rowptr[gr < rend ? gr : rend];
    gbase[g] = gr < rend ? A.base(gr) : 0;
    gon[g] = gr < rend && (!MASK || A.computed(gr));
  }
  gstart[4] = A.rowptr[rend];
  X sum = 0;
  for (int c0 = gstart[0]; c0 < gstart[4]; c0 += kEntryChunk) {
    const int c1 = c0 + kEntryChunk < gstart[4] ? c0 + kEntryChunk : gstart[4];
    int col[4];
    X v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = c0 + t + 256 * u;
      const int g = (p >= gstart[1]) + (p >= gstart[2]) + (p >= gstart[3]);
      col[u] = -1;
      v[u] = X(0);
      if (p < c1 && gon[g]) {
        if constexpr (C16) col[u] = gbase[g] >= 0 ? A.column(p, gbase[g]) : A.col[p];
        else col[u] = A.col[p];
        v[u] = (X)ldv(A.val[p]);
      }
    }
    X xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = col[u] >= 0 ? (X)x[col[u]] : X(0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (col[u] >= 0) prod[t + 256 * u] = v[u] * xv[u];
    __syncthreads();
    if (live) {
      const int e = re < c1 ? re : c1;
      for (int p = rs > c0 ? rs : c0; p < e; ++p) sum = sum + prod[p - c0];
    }
    __syncthreads();
  }
  if (live) epi(A.out_row(row), sum, pre);
}

// LDS-staged kernel (K = 1, shape bit 9, operators with compressed columns):
// a workgroup of 64 TPR threads takes one 64-row group, copies the group's
// window of x (columns cbase .. cbase + span - 1) into LDS with coalesced
// loads and gathers from LDS through the 16-bit column offsets.  Rows sum in
// the order of the TPR-lane row kernel, so the results are the same bit for
// bit.  A group that spans more than the LDS budget, or that kept int32
// columns, gathers from global memory instead.  The budget is the device's
// LDS per workgroup (160 KB on gfx950), 64 KB if the query fails.
static int64_t lds_budget_bytes() {
  static int64_t cached = 0;
  if (cached == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v >= 64 * 1024)
      cached = v;
    else
      cached = 64 * 1024;
  }
  return cached;
}

template <int TPR, class MV, class X, class Epi, bool MASK, class XI>
__global__ __launch_bounds__(64 * TPR) void spmv_lds_kernel(CSRT<MV, true> A,
                                                            const int32_t* __restrict__ cspan,
                                                            int64_t ngroups, int lds_cap,
                                                            const XI* __restrict__ x, Epi epi,
                                                            int xcd) {
  extern __shared__ unsigned char smem_raw[];
  X* xs = reinterpret_cast<X*>(smem_raw);
  const int64_t g = row_block_index(xcd);
  if (g >= ngroups) return;
  const int t = threadIdx.x;
  const int lane = t & (TPR - 1);
  const int64_t row = (g << kColBlockShift) + t / TPR;
  const bool live = row < A.rows;
  const int base = A.cbase[g];
  const int span = cspan[g];
  const bool on = !MASK || A.computed(g << kColBlockShift);
  // the same for the whole workgroup
  const bool staged = on && base >= 0 && span <= lds_cap;
  typename Epi::Pre pre{};
  if (live && lane == 0) pre = epi.pre(A.out_row(row));
  int s = 0, e = 0;
  if (live) {
    s = A.rowptr[row];
    e = on ? A.rowptr[row + 1] : s;
  }
  X sum = 0;
  constexpr int U = unroll_for<TPR>();
  if (staged) {
    // the lane's first U pairs are loaded before the x window, so the two
    // memory round trips overlap; the LDS gathers wait for the barrier
    const int qe = (e + 1) >> 1;
    int q0 = (s >> 1) + lane;
    int c0[U], c1[U];
    X v0[U], v1[U];
    load_pairs<TPR, U, true>(A, q0, qe, s, e, 0, c0, c1, v0, v1);
    for (int i = t; i < span; i += 64 * TPR) xs[i] = (X)x[base + i];
    __syncthreads();
    sum = add_pairs<U>((const X*)xs, c0, c1, v0, v1, sum);
    for (q0 += TPR * U; q0 < qe; q0 += TPR * U) {
      load_pairs<TPR, U, true>(A, q0, qe, s, e, 0, c0, c1, v0, v1);
      sum = add_pairs<U>((const X*)xs, c0, c1, v0, v1, sum);
    }
  } else if (live) {
    sum = row_dot_pairs<TPR, U>(A, s, e, base, lane, x, sum);
  }
  if constexpr (TPR > 1) {
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) sum = sum + __shfl_down(sum, o, TPR);
  }
  if (lane == 0 && live) epi(A.out_row(row), sum, pre);
}

// shape: lanes per row in bits 0-7 (0: the row-block kernel), the XCD
// mapping in bit 8, the LDS-staged kernel in bit 9, the entry-staged kernel in
// bit 10
// MASK: the launch honours Av.gmask (a separate instantiation, so that the
// unmasked products carry no test)
template <class MV, bool C16, bool MASK, class X, class XI, class Epi>
static void launch_spmv_t(const OpView& Av, int shape, int K, const XI* x, Epi epi, hipStream_t s) {
  if (Av.rows <= 0) return;
  const int tpr = shape & 0xff, xcd = (shape >> 8) & 1, lds = (shape >> 9) & 1;
  CSRT<MV, C16> A = csr_t<MV, C16>(Av);
  if (K == 1 && (shape & kShapeEntries)) {
    spmv_entries_kernel<MV, C16, X, Epi, MASK, XI><<<grid_for(Av.rows, 256, xcd), 256, 0, s>>>(
        A, x, epi, xcd);
    AIRG_CHECK_LAUNCH();
    return;
  }
  if (K == 1 && lds) {
    if constexpr (C16) {
      const int64_t ngroups = (Av.rows + 63) >> kColBlockShift;
      const int cap = (int)std::min<int64_t>(Av.max_span, lds_budget_bytes() / (int64_t)sizeof(X));
      const size_t smem = (size_t)std::max(cap, 1) * sizeof(X);
      const unsigned nb = grid_for(ngroups, 1, xcd);
      switch (tpr) {
        case 2: spmv_lds_kernel<2, MV, X, Epi, MASK, XI><<<nb, 128, smem, s>>>(A, Av.cspan, ngroups, cap, x, epi, xcd); break;
        case 4: spmv_lds_kernel<4, MV, X, Epi, MASK, XI><<<nb, 256, smem, s>>>(A, Av.cspan, ngroups, cap, x, epi, xcd); break;
        case 8: spmv_lds_kernel<8, MV, X, Epi, MASK, XI><<<nb, 512, smem, s>>>(A, Av.cspan, ngroups, cap, x, epi, xcd); break;
        case 16: spmv_lds_kernel<16, MV, X, Epi, MASK, XI><<<nb, 1024, smem, s>>>(A, Av.cspan, ngroups, cap, x, epi, xcd); break;
        default: fail(AIRG_ERR_INTERNAL, "LDS-staged product takes 2, 4, 8 or 16 lanes per row");
      }
      AIRG_CHECK_LAUNCH();
      return;
    } else {
      fail(AIRG_ERR_INTERNAL, "LDS-staged product needs compressed columns");
    }
  }
  if (K == 1 && tpr == 0) {
    if (!Av.rblk) fail(AIRG_ERR_INTERNAL, "row-block product without row blocks");
    spmv_rowblock_kernel<MV, C16, X, Epi, MASK, XI><<<grid_for(Av.nrblk, 1, xcd), 256, 0, s>>>(
        A, Av.rblk, Av.nrblk, x, epi, xcd);
    AIRG_CHECK_LAUNCH();
    return;
  }
  if (Av.rows * (int64_t)(K == 1 ? tpr : K) > (int64_t)INT32_MAX)
    fail(AIRG_ERR_INVALID, "product launch exceeds 2^31 threads (fewer lanes or columns needed)");
  if (K == 1) {
    unsigned nb = grid_for(Av.rows, 256 / tpr, xcd);
    switch (tpr) {
      case 1: spmv_kernel<1, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 2: spmv_kernel<2, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 4: spmv_kernel<4, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 8: spmv_kernel<8, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 16: spmv_kernel<16, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 32: spmv_kernel<32, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 64: spmv_kernel<64, MV, C16, X, Epi, MASK, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      default: fail(AIRG_ERR_INTERNAL, "bad lanes-per-row");
    }
  } else {
    unsigned nb = grid_for(Av.rows, 256 / K, xcd);
    switch (K) {
      case 2: spmm_kernel<2, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 4: spmm_kernel<4, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 8: spmm_kernel<8, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 16: spmm_kernel<16, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 32: spmm_kernel<32, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      case 64: spmm_kernel<64, MV, C16, X, Epi, XI><<<nb, 256, 0, s>>>(A, x, epi, xcd); break;
      default: fail(AIRG_ERR_INTERNAL, "column count must be a power of two <= 64");
    }
  }
  AIRG_CHECK_LAUNCH();
}

// dispatch on the matrix storage and column form: FP64 values go with FP64
// vectors, FP32 and BF16 values with FP32 vectors
template <class MV, class X, class XI, class Epi>
static void launch_cols(const OpView& A, int tpr, int K, const XI* x, Epi epi, hipStream_t s) {
  if (A.gmask && K == 1) {
    if (A.col16) launch_spmv_t<MV, true, true, X>(A, tpr, K, x, epi, s);
    else launch_spmv_t<MV, false, true, X>(A, tpr, K, x, epi, s);
    return;
  }
  if (A.col16) launch_spmv_t<MV, true, false, X>(A, tpr, K, x, epi, s);
  else launch_spmv_t<MV, false, false, X>(A, tpr, K, x, epi, s);
}
template <class Epi>
static void launch_spmv(const OpView& A, int tpr, int K, const double* x, Epi epi, hipStream_t s) {
  if (A.vt != VT_F64) fail(AIRG_ERR_INTERNAL, "FP64 vectors need FP64 values");
  launch_cols<double, double>(A, tpr, K, x, epi, s);
}
template <class Epi>
static void launch_spmv(const OpView& A, int tpr, int K, const float* x, Epi epi, hipStream_t s) {
  switch (A.vt) {
    case VT_F32: launch_cols<float, float>(A, tpr, K, x, epi, s); break;
    case VT_BF16: launch_cols<bf16, float>(A, tpr, K, x, epi, s); break;
    default: fail(AIRG_ERR_INTERNAL, "FP32 vectors need FP32 or BF16 values");
  }
}

int pick_tpr(int64_t rows, int64_t nnz) {
  double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
  if (avg <= 4.0) return 1;
  if (avg <= 8.0) return 2;
  if (avg <= 16.0) return 4;
  if (avg <= 32.0) return 8;
  if (avg <= 96.0) return 16;
  return 32;
}

// ------------------------------------------------------------------ epilogues
// i is the linear index row * K + c of the element.  pre(i) loads what the
// epilogue reads of the element before the row sum starts, so those loads
// overlap the row's gathers.
struct NoPre {};
template <class X>
struct EpiStore {
  X* y;
  using Pre = NoPre;
  __device__ Pre pre(int64_t) const { return {}; }
  __device__ void operator()(int64_t i, X t, const Pre&) const { y[i] = t; }
};
template <class X>
struct EpiHorner {
  X* out;
  const X* sv;
  X a, b;
  int acc;
  struct Pre {
    X s, o;
  };
  __device__ Pre pre(int64_t i) const { return {sv[i], acc ? out[i] : X(0)}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const {
    X v = a * t + b * p.s;
    out[i] = acc ? p.o + v : v;
  }
};
template <class X>
struct EpiRestrict {
  const X* src;
  X* dst;
  struct Pre {
    X s;
  };
  __device__ Pre pre(int64_t i) const { return {src[i]}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const { dst[i] = p.s + t; }
};
template <class X>
struct EpiNewtonReal {
  const X* w;
  X* wn;
  X* x;
  X inv, inv_last;
  int first;
  struct Pre {
    X w, x;
  };
  __device__ Pre pre(int64_t i) const { return {w[i], first ? X(0) : x[i]}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const {
    X xi = p.x + p.w * inv;
    X wni = p.w - t * inv;
    wn[i] = wni;
    if (inv_last != X(0)) xi = xi + wni * inv_last;
    x[i] = xi;
  }
};
template <class X>
struct EpiNewtonPair1 {
  const X* w;
  X* tv;
  X* x;
  X c1, c2;
  int first;
  struct Pre {
    X w, x;
  };
  __device__ Pre pre(int64_t i) const { return {w[i], first ? X(0) : x[i]}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const {
    tv[i] = t;
    x[i] = p.x + (c1 * p.w - c2 * t);
  }
};
template <class X>
struct EpiNewtonPair2 {
  const X* w;
  const X* tv;
  X* wn;
  X* x;
  X c1, c2, inv_last;
  struct Pre {
    X w, t, x;
  };
  __device__ Pre pre(int64_t i) const { return {w[i], tv[i], inv_last != X(0) ? x[i] : X(0)}; }
  __device__ void operator()(int64_t i, X u, const Pre& p) const {
    X wni = p.w - c1 * p.t + c2 * u;
    wn[i] = wni;
    if (inv_last != X(0)) x[i] = p.x + wni * inv_last;
  }
};

// F-point residual s = r_f - B e_c
template <class X>
struct EpiResidual {
  const X* rf;
  X* sv;
  struct Pre {
    X r;
  };
  __device__ Pre pre(int64_t i) const { return {rf[i]}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const { sv[i] = p.r - t; }
};
// last Horner step fused with the prolongation: e_f = W e_c + (a t + b s)
template <class X>
struct EpiHornerProlong {
  X* out;
  const X* sv;
  const int32_t* cmap;
  const X* ec;
  X a, b;
  int kshift;
  struct Pre {
    X s, e;
  };
  __device__ Pre pre(int64_t i) const {
    const int64_t row = i >> kshift;
    const int m = cmap[row];
    return {sv[i], m >= 0 ? ec[((int64_t)m << kshift) + (i - (row << kshift))] : X(0)};
  }
  __device__ void operator()(int64_t i, X t, const Pre& p) const { out[i] = p.e + (a * t + b * p.s); }
};

// nAIR's Jacobi-scaled Neumann step y' = y + D^{-1} (s - A y), and the last
// step fused with the prolongation: e_f = W e_c + (y + D^{-1} (s - A y)).
// y is the gathered vector; D^{-1} is per row.
template <class X>
struct EpiNeumann {
  X* out;
  const X* y;
  const X* sv;
  const X* dinv;
  int kshift;
  struct Pre {
    X y, s, d;
  };
  __device__ Pre pre(int64_t i) const { return {y[i], sv[i], dinv[i >> kshift]}; }
  __device__ void operator()(int64_t i, X t, const Pre& p) const { out[i] = p.y + p.d * (p.s - t); }
};
template <class X>
struct EpiNeumannProlong {
  X* out;
  const X* y;
  const X* sv;
  const X* dinv;
  const int32_t* cmap;
  const X* ec;
  int kshift;
  struct Pre {
    X y, s, d, e;
  };
  __device__ Pre pre(int64_t i) const {
    const int64_t row = i >> kshift;
    const int m = cmap[row];
    return {y[i], sv[i], dinv[row],
            m >= 0 ? ec[((int64_t)m << kshift) + (i - (row << kshift))] : X(0)};
  }
  __device__ void operator()(int64_t i, X t, const Pre& p) const {
    out[i] = p.e + (p.y + p.d * (p.s - t));
  }
};

static int log2_of(int K) {
  int k = 0;
  while ((1 << k) < K) ++k;
  return k;
}

template <class X>
void spmv_t(const OpView& A, int tpr, int K, const X* x, X* y, hipStream_t s) {
  launch_spmv(A, tpr, K, x, EpiStore<X>{y}, s);
}
template <class X>
void spmv_horner_t(const OpView& A, int tpr, int K, const X* y, const X* sv, X* out, double a,
                   double b, bool acc, hipStream_t st) {
  launch_spmv(A, tpr, K, y, EpiHorner<X>{out, sv, (X)a, (X)b, acc ? 1 : 0}, st);
}
template <class X>
void spmv_restrict_t(const OpView& Z, int tpr, int K, const X* rf, const X* src, X* dst,
                     hipStream_t s) {
  launch_spmv(Z, tpr, K, rf, EpiRestrict<X>{src, dst}, s);
}
template <class X>
void newton_real_t(const OpView& A, int tpr, int K, const X* w, X* wn, X* x, double inv,
                   bool first, double inv_last, hipStream_t s) {
  launch_spmv(A, tpr, K, w, EpiNewtonReal<X>{w, wn, x, (X)inv, (X)inv_last, first ? 1 : 0}, s);
}
template <class X>
void newton_pair1_t(const OpView& A, int tpr, int K, const X* w, X* t, X* x, double c1, double c2,
                    bool first, hipStream_t s) {
  launch_spmv(A, tpr, K, w, EpiNewtonPair1<X>{w, t, x, (X)c1, (X)c2, first ? 1 : 0}, s);
}
template <class X>
void newton_pair2_t(const OpView& A, int tpr, int K, const X* w, const X* t, X* wn, X* x,
                    double c1, double c2, double inv_last, hipStream_t s) {
  launch_spmv(A, tpr, K, t, EpiNewtonPair2<X>{w, t, wn, x, (X)c1, (X)c2, (X)inv_last}, s);
}

template <class X>
void spmv_residual_t(const OpView& B, int tpr, int K, const X* ec, const X* rf, X* sv,
                     hipStream_t s) {
  launch_spmv(B, tpr, K, ec, EpiResidual<X>{rf, sv}, s);
}
template <class X>
void spmv_horner_prolong_t(const OpView& A, int tpr, int K, const X* y, const X* sv, X* ef,
                           double a, double b, const int32_t* cmap, const X* ec, hipStream_t st) {
  launch_spmv(A, tpr, K, y, EpiHornerProlong<X>{ef, sv, cmap, ec, (X)a, (X)b, log2_of(K)}, st);
}

template <class X>
void spmv_neumann_t(const OpView& A, int tpr, int K, const X* y, const X* sv, const X* dinv, X* out,
                    hipStream_t st) {
  launch_spmv(A, tpr, K, y, EpiNeumann<X>{out, y, sv, dinv, log2_of(K)}, st);
}
template <class X>
void spmv_neumann_prolong_t(const OpView& A, int tpr, int K, const X* y, const X* sv,
                            const X* dinv, X* ef, const int32_t* cmap, const X* ec,
                            hipStream_t st) {
  launch_spmv(A, tpr, K, y,
              EpiNeumannProlong<X>{ef, y, sv, dinv, cmap, ec, log2_of(K)}, st);
}

// y = D^{-1} s, or (prolong) e_f = W e_c + D^{-1} s
template <class X>
__global__ void dinv_apply_kernel(X* out, const X* sv, const X* dinv, const int32_t* cmap,
                                  const X* ec, int kshift, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t row = i >> kshift;
  const X v = dinv[row] * sv[i];
  if (cmap) {
    const int m = cmap[row];
    const X e = m >= 0 ? ec[((int64_t)m << kshift) + (i - (row << kshift))] : X(0);
    out[i] = e + v;
  } else {
    out[i] = v;
  }
}
template <class X>
void dinv_apply_t(X* out, const X* sv, const X* dinv, const int32_t* cmap, const X* ec,
                  int64_t rows, int K, hipStream_t s) {
  const int64_t n = rows * K;
  if (n <= 0) return;
  dinv_apply_kernel<X><<<blocks_for(n, kBlock), kBlock, 0, s>>>(out, sv, dinv, cmap, ec,
                                                                 log2_of(K), n);
  AIRG_CHECK_LAUNCH();
}

template <class X>
__global__ void prolong_axpy_kernel(X* ef, const X* sv, const int32_t* cmap, const X* ec, X a,
                                    int kshift, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t row = i >> kshift;
  const int m = cmap[row];
  const X e = m >= 0 ? ec[((int64_t)m << kshift) + (i - (row << kshift))] : X(0);
  ef[i] = e + a * sv[i];
}
template <class X>
void prolong_axpy_t(X* ef, const X* sv, const int32_t* cmap, const X* ec, double a, int64_t rows,
                    int K, hipStream_t s) {
  const int64_t n = rows * K;
  if (n <= 0) return;
  prolong_axpy_kernel<X><<<blocks_for(n, kBlock), kBlock, 0, s>>>(ef, sv, cmap, ec, (X)a,
                                                                   log2_of(K), n);
  AIRG_CHECK_LAUNCH();
}

template <class X>
__global__ void axpy_first_kernel(X* x, const X* w, X a, int first, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (first ? X(0) : x[i]) + a * w[i];
}
template <class X>
void axpy_first_t(X* x, const X* w, double a, bool first, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  axpy_first_kernel<X><<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, w, (X)a, first ? 1 : 0, n);
  AIRG_CHECK_LAUNCH();
}

#define AIRG_INSTANTIATE(X)                                                                        \
  template void spmv_t<X>(const OpView&, int, int, const X*, X*, hipStream_t);                     \
  template void spmv_horner_t<X>(const OpView&, int, int, const X*, const X*, X*, double, double,  \
                                 bool, hipStream_t);                                               \
  template void spmv_restrict_t<X>(const OpView&, int, int, const X*, const X*, X*, hipStream_t);  \
  template void newton_real_t<X>(const OpView&, int, int, const X*, X*, X*, double, bool, double,  \
                                 hipStream_t);                                                     \
  template void newton_pair1_t<X>(const OpView&, int, int, const X*, X*, X*, double, double, bool, \
                                  hipStream_t);                                                    \
  template void newton_pair2_t<X>(const OpView&, int, int, const X*, const X*, X*, X*, double,     \
                                  double, double, hipStream_t);                                    \
  template void axpy_first_t<X>(X*, const X*, double, bool, int64_t, hipStream_t);                 \
  template void spmv_residual_t<X>(const OpView&, int, int, const X*, const X*, X*, hipStream_t);  \
  template void spmv_horner_prolong_t<X>(const OpView&, int, int, const X*, const X*, X*, double,  \
                                         double, const int32_t*, const X*, hipStream_t);           \
  template void prolong_axpy_t<X>(X*, const X*, const int32_t*, const X*, double, int64_t, int,    \
                                  hipStream_t);                                                    \
  template void spmv_neumann_t<X>(const OpView&, int, int, const X*, const X*, const X*, X*,       \
                                  hipStream_t);                                                    \
  template void spmv_neumann_prolong_t<X>(const OpView&, int, int, const X*, const X*, const X*,   \
                                          X*, const int32_t*, const X*, hipStream_t);              \
  template void dinv_apply_t<X>(X*, const X*, const X*, const int32_t*, const X*, int64_t, int,    \
                                hipStream_t);
AIRG_INSTANTIATE(double)
AIRG_INSTANTIATE(float)
#undef AIRG_INSTANTIATE

// y = A x with FP64 values and rows, x in FP32 (the outer loop's product with
// a basis kept in FP32): every x element is widened to FP64 as it is gathered
void spmv_x32(const OpView& A, int tpr, int K, const float* x, double* y, hipStream_t s) {
  if (A.vt != VT_F64) fail(AIRG_ERR_INTERNAL, "the FP32-vector product of the outer loop needs FP64 values");
  launch_cols<double, double>(A, tpr, K, x, EpiStore<double>{y}, s);
}

// ------------------------------------------------------------------ FP64 wrappers
void spmv_seq(const CSR& A, const double* x, double* y, hipStream_t s) {
  spmv_t(opview(A), 1, 1, x, y, s);
}
void spmv(const CSR& A, int tpr, const double* x, double* y, hipStream_t s) {
  spmv_t(opview(A), tpr, 1, x, y, s);
}

// ------------------------------------------------------------------ conversions
__global__ void d2f_kernel(float* y, const double* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void f2d_kernel(double* y, const float* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
// round to nearest even from FP32 (values are finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)((u + r) >> 16);
}
__global__ void d2bf_kernel(bf16* y, const double* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i].bits = f2bf((float)x[i]);
}
void convert_d2f(float* y, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  d2f_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, n);
  AIRG_CHECK_LAUNCH();
}
void convert_f2d(double* y, const float* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  f2d_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, n);
  AIRG_CHECK_LAUNCH();
}
void convert_d2bf(bf16* y, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  d2bf_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, n);
  AIRG_CHECK_LAUNCH();
}

}  // namespace airg
