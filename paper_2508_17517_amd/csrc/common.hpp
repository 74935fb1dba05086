// Shared host-side definitions of the AIRG library: error type, device
// buffers, CSR matrices and the launch helpers every translation unit uses.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "airg.h"
#include "error.hpp"

namespace airg {

#define AIRG_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      ::airg::fail(e_ == hipErrorOutOfMemory ? AIRG_ERR_NOMEM : AIRG_ERR_HIP,       \
                   std::string(#call) + ": " + hipGetErrorString(e_) + " (" +       \
                       std::to_string((int)e_) + ")");                              \
  } while (0)

#define AIRG_CHECK_LAUNCH() AIRG_HIP(hipGetLastError())

void launch_zero_bytes(void* p, size_t bytes, hipStream_t s);

// Device bytes the library's buffers hold, and an optional budget on them
// (a test hook: an allocation that would pass the budget fails as if the
// device were out of memory; 0 means no budget).
void account_device_bytes(int64_t delta);
void check_device_budget(size_t bytes);
void set_device_budget(int64_t bytes);

// Stream-ordered device buffer (hipMallocAsync / hipFreeAsync).
template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(size_t n, hipStream_t s) { alloc(n, s); }
  ~DBuf() { release(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_; n_ = o.n_; s_ = o.s_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  void alloc(size_t n, hipStream_t s) {
    release();
    s_ = s;
    if (n) {
      check_device_budget(n * sizeof(T) + 256);
      AIRG_HIP(hipMallocAsync((void**)&p_, n * sizeof(T) + 256, s));
      account_device_bytes((int64_t)(n * sizeof(T) + 256));
    }
    n_ = n;
  }
  void release() {
    if (p_) {
      (void)hipFreeAsync(p_, s_);
      account_device_bytes(-(int64_t)(n_ * sizeof(T) + 256));
    }
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  // cleared by a fill kernel (no memset nodes in code a caller may capture)
  void zero() { if (n_) launch_zero_bytes(p_, n_ * sizeof(T), s_); }
  void to_host(T* dst, size_t n) const {
    if (n) AIRG_HIP(hipMemcpyAsync(dst, p_, n * sizeof(T), hipMemcpyDeviceToHost, s_));
  }
  std::vector<T> host(size_t n) const {
    std::vector<T> v(n);
    to_host(v.data(), n);
    AIRG_HIP(hipStreamSynchronize(s_));
    return v;
  }
  void from_host(const T* src, size_t n) {
    if (n) AIRG_HIP(hipMemcpyAsync(p_, src, n * sizeof(T), hipMemcpyHostToDevice, s_));
  }
  hipStream_t stream() const { return s_; }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  hipStream_t s_ = nullptr;
};

// Device CSR matrix, int32 row pointers and columns.
// Rows per base of the compressed column form (see compress_columns).
constexpr int kColBlockShift = 6;

struct CSR {
  int64_t rows = 0, cols = 0, nnz = 0;
  DBuf<int32_t> rowptr, col;
  DBuf<double> val;
  // optional compressed columns for the solve kernels: the column of entry p
  // in row i is cbase[i >> kColBlockShift] + col16[p], or col[p] where that
  // base is negative
  DBuf<uint16_t> col16;
  DBuf<int32_t> cbase;
  // with col16: number of columns each 64-row group spans (max - min + 1),
  // and the largest span over the groups
  DBuf<int32_t> cspan;
  int64_t max_span = 0;
  // optional row blocks for the row-block product: block b holds rows
  // rblk[b] .. rblk[b+1]-1 (see build_row_blocks)
  DBuf<int32_t> rblk;
  int64_t nrblk = 0;
  // in a problem batch: the first of this operator's 64-row groups in the
  // batch's activity masks (-1: not masked)
  int64_t mask_off = -1;
  // optional stored row order of a solve operator: stored row r is the
  // operator's row rmap[r], so the products read and write their per-row
  // vectors at rmap[r] (see spatial_row_order); empty: row r is stored at r
  DBuf<int32_t> rmap;
  void alloc(int64_t r, int64_t c, int64_t nz, hipStream_t s) {
    rows = r; cols = c; nnz = nz;
    rowptr.alloc(r + 1, s);
    col.alloc(nz, s);
    val.alloc(nz, s);
    col16.release();
    cbase.release();
    cspan.release();
    max_span = 0;
    rblk.release();
    nrblk = 0;
    mask_off = -1;
    rmap.release();
  }
};

// Matrix value storage of a solve-phase operator.
enum ValType { VT_F64 = 0, VT_F32 = 1, VT_BF16 = 2 };
struct bf16 {
  uint16_t bits;
};

// Operator view for the solve kernels: structure plus values of type vt.
struct OpView {
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;
  ValType vt;
  int64_t rows;
  int64_t nnz;
  const uint16_t* col16;  // compressed columns, or null
  const int32_t* cbase;
  const int32_t* rblk;    // row blocks, or null
  int64_t nrblk;
  const int32_t* cspan;   // column span per 64-row group (with col16)
  int64_t max_span;
  // per 64-row group, 0 where every row belongs to a problem whose input is
  // zero in this product (its rows then skip the matrix: their sums are 0);
  // null: every row is computed
  const uint8_t* gmask;
  // stored row r is the operator's row rmap[r] (null: r)
  const int32_t* rmap;
};
inline OpView opview(const CSR& A) {
  return {A.rowptr.get(), A.col.get(), A.val.get(), VT_F64, A.rows, A.nnz, A.col16.get(),
          A.cbase.get(), A.rblk.get(), A.nrblk, A.cspan.get(), A.max_span, nullptr, A.rmap.get()};
}

// Read-only view passed to kernels.
struct CSRView {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  int64_t rows;
};
inline CSRView view(const CSR& A) { return {A.rowptr.get(), A.col.get(), A.val.get(), A.rows}; }

// A contiguous range of the nested numbering that belongs to one problem of
// a block-diagonal batch.
struct GroupRange {
  int64_t start, len;
  int32_t group;
};

inline unsigned blocks_for(int64_t n, int per_block) {
  int64_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b < 1 ? 1 : b);
}

// Host scalar fetched from device memory (synchronises the stream).
template <class T>
T fetch(const T* dptr, hipStream_t s) {
  T v;
  AIRG_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipStreamSynchronize(s));
  return v;
}

constexpr int kBlock = 256;

}  // namespace airg
