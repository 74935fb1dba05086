// CSR SpMV kernels of the solve and setup.  One group of TPR lanes (a power of
// two up to 64) handles one row: the lanes stride over the row's entries and
// then combine with a shuffle tree inside the group.  The row result goes to a
// fused epilogue (Horner step, restriction, Newton step, ...), so every
// smoother and coarse-solver step is one pass over its matrix.  With TPR = 1 a
// row is summed left to right from 0.0, the order the setup relies on.
#include "kernels.hpp"

namespace airg {

struct GatherX {
  const double* __restrict__ x;
  __device__ __forceinline__ double operator()(int j) const { return x[j]; }
};

template <int TPR, class Gather>
__device__ __forceinline__ double row_dot(const CSRView& A, int64_t row, int lane, const Gather& g) {
  double sum = 0.0;
  if (row < A.rows) {
    const int s = A.rowptr[row], e = A.rowptr[row + 1];
    for (int p = s + lane; p < e; p += TPR) sum = sum + A.val[p] * g(A.col[p]);
  }
  if constexpr (TPR > 1) {
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) sum = sum + __shfl_down(sum, o, TPR);
  }
  return sum;
}

template <int TPR, class Epi>
__global__ __launch_bounds__(256) void spmv_kernel(CSRView A, GatherX g, Epi epi) {
  const int lane = threadIdx.x & (TPR - 1);
  const int64_t row = (int64_t)blockIdx.x * (256 / TPR) + threadIdx.x / TPR;
  double sum = row_dot<TPR>(A, row, lane, g);
  if (lane == 0 && row < A.rows) epi(row, sum);
}

template <class Epi>
static void launch_spmv(const CSR& A, int tpr, const double* x, Epi epi, hipStream_t s) {
  if (A.rows <= 0) return;
  CSRView v = view(A);
  GatherX g{x};
  unsigned nb = blocks_for(A.rows, 256 / tpr);
  switch (tpr) {
    case 1: spmv_kernel<1, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 2: spmv_kernel<2, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 4: spmv_kernel<4, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 8: spmv_kernel<8, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 16: spmv_kernel<16, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 32: spmv_kernel<32, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    case 64: spmv_kernel<64, Epi><<<nb, 256, 0, s>>>(v, g, epi); break;
    default: fail(AIRG_ERR_INTERNAL, "bad lanes-per-row");
  }
  AIRG_CHECK_LAUNCH();
}

int pick_tpr(int64_t rows, int64_t nnz) {
  double avg = rows > 0 ? (double)nnz / (double)rows : 0.0;
  if (avg < 4.0) return 1;
  if (avg < 8.0) return 2;
  if (avg < 16.0) return 4;
  if (avg < 32.0) return 8;
  if (avg < 64.0) return 16;
  return 32;
}

// ------------------------------------------------------------------ epilogues
struct EpiStore {
  double* y;
  __device__ void operator()(int64_t i, double t) const { y[i] = t; }
};
struct EpiHorner {
  double* out;
  const double* sv;
  double a, b;
  int acc;
  __device__ void operator()(int64_t i, double t) const {
    double v = a * t + b * sv[i];
    out[i] = acc ? out[i] + v : v;
  }
};
struct EpiRestrict {
  const double* src;
  double* dst;
  __device__ void operator()(int64_t i, double t) const { dst[i] = src[i] + t; }
};
struct EpiNewtonReal {
  const double* w;
  double* wn;
  double* x;
  double inv, inv_last;
  int first;
  __device__ void operator()(int64_t i, double t) const {
    double wi = w[i];
    double xi = (first ? 0.0 : x[i]) + wi * inv;
    double wni = wi - t * inv;
    wn[i] = wni;
    if (inv_last != 0.0) xi = xi + wni * inv_last;
    x[i] = xi;
  }
};
struct EpiNewtonPair1 {
  const double* w;
  double* tv;
  double* x;
  double c1, c2;
  int first;
  __device__ void operator()(int64_t i, double t) const {
    tv[i] = t;
    x[i] = (first ? 0.0 : x[i]) + (c1 * w[i] - c2 * t);
  }
};
struct EpiNewtonPair2 {
  const double* w;
  const double* tv;
  double* wn;
  double* x;
  double c1, c2, inv_last;
  __device__ void operator()(int64_t i, double u) const {
    double wni = w[i] - c1 * tv[i] + c2 * u;
    wn[i] = wni;
    if (inv_last != 0.0) x[i] = x[i] + wni * inv_last;
  }
};

void spmv_seq(const CSR& A, const double* x, double* y, hipStream_t s) {
  launch_spmv(A, 1, x, EpiStore{y}, s);
}
void spmv(const CSR& A, int tpr, const double* x, double* y, hipStream_t s) {
  launch_spmv(A, tpr, x, EpiStore{y}, s);
}
void spmv_horner(const CSR& A, int tpr, const double* y, const double* sv, double* out, double a,
                 double b, bool acc, hipStream_t st) {
  launch_spmv(A, tpr, y, EpiHorner{out, sv, a, b, acc ? 1 : 0}, st);
}
void spmv_restrict(const CSR& Z, int tpr, const double* rf, const double* src, double* dst,
                   hipStream_t s) {
  launch_spmv(Z, tpr, rf, EpiRestrict{src, dst}, s);
}
void newton_real(const CSR& A, int tpr, const double* w, double* wn, double* x, double inv,
                 bool first, double inv_last, hipStream_t s) {
  launch_spmv(A, tpr, w, EpiNewtonReal{w, wn, x, inv, inv_last, first ? 1 : 0}, s);
}
void newton_pair1(const CSR& A, int tpr, const double* w, double* t, double* x, double c1,
                  double c2, bool first, hipStream_t s) {
  launch_spmv(A, tpr, w, EpiNewtonPair1{w, t, x, c1, c2, first ? 1 : 0}, s);
}
void newton_pair2(const CSR& A, int tpr, const double* w, const double* t, double* wn, double* x,
                  double c1, double c2, double inv_last, hipStream_t s) {
  launch_spmv(A, tpr, t, EpiNewtonPair2{w, t, wn, x, c1, c2, inv_last}, s);
}

__global__ void axpy_first_kernel(double* x, const double* w, double a, int first, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (first ? 0.0 : x[i]) + a * w[i];
}
void axpy_first(double* x, const double* w, double a, bool first, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  axpy_first_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, w, a, first ? 1 : 0, n);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ F-point residual
// s_i = r_i - sum_j Afc_ij e_c[j] - sum_j Aff_ij e_c[cmap[j]], ef_i = e_c[cmap[i]]
template <int TPR>
__global__ __launch_bounds__(256) void residual_kernel(CSRView Aff, CSRView Afc,
                                                       const int32_t* __restrict__ cmap,
                                                       const double* __restrict__ rf,
                                                       const double* __restrict__ ec,
                                                       double* __restrict__ ef,
                                                       double* __restrict__ sv) {
  const int lane = threadIdx.x & (TPR - 1);
  const int64_t row = (int64_t)blockIdx.x * (256 / TPR) + threadIdx.x / TPR;
  double sum = 0.0;
  if (row < Aff.rows) {
    int s = Afc.rowptr[row], e = Afc.rowptr[row + 1];
    for (int p = s + lane; p < e; p += TPR) sum = sum + Afc.val[p] * ec[Afc.col[p]];
    s = Aff.rowptr[row];
    e = Aff.rowptr[row + 1];
    for (int p = s + lane; p < e; p += TPR) {
      int c = cmap[Aff.col[p]];
      if (c >= 0) sum = sum + Aff.val[p] * ec[c];
    }
  }
  if constexpr (TPR > 1) {
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) sum = sum + __shfl_down(sum, o, TPR);
  }
  if (lane == 0 && row < Aff.rows) {
    int c = cmap[row];
    ef[row] = c >= 0 ? ec[c] : 0.0;
    sv[row] = rf[row] - sum;
  }
}

void residual_fpoint(const CSR& Aff, const CSR& Afc, const int32_t* cmap, int tpr,
                     const double* rf, const double* ec, double* ef, double* sv, hipStream_t s) {
  if (Aff.rows <= 0) return;
  CSRView a = view(Aff), b = view(Afc);
  unsigned nb = blocks_for(Aff.rows, 256 / tpr);
  switch (tpr) {
    case 1: residual_kernel<1><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 2: residual_kernel<2><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 4: residual_kernel<4><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 8: residual_kernel<8><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 16: residual_kernel<16><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 32: residual_kernel<32><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    case 64: residual_kernel<64><<<nb, 256, 0, s>>>(a, b, cmap, rf, ec, ef, sv); break;
    default: fail(AIRG_ERR_INTERNAL, "bad lanes-per-row");
  }
  AIRG_CHECK_LAUNCH();
}

}  // namespace airg
