// Vector kernels: counter-based random draws, elementwise updates, dot
// products in a fixed binary-tree order, permutations and prefix scans.
#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace airg {

// ------------------------------------------------------------------ RNG
// SplitMix64 (Steele, Lea & Flood 2014): output k of seed s is mix64(s + k g)
// with the golden gamma g; used here as a counter-based generator.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void uniform_kernel(double* out, int64_t n, uint64_t seed, uint64_t base) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t c = base + (uint64_t)i;
  uint64_t z = mix64(seed + (c + 1ull) * 0x9E3779B97F4A7C15ull);
  out[i] = (double)(z >> 11) * 0x1.0p-53;
}

void launch_uniform(double* out, int64_t n, uint64_t seed, int purpose, int level, hipStream_t s) {
  if (n <= 0) return;
  uint64_t base = ((uint64_t)purpose << 56) | ((uint64_t)level << 40);
  uniform_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(out, n, seed, base);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ elementwise
__global__ void fill_kernel(double* x, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void fill_i32_kernel(int32_t* x, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void zero_bytes_kernel(uint8_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
__global__ void copy_kernel(double* y, const double* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ void scale_kernel(double* y, const double* x, double a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}
__global__ void divide_kernel(double* y, const double* x, double d, int64_t n, float* y32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i] / d;
  y[i] = v;
  if (y32) y32[i] = (float)v;
}
// y = x / sqrt(d2[0]) (the square root taken here, correctly rounded like
// the host's), and y32 = (float) y when given
__global__ void divide_norm2_kernel(double* y, const double* x, const double* d2, int64_t n,
                                    float* y32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i] / sqrt(d2[0]);
  y[i] = v;
  if (y32) y32[i] = (float)v;
}
__global__ void divide_dev_kernel(double* y, const double* x, const double* d, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / d[0];
}
__global__ void sub_kernel(double* z, const double* x, const double* y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = x[i] - y[i];
}

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, n, v);
  AIRG_CHECK_LAUNCH();
}
void launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  fill_i32_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, n, v);
  AIRG_CHECK_LAUNCH();
}
void launch_zero_bytes(void* p, size_t bytes, hipStream_t s) {
  if (!bytes) return;
  zero_bytes_kernel<<<blocks_for((int64_t)bytes, kBlock), kBlock, 0, s>>>((uint8_t*)p, bytes);
  AIRG_CHECK_LAUNCH();
}
void launch_copy(double* y, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  copy_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, n);
  AIRG_CHECK_LAUNCH();
}
void launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  scale_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, a, n);
  AIRG_CHECK_LAUNCH();
}
void launch_divide(double* y, const double* x, double d, int64_t n, hipStream_t s, float* y32) {
  if (n <= 0) return;
  divide_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, d, n, y32);
  AIRG_CHECK_LAUNCH();
}
void launch_divide_norm2(double* y, const double* x, const double* d2, int64_t n, hipStream_t s,
                         float* y32) {
  if (n <= 0) return;
  divide_norm2_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, d2, n, y32);
  AIRG_CHECK_LAUNCH();
}
void launch_divide_dev(double* y, const double* x, const double* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  divide_dev_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, d, n);
  AIRG_CHECK_LAUNCH();
}
void launch_sub(double* z, const double* x, const double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  sub_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(z, x, y, n);
  AIRG_CHECK_LAUNCH();
}

__global__ void cgs_update_kernel(double* w, const double* V, int64_t ldv, const double* h, int nv,
                                  int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int k = 0; k < nv; ++k) acc = acc - h[k] * V[(int64_t)k * ldv + i];
  w[i] = acc;
}
void launch_cgs_update(double* w, const double* V, int64_t ldv, const double* h, int nv, int64_t n,
                       hipStream_t s) {
  if (n <= 0 || nv <= 0) return;
  cgs_update_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(w, V, ldv, h, nv, n);
  AIRG_CHECK_LAUNCH();
}

// Z in FP64, or in FP32 (widened to FP64 as it is read)
template <class ZT>
__global__ void basis_combine_kernel(double* x, const ZT* Z, int64_t ldz, const double* y, int nv,
                                     int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int k = 0; k < nv; ++k) acc = acc + y[k] * (double)Z[(int64_t)k * ldz + i];
  x[i] = acc;
}
template <class ZT>
static void launch_basis_combine_t(double* x, const ZT* Z, int64_t ldz, const double* y, int nv,
                                   int64_t n, hipStream_t s) {
  if (n <= 0 || nv <= 0) return;
  basis_combine_kernel<ZT><<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, Z, ldz, y, nv, n);
  AIRG_CHECK_LAUNCH();
}
void launch_basis_combine(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                          int64_t n, hipStream_t s) {
  launch_basis_combine_t(x, Z, ldz, y, nv, n, s);
}
void launch_basis_combine(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                          int64_t n, hipStream_t s) {
  launch_basis_combine_t(x, Z, ldz, y, nv, n, s);
}

// ------------------------------------------------------------------ tree dots
// A block reduces an aligned chunk of 1024 consecutive leaves: each of the 256
// threads sums 4 adjacent leaves as (l0 + l1) + (l2 + l3); lanes then pair up
// with offsets 1, 2, ..., 32 (lane L adds lane L + o when L is a multiple of
// 2o) and the four waves combine as (w0 + w1) + (w2 + w3).  Every partial is
// therefore an aligned subtree of the perfect binary tree over the zero-padded
// index range, and later stages repeat the scheme on the partials.
constexpr int kDotChunk = 1024;
constexpr int kMaxDotVecs = 64;

__device__ __forceinline__ double wave_tree(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double u = __shfl_down(v, o, 64);
    v = v + u;
  }
  return v;  // valid in lane 0
}

__global__ __launch_bounds__(256) void tree_dot_stage1(const double* __restrict__ V, int64_t ldv,
                                                       int nv, const double* __restrict__ w,
                                                       int64_t n, double* __restrict__ part,
                                                       int64_t nb) {
  __shared__ double red[kMaxDotVecs][4];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kDotChunk + 4 * t;
  double w4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) w4[q] = (i0 + q < n) ? w[i0 + q] : 0.0;
  const int lane = t & 63, wave = t >> 6;
  for (int k = 0; k < nv; ++k) {
    const double* v = V + (int64_t)k * ldv;
    double p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = (i0 + q < n) ? v[i0 + q] * w4[q] : 0.0;
    double local = (p[0] + p[1]) + (p[2] + p[3]);
    double ws = wave_tree(local);
    if (lane == 0) red[k][wave] = ws;
  }
  __syncthreads();
  if (t < nv) part[(int64_t)t * nb + blockIdx.x] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
}

__global__ __launch_bounds__(256) void tree_sum_stage(const double* __restrict__ in, int64_t m,
                                                      int64_t in_stride, double* __restrict__ out,
                                                      int64_t out_stride) {
  __shared__ double red[4];
  const int t = threadIdx.x;
  const int k = blockIdx.y;
  const double* src = in + (int64_t)k * in_stride;
  const int64_t i0 = (int64_t)blockIdx.x * kDotChunk + 4 * t;
  double p[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) p[q] = (i0 + q < m) ? src[i0 + q] : 0.0;
  double local = (p[0] + p[1]) + (p[2] + p[3]);
  double ws = wave_tree(local);
  if ((t & 63) == 0) red[t >> 6] = ws;
  __syncthreads();
  if (t == 0) out[(int64_t)k * out_stride + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

size_t dot_work_size(int64_t n, int nv) {
  int64_t nb = (n + kDotChunk - 1) / kDotChunk;
  if (nb < 1) nb = 1;
  int64_t nb2 = (nb + kDotChunk - 1) / kDotChunk;
  return (size_t)nv * (size_t)(nb + nb2 + 2);
}

void launch_tree_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* out,
                      double* work, hipStream_t s) {
  if (nv <= 0) return;
  if (nv > kMaxDotVecs) fail(AIRG_ERR_INVALID, "too many vectors in one dot launch");
  int64_t nb = (n + kDotChunk - 1) / kDotChunk;
  if (nb < 1) nb = 1;
  double* a = work;
  double* b = work + (size_t)nv * nb;
  tree_dot_stage1<<<(unsigned)nb, 256, 0, s>>>(V, ldv, nv, w, n, a, nb);
  AIRG_CHECK_LAUNCH();
  int64_t m = nb;
  int64_t stride = nb;
  for (;;) {
    // always at least one stage: a single partial is copied through as p + 0
    int64_t mb = (m + kDotChunk - 1) / kDotChunk;
    double* dst = (mb == 1) ? out : b;
    int64_t dstride = (mb == 1) ? 1 : mb;
    tree_sum_stage<<<dim3((unsigned)mb, (unsigned)nv), 256, 0, s>>>(a, m, stride, dst, dstride);
    AIRG_CHECK_LAUNCH();
    if (mb == 1) return;
    std::swap(a, b);
    m = mb;
    stride = dstride;
  }
}

__global__ void sqrt_kernel(double* v) { v[0] = sqrt(v[0]); }
void launch_sqrt_inplace(double* v, hipStream_t s) {
  sqrt_kernel<<<1, 1, 0, s>>>(v);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ fused Gram-Schmidt sweeps
// A classical Gram-Schmidt sweep with the reduction that follows it: MODE 0
// forms out[k] = V_k . w; MODE 1 updates w = w - sum_k h[k] V_k (k ascending
// per element, as in cgs_update_kernel) and then forms out[k] = V_k . w;
// MODE 2 updates w the same way and forms out[0] = w . w.  An element's V_k
// values stay in registers between the update and the products, so the
// basis is read once per sweep.  Block b takes the kFusedSpan elements from
// b * kFusedSpan, four per thread at stride 256 (coalesced); a thread adds its
// four products in order, the shuffle tree and the four waves in pairs give
// the block's partial, and one more launch sums the partials of each k in
// block order (sum_partials_kernel).  Fixed orders throughout: the result is
// the same on every run.
constexpr int kFusedPerThread = 4;
constexpr int64_t kFusedSpan = 256 * kFusedPerThread;

template <int MODE, int NV>
__global__ __launch_bounds__(256) void cgs_fused_kernel(
    double* __restrict__ w, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
    int64_t n, double* __restrict__ part, int64_t nb) {
  constexpr int CNT = MODE == 2 ? 1 : NV;
  __shared__ double red[CNT][4];
  const int t = threadIdx.x;
  double hk[MODE == 0 ? 1 : NV];
  if constexpr (MODE != 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) hk[k] = h[k];
  }
  double acc[CNT];
#pragma unroll
  for (int k = 0; k < CNT; ++k) acc[k] = 0.0;
  for (int u = 0; u < kFusedPerThread; ++u) {
    const int64_t i = (int64_t)blockIdx.x * kFusedSpan + u * 256 + t;
    if (i >= n) break;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = V[(int64_t)k * ldv + i];
    double wi = w[i];
    if constexpr (MODE != 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) wi = wi - hk[k] * v[k];
      w[i] = wi;
    }
#pragma unroll
    for (int k = 0; k < CNT; ++k) acc[k] = acc[k] + (MODE == 2 ? wi * wi : v[k] * wi);
  }
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const double s = wave_tree(acc[k]);
    if (lane == 0) red[k][wave] = s;
  }
  __syncthreads();
  if (t < CNT) part[(int64_t)t * nb + blockIdx.x] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
}

// out[k] = sum of part[k * nb + q] over q < nb, block k: thread t adds
// q = t, t + 256, ... in order, then the shuffle tree and the waves in pairs
__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ part,
                                                           int64_t nb, double* __restrict__ out) {
  __shared__ double red[4];
  const int t = threadIdx.x;
  const double* p = part + (int64_t)blockIdx.x * nb;
  double acc = 0.0;
#pragma unroll 4
  for (int64_t q = t; q < nb; q += 256) acc = acc + p[q];
  const double s = wave_tree(acc);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int MODE, int NV>
static void launch_fused_nv(int nv, double* w, const double* V, int64_t ldv, const double* h,
                            int64_t n, double* part, int64_t nb, hipStream_t s) {
  if constexpr (NV > kFusedVecs) {
    fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  } else {
    if (nv != NV) return launch_fused_nv<MODE, NV + 1>(nv, w, V, ldv, h, n, part, nb, s);
    cgs_fused_kernel<MODE, NV><<<(unsigned)nb, 256, 0, s>>>(w, V, ldv, h, n, part, nb);
  }
}

static int64_t fused_blocks(int64_t n) { return n < 1 ? 1 : (n + kFusedSpan - 1) / kFusedSpan; }

size_t cgs_fused_work_size(int64_t n) { return (size_t)kFusedVecs * (size_t)fused_blocks(n); }

template <int MODE>
static void launch_cgs_fused(double* w, const double* V, int64_t ldv, const double* h, int nv,
                             int64_t n, double* out, double* work, hipStream_t s) {
  if (nv < 1 || nv > kFusedVecs) fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  if (n <= 0) return;
  const int64_t nb = fused_blocks(n);
  launch_fused_nv<MODE, 1>(nv, w, V, ldv, h, n, work, nb, s);
  AIRG_CHECK_LAUNCH();
  sum_partials_kernel<<<MODE == 2 ? 1 : nv, 256, 0, s>>>(work, nb, out);
  AIRG_CHECK_LAUNCH();
}
void launch_cgs_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                     double* out, double* work, hipStream_t s) {
  // MODE 0 neither writes w nor reads h
  launch_cgs_fused<0>(const_cast<double*>(w), V, ldv, nullptr, nv, n, out, work, s);
}
void launch_cgs_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                            int64_t n, double* out, double* work, hipStream_t s) {
  launch_cgs_fused<1>(w, V, ldv, h, nv, n, out, work, s);
}
void launch_cgs_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                             int64_t n, double* out, double* work, hipStream_t s) {
  launch_cgs_fused<2>(w, V, ldv, h, nv, n, out, work, s);
}

// ------------------------------------------------------------------ per-column Krylov
// K interleaved columns (element e = r K + c of an [n][K] array, K a power of
// two): the orthogonalisation of one FGMRES per column, all columns per launch.
__global__ void cgs_update_cols_kernel(double* w, const double* V, int64_t ldv, const double* h,
                                       int nv, int64_t n, int K) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e & (K - 1));
  double acc = w[e];
  for (int k = 0; k < nv; ++k) acc = acc - h[k * K + c] * V[(int64_t)k * ldv + e];
  w[e] = acc;
}
template <class ZT>
__global__ void basis_combine_cols_kernel(double* x, const ZT* Z, int64_t ldz, const double* y,
                                          int nv, int64_t n, int K) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e & (K - 1));
  double acc = x[e];
  for (int k = 0; k < nv; ++k) acc = acc + y[k * K + c] * (double)Z[(int64_t)k * ldz + e];
  x[e] = acc;
}
__global__ void divide_cols_kernel(double* y, const double* x, const double* d, int64_t n, int K,
                                   float* y32) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double dc = d[e & (K - 1)];
  const double v = dc != 0.0 ? x[e] / dc : 0.0;
  y[e] = v;
  if (y32) y32[e] = (float)v;
}

static void check_cols(int K) {
  if (K < 1 || K > 64 || (K & (K - 1)) != 0) fail(AIRG_ERR_INTERNAL, "bad column count");
}
void launch_cgs_update_cols(double* w, const double* V, int64_t ldv, const double* h, int nv,
                            int64_t n0, int K, hipStream_t s) {
  check_cols(K);
  const int64_t n = n0 * K;
  if (n <= 0 || nv <= 0) return;
  cgs_update_cols_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(w, V, ldv, h, nv, n, K);
  AIRG_CHECK_LAUNCH();
}
template <class ZT>
static void launch_basis_combine_cols_t(double* x, const ZT* Z, int64_t ldz, const double* y,
                                        int nv, int64_t n0, int K, hipStream_t s) {
  check_cols(K);
  const int64_t n = n0 * K;
  if (n <= 0 || nv <= 0) return;
  basis_combine_cols_kernel<ZT><<<blocks_for(n, kBlock), kBlock, 0, s>>>(x, Z, ldz, y, nv, n, K);
  AIRG_CHECK_LAUNCH();
}
void launch_basis_combine_cols(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                               int64_t n0, int K, hipStream_t s) {
  launch_basis_combine_cols_t(x, Z, ldz, y, nv, n0, K, s);
}
void launch_basis_combine_cols(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                               int64_t n0, int K, hipStream_t s) {
  launch_basis_combine_cols_t(x, Z, ldz, y, nv, n0, K, s);
}
void launch_divide_cols(double* y, const double* x, const double* d, int64_t n0, int K,
                        hipStream_t s, float* y32) {
  check_cols(K);
  const int64_t n = n0 * K;
  if (n <= 0) return;
  divide_cols_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, d, n, K, y32);
  AIRG_CHECK_LAUNCH();
}

// Per-column dot products out[k K + c] = sum_r V_k[r K + c] w[r K + c], up to
// kColDotVecs vectors per pass.  Block b walks the 256-element slabs b, b + G,
// b + 2G, ... of the array (a slab holds whole rows, so thread t always meets
// column t mod K) adding its products in sequence; the lanes of a column then
// combine by a shuffle tree, the four waves in order, and the G block
// partials of each (k, c) by the tree sum.  w is read once per pass.
constexpr int kColDotVecs = 16;
constexpr int kColDotBlocks = 1024;

static int64_t col_dot_blocks(int64_t n) {
  int64_t g = (n + 255) / 256;
  return g < 1 ? 1 : (g > kColDotBlocks ? kColDotBlocks : g);
}

__global__ __launch_bounds__(256) void col_dots_stage1(const double* __restrict__ V, int64_t ldv,
                                                       int nv, const double* __restrict__ w,
                                                       int64_t n, int K, double* __restrict__ part) {
  __shared__ double red[kColDotVecs][4][64];
  const int t = threadIdx.x;
  double acc[kColDotVecs];
#pragma unroll
  for (int k = 0; k < kColDotVecs; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + t; e < n; e += stride) {
    const double wv = w[e];
#pragma unroll
    for (int k = 0; k < kColDotVecs; ++k)
      if (k < nv) acc[k] = acc[k] + V[(int64_t)k * ldv + e] * wv;
  }
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < kColDotVecs; ++k) {
    if (k < nv) {
      double v = acc[k];
      for (int o = K; o < 64; o <<= 1) v = v + __shfl_down(v, o, 64);
      if (lane < K) red[k][wave][lane] = v;
    }
  }
  __syncthreads();
  for (int q = t; q < nv * K; q += 256) {
    const int k = q / K, c = q % K;
    part[(int64_t)q * gridDim.x + blockIdx.x] =
        (red[k][0][c] + red[k][1][c]) + (red[k][2][c] + red[k][3][c]);
  }
}

size_t col_dots_work_size(int64_t n0, int K) {
  return (size_t)kColDotVecs * (size_t)K * (size_t)col_dot_blocks(n0 * K);
}
void launch_col_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n0, int K,
                     double* out, double* work, hipStream_t s) {
  check_cols(K);
  if (nv <= 0) return;
  const int64_t n = n0 * K;
  const int64_t G = col_dot_blocks(n);
  for (int k0 = 0; k0 < nv; k0 += kColDotVecs) {
    const int cnt = nv - k0 < kColDotVecs ? nv - k0 : kColDotVecs;
    col_dots_stage1<<<(unsigned)G, 256, 0, s>>>(V + (int64_t)k0 * ldv, ldv, cnt, w, n, K, work);
    AIRG_CHECK_LAUNCH();
    // G <= kDotChunk partials per (k, c): one tree stage per pair
    tree_sum_stage<<<dim3(1u, (unsigned)(cnt * K)), 256, 0, s>>>(work, G, G, out + (int64_t)k0 * K, 1);
    AIRG_CHECK_LAUNCH();
  }
}

// The fused sweeps of cgs_fused_kernel per column: the update of
// cgs_update_cols_kernel, then the products of col_dots_stage1 (DOTS, the
// same walk and sum order) or the column sums of squares, with the element's
// basis values kept in registers in between.  The coefficients h[k K + c]
// sit in LDS.
template <bool DOTS, int NV>
__global__ __launch_bounds__(256) void col_fused_kernel(double* __restrict__ w,
                                                        const double* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ h, int64_t n,
                                                        int K, double* __restrict__ part) {
  constexpr int CNT = DOTS ? NV : 1;
  __shared__ double hs[NV][64];
  __shared__ double red[4][64];
  const int t = threadIdx.x;
  for (int q = t; q < NV * K; q += 256) hs[q / K][q % K] = h[q];
  __syncthreads();
  const int c = t & (K - 1);  // every element a thread meets is in column c
  double acc[CNT];
#pragma unroll
  for (int k = 0; k < CNT; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e = (int64_t)blockIdx.x * 256 + t; e < n; e += stride) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = V[(int64_t)k * ldv + e];
    double wi = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k) wi = wi - hs[k][c] * v[k];
    w[e] = wi;
    if constexpr (DOTS) {
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k] = acc[k] + v[k] * wi;
    } else {
      acc[0] = acc[0] + wi * wi;
    }
  }
  // one k at a time through a small LDS buffer (the sums of col_dots_stage1)
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    double v = acc[k];
    for (int o = K; o < 64; o <<= 1) v = v + __shfl_down(v, o, 64);
    if (lane < K) red[wave][lane] = v;
    __syncthreads();
    if (t < K)
      part[(int64_t)(k * K + t) * gridDim.x + blockIdx.x] =
          (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    __syncthreads();
  }
}

template <bool DOTS, int NV>
static void launch_col_fused_nv(int nv, double* w, const double* V, int64_t ldv, const double* h,
                                int64_t n, int K, double* part, int64_t G, hipStream_t s) {
  if constexpr (NV > kFusedVecs) {
    fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  } else {
    if (nv != NV) return launch_col_fused_nv<DOTS, NV + 1>(nv, w, V, ldv, h, n, K, part, G, s);
    col_fused_kernel<DOTS, NV><<<(unsigned)G, 256, 0, s>>>(w, V, ldv, h, n, K, part);
  }
}

size_t col_fused_work_size(int64_t n0, int K) {
  return (size_t)kFusedVecs * (size_t)K * (size_t)col_dot_blocks(n0 * K);
}

static void launch_col_fused(bool dots, double* w, const double* V, int64_t ldv, const double* h,
                             int nv, int64_t n0, int K, double* out, double* work, hipStream_t s) {
  check_cols(K);
  if (nv < 1 || nv > kFusedVecs) fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  const int64_t n = n0 * K;
  if (n <= 0) return;
  const int64_t G = col_dot_blocks(n);
  if (dots) launch_col_fused_nv<true, 1>(nv, w, V, ldv, h, n, K, work, G, s);
  else launch_col_fused_nv<false, 1>(nv, w, V, ldv, h, n, K, work, G, s);
  AIRG_CHECK_LAUNCH();
  // G <= kDotChunk partials per (k, c): one tree stage per pair
  tree_sum_stage<<<dim3(1u, (unsigned)((dots ? nv : 1) * K)), 256, 0, s>>>(work, G, G, out, 1);
  AIRG_CHECK_LAUNCH();
}
void launch_cols_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                             int64_t n0, int K, double* out, double* work, hipStream_t s) {
  launch_col_fused(true, w, V, ldv, h, nv, n0, K, out, work, s);
}
void launch_cols_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                              int64_t n0, int K, double* out, double* work, hipStream_t s) {
  launch_col_fused(false, w, V, ldv, h, nv, n0, K, out, work, s);
}

// ------------------------------------------------------------------ per-problem Krylov
// One outer process per problem of a batch ordered problem-major: work item
// q covers elements start[q] .. start[q] + len[q] - 1 (len <= kDotChunk) of
// problem grp[q]; coefficient arrays hold entry (k, g) at k G + g.
void build_group_items(const std::vector<GroupRange>& ranges, int G, GroupItems& out,
                       hipStream_t s, int chunk) {
  if (chunk < 1 || chunk > kDotChunk) fail(AIRG_ERR_INTERNAL, "item length must be 1..1024");
  std::vector<int64_t> st;
  std::vector<int32_t> ln, gp;
  for (const GroupRange& r : ranges)
    for (int64_t a = 0; a < r.len; a += chunk) {
      st.push_back(r.start + a);
      ln.push_back((int32_t)std::min<int64_t>(chunk, r.len - a));
      gp.push_back(r.group);
    }
  // items of each problem in list order: the fixed order of its sums
  std::vector<int32_t> gptr(G + 1, 0), glist(gp.size());
  for (int32_t g : gp) ++gptr[g + 1];
  for (int g = 0; g < G; ++g) gptr[g + 1] += gptr[g];
  std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
  for (size_t q = 0; q < gp.size(); ++q) glist[fill[gp[q]]++] = (int32_t)q;
  out.n = (int64_t)st.size();
  out.G = G;
  out.start.alloc(st.size(), s);
  out.len.alloc(ln.size(), s);
  out.grp.alloc(gp.size(), s);
  out.gptr.alloc(gptr.size(), s);
  out.glist.alloc(glist.size(), s);
  out.start.from_host(st.data(), st.size());
  out.len.from_host(ln.data(), ln.size());
  out.grp.from_host(gp.data(), gp.size());
  out.gptr.from_host(gptr.data(), gptr.size());
  out.glist.from_host(glist.data(), glist.size());
  AIRG_HIP(hipStreamSynchronize(s));
}

// block q: partial products of its item, by the tree of tree_dot_stage1; an
// item of a problem whose process is not running (active[grp] == 0, when
// active is given) leaves zero partials without reading anything: its w is
// zero there, so its products would be zero too
__global__ __launch_bounds__(256) void group_dots_stage1(const double* __restrict__ V, int64_t ldv,
                                                         int nv, const double* __restrict__ w,
                                                         const int64_t* __restrict__ start,
                                                         const int32_t* __restrict__ len,
                                                         const int32_t* __restrict__ grp,
                                                         const uint8_t* __restrict__ active,
                                                         double* __restrict__ part, int64_t nq) {
  __shared__ double red[kMaxDotVecs][4];
  const int t = threadIdx.x;
  if (active && !active[grp[blockIdx.x]]) {
    if (t < nv) part[(int64_t)t * nq + blockIdx.x] = 0.0;
    return;
  }
  const int64_t b = start[blockIdx.x];
  const int m = len[blockIdx.x];
  double w4[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) w4[q] = (4 * t + q < m) ? w[b + 4 * t + q] : 0.0;
  const int lane = t & 63, wave = t >> 6;
  for (int k = 0; k < nv; ++k) {
    const double* v = V + (int64_t)k * ldv + b;
    double p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = (4 * t + q < m) ? v[4 * t + q] * w4[q] : 0.0;
    const double ws = wave_tree((p[0] + p[1]) + (p[2] + p[3]));
    if (lane == 0) red[k][wave] = ws;
  }
  __syncthreads();
  if (t < nv) part[(int64_t)t * nq + blockIdx.x] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
}
// block (g, k): out[k G + g] = the partials of problem g's items, each thread
// adding its share of the list in order, then the shuffle tree and the waves
__global__ __launch_bounds__(256) void group_sum_kernel(const double* __restrict__ part, int64_t nq,
                                                        const int32_t* __restrict__ gptr,
                                                        const int32_t* __restrict__ glist, int G,
                                                        double* __restrict__ out) {
  __shared__ double red[4];
  const int g = blockIdx.x, k = blockIdx.y, t = threadIdx.x;
  const double* src = part + (int64_t)k * nq;
  double acc = 0.0;
  for (int q = gptr[g] + t; q < gptr[g + 1]; q += 256) acc = acc + src[glist[q]];
  const double ws = wave_tree(acc);
  if ((t & 63) == 0) red[t >> 6] = ws;
  __syncthreads();
  if (t == 0) out[(int64_t)k * G + g] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(256) void group_update_kernel(double* __restrict__ w,
                                                           const double* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ h, int nv,
                                                           int G, const int64_t* __restrict__ start,
                                                           const int32_t* __restrict__ len,
                                                           const int32_t* __restrict__ grp) {
  const int64_t b = start[blockIdx.x];
  const int m = len[blockIdx.x], g = grp[blockIdx.x];
  for (int e = threadIdx.x; e < m; e += 256) {
    const int64_t i = b + e;
    double acc = w[i];
    for (int k = 0; k < nv; ++k) acc = acc - h[(int64_t)k * G + g] * V[(int64_t)k * ldv + i];
    w[i] = acc;
  }
}
template <class ZT>
__global__ __launch_bounds__(256) void group_combine_kernel(double* __restrict__ x,
                                                            const ZT* __restrict__ Z, int64_t ldz,
                                                            const double* __restrict__ y, int nv,
                                                            int G, const int64_t* __restrict__ start,
                                                            const int32_t* __restrict__ len,
                                                            const int32_t* __restrict__ grp) {
  const int64_t b = start[blockIdx.x];
  const int m = len[blockIdx.x], g = grp[blockIdx.x];
  for (int e = threadIdx.x; e < m; e += 256) {
    const int64_t i = b + e;
    double acc = x[i];
    for (int k = 0; k < nv; ++k)
      acc = acc + y[(int64_t)k * G + g] * (double)Z[(int64_t)k * ldz + i];
    x[i] = acc;
  }
}
__global__ __launch_bounds__(256) void group_divide_kernel(double* __restrict__ y,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ d,
                                                           const int64_t* __restrict__ start,
                                                           const int32_t* __restrict__ len,
                                                           const int32_t* __restrict__ grp,
                                                           float* __restrict__ y32) {
  const int64_t b = start[blockIdx.x];
  const int m = len[blockIdx.x];
  const double dg = d[grp[blockIdx.x]];
  for (int e = threadIdx.x; e < m; e += 256) {
    const double v = dg != 0.0 ? x[b + e] / dg : 0.0;
    y[b + e] = v;
    if (y32) y32[b + e] = (float)v;
  }
}

size_t group_dots_work_size(const GroupItems& it) { return (size_t)kMaxDotVecs * (size_t)std::max<int64_t>(it.n, 1); }
void launch_group_dots(const double* V, int64_t ldv, int nv, const double* w, const GroupItems& it,
                       double* out, double* work, hipStream_t s, const uint8_t* active) {
  if (nv <= 0 || it.n <= 0) return;
  for (int k0 = 0; k0 < nv; k0 += kMaxDotVecs) {
    const int cnt = std::min(kMaxDotVecs, nv - k0);
    group_dots_stage1<<<(unsigned)it.n, 256, 0, s>>>(V + (int64_t)k0 * ldv, ldv, cnt, w,
                                                      it.start.get(), it.len.get(), it.grp.get(),
                                                      active, work, it.n);
    AIRG_CHECK_LAUNCH();
    group_sum_kernel<<<dim3((unsigned)it.G, (unsigned)cnt), 256, 0, s>>>(
        work, it.n, it.gptr.get(), it.glist.get(), it.G, out + (int64_t)k0 * it.G);
    AIRG_CHECK_LAUNCH();
  }
}
void launch_group_update(double* w, const double* V, int64_t ldv, const double* h, int nv,
                         const GroupItems& it, hipStream_t s) {
  if (nv <= 0 || it.n <= 0) return;
  group_update_kernel<<<(unsigned)it.n, 256, 0, s>>>(w, V, ldv, h, nv, it.G, it.start.get(),
                                                      it.len.get(), it.grp.get());
  AIRG_CHECK_LAUNCH();
}
template <class ZT>
static void launch_group_combine_t(double* x, const ZT* Z, int64_t ldz, const double* y, int nv,
                                   const GroupItems& it, hipStream_t s) {
  if (nv <= 0 || it.n <= 0) return;
  group_combine_kernel<ZT><<<(unsigned)it.n, 256, 0, s>>>(x, Z, ldz, y, nv, it.G, it.start.get(),
                                                           it.len.get(), it.grp.get());
  AIRG_CHECK_LAUNCH();
}
void launch_group_combine(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                          const GroupItems& it, hipStream_t s) {
  launch_group_combine_t(x, Z, ldz, y, nv, it, s);
}
void launch_group_combine(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                          const GroupItems& it, hipStream_t s) {
  launch_group_combine_t(x, Z, ldz, y, nv, it, s);
}
void launch_group_divide(double* y, const double* x, const double* d, const GroupItems& it,
                         hipStream_t s, float* y32) {
  if (it.n <= 0) return;
  group_divide_kernel<<<(unsigned)it.n, 256, 0, s>>>(y, x, d, it.start.get(), it.len.get(),
                                                      it.grp.get(), y32);
  AIRG_CHECK_LAUNCH();
}

// The fused sweeps of cgs_fused_kernel per problem: block q takes item q (at
// most 256 elements of problem grp[q], one per thread) and forms the item's
// partial products (MODE 0: V_k . w), or first updates w with that problem's
// coefficients (MODE 1: then V_k . w; MODE 2: then w . w); group_sum_kernel
// adds the partials per problem in list order.  An item of a problem whose
// process is not running (active given and active[grp] == 0) has w = 0 and
// coefficients 0: it leaves w as it is and zero partials, reading nothing.
template <int MODE, int NV>
__global__ __launch_bounds__(256) void group_fused_kernel(
    double* __restrict__ w, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
    int G, const int64_t* __restrict__ start, const int32_t* __restrict__ len,
    const int32_t* __restrict__ grp, const uint8_t* __restrict__ active, double* __restrict__ part,
    int64_t nq) {
  constexpr int CNT = MODE == 2 ? 1 : NV;
  __shared__ double red[CNT][4];
  const int t = threadIdx.x;
  const int g = grp[blockIdx.x];
  if (active && !active[g]) {
    if (t < CNT) part[(int64_t)t * nq + blockIdx.x] = 0.0;
    return;
  }
  const int64_t b = start[blockIdx.x];
  const bool in = t < len[blockIdx.x];
  const int64_t i = in ? b + t : b;  // in-range address for the padding lanes
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = V[(int64_t)k * ldv + i];
  double wi = w[i];
  if constexpr (MODE != 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) wi = wi - h[(int64_t)k * G + g] * v[k];
    if (in) w[i] = wi;
  }
  const int lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int k = 0; k < CNT; ++k) {
    const double s = wave_tree(in ? (MODE == 2 ? wi * wi : v[k] * wi) : 0.0);
    if (lane == 0) red[k][wave] = s;
  }
  __syncthreads();
  if (t < CNT) part[(int64_t)t * nq + blockIdx.x] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
}

template <int MODE, int NV>
static void launch_group_fused_nv(int nv, double* w, const double* V, int64_t ldv, const double* h,
                                  const GroupItems& it, const uint8_t* active, double* part,
                                  hipStream_t s) {
  if constexpr (NV > kFusedVecs) {
    fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  } else {
    if (nv != NV)
      return launch_group_fused_nv<MODE, NV + 1>(nv, w, V, ldv, h, it, active, part, s);
    group_fused_kernel<MODE, NV><<<(unsigned)it.n, 256, 0, s>>>(
        w, V, ldv, h, it.G, it.start.get(), it.len.get(), it.grp.get(), active, part, it.n);
  }
}

size_t group_fused_work_size(const GroupItems& it) {
  return (size_t)kFusedVecs * (size_t)std::max<int64_t>(it.n, 1);
}

template <int MODE>
static void launch_group_fused(double* w, const double* V, int64_t ldv, const double* h, int nv,
                               const GroupItems& it, double* out, double* work, hipStream_t s,
                               const uint8_t* active) {
  if (nv < 1 || nv > kFusedVecs) fail(AIRG_ERR_INTERNAL, "fused Gram-Schmidt takes 1 to 32 vectors");
  if (it.n <= 0) return;
  launch_group_fused_nv<MODE, 1>(nv, w, V, ldv, h, it, active, work, s);
  AIRG_CHECK_LAUNCH();
  group_sum_kernel<<<dim3((unsigned)it.G, (unsigned)(MODE == 2 ? 1 : nv)), 256, 0, s>>>(
      work, it.n, it.gptr.get(), it.glist.get(), it.G, out);
  AIRG_CHECK_LAUNCH();
}
void launch_group_fused_dots(const double* V, int64_t ldv, int nv, const double* w,
                             const GroupItems& it, double* out, double* work, hipStream_t s,
                             const uint8_t* active) {
  // MODE 0 neither writes w nor reads h
  launch_group_fused<0>(const_cast<double*>(w), V, ldv, nullptr, nv, it, out, work, s, active);
}
void launch_group_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                              const GroupItems& it, double* out, double* work, hipStream_t s,
                              const uint8_t* active) {
  launch_group_fused<1>(w, V, ldv, h, nv, it, out, work, s, active);
}
void launch_group_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                               const GroupItems& it, double* out, double* work, hipStream_t s,
                               const uint8_t* active) {
  launch_group_fused<2>(w, V, ldv, h, nv, it, out, work, s, active);
}

// mask[i] = 1 where any problem g0[i] .. g1[i] of 64-row group i is active
__global__ void group_mask_kernel(const int32_t* __restrict__ g0, const int32_t* __restrict__ g1,
                                  const uint8_t* __restrict__ active, int64_t n,
                                  uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t m = 0;
  for (int32_t p = g0[i]; p <= g1[i]; ++p) m |= active[p];
  mask[i] = m != 0 ? 1 : 0;
}
void launch_group_mask(const int32_t* g0, const int32_t* g1, const uint8_t* active, int64_t n,
                       uint8_t* mask, hipStream_t s) {
  if (n <= 0) return;
  group_mask_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(g0, g1, active, n, mask);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ permutations
__global__ void scatter_kernel(double* y, const double* x, const int32_t* perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[perm[i]] = x[i];
}
__global__ void gather_kernel(double* y, const double* x, const int32_t* perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[perm[i]];
}
void launch_scatter(double* y, const double* x, const int32_t* perm, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  scatter_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, perm, n);
  AIRG_CHECK_LAUNCH();
}
__global__ void scatter_i32_kernel(int32_t* y, const int32_t* x, const int32_t* perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[perm[i]] = x[i];
}
void launch_scatter_i32(int32_t* y, const int32_t* x, const int32_t* perm, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  scatter_i32_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, perm, n);
  AIRG_CHECK_LAUNCH();
}
void launch_gather(double* y, const double* x, const int32_t* perm, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  gather_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(y, x, perm, n);
  AIRG_CHECK_LAUNCH();
}

// K columns: ys[pos[i] * K + c] = b[c * ldb + i] and back; columns c >= kv
// are padding (zero in ys, not written back).
__global__ void scatter_cols_kernel(double* ys, const double* b, int64_t ldb, const int32_t* pos,
                                    int64_t n, int K, int kv) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t i = t / K;
  const int c = (int)(t % K);
  ys[(int64_t)pos[i] * K + c] = c < kv ? b[(int64_t)c * ldb + i] : 0.0;
}
__global__ void gather_cols_kernel(double* x, int64_t ldx, const double* xs, const int32_t* pos,
                                   int64_t n, int K, int kv) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K) return;
  const int64_t i = t / K;
  const int c = (int)(t % K);
  if (c < kv) x[(int64_t)c * ldx + i] = xs[(int64_t)pos[i] * K + c];
}
void launch_scatter_cols(double* ys, const double* b, int64_t ldb, const int32_t* pos, int64_t n,
                         int K, int kv, hipStream_t s) {
  if (n <= 0) return;
  scatter_cols_kernel<<<blocks_for(n * K, kBlock), kBlock, 0, s>>>(ys, b, ldb, pos, n, K, kv);
  AIRG_CHECK_LAUNCH();
}
void launch_gather_cols(double* x, int64_t ldx, const double* xs, const int32_t* pos, int64_t n,
                        int K, int kv, hipStream_t s) {
  if (n <= 0) return;
  gather_cols_kernel<<<blocks_for(n * K, kBlock), kBlock, 0, s>>>(x, ldx, xs, pos, n, K, kv);
  AIRG_CHECK_LAUNCH();
}

// Per-column sums of squares of an [n][K] array: block b sums rows
// b*R .. b*R+R-1 of every column sequentially per thread, the threads of a
// column combine in a fixed order, then one thread per column adds the block
// partials in order.
constexpr int kColRows = 4096;
__global__ __launch_bounds__(256) void col_sumsq_stage1(const double* x, int64_t n, int K,
                                                        double* part) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int c = t % K;
  const int lanes = 256 / K;  // threads per column
  const int q = t / K;
  const int64_t r0 = (int64_t)blockIdx.x * kColRows;
  double acc = 0.0;
  for (int64_t r = r0 + q; r < r0 + kColRows && r < n; r += lanes) {
    double v = x[r * K + c];
    acc = acc + v * v;
  }
  sh[t] = acc;
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int j = 0; j < lanes; ++j) s = s + sh[j * K + t];
    part[(int64_t)t * gridDim.x + blockIdx.x] = s;
  }
}
__global__ void col_sumsq_stage2(const double* part, int64_t nb, int K, double* out) {
  int c = threadIdx.x;
  if (c >= K) return;
  double s = 0.0;
  for (int64_t b = 0; b < nb; ++b) s = s + part[(int64_t)c * nb + b];
  out[c] = s;
}
size_t col_sumsq_work_size(int64_t n, int K) {
  return (size_t)K * (size_t)((n + kColRows - 1) / kColRows + 1);
}
void launch_col_sumsq(const double* x, int64_t n, int K, double* out, double* work, hipStream_t s) {
  if (K < 1 || K > 256 || (256 % K) != 0) fail(AIRG_ERR_INTERNAL, "bad column count");
  int64_t nb = (n + kColRows - 1) / kColRows;
  if (nb < 1) nb = 1;
  col_sumsq_stage1<<<(unsigned)nb, 256, 0, s>>>(x, n, K, work);
  AIRG_CHECK_LAUNCH();
  col_sumsq_stage2<<<1, 256, 0, s>>>(work, nb, K, out);
  AIRG_CHECK_LAUNCH();
}

__global__ void offset_copy_i32_kernel(int32_t* dst, const int32_t* src, int64_t n, int64_t add) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (int32_t)(src[i] + add);
}
void launch_offset_copy_i32(int32_t* dst, const int32_t* src, int64_t n, int64_t add,
                            hipStream_t s) {
  if (n <= 0) return;
  offset_copy_i32_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(dst, src, n, add);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ scans
// Three phases over chunks of 1024: chunk totals, a single-block exclusive scan
// of the totals, then per-chunk exclusive scans offset by the chunk prefix.
constexpr int kScanChunk = 1024;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  // 256 threads: Hillis-Steele inclusive scan in LDS
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int64_t a = (t >= o) ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int64_t incl = sh[t];
  if (total) *total = sh[255];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void scan_totals_kernel(const int64_t* in, int64_t n,
                                                          int64_t* totals) {
  __shared__ int64_t sh[256];
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + 4 * threadIdx.x;
  int64_t v = 0;
  for (int q = 0; q < 4; ++q)
    if (i0 + q < n) v += in[i0 + q];
  int64_t tot;
  block_exclusive_scan(v, sh, &tot);
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_single_kernel(int64_t* a, int64_t m) {
  // exclusive scan of a[0..m) in place by one block; a[m] = total
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  const int64_t per = (m + 255) / 256;
  const int64_t lo = t * per, hi = (lo + per < m) ? lo + per : m;
  int64_t v = 0;
  for (int64_t i = lo; i < hi; ++i) v += a[i];
  int64_t tot;
  int64_t base = block_exclusive_scan(v, sh, &tot);
  for (int64_t i = lo; i < hi; ++i) {
    int64_t x = a[i];
    a[i] = base;
    base += x;
  }
  if (t == 0) a[m] = tot;
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const int64_t* in, int64_t* out, int64_t n,
                                                         const int64_t* prefix) {
  __shared__ int64_t sh[256];
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + 4 * threadIdx.x;
  int64_t v[4];
  int64_t tsum = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = (i0 + q < n) ? in[i0 + q] : 0;
    tsum += v[q];
  }
  __syncthreads();  // in and out may alias: every read of this block is done
  int64_t base = block_exclusive_scan(tsum, sh, nullptr) + prefix[blockIdx.x];
  for (int q = 0; q < 4; ++q) {
    if (i0 + q < n) out[i0 + q] = base;
    base += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = prefix[gridDim.x];
}

size_t scan_work_size(int64_t n) {
  int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  return (size_t)(nb + 2);
}

void launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* work, hipStream_t s) {
  if (n <= 0) {
    launch_zero_bytes(out, sizeof(int64_t), s);
    return;
  }
  int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  scan_totals_kernel<<<(unsigned)nb, 256, 0, s>>>(in, n, work);
  AIRG_CHECK_LAUNCH();
  scan_single_kernel<<<1, 256, 0, s>>>(work, nb);
  AIRG_CHECK_LAUNCH();
  scan_apply_kernel<<<(unsigned)nb, 256, 0, s>>>(in, out, n, work);
  AIRG_CHECK_LAUNCH();
}

__global__ void offsets_to_i32_kernel(const int64_t* off, int32_t* rp, int64_t n1, int32_t* ovf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  int64_t v = off[i];
  if (v > 2147483647ll) {
    atomicOr(ovf, 1);
    v = 0;
  }
  rp[i] = (int32_t)v;
}
void launch_offsets_to_i32(const int64_t* off, int32_t* rowptr, int64_t n1, int32_t* overflow,
                           hipStream_t s) {
  if (n1 <= 0) return;
  offsets_to_i32_kernel<<<blocks_for(n1, kBlock), kBlock, 0, s>>>(off, rowptr, n1, overflow);
  AIRG_CHECK_LAUNCH();
}

}  // namespace airg
