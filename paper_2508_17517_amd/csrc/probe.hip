// Streaming probes: the bandwidth a plain read stream and a plain copy reach
// on this device, measured with the library's own kernels.  They give the
// practical ceiling the sparse products are compared with (the products
// mostly read: matrix entries and gathered vector elements) and, on a buffer
// small enough to stay in the on-die caches, what repeated passes over a
// cache-resident operator can reach.
#include "kernels.hpp"

namespace airg {

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

// Sum of every 16-byte element (the sum is only kept so that the loads are
// not removed: it is written if it ever equals a value no input produces).
__global__ __launch_bounds__(kProbeBlock) void probe_read_kernel(const d2* __restrict__ src,
                                                                 int64_t n16, double* sink) {
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  double acc = 0.0;
  for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
    d2 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += v[u].x + v[u].y;
  }
  for (; i < n16; i += stride) {
    d2 v = src[i];
    acc += v.x + v.y;
  }
  if (acc == -1.0e300) sink[0] = acc;
}

__global__ __launch_bounds__(kProbeBlock) void probe_copy_kernel(const d2* __restrict__ src,
                                                                 d2* __restrict__ dst,
                                                                 int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
  int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
    d2 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

double stream_probe(int kind, const void* src, void* dst, int64_t bytes, int reps, int blocks,
                    hipStream_t s) {
  const int64_t n16 = bytes / 16;
  hipEvent_t e0, e1;
  AIRG_HIP(hipEventCreate(&e0));
  AIRG_HIP(hipEventCreate(&e1));
  auto launch = [&]() {
    if (kind == 0)
      probe_read_kernel<<<blocks, kProbeBlock, 0, s>>>(static_cast<const d2*>(src), n16,
                                                       static_cast<double*>(dst));
    else
      probe_copy_kernel<<<blocks, kProbeBlock, 0, s>>>(static_cast<const d2*>(src),
                                                       static_cast<d2*>(dst), n16);
    AIRG_CHECK_LAUNCH();
  };
  launch();  // warm-up
  AIRG_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) launch();
  AIRG_HIP(hipEventRecord(e1, s));
  AIRG_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  AIRG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

}  // namespace airg
