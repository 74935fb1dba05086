// Grid-wide barrier for persistent launches (the coarsest level's Newton
// steps, the breadth-first passes of the locality order).  Such a launch must
// not hold more workgroups than the device keeps resident at once.
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace airg {

// Wait until every workgroup has arrived: a device-scope release fence
// publishes the workgroup's writes before its arrival is counted, and a
// device-scope acquire fence after the wait makes the other workgroups'
// writes visible to it (on this GPU: a write-back of the XCD's L2 before the
// arrival, an invalidation after the wait).  The counter only grows:
// arrival number k belongs to the barrier that completes at the next
// multiple of the grid size, so it must hold 0 (or a multiple of the grid
// size) when the launch starts.  A wait that exceeds the poll limit, or sees
// another workgroup's failure, stops waiting and sets *err, so every
// workgroup always finishes.
__device__ inline void grid_barrier(unsigned long long* bar, int* err, int64_t spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned long long g = gridDim.x;
    const unsigned long long k = atomicAdd(bar, 1ull);
    const unsigned long long target = k - k % g + g;
    int64_t polls = 0;
    for (;;) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++polls > spin_limit) {
        atomicOr(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// The error flag as every thread of the workgroup sees it (one load by
// thread 0, shared through LDS), so that a workgroup leaves its loop as one.
__device__ inline bool grid_failed(const int* err) {
  __shared__ int s_err;
  if (threadIdx.x == 0)
    s_err = __hip_atomic_load(const_cast<int*>(err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool f = s_err != 0;
  __syncthreads();
  return f;
}

}  // namespace airg
