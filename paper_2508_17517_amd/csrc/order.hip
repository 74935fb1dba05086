// Locality order of the solve numbering.
//
// The hierarchy is built in the input's numbering (which may be a random
// permutation).  For the solve only the block structure [F_l | C_l] of the
// nested numbering matters, so the F points of every level, and the points of
// the coarsest level, may be placed in any order.  They are placed by a key
// made of two breadth-first distances on the graph of A + A^T (ties by
// index), which keeps the gathers of every SpMV within a few neighbouring
// stretches of the vector that stay in cache.  Coarse points inherit the key
// of the fine point they are.  The two distances act as coordinates of the
// grid, and the inherited key is the point's index along a Hilbert curve
// through them: points near each other in both distances stay near each
// other in the order at every scale, so the rows of a coarse level, whose
// couplings reach many fine grid lines, still gather from a few cache lines
// each.  The coarsest level, ordered by its own graph for its LDS-staged
// products, takes the anti-diagonal key, whose 64-row groups span one
// narrow window of columns.
#include <algorithm>
#include <functional>

#include "grid_sync.hpp"
#include "kernels.hpp"

namespace airg {

// Expand one frontier: every unreached neighbour (in A or A^T) of a node
// q_in[t], t < n_in, gets level dn and joins q_out (count *n_out).  Waves
// take 64 consecutive frontier nodes from wave_first on, in steps of stride.
// A lane takes its node's neighbours 8 at a time: it loads their indices,
// then tries to claim each of them (a compare-and-swap from -1; a neighbour
// already reached keeps its level), all 8 in flight at once, and one atomic
// per wave then reserves the queue slots of the nodes the wave claimed.  So
// that no branch separates the 8 swaps, a slot with no neighbour (and a lane
// past the frontier's end) swaps on the level of a frontier node instead,
// which is never -1 and so never changes.  Which lane claims a node does not
// matter: the levels are the breadth-first distances either way.
constexpr int kExpandChunk = 8;
__device__ __forceinline__ void expand_frontier(const CSRView& A, const CSRView& At, int32_t* level,
                                                int32_t dn, const int32_t* q_in, int64_t n_in,
                                                int32_t* q_out, int32_t* n_out, int64_t wave_first,
                                                int64_t stride) {
  const int lane = threadIdx.x & 63;
  for (int64_t b = wave_first; b < n_in; b += stride) {
    const int64_t t = b + lane;
    const bool live = t < n_in;
    const int u = q_in[live ? t : t % n_in];
    int a0 = 0, na = 0, t0 = 0, deg = 0;
    if (live) {
      a0 = A.rowptr[u];
      na = A.rowptr[u + 1] - a0;
      t0 = At.rowptr[u];
      deg = na + (At.rowptr[u + 1] - t0);
    }
    int dmax = deg;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, 64));
    for (int j0 = 0; j0 < dmax; j0 += kExpandChunk) {
      int v[kExpandChunk];
#pragma unroll
      for (int c = 0; c < kExpandChunk; ++c) {
        const int j = j0 + c;
        v[c] = j < deg ? (j < na ? A.col[a0 + j] : At.col[t0 + j - na]) : u;
      }
      bool got[kExpandChunk];
#pragma unroll
      for (int c = 0; c < kExpandChunk; ++c) got[c] = atomicCAS(&level[v[c]], -1, dn) == -1;
      unsigned long long m[kExpandChunk];
      int total = 0;
#pragma unroll
      for (int c = 0; c < kExpandChunk; ++c) {
        m[c] = __ballot(got[c]);
        total += (int)__popcll(m[c]);
      }
      if (total == 0) continue;
      int base = 0;
      if (lane == 0) base = atomicAdd(n_out, total);
      base = __shfl(base, 0, 64);
#pragma unroll
      for (int c = 0; c < kExpandChunk; ++c) {
        const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m[c] >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m[c], 0u));
        if (got[c]) q_out[base + below] = v[c];
        base += (int)__popcll(m[c]);
      }
    }
  }
}

// One breadth-first step over the frontier of step d (q_in, count
// cnt[d % 3]) into q_out (count cnt[(d + 1) % 3]).  The counter for step
// d + 2 is cleared here.
__global__ void bfs_frontier_kernel(CSRView A, CSRView At, int32_t* level, int32_t d,
                                    const int32_t* q_in, int32_t* q_out, int32_t* cnt) {
  const int32_t n_in = cnt[d % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(d + 2) % 3] = 0;
  expand_frontier(A, At, level, d + 1, q_in, n_in, q_out, cnt + (d + 1) % 3,
                  (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63), (int64_t)gridDim.x * blockDim.x);
}

constexpr int kBfsThreads = 256;

// Steps d0, d0 + 1, .. of bfs_frontier_kernel in one launch, with a grid
// barrier after each, until a step finds its frontier empty or `steps` steps
// have run; ctl[0] receives the step it stopped at (d0 + steps when none was
// empty).  The frontier of step d is qa for even d and qb for odd d.  Every
// workgroup reads the same count after a barrier, so all leave together; a
// barrier wait that gives up sets *err and every workgroup leaves.
__global__ __launch_bounds__(kBfsThreads) void bfs_persistent_kernel(CSRView A, CSRView At, int32_t* level,
                                                                int32_t d0, int32_t steps, int32_t* qa,
                                                                int32_t* qb, int32_t* cnt, int32_t* ctl,
                                                                unsigned long long* bar, int* err,
                                                                int64_t spin_limit) {
  __shared__ int s_n;
  const int64_t wave_first = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t d = d0;
  for (int k = 0; k < steps; ++k, ++d) {
    if (threadIdx.x == 0) s_n = __hip_atomic_load(cnt + d % 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int n_in = s_n;
    if (n_in == 0) break;
    if (blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(cnt + (d + 2) % 3, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    expand_frontier(A, At, level, d + 1, (d & 1) ? qb : qa, n_in, (d & 1) ? qa : qb,
                    cnt + (d + 1) % 3, wave_first, stride);
    grid_barrier(bar, err, spin_limit);
    if (grid_failed(err)) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl[0] = d;
}

// Workgroups of a persistent breadth-first launch: enough for the wide
// frontiers, few enough that a barrier stays cheap, never more than the
// device holds at once (0 when that cannot be found out).
constexpr int kBfsBlocks = 64;
// steps per persistent launch (the host reads the state back once per launch)
constexpr int32_t kBfsSteps = 4096;

static int bfs_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, bfs_persistent_kernel, kBfsThreads, 0) != hipSuccess)
    return 0;
  return std::min(kBfsBlocks, cus * per);
}

// Steps from d on until a frontier is empty; d becomes a step at or after
// the first one whose frontier is empty (the callers restart from the
// levels, not from d).  Persistent launches when `persistent` (false when a
// barrier wait gave up: the levels are then incomplete), else one launch per
// step, 32 steps between reads of the count (steps past the end do nothing).
static bool bfs_steps(const CSR& A, const CSR& At, int32_t* level, int32_t& d, int32_t* const q[2],
                      int32_t* cnt, bool persistent, hipStream_t s) {
  const int64_t n = A.rows;
  if (persistent) {
    const int g = bfs_blocks();
    if (g <= 0) return false;
    DBuf<int32_t> ctl(2, s);
    DBuf<unsigned long long> bar(1, s);
    const int64_t lim = grid_spin_limit();
    for (;;) {
      bar.zero();
      ctl.zero();
      bfs_persistent_kernel<<<g, kBfsThreads, 0, s>>>(view(A), view(At), level, d, kBfsSteps, q[0], q[1],
                                                 cnt, ctl.get(), bar.get(), ctl.get() + 1, lim);
      AIRG_CHECK_LAUNCH();
      const std::vector<int32_t> h = ctl.host(2);
      if (h[1] != 0) return false;
      const bool done = h[0] < d + kBfsSteps;
      d = h[0];
      if (done) return true;
    }
  }
  const unsigned nb = blocks_for(std::min<int64_t>(n, 256 * 1024), kBlock);
  for (;;) {
    for (int k = 0; k < 32; ++k, ++d) {
      bfs_frontier_kernel<<<nb, kBlock, 0, s>>>(view(A), view(At), level, d, q[d & 1], q[(d + 1) & 1],
                                                cnt);
      AIRG_CHECK_LAUNCH();
    }
    if (fetch(cnt + d % 3, s) == 0) return true;
  }
}

// Largest level, ties to the smallest index, packed as level << 32 | ~index.
__global__ void far_node_kernel(const int32_t* level, int64_t n, unsigned long long* best) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t l = level[i];
  if (l < 0) return;
  unsigned long long k = ((unsigned long long)(uint32_t)l << 32) | (0xffffffffull - (uint64_t)i);
  atomicMax(best, k);
}

// Smallest index not reached yet.
__global__ void first_unvisited_kernel(const int32_t* level, int64_t n, unsigned long long* first) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && level[i] < 0) atomicMin(first, (unsigned long long)i);
}

// Start a frontier: level[i] = v, q[0] = i, cnt[slot] = 1.
__global__ void seed_frontier_kernel(int32_t* level, int64_t i, int32_t v, int32_t* q, int32_t* cnt,
                                     int slot) {
  level[i] = v;
  q[0] = (int32_t)i;
  cnt[0] = cnt[1] = cnt[2] = 0;
  cnt[slot] = 1;
}

// Breadth-first levels of the graph of A + A^T from src; unreached
// components restart from their smallest index at the next level.
static bool bfs_levels_pass(const CSR& A, const CSR& At, int64_t src, int32_t* level, bool persistent,
                            hipStream_t s) {
  const int64_t n = A.rows;
  launch_fill_i32(level, n, -1, s);
  DBuf<int32_t> qa(n, s), qb(n, s), cnt(3, s);
  DBuf<unsigned long long> red(1, s);
  int32_t d = 0;
  seed_frontier_kernel<<<1, 1, 0, s>>>(level, src, 0, qa.get(), cnt.get(), 0);
  AIRG_CHECK_LAUNCH();
  int32_t* const q[2] = {qa.get(), qb.get()};
  for (;;) {
    if (!bfs_steps(A, At, level, d, q, cnt.get(), persistent, s)) return false;
    // the frontier is empty: every component reached so far is done
    unsigned long long first = ~0ull;
    red.from_host(&first, 1);
    first_unvisited_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(level, n, red.get());
    AIRG_CHECK_LAUNCH();
    first = fetch(red.get(), s);
    if (first == ~0ull) return true;
    unsigned long long zero = 0;
    red.from_host(&zero, 1);
    far_node_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(level, n, red.get());
    AIRG_CHECK_LAUNCH();
    const int32_t dmax = (int32_t)(fetch(red.get(), s) >> 32);
    d = dmax + 1;
    seed_frontier_kernel<<<1, 1, 0, s>>>(level, (int64_t)first, d, q[d & 1], cnt.get(), d % 3);
    AIRG_CHECK_LAUNCH();
  }
}

// The persistent steps first; where a barrier wait gives up, the pass runs
// again with one launch per step.
void bfs_levels(const CSR& A, const CSR& At, int64_t src, int32_t* level, hipStream_t s) {
  if (!bfs_levels_pass(A, At, src, level, true, s)) bfs_levels_pass(A, At, src, level, false, s);
}

int64_t far_node(const int32_t* level, int64_t n, hipStream_t s) {
  DBuf<unsigned long long> red(1, s);
  unsigned long long zero = 0;
  red.from_host(&zero, 1);
  far_node_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(level, n, red.get());
  AIRG_CHECK_LAUNCH();
  unsigned long long k = fetch(red.get(), s);
  return (int64_t)(0xffffffffull - (k & 0xffffffffull));
}

// Smallest index on a given level.
__global__ void band_first_kernel(const int32_t* level, int64_t n, int32_t target,
                                  unsigned long long* first) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && level[i] == target) atomicMin(first, (unsigned long long)i);
}
// Node of largest dist among the nodes with band[i] == target (ties: smallest index).
__global__ void far_in_band_kernel(const int32_t* dist, const int32_t* band, int64_t n,
                                   int32_t target, unsigned long long* best) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || band[i] != target) return;
  unsigned long long k =
      ((unsigned long long)(uint32_t)dist[i] << 32) | (0xffffffffull - (uint64_t)i);
  atomicMax(best, k);
}
__global__ void combine_keys_kernel(int32_t* d1, const int32_t* d2, int64_t n, int64_t mult) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d1[i] = (int32_t)((int64_t)d1[i] * mult + d2[i]);
}
// Index of cell (x, y) along the Hilbert curve over a side x side square
// (side a power of two): at each scale the quadrant's place in the curve's
// visiting order is added, and the coordinates are turned into that
// quadrant's frame (flipped and/or transposed), so that the curve enters
// every sub-square where the previous one left it.
__device__ __forceinline__ uint32_t hilbert_index(uint32_t side, uint32_t x, uint32_t y) {
  uint32_t d = 0;
  for (uint32_t h = side >> 1; h > 0; h >>= 1) {
    const uint32_t rx = (x & h) ? 1u : 0u, ry = (y & h) ? 1u : 0u;
    d += h * h * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = side - 1 - x;
        y = side - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}
__global__ void hilbert_keys_kernel(int32_t* d1, const int32_t* d2, int64_t n, uint32_t side) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d1[i] = (int32_t)hilbert_index(side, (uint32_t)d1[i], (uint32_t)d2[i]);
}
// key = Hilbert index of (d1, d2) when asked for and both distances are below
// 2^15 (the index then fits 30 bits), else d1 * (d2max + 1) + d2 when that
// fits 31 bits; otherwise the key stays d1
static void combine_keys(int32_t* key, const int32_t* d2, int64_t n, int32_t d1max,
                         int32_t d2max, bool hilbert, hipStream_t s) {
  const unsigned nb = blocks_for(n, kBlock);
  const int32_t dm = std::max(d1max, d2max);
  if (hilbert && dm < (1 << 15)) {
    uint32_t side = 1;
    while (side <= (uint32_t)dm) side <<= 1;
    hilbert_keys_kernel<<<nb, kBlock, 0, s>>>(key, d2, n, side);
    AIRG_CHECK_LAUNCH();
    return;
  }
  const int64_t mult = (int64_t)d2max + 1;
  if (((int64_t)d1max + 1) * mult >= (int64_t)1 << 31) return;
  combine_keys_kernel<<<nb, kBlock, 0, s>>>(key, d2, n, mult);
  AIRG_CHECK_LAUNCH();
}

// Connected components of the graph of A + A^T: every node's label falls to
// the smallest index of its component by hooking (an edge whose ends carry
// different labels lowers the larger label's entry to the smaller) and
// pointer jumping, repeated until no edge joins two labels.  The fixed point
// does not depend on the order of the atomics.
__global__ void cc_hook_kernel(CSRView A, int32_t* lab, int32_t* changed) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= A.rows) return;
  bool any = false;
  for (int p = A.rowptr[u]; p < A.rowptr[u + 1]; ++p) {
    const int32_t lu = lab[u], lv = lab[A.col[p]];
    if (lu == lv) continue;
    atomicMin(&lab[lu > lv ? lu : lv], lu < lv ? lu : lv);
    any = true;
  }
  if (any) atomicOr(changed, 1);
}
__global__ void cc_jump_kernel(int32_t* lab, int64_t n, int32_t* changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t l = lab[i], ll = lab[l];
  if (ll != l) {
    lab[i] = ll;
    atomicOr(changed, 1);
  }
}
__global__ void cc_root_flag_kernel(const int32_t* lab, int64_t n, int64_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = lab[i] == i ? 1 : 0;
}
__global__ void cc_rank_kernel(const int32_t* lab, const int64_t* rank, int64_t n, int32_t* sid) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sid[i] = (int32_t)rank[lab[i]];
}
// sid[i] = rank of i's component (components ordered by smallest index);
// returns the number of components
static int component_ids(const CSR& A, int32_t* sid, hipStream_t s) {
  const int64_t n = A.rows;
  const unsigned nb = blocks_for(n, kBlock);
  DBuf<int32_t> flag(1, s);
  launch_iota(sid, n, s);
  for (;;) {
    launch_fill_i32(flag.get(), 1, 0, s);
    cc_hook_kernel<<<nb, kBlock, 0, s>>>(view(A), sid, flag.get());
    AIRG_CHECK_LAUNCH();
    const int32_t hooked = fetch(flag.get(), s);
    for (;;) {
      launch_fill_i32(flag.get(), 1, 0, s);
      cc_jump_kernel<<<nb, kBlock, 0, s>>>(sid, n, flag.get());
      AIRG_CHECK_LAUNCH();
      if (!fetch(flag.get(), s)) break;
    }
    if (!hooked) break;
  }
  DBuf<int64_t> rk(n + 1, s), work(scan_work_size(n), s);
  cc_root_flag_kernel<<<nb, kBlock, 0, s>>>(sid, n, rk.get());
  AIRG_CHECK_LAUNCH();
  launch_scan_i64(rk.get(), rk.get(), n, work.get(), s);
  const int64_t nc = fetch(rk.get() + n, s);
  cc_rank_kernel<<<nb, kBlock, 0, s>>>(sid, rk.get(), n, sid);
  AIRG_CHECK_LAUNCH();
  return (int)nc;
}

void locality_keys(const CSR& A, int32_t* key, hipStream_t s, bool hilbert) {
  const int64_t n = A.rows;
  if (n <= 0) return;
  // several components (a flow along the grid lines decouples them): the
  // keys of every component at once, then component-major
  {
    DBuf<int32_t> sid(n, s);
    const int nc = component_ids(A, sid.get(), s);
    if (nc > 1) {
      locality_keys_seg(A, sid.get(), nc, key, s, hilbert);
      const int64_t m = (int64_t)max_key(key, n, s) + 1;
      if ((int64_t)nc * m <= (int64_t)INT32_MAX) problem_major_keys(key, sid.get(), n, m, s);
      return;
    }
  }
  const unsigned nb = blocks_for(n, kBlock);
  CSR At;
  transpose(A, At, s);
  DBuf<int32_t> d2(n, s);
  DBuf<unsigned long long> red(1, s);
  // d1: distance from a far node (the node farthest from node 0)
  bfs_levels(A, At, 0, key, s);
  bfs_levels(A, At, far_node(key, n, s), key, s);
  const int64_t f1 = far_node(key, n, s);
  const int32_t d1max = fetch(key + f1, s);
  if (d1max < 2) return;
  // an end of the middle band: the band node farthest from some band node
  const int32_t mid = d1max / 2;
  unsigned long long first = ~0ull;
  red.from_host(&first, 1);
  band_first_kernel<<<nb, kBlock, 0, s>>>(key, n, mid, red.get());
  AIRG_CHECK_LAUNCH();
  first = fetch(red.get(), s);
  if (first == ~0ull) return;
  bfs_levels(A, At, (int64_t)first, d2.get(), s);
  unsigned long long zero = 0;
  red.from_host(&zero, 1);
  far_in_band_kernel<<<nb, kBlock, 0, s>>>(d2.get(), key, n, mid, red.get());
  AIRG_CHECK_LAUNCH();
  const int64_t f2 = (int64_t)(0xffffffffull - (fetch(red.get(), s) & 0xffffffffull));
  bfs_levels(A, At, f2, d2.get(), s);
  const int32_t d2max = fetch(d2.get() + far_node(d2.get(), n, s), s);
  combine_keys(key, d2.get(), n, d1max, d2max, hilbert, s);
}

// ------------------------------------------------------------------ ranking
__global__ void make_keys_kernel(const int8_t* state, const int64_t* fidx, const int32_t* key,
                                 int64_t n, uint64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && state[i] == 1)
    out[fidx[i]] = ((uint64_t)(uint32_t)key[i] << 32) | (uint64_t)fidx[i];
}
__global__ void pad_keys_kernel(uint64_t* k, int64_t from, int64_t to) {
  int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) k[i] = ~0ull;
}
__global__ void bitonic_step_kernel(uint64_t* keys, int64_t P, int64_t j, int64_t k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  int64_t l = i ^ j;
  if (l <= i) return;
  const bool asc = (i & k) == 0;
  uint64_t a = keys[i], b = keys[l];
  if ((a > b) == asc) {
    keys[i] = b;
    keys[l] = a;
  }
}
static void bitonic_sort(uint64_t* keys, int64_t P, hipStream_t s) {
  const unsigned nb = blocks_for(P, kBlock);
  for (int64_t k = 2; k <= P; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      bitonic_step_kernel<<<nb, kBlock, 0, s>>>(keys, P, j, k);
      AIRG_CHECK_LAUNCH();
    }
}
__global__ void rank_kernel(const uint64_t* sorted, int64_t nf, int32_t* rank) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nf) rank[sorted[r] & 0xffffffffull] = (int32_t)r;
}

// rank[f] = position of F point f when the F points are ordered by
// (key, F index); keys are unique, so any correct sort gives the same ranks.
void rank_f_points(const int8_t* state, const int64_t* fidx, const int32_t* key, int64_t n,
                   int64_t nf, int32_t* rank, hipStream_t s) {
  if (nf <= 0) return;
  int64_t P = 1;
  while (P < nf) P <<= 1;
  DBuf<uint64_t> keys(P, s);
  make_keys_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, fidx, key, n, keys.get());
  AIRG_CHECK_LAUNCH();
  if (P > nf) {
    pad_keys_kernel<<<blocks_for(P - nf, kBlock), kBlock, 0, s>>>(keys.get(), nf, P);
    AIRG_CHECK_LAUNCH();
  }
  bitonic_sort(keys.get(), P, s);
  rank_kernel<<<blocks_for(nf, kBlock), kBlock, 0, s>>>(keys.get(), nf, rank);
  AIRG_CHECK_LAUNCH();
}

__global__ void point_keys_kernel(const int32_t* key, int64_t n, uint64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ((uint64_t)(uint32_t)key[i] << 32) | (uint64_t)i;
}
void rank_points(const int32_t* key, int64_t n, int32_t* rank, hipStream_t s) {
  if (n <= 0) return;
  int64_t P = 1;
  while (P < n) P <<= 1;
  DBuf<uint64_t> keys(P, s);
  point_keys_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(key, n, keys.get());
  AIRG_CHECK_LAUNCH();
  if (P > n) {
    pad_keys_kernel<<<blocks_for(P - n, kBlock), kBlock, 0, s>>>(keys.get(), n, P);
    AIRG_CHECK_LAUNCH();
  }
  bitonic_sort(keys.get(), P, s);
  rank_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(keys.get(), n, rank);
  AIRG_CHECK_LAUNCH();
}
__global__ void invert_perm_kernel(const int32_t* pos, int64_t n, int32_t* inv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[pos[i]] = (int32_t)i;
}
void invert_perm(const int32_t* pos, int64_t n, int32_t* inv, hipStream_t s) {
  if (n <= 0) return;
  invert_perm_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(pos, n, inv);
  AIRG_CHECK_LAUNCH();
}

// key_next[c] = key[clist[c]]
__global__ void inherit_key_kernel(const int32_t* key, const int64_t* clist, int64_t nc,
                                   int32_t* out) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) out[c] = key[clist[c]];
}
void inherit_keys(const int32_t* key, const int64_t* clist, int64_t nc, int32_t* out,
                  hipStream_t s) {
  if (nc <= 0) return;
  inherit_key_kernel<<<blocks_for(nc, kBlock), kBlock, 0, s>>>(key, clist, nc, out);
  AIRG_CHECK_LAUNCH();
}

// ------------------------------------------------------------------ per-segment keys
// The keys of a graph made of independent segments (the problems of a
// batch: sid[i] is node i's segment, constant over long runs of indices)
// are the keys above taken in every segment at once: each breadth-first
// pass starts from one node per segment, and every choice of a start node
// is made per segment.  The per-segment choices reduce packed (value,
// index) words with atomics, first inside a wavefront whose lanes share a
// segment, so the result does not depend on thread order.
constexpr unsigned long long kNone = ~0ull;

__device__ __forceinline__ void seg_atomic_min(unsigned long long* slot, int sid, unsigned long long v,
                                               bool live) {
  const int s0 = __shfl(sid, 0, 64);
  const bool uniform = __all(sid == s0);
  if (uniform) {
    unsigned long long m = live ? v : kNone;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long u = __shfl_down(m, o, 64);
      m = u < m ? u : m;
    }
    if ((threadIdx.x & 63) == 0 && m != kNone) atomicMin(slot + s0, m);
  } else if (live) {
    atomicMin(slot + sid, v);
  }
}
__device__ __forceinline__ void seg_atomic_max(unsigned long long* slot, int sid, unsigned long long v,
                                               bool live) {
  const int s0 = __shfl(sid, 0, 64);
  const bool uniform = __all(sid == s0);
  if (uniform) {
    unsigned long long m = live ? v : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long u = __shfl_down(m, o, 64);
      m = u > m ? u : m;
    }
    if ((threadIdx.x & 63) == 0 && m != 0ull) atomicMax(slot + s0, m);
  } else if (live) {
    atomicMax(slot + sid, v);
  }
}
// smallest index per segment among the unreached nodes (all nodes when all)
__global__ void seg_first_kernel(const int32_t* level, const int32_t* sid, int64_t n, int all,
                                 unsigned long long* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int sg = in ? sid[i] : 0;
  seg_atomic_min(slot, sg, (unsigned long long)i, in && (all || level[i] < 0));
}
// per segment, the node of largest level (ties: smallest index); with band,
// only the nodes whose band value equals the segment's target count
__global__ void seg_far_kernel(const int32_t* level, const int32_t* band, const int32_t* target,
                               const int32_t* sid, int64_t n, unsigned long long* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int sg = in ? sid[i] : 0;
  bool live = in && level[i] >= 0;
  if (band && live) live = band[i] == target[sg];
  const unsigned long long k =
      live ? (((unsigned long long)(uint32_t)level[i] << 32) | (0xffffffffull - (uint64_t)i)) : 0ull;
  seg_atomic_max(slot, sg, k, live);
}
// per segment, the smallest index on the segment's target level
__global__ void seg_band_first_kernel(const int32_t* level, const int32_t* target, const int32_t* sid,
                                      int64_t n, unsigned long long* slot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < n;
  const int sg = in ? sid[i] : 0;
  seg_atomic_min(slot, sg, (unsigned long long)i, in && level[i] == target[sg]);
}
// start a frontier from a list of nodes at level v
__global__ void seed_list_kernel(int32_t* level, const int32_t* seeds, int ns, int32_t v, int32_t* q,
                                 int32_t* cnt, int slot) {
  for (int t = threadIdx.x; t < ns; t += blockDim.x) {
    level[seeds[t]] = v;
    q[t] = seeds[t];
  }
  if (threadIdx.x == 0) {
    cnt[0] = cnt[1] = cnt[2] = 0;
    cnt[slot] = ns;
  }
}

static std::vector<unsigned long long> seg_reduce(int nseg, unsigned long long init,
                                                  const std::function<void(unsigned long long*)>& run,
                                                  hipStream_t s) {
  DBuf<unsigned long long> slot(nseg, s);
  std::vector<unsigned long long> h(nseg, init);
  slot.from_host(h.data(), nseg);
  run(slot.get());
  return slot.host(nseg);
}

// breadth-first levels from one start node per segment (none where -1);
// unreached parts restart, every segment at once, from their smallest
// index at the next step
static bool bfs_levels_seg_pass(const CSR& A, const CSR& At, const std::vector<int32_t>& start,
                                const int32_t* sid, int nseg, int32_t* level, bool persistent,
                                hipStream_t s) {
  const int64_t n = A.rows;
  launch_fill_i32(level, n, -1, s);
  DBuf<int32_t> qa(n, s), qb(n, s), cnt(3, s), sd(std::max(nseg, 1), s);
  int32_t* const q[2] = {qa.get(), qb.get()};
  std::vector<int32_t> seeds;
  for (int32_t v : start)
    if (v >= 0) seeds.push_back(v);
  int32_t d = 0;
  for (;;) {
    if (seeds.empty()) return true;
    sd.from_host(seeds.data(), seeds.size());
    seed_list_kernel<<<1, 256, 0, s>>>(level, sd.get(), (int)seeds.size(), d, q[d & 1], cnt.get(),
                                       d % 3);
    AIRG_CHECK_LAUNCH();
    if (!bfs_steps(A, At, level, d, q, cnt.get(), persistent, s)) return false;
    // the frontier is empty: restart every segment that has unreached nodes
    const std::vector<unsigned long long> first = seg_reduce(nseg, kNone, [&](unsigned long long* sl) {
      seg_first_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(level, sid, n, 0, sl);
      AIRG_CHECK_LAUNCH();
    }, s);
    seeds.clear();
    for (unsigned long long f : first)
      if (f != kNone) seeds.push_back((int32_t)f);
    // the restarted parts begin one level past the deepest level so far
    if (!seeds.empty()) d = fetch(level + far_node(level, n, s), s) + 1;
  }
}

static void bfs_levels_seg(const CSR& A, const CSR& At, const std::vector<int32_t>& start,
                           const int32_t* sid, int nseg, int32_t* level, hipStream_t s) {
  if (!bfs_levels_seg_pass(A, At, start, sid, nseg, level, true, s))
    bfs_levels_seg_pass(A, At, start, sid, nseg, level, false, s);
}

void locality_keys_seg(const CSR& A, const int32_t* sid, int nseg, int32_t* key, hipStream_t s,
                       bool hilbert) {
  const int64_t n = A.rows;
  if (n <= 0) return;
  const unsigned nb = blocks_for(n, kBlock);
  CSR At;
  transpose(A, At, s);
  DBuf<int32_t> d2(n, s), tgt(nseg, s);
  auto unpack_index = [](unsigned long long k) { return (int32_t)(0xffffffffull - (k & 0xffffffffull)); };
  auto far = [&](const int32_t* lv, const int32_t* band) {
    return seg_reduce(nseg, 0ull, [&](unsigned long long* sl) {
      seg_far_kernel<<<nb, kBlock, 0, s>>>(lv, band, tgt.get(), sid, n, sl);
      AIRG_CHECK_LAUNCH();
    }, s);
  };
  // from each segment's smallest index, then from the node farthest from it
  std::vector<int32_t> start(nseg, -1);
  {
    const std::vector<unsigned long long> f = seg_reduce(nseg, kNone, [&](unsigned long long* sl) {
      seg_first_kernel<<<nb, kBlock, 0, s>>>(key, sid, n, 1, sl);
      AIRG_CHECK_LAUNCH();
    }, s);
    for (int g = 0; g < nseg; ++g) start[g] = f[g] == kNone ? -1 : (int32_t)f[g];
  }
  bfs_levels_seg(A, At, start, sid, nseg, key, s);
  std::vector<unsigned long long> fk = far(key, nullptr);
  for (int g = 0; g < nseg; ++g) start[g] = fk[g] ? unpack_index(fk[g]) : -1;
  bfs_levels_seg(A, At, start, sid, nseg, key, s);  // d1
  // an end of each segment's middle band
  fk = far(key, nullptr);
  std::vector<int32_t> mid(nseg, 0);
  int32_t d1max = 0;
  for (int g = 0; g < nseg; ++g) {
    const int32_t m = fk[g] ? (int32_t)(fk[g] >> 32) : 0;
    d1max = std::max(d1max, m);
    mid[g] = m / 2;
  }
  tgt.from_host(mid.data(), nseg);
  {
    const std::vector<unsigned long long> f = seg_reduce(nseg, kNone, [&](unsigned long long* sl) {
      seg_band_first_kernel<<<nb, kBlock, 0, s>>>(key, tgt.get(), sid, n, sl);
      AIRG_CHECK_LAUNCH();
    }, s);
    for (int g = 0; g < nseg; ++g) start[g] = f[g] == kNone ? -1 : (int32_t)f[g];
  }
  bfs_levels_seg(A, At, start, sid, nseg, d2.get(), s);
  fk = far(d2.get(), key);
  for (int g = 0; g < nseg; ++g) start[g] = fk[g] ? unpack_index(fk[g]) : -1;
  bfs_levels_seg(A, At, start, sid, nseg, d2.get(), s);  // d2
  const int32_t d2max = fetch(d2.get() + far_node(d2.get(), n, s), s);
  combine_keys(key, d2.get(), n, d1max, d2max, hilbert, s);
}

void locality_keys_by_component(const CSR& A, int32_t* key, hipStream_t s, bool hilbert) {
  const int64_t n = A.rows;
  if (n <= 0) return;
  DBuf<int32_t> sid(n, s);
  const int nc = component_ids(A, sid.get(), s);
  if (nc > 1) locality_keys_seg(A, sid.get(), nc, key, s, hilbert);
  else locality_keys(A, key, s, hilbert);
}

// ------------------------------------------------------------------ problem-major keys
// For a block-diagonal batch: key = p * mult + key with p the problem of the
// point, so that every ordered block of points keeps each problem together.
__global__ void problem_major_seg_kernel(int32_t* key, int64_t n, const int64_t* seg, int np,
                                         int64_t mult) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = np - 1;  // the largest p with seg[p] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  key[i] = (int32_t)((int64_t)lo * mult + key[i]);
}
__global__ void problem_major_pid_kernel(int32_t* key, const int32_t* pid, int64_t n, int64_t mult) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) key[i] = (int32_t)((int64_t)pid[i] * mult + key[i]);
}
__global__ void key_problem_kernel(const int32_t* key, int64_t n, int64_t mult, int32_t* pid) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pid[i] = (int32_t)(key[i] / mult);
}
__global__ void count_problems_kernel(const int8_t* state, const int32_t* key, int64_t n,
                                      int64_t mult, int np, int32_t* counts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (state && state[i] != 1)) return;
  const int64_t p = key[i] / mult;
  if (p >= 0 && p < np) atomicAdd(&counts[p], 1);
}

int32_t max_key(const int32_t* key, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  return fetch(key + far_node(key, n, s), s);
}
void problem_major_keys(int32_t* key, int64_t n, const std::vector<int64_t>& seg, int64_t mult,
                        hipStream_t s) {
  const int np = (int)seg.size() - 1;
  if (n <= 0 || np < 1) return;
  DBuf<int64_t> sd(seg.size(), s);
  sd.from_host(seg.data(), seg.size());
  problem_major_seg_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(key, n, sd.get(), np, mult);
  AIRG_CHECK_LAUNCH();
  AIRG_HIP(hipStreamSynchronize(s));
}
void problem_major_keys(int32_t* key, const int32_t* pid, int64_t n, int64_t mult, hipStream_t s) {
  if (n <= 0) return;
  problem_major_pid_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(key, pid, n, mult);
  AIRG_CHECK_LAUNCH();
}
void key_problems(const int32_t* key, int64_t n, int64_t mult, int32_t* pid, hipStream_t s) {
  if (n <= 0) return;
  key_problem_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(key, n, mult, pid);
  AIRG_CHECK_LAUNCH();
}
std::vector<int32_t> count_problems(const int8_t* state, const int32_t* key, int64_t n,
                                    int64_t mult, int np, hipStream_t s) {
  DBuf<int32_t> c(np, s);
  launch_fill_i32(c.get(), np, 0, s);
  if (n > 0) {
    count_problems_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, key, n, mult, np, c.get());
    AIRG_CHECK_LAUNCH();
  }
  return c.host(np);
}

// Nested positions with ordered F points, and the permuted prolongation map.
__global__ void nested_pos_ranked_kernel(const int8_t* state, const int64_t* fidx,
                                         const int64_t* cidx, const int32_t* frank, int64_t nF,
                                         const int32_t* pos_next, int64_t n, int32_t* pos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pos[i] = state[i] == 1 ? frank[fidx[i]] : (int32_t)(nF + pos_next[cidx[i]]);
}
void launch_nested_pos_ranked(const int8_t* state, const int64_t* fidx, const int64_t* cidx,
                              const int32_t* frank, int64_t nF, const int32_t* pos_next, int64_t n,
                              int32_t* pos, hipStream_t s) {
  if (n <= 0) return;
  nested_pos_ranked_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(state, fidx, cidx, frank, nF,
                                                                    pos_next, n, pos);
  AIRG_CHECK_LAUNCH();
}
__global__ void remap_ranked_kernel(const int32_t* cmap, const int32_t* pos_next,
                                    const int32_t* frank, int64_t nf, int32_t* out) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int32_t c = cmap[f];
  out[frank[f]] = c >= 0 ? pos_next[c] : -1;
}
void launch_remap_ranked(const int32_t* cmap, const int32_t* pos_next, const int32_t* frank,
                         int64_t nf, int32_t* out, hipStream_t s) {
  if (nf <= 0) return;
  remap_ranked_kernel<<<blocks_for(nf, kBlock), kBlock, 0, s>>>(cmap, pos_next, frank, nf, out);
  AIRG_CHECK_LAUNCH();
}

}  // namespace airg
