// The coarsest level's Newton polynomial (Sec. 2.3) in one persistent launch.
//
// The per-step form launches one product per Newton step, and every launch
// streams the whole coarsest matrix from HBM again (about 20 times per
// V-cycle).  Here one launch runs every step: each workgroup owns a range of
// rows, loads that range's matrix entries once (32 values per thread in
// registers, read at consecutive addresses through an LDS staging area; their
// 16-bit columns in LDS; 1024 threads), and keeps its rows' Newton vectors
// (w, t, x) in registers too.  Between steps only the vector that the next product gathers
// crosses workgroups: every workgroup writes its rows of it, and a grid-wide
// barrier (an arrival counter with a bounded wait) orders the writes before
// the next step's gathers.
//
// Row sums: thread t takes the entries t * 32 .. t * 32 + 31 of its
// workgroup's range in storage order and adds each row piece left to right;
// the thread that owns a row adds the pieces of its row in thread order.  The
// order is fixed, so results repeat bit for bit; it is not the per-step
// kernels' order, so the two forms agree to rounding.
//
// The steps, their coefficients and the vector each one updates are those of
// the per-step form (newton_apply_t): a real root theta updates
// x += w / theta and w -= A w / theta; a complex pair (a, b) first forms
// t = A w and x += (2a w - t) / (a^2 + b^2), then w -= (2a t - A t) / (a^2 +
// b^2); a final real root adds w / theta without a product; a real root that
// directly follows the last product is folded into it.
#include <atomic>
#include <type_traits>
#include <vector>

#include "grid_sync.hpp"
#include "hierarchy.hpp"
#include "kernels.hpp"

namespace airg {

namespace {

constexpr int kPcThreads = 1024;
constexpr int kPcEntries = 32;
constexpr int kPcCapacity = kPcThreads * kPcEntries;
// values staged per round of the initial load (32 KB in FP64)
constexpr int kPcStage = 4096;

__device__ __forceinline__ double to_x(double v, double) { return v; }
__device__ __forceinline__ float to_x(float v, float) { return v; }
__device__ __forceinline__ float to_x(bf16 v, float) { return __uint_as_float((uint32_t)v.bits << 16); }

template <class MV, class X>
__global__ __launch_bounds__(kPcThreads) void newton_persistent_kernel(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const MV* __restrict__ val, const int32_t* __restrict__ wrows,
    const CoarseStep* __restrict__ steps, int nsteps, int fin, double fin_inv, int fin_first,
    const X* r, X* __restrict__ x, X* pub, int64_t n, unsigned long long* bar, int* err,
    int64_t spin_limit) {
  // the workgroup's 16-bit columns (thread t's at t * 32 ..), its row starts,
  // the row pieces' sums (each thread's first and last piece, and the rows
  // that lie inside one thread's entries), and a staging area for the values
  __shared__ __align__(16) uint16_t scol[kPcCapacity];
  __shared__ int srp[kPcThreads + 1];
  __shared__ X pfirst[kPcThreads], plast[kPcThreads], prow[kPcThreads];
  __shared__ MV stage[kPcStage];
  const int t = threadIdx.x;
  const int r0 = wrows[blockIdx.x], r1 = wrows[blockIdx.x + 1];
  const int nrows = r1 - r0;
  const int e0 = rowptr[r0];
  const int cnt = rowptr[r1] - e0;
  const int q0 = t * kPcEntries;
  // every load of a phase is issued before any is used: one memory round
  // trip for the row starts and columns, one per staging round
  {
    int rp0 = 0, rp1 = 0;
    if (t <= nrows) rp0 = rowptr[r0 + t];
    if (t == 0) rp1 = rowptr[r1];
    int c[kPcEntries];
#pragma unroll
    for (int j = 0; j < kPcEntries; ++j) {
      const int q = t + j * kPcThreads;
      c[j] = q < cnt ? col[e0 + q] : 0;
    }
    if (t < nrows) srp[t] = rp0 - e0;
    if (t == 0) srp[nrows] = rp1 - e0;
#pragma unroll
    for (int j = 0; j < kPcEntries; ++j) {
      const int q = t + j * kPcThreads;
      if (q < cnt) scol[q] = (uint16_t)c[j];
    }
  }

  // this thread's values, read from HBM at consecutive addresses through
  // the staging area: round g stages entries g * kPcStage .., which belong to
  // threads g * kPcStage / 32 ..
  MV v[kPcEntries];
#pragma unroll
  for (int u = 0; u < kPcEntries; ++u) v[u] = MV{};
  constexpr int kPer = kPcStage / kPcThreads;
  for (int g = 0; g * kPcStage < cnt; ++g) {
    MV tmp[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int q = g * kPcStage + t + j * kPcThreads;
      tmp[j] = q < cnt ? val[e0 + q] : MV{};
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) stage[t + j * kPcThreads] = tmp[j];
    __syncthreads();
    if (t >= g * (kPcStage / kPcEntries) && t < (g + 1) * (kPcStage / kPcEntries)) {
      const int base = q0 - g * kPcStage;
#pragma unroll
      for (int u = 0; u < kPcEntries; ++u)
        if (q0 + u < cnt) v[u] = stage[base + u];
    }
  }
  __syncthreads();

  // the row of entry q0, and the pieces' boundaries: bit u is set where
  // entry q0 + u starts a row (u > 0; rows are never empty here)
  uint32_t bmask = 0;
  int rowa = r0;
  if (q0 < cnt) {
    int lo = 0, hi = nrows - 1;  // the last row that starts at or before q0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (srp[mid] <= q0) lo = mid;
      else hi = mid - 1;
    }
    rowa = r0 + lo;
    for (int rr = lo + 1; rr < nrows && srp[rr] < q0 + kPcEntries; ++rr)
      bmask |= 1u << (srp[rr] - q0);
  }

  // the row this thread owns, with its Newton vectors
  const int row = r0 + t;
  const bool own = t < nrows;
  int sj = 0, ej = 0;
  X w = X(0), tv = X(0), xr = X(0);
  if (own) {
    sj = srp[t];
    ej = srp[t + 1];
    w = r[row];
  }

  const X* src = r;
  for (int k = 0; k < nsteps; ++k) {
    const CoarseStep st = steps[k];
    // products of this thread's entries, one sum per row piece, eight
    // gathers at a time
    if (q0 < cnt) {
      X s = X(0);
      bool first_piece = true;
      int rw = rowa;
#pragma unroll
      for (int b8 = 0; b8 < kPcEntries / 8; ++b8) {
        const uint4 cc = *reinterpret_cast<const uint4*>(&scol[q0 + 8 * b8]);
        const uint32_t cw[4] = {cc.x, cc.y, cc.z, cc.w};
        X xv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int c = (int)((cw[i >> 1] >> (16 * (i & 1))) & 0xffffu);
          xv[i] = q0 + 8 * b8 + i < cnt ? src[c] : X(0);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int u = 8 * b8 + i;
          if (q0 + u < cnt) {
            if ((bmask >> u) & 1u) {
              if (first_piece) pfirst[t] = s;
              else prow[rw - r0] = s;
              first_piece = false;
              ++rw;
              s = X(0);
            }
            s = s + to_x(v[u], X(0)) * xv[i];
          }
        }
      }
      if (first_piece) pfirst[t] = s;
      else plast[t] = s;
    }
    __syncthreads();
    if (own) {
      // the row's pieces in thread order
      X sum = X(0);
      if (ej > sj) {
        const int t0 = sj / kPcEntries, t1 = (ej - 1) / kPcEntries;
        if (t0 == t1) {
          const int tend = min(cnt, (t0 + 1) * kPcEntries);
          sum = sj == t0 * kPcEntries ? pfirst[t0] : (ej == tend ? plast[t0] : prow[t]);
        } else {
          sum = sj == t0 * kPcEntries ? pfirst[t0] : plast[t0];
          for (int tt = t0 + 1; tt <= t1; ++tt) sum = sum + pfirst[tt];
        }
      }
      const X a = (X)st.a, b = (X)st.b, c = (X)st.c;
      X out;
      if (st.kind == kCoarseReal) {
        // a = 1 / theta, b = 1 / theta of a folded final root (or 0)
        X xi = (st.first ? X(0) : xr) + w * a;
        const X wn = w - sum * a;
        if (b != X(0)) xi = xi + wn * b;
        xr = xi;
        w = wn;
        out = wn;
      } else if (st.kind == kCoarsePair1) {
        // a = 2 Re / |z|^2, b = 1 / |z|^2
        tv = sum;
        xr = (st.first ? X(0) : xr) + (a * w - b * sum);
        out = sum;
      } else {
        // a, b as above, c = 1 / theta of a folded final root (or 0)
        const X wn = w - a * tv + b * sum;
        if (c != X(0)) xr = xr + wn * c;
        w = wn;
        out = wn;
      }
      if (k + 1 < nsteps) pub[(int64_t)(k & 1) * n + row] = out;
    }
    if (k + 1 < nsteps) {
      grid_barrier(bar, err, spin_limit);
      src = pub + (int64_t)(k & 1) * n;
    }
  }
  if (own) {
    if (fin) xr = (fin_first ? X(0) : xr) + (X)fin_inv * w;
    x[row] = xr;
  }
}

template <class MV, class X>
int max_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, newton_persistent_kernel<MV, X>, kPcThreads,
                                                   0) != hipSuccess)
    return 0;
  return cus * per;
}

}  // namespace

// polls of the barrier counter before a wait gives up (about a second)
constexpr int64_t kSpinDefault = int64_t(1) << 20;
static std::atomic<int64_t> g_grid_spin_limit{kSpinDefault};
void set_grid_spin_limit(int64_t polls) { g_grid_spin_limit.store(polls > 0 ? polls : kSpinDefault); }
int64_t grid_spin_limit() { return g_grid_spin_limit.load(); }

bool coarse_plan_build(CoarsePlan& pc, const CSR& A, const std::vector<cplx>& roots, int prec,
                       hipStream_t s) {
  pc.ok = false;
  const int64_t n = A.rows;
  const int m = (int)roots.size();
  if (n < 1 || n > 65535 || m < 2 || A.rmap.get() != nullptr) return false;
  // the steps, as the per-step form takes them
  std::vector<CoarseStep> st;
  pc.fin = 0;
  pc.fin_inv = 0.0;
  pc.fin_first = 0;
  bool first = true;
  for (int i = 0; i < m;) {
    const cplx z = roots[i];
    if (z.imag() == 0.0) {
      const double inv = 1.0 / z.real();
      if (i == m - 1) {
        pc.fin = 1;
        pc.fin_inv = inv;
        pc.fin_first = first ? 1 : 0;
        break;
      }
      double inv_last = 0.0;
      int skip = 0;
      if (i + 1 == m - 1 && roots[i + 1].imag() == 0.0) {
        inv_last = 1.0 / roots[i + 1].real();
        skip = 1;
      }
      st.push_back({kCoarseReal, first ? 1 : 0, inv, inv_last, 0.0});
      first = false;
      i += 1 + skip;
    } else {
      const double a = z.real(), b = z.imag();
      const double mod2 = a * a + b * b;
      const double c1 = 2.0 * a / mod2, c2 = 1.0 / mod2;
      st.push_back({kCoarsePair1, first ? 1 : 0, c1, c2, 0.0});
      first = false;
      if (i + 1 == m - 1) break;
      double inv_last = 0.0;
      int skip = 0;
      if (i + 2 == m - 1 && roots[i + 2].imag() == 0.0) {
        inv_last = 1.0 / roots[i + 2].real();
        skip = 1;
      }
      st.push_back({kCoarsePair2, 0, c1, c2, inv_last});
      i += 2 + skip;
    }
  }
  if (st.empty()) return false;
  // rows to workgroups: consecutive rows while the entries fit the registers
  std::vector<int32_t> rp(n + 1);
  AIRG_HIP(hipMemcpyAsync(rp.data(), A.rowptr.get(), (n + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> wr{0};
  for (int64_t i = 0; i < n; ++i) {
    const int64_t len = rp[i + 1] - rp[i];
    if (len < 1 || len > kPcCapacity) return false;
    const int64_t start = wr.back();
    if (i - start + 1 > kPcThreads || rp[i + 1] - rp[start] > kPcCapacity) wr.push_back((int32_t)i);
  }
  wr.push_back((int32_t)n);
  const int g = (int)wr.size() - 1;
  const int cap = prec == AIRG_FP64   ? max_resident_blocks<double, double>()
                  : prec == AIRG_FP32 ? max_resident_blocks<float, float>()
                                      : max_resident_blocks<bf16, float>();
  if (g > cap) return false;
  pc.blocks = g;
  pc.n = n;
  pc.nsteps = (int)st.size();
  pc.wrows.alloc(g + 1, s);
  pc.steps.alloc(st.size(), s);
  AIRG_HIP(hipMemcpyAsync(pc.wrows.get(), wr.data(), wr.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  AIRG_HIP(hipMemcpyAsync(pc.steps.get(), st.data(), st.size() * sizeof(CoarseStep),
                          hipMemcpyHostToDevice, s));
  pc.pub.alloc(2 * n, s);
  pc.bar.alloc(1, s);
  pc.err.alloc(1, s);
  AIRG_HIP(hipMemsetAsync(pc.bar.get(), 0, sizeof(unsigned long long), s));
  AIRG_HIP(hipMemsetAsync(pc.err.get(), 0, sizeof(int), s));
  AIRG_HIP(hipStreamSynchronize(s));
  pc.ok = true;
  return true;
}

template <class X>
void coarse_persistent_t(const CoarsePlan& pc, const OpView& A, const X* r, X* x, hipStream_t s) {
  if (!pc.ok || A.rows != pc.n) fail(AIRG_ERR_INTERNAL, "persistent coarse solve without a plan");
  X* pub = reinterpret_cast<X*>(pc.pub.get());
  const int64_t lim = grid_spin_limit();
  if constexpr (std::is_same<X, double>::value) {
    if (A.vt != VT_F64) fail(AIRG_ERR_INTERNAL, "FP64 coarse solve needs FP64 values");
    newton_persistent_kernel<double, double><<<pc.blocks, kPcThreads, 0, s>>>(
        A.rowptr, A.col, (const double*)A.val, pc.wrows.get(), pc.steps.get(), pc.nsteps, pc.fin,
        pc.fin_inv, pc.fin_first, r, x, pub, pc.n, pc.bar.get(), pc.err.get(), lim);
  } else {
    if (A.vt == VT_F32)
      newton_persistent_kernel<float, float><<<pc.blocks, kPcThreads, 0, s>>>(
          A.rowptr, A.col, (const float*)A.val, pc.wrows.get(), pc.steps.get(), pc.nsteps, pc.fin,
          pc.fin_inv, pc.fin_first, r, x, pub, pc.n, pc.bar.get(), pc.err.get(), lim);
    else if (A.vt == VT_BF16)
      newton_persistent_kernel<bf16, float><<<pc.blocks, kPcThreads, 0, s>>>(
          A.rowptr, A.col, (const bf16*)A.val, pc.wrows.get(), pc.steps.get(), pc.nsteps, pc.fin,
          pc.fin_inv, pc.fin_first, r, x, pub, pc.n, pc.bar.get(), pc.err.get(), lim);
    else
      fail(AIRG_ERR_INTERNAL, "FP32 coarse solve needs FP32 or BF16 values");
  }
  AIRG_CHECK_LAUNCH();
}

int coarse_plan_error(const CoarsePlan& pc, hipStream_t s) {
  if (!pc.ok) return 0;
  int e = 0;
  AIRG_HIP(hipMemcpyAsync(&e, pc.err.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  AIRG_HIP(hipStreamSynchronize(s));
  if (e != 0) launch_fill_i32(pc.err.get(), 1, 0, s);
  return e;
}

template void coarse_persistent_t<double>(const CoarsePlan&, const OpView&, const double*, double*,
                                          hipStream_t);
template void coarse_persistent_t<float>(const CoarsePlan&, const OpView&, const float*, float*,
                                         hipStream_t);

}  // namespace airg
