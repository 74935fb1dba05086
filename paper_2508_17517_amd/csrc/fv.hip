// Upwind finite-volume discretisation of v.grad(u) = 0 on an nx x ny grid of
// square cells (paper Eqs. advection and advection_bc; fluxes divided by the
// cell size h, inflow faces on the right-hand side), assembled on the device,
// and the gradient contractions of the differentiable solve.
//
// Unknown k = j nx + i.  Row k: (vx + vy) u_k - vx u_{k-1} [i > 0]
// - vy u_{k-nx} [j > 0]; b_k = vx g_W(j) [i = 0] + vy g_S(i) [j = 0], with
// v = (cos theta, sin theta).  Entries with a zero coefficient are not stored.
#include <cmath>
#include <mutex>

#include "kernels.hpp"

namespace airg {

__device__ __forceinline__ int64_t fv_rowptr(int64_t k, int64_t nx, bool has_s, bool has_w) {
  // rows before k holding a south entry (k' >= nx) and a west entry (k' % nx != 0)
  int64_t s = has_s ? (k > nx ? k - nx : 0) : 0;
  int64_t w = has_w ? k - (k + nx - 1) / nx : 0;
  return k + s + w;
}

__global__ void fv_assemble_kernel(int64_t nx, int64_t ny, double vx, double vy, double dvx,
                                   double dvy, const double* gw, const double* gs, int32_t* rowptr,
                                   int32_t* col, double* val, double* b, double* dval, double* db) {
  const int64_t n = nx * ny;
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n) return;
  const bool has_s = vy != 0.0, has_w = vx != 0.0;
  rowptr[k] = (int32_t)fv_rowptr(k, nx, has_s, has_w);
  if (k == n) return;
  const int64_t i = k % nx, j = k / nx;
  int64_t p = fv_rowptr(k, nx, has_s, has_w);
  if (has_s && j > 0) {
    col[p] = (int32_t)(k - nx);
    val[p] = -vy;
    if (dval) dval[p] = -dvy;
    ++p;
  }
  if (has_w && i > 0) {
    col[p] = (int32_t)(k - 1);
    val[p] = -vx;
    if (dval) dval[p] = -dvx;
    ++p;
  }
  col[p] = (int32_t)k;
  val[p] = vx + vy;
  if (dval) dval[p] = dvx + dvy;
  double bk = 0.0, dbk = 0.0;
  if (has_w && i == 0) {
    bk = bk + vx * gw[j];
    dbk = dbk + dvx * gw[j];
  }
  if (has_s && j == 0) {
    bk = bk + vy * gs[i];
    dbk = dbk + dvy * gs[i];
  }
  b[k] = bk;
  if (db) db[k] = dbk;
}

int64_t fv_nnz(int64_t nx, int64_t ny, double theta) {
  const double vx = std::cos(theta), vy = std::sin(theta);
  const int64_t n = nx * ny;
  return n + (vy != 0.0 ? (ny - 1) * nx : 0) + (vx != 0.0 ? (nx - 1) * ny : 0);
}

void fv_assemble(int64_t nx, int64_t ny, double theta, const double* gw, const double* gs,
                 int32_t* rowptr, int32_t* col, double* val, double* b, double* dval, double* db,
                 hipStream_t s) {
  const double vx = std::cos(theta), vy = std::sin(theta);
  const double dvx = -std::sin(theta), dvy = std::cos(theta);
  const int64_t n = nx * ny;
  fv_assemble_kernel<<<blocks_for(n + 1, kBlock), kBlock, 0, s>>>(nx, ny, vx, vy, dvx, dvy, gw, gs,
                                                                 rowptr, col, val, b, dval, db);
  AIRG_CHECK_LAUNCH();
}

// r_k = db_k - (dA u)_k for the theta contraction lam^T (db/dtheta - dA/dtheta u)
__global__ void fv_theta_terms_kernel(const int32_t* rowptr, const int32_t* col, const double* dval,
                                      const double* db, const double* u, int64_t n, double* r) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t = 0.0;
  for (int p = rowptr[k]; p < rowptr[k + 1]; ++p) t = t + dval[p] * u[col[p]];
  r[k] = db[k] - t;
}
__global__ void fv_inflow_grads_kernel(int64_t nx, int64_t ny, double vx, double vy,
                                       const double* lam, double* dgw, double* dgs) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ny) dgw[t] = vx != 0.0 ? vx * lam[t * nx] : 0.0;
  if (t < nx) dgs[t] = vy != 0.0 ? vy * lam[t] : 0.0;
}

void fv_gradients(int64_t nx, int64_t ny, double theta, const int32_t* rowptr, const int32_t* col,
                  const double* dval, const double* db, const double* u, const double* lam,
                  double* dgw, double* dgs, double* dtheta, hipStream_t s) {
  const int64_t n = nx * ny;
  const double vx = std::cos(theta), vy = std::sin(theta);
  const int64_t m = nx > ny ? nx : ny;
  fv_inflow_grads_kernel<<<blocks_for(m, kBlock), kBlock, 0, s>>>(nx, ny, vx, vy, lam, dgw, dgs);
  AIRG_CHECK_LAUNCH();
  DBuf<double> r(n, s), work(dot_work_size(n, 1), s);
  fv_theta_terms_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(rowptr, col, dval, db, u, n, r.get());
  AIRG_CHECK_LAUNCH();
  launch_tree_dots(lam, 0, 1, r.get(), n, dtheta, work.get(), s);
  AIRG_HIP(hipStreamSynchronize(s));
}

// ---- the same gradients without allocating --------------------------------
// The theta terms r (n doubles) and the partial sums of lam . r live in one
// file-scope device array instead of stream-ordered allocations.  Every
// device that runs the entry point holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is a host-side stand-in).
constexpr int64_t kNoallocWorkDoubles = 2 * ((kFvNoallocMaxN + 1023) / 1024) + 8;
static __device__ __align__(256) double scratch[kFvNoallocMaxN + kNoallocWorkDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device, looked up once per device.
double* scratch_on_current_device() {
  int dev = 0;
  AIRG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(AIRG_ERR_INVALID, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    AIRG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(AIRG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

void fv_gradients_noalloc(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                          const int32_t* col, const double* dval, const double* db, const double* u,
                          const double* lam, double* dgw, double* dgs, double* dtheta, hipStream_t s) {
  const int64_t n = nx * ny;
  if (n > kFvNoallocMaxN) fail(AIRG_ERR_INVALID, "grid beyond the no-allocation limit of 4194304 unknowns");
  if (dot_work_size(n, 1) > (size_t)kNoallocWorkDoubles)
    fail(AIRG_ERR_INTERNAL, "no-allocation scratch too small for the dot partials");
  double* base = scratch_on_current_device();
  double* r = base;
  double* work = base + kFvNoallocMaxN;
  const double vx = std::cos(theta), vy = std::sin(theta);
  const int64_t m = nx > ny ? nx : ny;
  fv_inflow_grads_kernel<<<blocks_for(m, kBlock), kBlock, 0, s>>>(nx, ny, vx, vy, lam, dgw, dgs);
  AIRG_CHECK_LAUNCH();
  fv_theta_terms_kernel<<<blocks_for(n, kBlock), kBlock, 0, s>>>(rowptr, col, dval, db, u, n, r);
  AIRG_CHECK_LAUNCH();
  launch_tree_dots(lam, 0, 1, r, n, dtheta, work, s);
}

}  // namespace airg
