// Solve phase: FGMRES preconditioned by AIRG V-cycles (device vectors in the
// nested numbering of the hierarchy, K interleaved columns).
#pragma once

#include "hierarchy.hpp"
#include "kernels.hpp"

namespace airg {

// One captured V-cycle (see vcycle): its input and output vectors, whether
// the activity masks were on, and the launch-shape epoch it was captured in.
struct VcycleGraph {
  const double* in;
  double* e64;
  float* e32;
  bool in32_ready;
  bool mask;
  uint64_t epoch;
  hipGraphExec_t exec;
};

struct Workspace {
  int K = 1;           // interleaved columns (right-hand sides solved together)
  int64_t ld = 0;      // leading dimension of the Krylov bases (>= n K)
  int restart = 0;
  DBuf<double> V, Zb;  // (restart + 1) and restart basis vectors
  // the Z basis in FP32 (FGMRES with FP32 or BF16 storage in the V-cycle)
  DBuf<float> Zb32;
  bool z32 = false;
  DBuf<double> w, rr, sv, y0, y1;
  DBuf<double> cw0, cw1, ct;
  // the coarsest level's Newton steps in one persistent launch (single
  // right-hand side, single problem, params.coarse_persistent; ok where it fits)
  CoarsePlan pc;
  // FP32 vectors of the mixed-precision V-cycle
  DBuf<float> in32, e32, rr32, sv32, y032, y132, cw032, cw132, ct32;
  // each level's residual kept for C-point smoothing (stacked segments)
  DBuf<double> rin;
  DBuf<float> rin32;
  DBuf<double> bperm, xperm, nat;
  DBuf<double> hbuf, ybuf, gbuf, dot_work, col_work;
  DBuf<double> cdiv, cdot_work;  // per-column divisors and dot partials (K > 1)
  DBuf<double> cfused_work;      // partials of the fused per-column sweeps (K > 1)
  DBuf<double> fused_work;       // partials of the fused Gram-Schmidt sweeps (K = 1)
  GroupItems gitems;             // per-problem work items of a batch (K = 1)
  DBuf<double> gdot_work;
  GroupItems gitems_f;           // the same ranges in items of 256, for the fused sweeps
  DBuf<double> gfused_work;
  // activity of the problems and its 64-row-group masks (Hierarchy::mgp0);
  // with mask_on the V-cycle's masked products skip the inactive groups
  DBuf<uint8_t> active, gmask;
  bool mask_on = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // pinned host staging for the small per-iteration reads of the outer loop;
  // the single-process FGMRES uses two slots of pin_slot doubles at pin,
  // each with the event that marks its copy (evh), so that the next Arnoldi
  // step can be queued while the host reads the last one's coefficients
  double* pin = nullptr;
  size_t pin_n = 0, pin_slot = 0;
  hipEvent_t evh[2] = {nullptr, nullptr};
  // captured V-cycles (params.graph) and the stream they are captured on
  std::vector<VcycleGraph> graphs;
  hipStream_t cap = nullptr;
  ~Workspace();
};

void workspace_init(const Hierarchy& H, Workspace& W, int K = 1);

// One V-cycle: e = M r for a top-level vector `in` (nested numbering, W.K
// columns), launched kernel by kernel, or replayed from a captured HIP graph
// with params.graph.  The output goes to e64, or with FP32 or BF16 storage
// to e32 in FP32 when e32 is given; in32_ready says that W.in32 already holds
// (float) in.
void vcycle(const Hierarchy& H, Workspace& W, const double* in, double* e64,
            float* e32 = nullptr, bool in32_ready = false);

// The outer solve of A x = b for W.K right-hand sides solved together: column
// c of b starts at b + c ldb and of x at x + c ldx (setup numbering, device);
// only the first kvalid columns are read and written.  With K > 1 every
// column runs its own FGMRES (or Richardson) process with its own stopping
// test, iteration count and restarts, while the V-cycle, the top-level
// product and the orthogonalisation kernels cover all K columns per launch.
// A batch of problems (H.seg) ordered problem-major (H.granges) likewise runs
// one process per problem, with kernels over each problem's ranges of the
// nested numbering; otherwise one process runs over the block-diagonal
// system until every problem reaches |r_p| <= rtol |b_p|.  info receives
// one entry per column or problem.
int fgmres_solve(const Hierarchy& H, Workspace& W, const double* b, int64_t ldb, double* x,
                 int64_t ldx, int kvalid, bool guess, airg_solve_info* info);

// Replays one V-cycle's launches of a kernel class `reps` times between HIP
// events (airg_time_kernels).
int time_kernels(const Hierarchy& H, Workspace& W, int cls, int reps, airg_kernel_timing* out);
// Launch-shape tuner (see airg_autotune) and its manual setter.
int autotune(Hierarchy& H, Workspace& W, int reps, std::vector<airg_tune_entry>& out);
void set_lanes(Hierarchy& H, int level, int op, int lanes, int xcd_map, int lds);

}  // namespace airg
