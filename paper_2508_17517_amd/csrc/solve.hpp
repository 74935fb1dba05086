// Solve phase: FGMRES preconditioned by AIRG V-cycles (device vectors in the
// nested numbering of the hierarchy).
#pragma once

#include "hierarchy.hpp"

namespace airg {

struct Workspace {
  int64_t ld = 0;      // leading dimension of the Krylov bases
  int restart = 0;
  DBuf<double> V, Zb;  // (restart + 1) and restart basis vectors
  DBuf<double> w, rr, sv, y0, y1;
  DBuf<double> cw0, cw1, ct;
  // FP32 vectors of the mixed-precision V-cycle
  DBuf<float> in32, e32, rr32, sv32, y032, y132, cw032, cw132, ct32;
  DBuf<double> bperm, xperm;
  DBuf<double> hbuf, ybuf, dot_work;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  ~Workspace();
};

void workspace_init(const Hierarchy& H, Workspace& W);

// One V-cycle: e = M r for a top-level vector `in` (nested numbering).
void vcycle(const Hierarchy& H, Workspace& W, const double* in, double* e);

// FGMRES on A x = b for one right-hand side (b, x in setup numbering, device).
int fgmres_solve(const Hierarchy& H, Workspace& W, const double* b, double* x, bool guess,
                 airg_solve_info* info);

// Replays one V-cycle's launches of a kernel class `reps` times between HIP
// events (airg_time_kernels).
int time_kernels(const Hierarchy& H, Workspace& W, int cls, int reps, airg_kernel_timing* out);

}  // namespace airg
