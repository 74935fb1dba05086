// AIRG hierarchy: per-level operators in two numberings.
//
// Setup numbering: the natural order of level l (F and C points in ascending
// level index, coarse index = rank among the C points).  All setup decisions
// are taken here.
//
// Solve numbering ("nested"): every level orders its unknowns F first, then
// its C points in the nested order of level l+1.  Level l's vector is then
// the suffix of the top-level vector starting at off_l = n_F(0) + ... +
// n_F(l-1), so restriction, prolongation and smoothing touch contiguous
// ranges and the V-cycle needs no gathers between levels.
#pragma once

#include <cmath>
#include <complex>
#include <limits>
#include <vector>

#include "common.hpp"
#include "dense.hpp"

namespace airg {

OpView op_view(const CSR& A, const DBuf<float>& v32, const DBuf<bf16>& v16, int prec);

// A solve-phase operator with its low-precision value copy and launch shape.
struct SolveOp {
  CSR m;
  DBuf<float> v32;
  DBuf<bf16> v16;
  int tpr = 1;
  OpView view(int prec) const { return op_view(m, v32, v16, prec); }
};

struct Level {
  int64_t n = 0, nF = 0, nC = 0;
  int64_t off = 0;
  bool coarsest = false;

  // setup numbering (freed after finalize unless keep_setup_data)
  CSR A;                    // level matrix (kept on the coarsest level)
  DBuf<int8_t> state;       // 1 = F, 2 = C
  DBuf<int64_t> fidx, cidx; // exclusive scans of the F / C flags
  CSR Afc_nat, Z_nat;
  CSR Aff_nat;              // A_ff in setup numbering when the solve order differs
  DBuf<int32_t> cmap_nat;

  // solve numbering
  CSR Aff, Z;               // Z rows in level l+1's nested order
  CSR Afc;                  // A_fc in solve numbering (only until B is built)
  CSR B;                    // A_fc + A_ff W: the F-point residual operator on e_c
  CSR Ahat;                 // assembled Ahat^{-1} (AIRG_SMOOTH_ASSEMBLED), A_ff's pattern
  DBuf<double> dinv;        // 1 / diag(A_ff) for the matrix-free Neumann smoother
  DBuf<float> dinv32;
  DBuf<int32_t> cmap;       // nested position on level l+1, or -1
  DBuf<int32_t> pos;        // setup index -> nested position on this level
  std::vector<double> alpha;
  std::vector<cplx> roots;
  // C-point smoothing (FC / FCF): A_cf and A_cc in setup numbering until
  // finalize; then A_cf (rows in level l+1's nested order, columns in F
  // order), A_cc (both in level l+1's nested order), its assembled
  // approximate inverse (AIRG_SMOOTH_ASSEMBLED) and, for FCF, A_fc
  CSR Acf_nat, Acc_nat;
  SolveOp cf, cc, hat_cc, fc;
  std::vector<double> alpha_c;  // GMRES polynomial coefficients of A_cc
  int64_t in_off = 0;           // this level's segment of the stacked residuals (levels >= 1)
  // launch shapes of the products: lanes per row (bits 0-7, 0 = row-block
  // kernel) and the XCD mapping (bit 8)
  int tpr_ff = 1, tpr_b = 1, tpr_z = 1, tpr_a = 1, tpr_hat = 1;
  // the coarsest level's A is stored in its solve order (pos) when true
  bool a_permuted = false;

  // low-precision copies of the solve operators' values (FP32 or BF16 storage)
  DBuf<float> ff32, b32, z32, a32, hat32;
  DBuf<bf16> ff16, b16, z16, a16, hat16;

  // statistics
  int64_t nnz_a = 0, nnz_fc = 0;
  int pmisr_rounds = 0;
  double trunc_rel = std::numeric_limits<double>::quiet_NaN();
};

struct Hierarchy {
  airg_params p{};
  hipStream_t s = nullptr;
  int64_t n0 = 0, nnz0 = 0;
  CSR A0;                   // top matrix, setup numbering
  CSR Aperm;                // top matrix, nested numbering
  int tpr_top = 1;
  std::vector<Level> levels;
  int64_t stacked_len = 0;  // sum of the level sizes below the top (C-point smoothing)
  double setup_ms = 0.0;
  double comp_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // a block-diagonal batch of problems: block p holds setup-numbering rows
  // seg[p] .. seg[p+1]-1 (empty for a single problem)
  std::vector<int64_t> seg;
  // with a batch ordered problem-major, every problem's unknowns in the
  // nested numbering as ranges (each level's F block, then the coarsest
  // block, problems ascending inside each); empty otherwise
  std::vector<GroupRange> granges;
  // with granges: for every 64-row group of the masked solve operators
  // (A_ff, B and Z of each level, the coarsest matrix, the top matrix; each
  // CSR's mask_off is its first group), the lowest and highest problem of
  // its rows
  DBuf<int32_t> mgp0, mgp1;
  int64_t mgroups = 0;
  // bumped whenever a solve operator's launch shape changes (captured
  // V-cycles of an older epoch are stale)
  uint64_t shape_epoch = 0;
};

// The coarsest level's Newton polynomial in one persistent launch (coarse.hip):
// the steps of the per-step form, the rows each workgroup owns and the
// barrier state.  ok is false where the launch does not apply (more than
// 65535 rows, an empty row, a row map, or entries that do not fit the
// registers of the workgroups the device holds at once).
enum { kCoarseReal = 0, kCoarsePair1 = 1, kCoarsePair2 = 2 };
struct CoarseStep {
  int32_t kind;   // kCoarseReal (a = 1 / theta, b = a folded final root's 1 / theta or 0),
                  // kCoarsePair1 (a = 2 Re z / |z|^2, b = 1 / |z|^2),
                  // kCoarsePair2 (a, b as Pair1, c = a folded final root's 1 / theta or 0)
  int32_t first;  // x starts here (it is not read)
  double a, b, c;
};
struct CoarsePlan {
  bool ok = false;
  int blocks = 0, nsteps = 0;
  int fin = 0, fin_first = 0;  // a final real root applied without a product
  double fin_inv = 0.0;
  int64_t n = 0;
  DBuf<int32_t> wrows;         // blocks + 1 row bounds
  DBuf<CoarseStep> steps;
  DBuf<double> pub;            // two vectors of n (FP64 or FP32 elements)
  DBuf<unsigned long long> bar;
  DBuf<int> err;
};
bool coarse_plan_build(CoarsePlan& pc, const CSR& A, const std::vector<cplx>& roots, int prec,
                       hipStream_t s);
template <class X>
void coarse_persistent_t(const CoarsePlan& pc, const OpView& A, const X* r, X* x, hipStream_t s);
// nonzero when a launch's barrier wait gave up (cleared by the call)
int coarse_plan_error(const CoarsePlan& pc, hipStream_t s);

// Build the hierarchy for A (device CSR, validated) with parameters p.
void build_hierarchy(Hierarchy& H, CSR&& A);
// Nested numbering and solve-form operators; frees setup data unless kept.
void finalize_hierarchy(Hierarchy& H);
// Build from host arrays in setup numbering (see airg_import_hierarchy).
void import_hierarchy(Hierarchy& H, int nlevels, const airg_level_info* infos,
                      const airg_level_arrays* arr);
// Upload a host CSR.
void upload_csr(CSR& out, int64_t rows, int64_t cols, int64_t nnz, const int32_t* rowptr,
                const int32_t* col, const double* val, hipStream_t s);
// Statistics.
void hierarchy_stats(const Hierarchy& H, airg_stats* st);

// Launch count and algorithmic traffic of a sequence of kernel launches: each
// matrix entry (12 bytes with its column), row pointer and vector element read
// or written once; flops count 2 per matrix entry plus the vector updates.
// `stored` counts what the kernels actually move: `saving` is subtracted for
// operators kept with compressed columns.
struct LaunchTally {
  int launches = 0;
  double bytes = 0.0, flops = 0.0, stored = 0.0;
  void add(double b, double f, double saving = 0.0) {
    ++launches;
    bytes += b;
    flops += f;
    stored += b - saving;
  }
};
inline double csr_bytes(int64_t rows, int64_t nnz, double vbytes = 8.0) {
  return (4.0 + vbytes) * nnz + 4.0 * (rows + 1);
}
// Bytes the compressed column form saves on one pass over A (at most 1 in 16
// row blocks keeps int32 columns; counted as if none did).
inline double col_saving(const OpView& A) {
  return A.col16 ? 2.0 * (double)A.nnz - 4.0 * (double)((A.rows + 63) / 64) : 0.0;
}

// Operator view of A in the storage precision prec (airg_precision): FP64
// values, or the FP32 / BF16 copy.
OpView op_view(const CSR& A, const DBuf<float>& v32, const DBuf<bf16>& v16, int prec);
// Bytes of one stored matrix value in precision prec.
inline double value_bytes(int prec) { return prec == AIRG_FP64 ? 8.0 : prec == AIRG_FP32 ? 4.0 : 2.0; }

// Coarse solver: x = q(A) r with the Newton roots (r, x device vectors of
// A.rows x K interleaved columns; w0, w1, t scratch of the same size).  X is
// the vector type.
template <class X>
void newton_apply_t(const OpView& A, int tpr, int K, const std::vector<cplx>& roots, const X* r,
                    X* x, X* w0, X* w1, X* t, hipStream_t s, LaunchTally* tally = nullptr);
inline void newton_apply_dev(const CSR& A, int tpr, const std::vector<cplx>& roots, const double* r,
                             double* x, double* w0, double* w1, double* t, hipStream_t s,
                             LaunchTally* tally = nullptr) {
  newton_apply_t<double>(opview(A), tpr, 1, roots, r, x, w0, w1, t, s, tally);
}

// Validates a device CSR and returns its diagonal; throws on error.
void validate_csr(const CSR& A, DBuf<double>& diag, hipStream_t s, bool top);

}  // namespace airg
