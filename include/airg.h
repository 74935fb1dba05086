/*
 * airg.h -- C ABI of the MI355X AIRG reduction-multigrid solver.
 *
 * The library solves A x = b for a sparse nonsymmetric A (for example an
 * upwind discretisation of v.grad(u) = 0, the paper's Eqs. advection and
 * advection_bc) with FGMRES preconditioned by AIRG V-cycles:
 *   - setup: PMISR DDC CF splitting (Sec. 2.1), GMRES-polynomial smoother
 *     coefficients by Arnoldi (Sec. 2.2, Eq. gmres_poly), the fixed-sparsity
 *     assembled inverse (Eq. fixed_sparsity), the approximate ideal restrictor
 *     Z = -A_cf Ahat^{-1} (Eq. z), one-point prolongation, A_coarse = R A P with
 *     relative drop and lumping, and automatic truncation with a high-order
 *     Newton-form coarse polynomial (Sec. 2.3, 2.4);
 *   - solve: V-cycles with only up F-point smoothing (Eq. f_point), the
 *     polynomials applied matrix-free (or the assembled Ahat^{-1}), inside
 *     FGMRES or the paper's undamped Richardson.
 *
 * Conventions
 *   - Every function returns an int status: AIRG_OK (0), a warning (> 0) or an
 *     error (< 0).  Nothing throws across the ABI.  airg_last_error() returns
 *     the message of the most recent error on the calling thread.
 *   - Matrices are CSR with int32 row pointers and column indices, the columns
 *     of each row strictly ascending, every row holding a nonzero diagonal.
 *   - Vectors are FP64.  Solve-phase vectors (b, x, w, lam) are DEVICE pointers
 *     on the current HIP device; setup matrices may be host or device pointers
 *     (flag on_device).
 *   - All device work is enqueued on the hip_stream given at setup (NULL: the
 *     null stream); a call returns after its results are complete.
 *   - A handle is not re-entrant: calls on one handle must not overlap.
 *     Separate handles are independent.
 */
#ifndef AIRG_H
#define AIRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AIRG_MAX_LEVELS 64

enum airg_status {
  AIRG_OK = 0,
  AIRG_NOT_CONVERGED = 1,   /* max_it reached; x holds the last iterate */
  AIRG_ERR_INVALID = -1,    /* bad shape, pointer, parameter or CSR structure */
  AIRG_ERR_ZERO_DIAG = -2,  /* a level matrix has a zero or missing diagonal */
  AIRG_ERR_NONFINITE = -3,  /* NaN or Inf in the matrix or a right-hand side */
  AIRG_ERR_HIP = -4,        /* a HIP runtime call failed (code in the message) */
  AIRG_ERR_NOMEM = -5,      /* device allocation failed */
  AIRG_ERR_BREAKDOWN = -6,  /* unrecoverable Krylov breakdown */
  AIRG_ERR_INTERNAL = -7
};

typedef enum { AIRG_FP64 = 0, AIRG_FP32 = 1, AIRG_BF16 = 2 } airg_precision;

typedef struct airg_ctx* airg_handle;

/* Solver options: one field per option of the paper's solver (Sec. 3 option
 * set); airg_params_default() fills the defaults listed here. */
typedef struct {
  double strong_threshold;   /* theta_s of the strength test, 0.99 (Sec. 2.1) */
  double ddc_fraction;       /* F points converted per DDC pass, 0.01 (Sec. 2.1) */
  double a_drop;             /* relative drop on A_coarse, 1e-6 (Sec. 2) */
  double r_drop;             /* relative drop on R, 0.01 (value not in the paper) */
  double trunc_tol;          /* automatic truncation tolerance, 1e-2; <= 0 disables (Sec. 2.4) */
  double rtol;               /* relative tolerance of the outer loop on |b - A x|, 1e-10 */
  uint64_t seed;             /* every random draw of the setup, 17517 */
  int64_t min_coarse_rows;   /* a level this small is always the coarsest, 64 */
  int32_t ddc_its;           /* DDC passes, 2 */
  int32_t lump;              /* lump dropped A_coarse entries to the diagonal, 1 */
  int32_t poly_order;        /* smoother polynomial degree d, 4 */
  int32_t coarse_poly_order; /* Newton coarse polynomial degree, 20 */
  int32_t trunc_start_level; /* first level tested for truncation, 1 */
  int32_t max_levels;        /* <= AIRG_MAX_LEVELS, 64 */
  int32_t added_roots;       /* extra copies of outlying Newton roots, 1 */
  int32_t precision;         /* airg_precision of the V-cycle storage, AIRG_FP64 */
  int32_t max_it;            /* outer iteration cap (V-cycles), 500 */
  int32_t restart;           /* FGMRES restart length, 30 (unused by Richardson) */
  int32_t keep_setup_data;   /* keep level data in setup numbering for export, 0 */
  int32_t locality_order;    /* order each level's F points and the coarsest level's
                                points in the solve numbering by a locality key of two
                                breadth-first distances on A + A^T (cache locality of the
                                SpMV gathers; the hierarchy itself is unchanged), 1 */
  int32_t outer;             /* airg_outer: the outer iteration, AIRG_OUTER_FGMRES */
  int32_t smoother;          /* airg_smoother: the F-point smoother, AIRG_SMOOTH_POLY */
  int32_t inverse_type;      /* airg_inverse: the polynomial approximating A_ff^{-1},
                                AIRG_INVERSE_ARNOLDI */
  int32_t smooth_type;       /* airg_smooth_type: the up-smooths of each level,
                                AIRG_SMOOTH_TYPE_F */
  double atol;               /* absolute tolerance of the outer loop: a residual norm at
                                or below max(rtol |b|, atol) stops it, 1e-50 (Sec. 3
                                option set) */
  int32_t graph;             /* 1: replay each V-cycle from a captured HIP graph (captured
                                on first use per pair of vectors, recaptured after a
                                launch-shape change; the same launches, bit for bit the
                                same results); 0: launch its kernels one by one, 0 */
  int32_t stagnation_check;  /* 1: a process (right-hand side, problem) whose true residual
                                norm falls by less than 1% over a restart cycle (Richardson:
                                over `restart` steps) stops there, not converged, with
                                airg_solve_info.stagnated set; 0: only rtol, atol and max_it
                                stop it, 0 */
  int32_t coarse_persistent; /* 1: apply the coarsest level's Newton polynomial (Sec. 2.3) in
                                one persistent launch that keeps the coarsest matrix in
                                registers across its steps, with a grid-wide barrier between
                                steps, where it fits (one right-hand side of a single problem,
                                at most 65535 coarsest rows, no empty row, 32 entries per
                                thread of the workgroups the device holds at once); the same
                                steps as the per-step launches, rows summed in another fixed
                                order.  Such a launch needs the whole device: solves of other
                                handles that overlap it on other streams may fail with
                                AIRG_ERR_INTERNAL.  0: one product launch per step (faster on
                                the MI355X: a barrier across its XCDs costs about as much as a
                                launch), 0 */
  int32_t lookahead;         /* 1: the outer FGMRES of one right-hand side of a single problem
                                queues Arnoldi step j + 1 on the device before it reads step
                                j's coefficients back, when the residual estimates predict
                                that step j does not converge (the GPU then works while the
                                host updates the least-squares problem); the same results bit
                                for bit, a wrong prediction costs one step's work; 0: every
                                step waits for the host, 1 */
} airg_params;

/* The polynomial approximation of A_ff^{-1} in the smoother and in Ahat^{-1}.
 * AIRG_INVERSE_ARNOLDI: the GMRES polynomial of AIRG (Sec. 2.2).
 * AIRG_INVERSE_NEUMANN: nAIR's Neumann polynomial of the same degree d (the
 * paper's comparison, Sec. 3.3), read as the Jacobi-scaled series
 * sum_{k=0}^{d} N^k D^{-1} with D = diag(A_ff), N = I - D^{-1} A_ff; matrix-free
 * it is d + 1 Jacobi sweeps from zero, assembled it keeps the powers of N on
 * A_ff's pattern as Eq. fixed_sparsity does. */
typedef enum { AIRG_INVERSE_ARNOLDI = 0, AIRG_INVERSE_NEUMANN = 1 } airg_inverse;

/* F-point smoothers.  AIRG_SMOOTH_POLY applies the GMRES polynomial
 * matrix-free (d products with A_ff, Sec. 2.2); AIRG_SMOOTH_ASSEMBLED applies
 * the assembled fixed-sparsity Ahat^{-1} of Eq. fixed_sparsity (one product
 * with an operator of A_ff's pattern, kept per level). */
typedef enum { AIRG_SMOOTH_POLY = 0, AIRG_SMOOTH_ASSEMBLED = 1 } airg_smoother;

/* Up-smooths of each level after its coarse-grid correction (Sec. 2; the
 * paper's option set uses F only and measures the storage of FC and FCF in
 * Sec. 3.3).  F: one F-point smooth.  FC: then a C-point smooth
 * e_c += q_c(A_cc) (r_c - A_cf e_f - A_cc e_c), q_c the GMRES polynomial of
 * A_cc of degree poly_order from its own random right-hand side (matrix-free,
 * or assembled on A_cc's pattern with AIRG_SMOOTH_ASSEMBLED); every level
 * then also keeps A_cf and A_cc and the V-cycle keeps each level's residual.
 * FCF: then a second F-point smooth with the updated e_c.  FC and FCF need
 * AIRG_INVERSE_ARNOLDI and a hierarchy built by setup (not imported). */
typedef enum {
  AIRG_SMOOTH_TYPE_F = 0,
  AIRG_SMOOTH_TYPE_FC = 1,
  AIRG_SMOOTH_TYPE_FCF = 2
} airg_smooth_type;

/* Outer iterations.  AIRG_OUTER_RICHARDSON is the paper's undamped Richardson
 * x <- x + M (b - A x) with M one V-cycle (Sec. 3), stopped when the true
 * residual |b - A x| <= rtol |b|, or rtol |b - A x0| when b = 0; its
 * iteration count is the number of V-cycles. */
typedef enum { AIRG_OUTER_FGMRES = 0, AIRG_OUTER_RICHARDSON = 1 } airg_outer;

typedef struct {
  int32_t iterations;        /* V-cycles applied */
  int32_t converged;         /* 1 when the true relative residual <= rtol (or the residual
                                norm <= atol) */
  int32_t restarts;
  int32_t stagnated;         /* 1 when the stagnation check stopped it (stagnation_check) */
  double rel_residual;       /* true |b - A x| / |b| at exit (Richardson with b = 0:
                                relative to |b - A x0|) */
  double rel_residual_estimate; /* Arnoldi estimate at exit */
  double solve_ms;           /* device time of the solve */
} airg_solve_info;

typedef struct {
  int32_t levels;
  int32_t coarse_roots;                    /* Newton roots on the coarsest level */
  int64_t n[AIRG_MAX_LEVELS];              /* rows of A_l */
  int64_t nnz[AIRG_MAX_LEVELS];            /* nnz of A_l */
  int64_t n_f[AIRG_MAX_LEVELS];            /* F points (0 on the coarsest) */
  int64_t nnz_ff[AIRG_MAX_LEVELS];
  int64_t nnz_fc[AIRG_MAX_LEVELS];
  int64_t nnz_z[AIRG_MAX_LEVELS];          /* Z after the relative drop */
  int32_t poly_degree[AIRG_MAX_LEVELS];    /* smoother degree actually used */
  int32_t pmisr_rounds[AIRG_MAX_LEVELS];
  double trunc_rel[AIRG_MAX_LEVELS];       /* truncation test result (NaN if not tested) */
  double grid_complexity;                  /* sum n_l / n_0 */
  double cycle_complexity;                 /* V-cycle FLOPs / FLOPs of one top-grid SpMV */
  double storage_complexity;               /* nnz kept for the solve / nnz(A_0) */
  double vcycle_bytes;                     /* algorithmic HBM bytes of one V-cycle */
  double setup_ms;                         /* device+host time of airg_setup */
  double setup_component_ms[8];            /* cf split, prolongator, gmres poly,
                                              restrictor spgemm, coarse spgemm,
                                              extract, drop, truncation */
} airg_stats;

/* Sizes of one level (for allocating export buffers). */
typedef struct {
  int64_t n, n_f, n_c;
  int64_t nnz_a, nnz_ff, nnz_fc, nnz_z;
  int32_t is_coarsest;
  int32_t poly_len;      /* number of smoother coefficients (degree + 1) */
  int32_t n_roots;       /* Newton roots (coarsest level) */
  int32_t c_poly_len;    /* C-point smoother coefficients (0 without FC / FCF) */
} airg_level_info;

/* Host arrays of one level in setup numbering: F and C points in ascending
 * level index, coarse index = rank among the C points.  Caller allocated from
 * airg_level_info; a NULL pointer skips that array. */
typedef struct {
  int8_t* state;                                   /* n: 1 = F, 2 = C */
  int32_t* a_rowptr; int32_t* a_col; double* a_val;     /* A_l */
  int32_t* ff_rowptr; int32_t* ff_col; double* ff_val;  /* A_ff */
  int32_t* fc_rowptr; int32_t* fc_col; double* fc_val;  /* A_fc */
  int32_t* z_rowptr; int32_t* z_col; double* z_val;     /* Z (n_c x n_f) */
  int32_t* cmap;                                   /* n_f: coarse index or -1 */
  double* alpha;                                   /* poly_len smoother coefficients
                                                      (zeros for AIRG_INVERSE_NEUMANN:
                                                      only the degree counts) */
  double* roots_re; double* roots_im;              /* n_roots, applied order */
  double* alpha_c;                                 /* c_poly_len coefficients of the
                                                      C-point smoother (export only) */
} airg_level_arrays;

/* Fill *p with the defaults above. */
int airg_params_default(airg_params* p);

/* Build the hierarchy for the n x n CSR matrix (rowptr[n+1], colidx[nnz],
 * vals[nnz]).  The arrays are read during the call only (the library copies A);
 * on_device says whether they are device pointers.  On success *out owns all
 * device memory of the solver until airg_destroy. */
int airg_setup(airg_handle* out, int64_t n, int64_t nnz, const int32_t* rowptr,
               const int32_t* colidx, const double* vals, int on_device,
               const airg_params* p, void* hip_stream);

/* Solve A x = b for nrhs right-hand sides: column k of b starts at b + k*ldb,
 * of x at x + k*ldx (device pointers, FP64).  x is the initial guess when
 * use_x_as_guess, else the guess is 0.  info (nrhs entries, may be NULL)
 * receives per right-hand-side results.  Returns AIRG_NOT_CONVERGED if any
 * column missed rtol within max_it.
 * Several columns are solved together, K at a time (K a power of two, at
 * most 64 and with n K < 2^31): every V-cycle kernel then reads each matrix
 * entry once for all K columns (SpMM on interleaved columns), and so do the
 * top-level product and the orthogonalisation kernels, while each column
 * runs its own outer process (FGMRES or Richardson) with its own stopping
 * test |b_k - A x_k| <= rtol |b_k|, restarts and iteration count, as if it
 * were solved alone; a column that has stopped rides along as zeros until
 * the others stop.  The Krylov bases then hold (2 restart + 1) vectors of
 * n K doubles (136 GB for n = 2048^2, K = 64, restart 30). */
int airg_solve(airg_handle h, int nrhs, const double* b, int64_t ldb, double* x,
               int64_t ldx, int use_x_as_guess, airg_solve_info* info);

/* A batch of nprob independent systems (problem p: n[p] rows, nnz[p]
 * entries, CSR arrays rowptr[p], colidx[p], vals[p]) set up as one
 * block-diagonal matrix: every setup kernel and every V-cycle launch covers
 * all problems at once.  on_device as in airg_setup. */
int airg_setup_batch(airg_handle* out, int nprob, const int64_t* n, const int64_t* nnz,
                     const int32_t* const* rowptr, const int32_t* const* colidx,
                     const double* const* vals, int on_device, const airg_params* p,
                     void* hip_stream);

/* Solve every problem of a batch handle: b[p], x[p] device pointers of n[p]
 * doubles; info has nprob entries.  Each problem runs its own outer process
 * (FGMRES or Richardson, with its own stopping test |b_p - A_p x_p| <=
 * rtol |b_p|, restarts and iteration count), the V-cycle and every other
 * kernel covering all problems per launch; the solve numbering orders each
 * level problem-major for that.  (Should the problem-major keys not fit 31
 * bits, or with locality_order = 0, one process runs over the block-diagonal
 * system until every problem meets its test.)  A batch handle takes no
 * airg_solve or airg_adjoint_solve call. */
int airg_solve_batch(airg_handle h, const double* const* b, double* const* x,
                     int use_x_as_guess, airg_solve_info* info);

/* Solve A^T lam = w (adjoint) with an AIRG hierarchy built on the explicit
 * transpose, with the same parameters and seed; built on the first call and
 * kept by the handle.  Pointers and layout as in airg_solve. */
int airg_adjoint_solve(airg_handle h, int nrhs, const double* w, int64_t ldw,
                       double* lam, int64_t ldl, int use_guess, airg_solve_info* info);

/* Free the Krylov workspaces that multi-column solves (nrhs > 1, forward or
 * adjoint) keep in the handle for reuse (up to (2 restart + 1) n K doubles
 * each); the next multi-column solve makes them again.  The hierarchies and
 * the single-column workspace stay. */
int airg_trim(airg_handle h);

/* Hierarchy statistics. */
int airg_get_stats(airg_handle h, airg_stats* s);

/* Level sizes and level arrays (the arrays need keep_setup_data = 1, except
 * for the coarsest level's matrix and roots and every level's coefficients). */
int airg_level_info_get(airg_handle h, int level, airg_level_info* out);
int airg_export_level(airg_handle h, int level, airg_level_arrays* out);

/* Build a solver from a given hierarchy (host arrays in setup numbering, as
 * airg_export_level writes them): level 0's a_* arrays hold the top matrix,
 * every non-coarsest level holds state, ff, fc, z, cmap and alpha, and the
 * coarsest holds a_* and the roots in applied order. */
int airg_import_hierarchy(airg_handle* out, int nlevels, const airg_level_info* infos,
                          const airg_level_arrays* levels, const airg_params* p,
                          void* hip_stream);

/* Kernel classes of the solve, for airg_time_kernels. */
enum airg_kernel_class {
  AIRG_K_POLY = 0,      /* every polynomial SpMV of a V-cycle: Horner smoother steps on
                           all levels and the Newton steps of the coarse solve */
  AIRG_K_HORNER = 1,    /* smoother products only: Horner or Neumann steps, or the
                           assembled Ahat^{-1} (Sec. 2.2) */
  AIRG_K_NEWTON = 2,    /* coarse Newton steps only (Sec. 2.3) */
  AIRG_K_RESIDUAL = 3,  /* F-point residual s = r_f - (A_fc + A_ff W) e_c (Eq. f_point) */
  AIRG_K_RESTRICT = 4,  /* restriction r_c + Z r_f */
  AIRG_K_TOP_SPMV = 5   /* top-level y = A x of the outer loop */
};

typedef struct {
  int32_t launches;          /* launches of the class in one V-cycle (1 for AIRG_K_TOP_SPMV) */
  int32_t reserved;
  double avg_launch_ms;      /* device time per launch, HIP events around reps passes */
  double bytes_per_launch;   /* algorithmic HBM bytes per launch: each matrix entry and
                                each vector element read or written once */
  double flops_per_launch;   /* 2 per matrix entry plus the vector updates */
  double stored_bytes_per_launch; /* the same with the bytes the operators' stored form
                                     actually has (16-bit compressed columns) */
} airg_kernel_timing;

/* Diagnostics for benchmarks: enqueue `reps` passes of exactly the launches
 * one V-cycle makes of kernel class `cls` (same operators, same launch
 * shapes, on the handle's scratch vectors) between two HIP events on the
 * handle's stream, and report the average launch time and the algorithmic
 * bytes and flops per launch.  Does not change the solver's state. */
int airg_time_kernels(airg_handle h, int cls, int reps, airg_kernel_timing* out);

/* Streaming probe, for benchmarks: the average device time (*avg_ms) of one
 * pass of the library's streaming read (kind 0: reads `bytes` from src,
 * writes nothing to dst, which must still be a valid device pointer of 8
 * bytes or more) or copy (kind 1: src to dst, `bytes` each) kernel, with
 * `blocks` workgroups of 256 threads, 16-byte loads and stores, timed with
 * HIP events over `reps` back-to-back launches on hip_stream after one
 * warm-up launch.  Device pointers, 16-byte aligned; bytes a positive
 * multiple of 16.  It gives the bandwidth a plain stream reaches on this
 * device (from HBM for buffers far above the on-die caches, from the caches
 * for small ones), the ceiling the sparse products are compared with. */
int airg_stream_probe(int kind, const void* src, void* dst, int64_t bytes, int reps, int blocks,
                      double* avg_ms, void* hip_stream);

/* Solve operators, for the launch-shape tuner. */
enum airg_operator {
  AIRG_OP_FF = 0,   /* A_ff of a level (smoother steps) */
  AIRG_OP_B = 1,    /* A_fc + A_ff W of a level (F-point residual) */
  AIRG_OP_Z = 2,    /* Z of a level (restriction) */
  AIRG_OP_A = 3,    /* the coarsest matrix (Newton steps) */
  AIRG_OP_TOP = 4,  /* the top matrix of the outer loop (level 0) */
  AIRG_OP_HAT = 5   /* the assembled Ahat^{-1} of a level (AIRG_SMOOTH_ASSEMBLED) */
};

typedef struct {
  int32_t level;
  int32_t op;          /* airg_operator */
  int32_t lanes;       /* lanes per row of single-column products (1..64, power of two),
                          or 0: the row-block kernel (a workgroup loads a block of rows
                          with at most 2048 entries at once and each row's thread sums
                          its products in order; operators with 8 or more entries per
                          row on average) */
  int32_t xcd_map;     /* 1: workgroups of one XCD take one contiguous eighth of the rows
                          (each XCD has its own L2); 0: workgroup i takes row block i */
  int32_t lds;         /* what the product stages in LDS.  0: nothing.  1: the window of x
                          (a workgroup per 64-row group copies the group's window of x to
                          LDS and gathers there; operators with compressed columns; lanes
                          2..16).  2: the entries (a workgroup per 256 consecutive rows
                          loads their entries at consecutive addresses and leaves the
                          products in LDS, where each row's thread adds its own in order:
                          the one-lane kernel's sums, bit for bit; lanes 1) */
  int32_t default_lanes;
  int32_t default_xcd_map;
  int32_t default_lds;
  double best_us;      /* device time of one product with the chosen shape */
  double default_us;   /* ... with the default shape (a rule on the mean row length) */
} airg_tune_entry;

/* Launch-shape tuner: time every solve operator's single-column product with
 * 1, 2, ..., 64 lanes per row, the row-block kernel and the LDS-staged kernel
 * where they exist and the entry-staged kernel, each with and without the XCD
 * mapping (`reps` launches
 * each, HIP events on the handle's stream), and keep the fastest per
 * operator.  A row split over more
 * lanes sums in a different order, so solves after tuning agree with untuned
 * ones to rounding, not bit for bit; timings vary run to run, so a caller
 * that needs reproducible results pins the shapes with airg_set_lanes.
 * Writes at most max_out entries to out (may be NULL) and the number of
 * operators to *n_out (may be NULL). */
int airg_autotune(airg_handle h, int reps, airg_tune_entry* out, int max_out, int* n_out);

/* Set the launch shape (lanes per row, XCD mapping and LDS staging, as in
 * airg_tune_entry) of one solve operator (level is ignored for AIRG_OP_TOP
 * and AIRG_OP_A).  AIRG_ERR_INVALID for an unknown operator, lanes not 0 or a
 * power of two in 1..64, 0 for an operator without row blocks, xcd_map not 0
 * or 1, lds not 0, 1 or 2, lds = 1 with lanes outside 2..16 or for an operator
 * without compressed columns, or lds = 2 with lanes other than 1. */
int airg_set_lanes(airg_handle h, int level, int op, int lanes, int xcd_map, int lds);

/* ---- differentiable advection solve -------------------------------------
 * The upwind finite-volume system of v.grad(u) = 0 with inflow values g
 * (paper Eqs. advection and advection_bc) on an nx x ny grid of square cells,
 * v = (cos theta, sin theta), theta in [0, pi/2]: fluxes are divided by the
 * cell size, inflow faces (west, south) move to the right-hand side.  Unknown
 * k = j nx + i; row k holds -vy at k - nx (j > 0), -vx at k - 1 (i > 0) and
 * vx + vy on the diagonal; b_k = vx g_west[j] (i = 0) + vy g_south[i] (j = 0).
 * All pointers are device pointers. */

/* Number of stored entries of the system. */
int airg_fv_nnz(int64_t nx, int64_t ny, double theta, int64_t* nnz);

/* Assemble rowptr[n+1], col[nnz], val[nnz], b[n] (n = nx ny); if not NULL,
 * dval_dtheta[nnz] and db_dtheta[n] receive the derivatives in theta. */
int airg_fv_assemble(int64_t nx, int64_t ny, double theta, const double* g_west,
                     const double* g_south, int32_t* rowptr, int32_t* col, double* val,
                     double* b, double* dval_dtheta, double* db_dtheta, void* hip_stream);

/* Gradients of a loss L(u) with u = A^{-1} b, given the adjoint solution
 * lam = A^{-T} dL/du: dg_west[ny] = vx lam at the west inflow cells,
 * dg_south[nx] = vy lam at the south inflow cells and
 * *dtheta = lam^T (db/dtheta - dA/dtheta u) (one device double). */
int airg_fv_gradients(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                      const int32_t* col, const double* dval_dtheta, const double* db_dtheta,
                      const double* u, const double* lam, double* dg_west, double* dg_south,
                      double* dtheta, void* hip_stream);

/* airg_fv_gradients without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same kernels,
 * bit for bit the same results; the theta terms and the partial sums of the
 * contraction live in one static device array of the library (about 34 MB,
 * held by each device that runs this call until the process ends), whose
 * address is looked up once per device on the first call there.
 *   - n = nx ny must be at most 4194304 (2048 x 2048); larger grids get
 *     AIRG_ERR_INVALID and nothing is enqueued.
 *   - The work is enqueued on hip_stream and the call returns without
 *     waiting: dg_west, dg_south and *dtheta are complete when the stream
 *     reaches that point.
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents: calls whose work can overlap on one device (other
 *     streams, other threads, before the stream has drained the previous
 *     call) race and must be serialised by the caller. */
int airg_fv_gradients_noalloc(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                              const int32_t* col, const double* dval_dtheta,
                              const double* db_dtheta, const double* u, const double* lam,
                              double* dg_west, double* dg_south, double* dtheta,
                              void* hip_stream);

/* Failure-handling hook (for tests and for callers that cap the library's
 * memory): from now on, a device allocation of the library that would take
 * the bytes its buffers hold past `bytes` fails with AIRG_ERR_NOMEM, as if
 * the device were out of memory (the call that needed it returns that code
 * and releases what it had allocated).  bytes <= 0 removes the budget.
 * *in_use (may be NULL) receives the bytes the library's buffers hold now,
 * over every handle of the process. */
int airg_set_alloc_budget(int64_t bytes, int64_t* in_use);

/* Failure-handling hook (for tests): a grid-wide barrier wait of a
 * persistent launch gives up after `polls` polls of its counter (polls <= 0:
 * the default, about a second); every workgroup still finishes.  In the
 * persistent coarse solve (airg_params.coarse_persistent) the solve then
 * fails with AIRG_ERR_INTERNAL; in the breadth-first passes of the locality
 * order (setup) the pass runs again with one launch per step, with the same
 * result.  Applies to launches enqueued after the call. */
int airg_set_spin_limit(int64_t polls);

/* Release the handle and all its device memory (NULL is a no-op). */
void airg_destroy(airg_handle h);

/* Static text for a status code; the last error message of this thread. */
const char* airg_status_string(int code);
const char* airg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AIRG_H */
