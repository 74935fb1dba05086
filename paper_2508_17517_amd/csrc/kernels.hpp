// Host launchers of the HIP kernels (vec.hip, spmv.hip, cf.hip, spgemm.hip).
// Every launcher enqueues on the given stream and returns without syncing.
#pragma once

#include "common.hpp"

namespace airg {

// ---------------------------------------------------------------- vec.hip
// Random draws of the setup: U[0,1) from counter-based SplitMix64, element i
// of stream (purpose, level) being output c + 1 of `seed`, c = purpose << 56 |
// level << 40 | i.
enum RngPurpose {
  RNG_PMISR = 1,
  RNG_POLY_RHS = 2,
  RNG_COARSE_RHS = 3,
  RNG_TRUNC_RHS = 4,
  RNG_CPOLY_RHS = 5  // the C-point smoother's polynomial
};
void launch_uniform(double* out, int64_t n, uint64_t seed, int purpose, int level, hipStream_t s);

void launch_fill(double* x, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);
void launch_zero_bytes(void* p, size_t bytes, hipStream_t s);
void launch_copy(double* y, const double* x, int64_t n, hipStream_t s);
void launch_scale(double* y, const double* x, double a, int64_t n, hipStream_t s);   // y = a x
// y = x / d, and y32 = (float) y when y32 is given
void launch_divide(double* y, const double* x, double d, int64_t n, hipStream_t s,
                   float* y32 = nullptr);
void launch_divide_dev(double* y, const double* x, const double* d, int64_t n, hipStream_t s);
// y = x / sqrt(d2[0]) with the norm's square on the device (y32 as above)
void launch_divide_norm2(double* y, const double* x, const double* d2, int64_t n, hipStream_t s,
                         float* y32 = nullptr);
void launch_sub(double* z, const double* x, const double* y, int64_t n, hipStream_t s);  // z = x - y
// w = w - h[0] V_0 - h[1] V_1 - ... (k sequential per element; V_k = V + k ldv)
void launch_cgs_update(double* w, const double* V, int64_t ldv, const double* h, int nv,
                       int64_t n, hipStream_t s);
// x = x + sum_k y[k] Z_k (y on device; Z in FP64 or FP32)
void launch_basis_combine(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                          int64_t n, hipStream_t s);
void launch_basis_combine(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                          int64_t n, hipStream_t s);

// Dot products by the perfect binary tree over the index range (adjacent pairs
// first, zero padded): out[k] = V_k . w for k < nv.  `work` needs
// dot_work_size(n, nv) doubles.
size_t dot_work_size(int64_t n, int nv);
void launch_tree_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                      double* out, double* work, hipStream_t s);
// A Gram-Schmidt sweep fused with the reduction after it (1 <= nv <= 32):
// out[k] = V_k . w (launch_cgs_dots), or w = w - sum_k h[k] V_k and then
// out[k] = V_k . w (k < nv) or out[0] = w . w; every sum in a fixed order.
// `work` needs cgs_fused_work_size(n) doubles.
size_t cgs_fused_work_size(int64_t n);
void launch_cgs_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                     double* out, double* work, hipStream_t s);
void launch_cgs_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                            int64_t n, double* out, double* work, hipStream_t s);
void launch_cgs_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                             int64_t n, double* out, double* work, hipStream_t s);
// One FGMRES per column of K interleaved columns ([n0][K] arrays, K a power
// of two, at most 64; h, y and out hold entry (k, c) at k K + c):
//   w = w - sum_k h[k, c] V_k (k sequential per element),
//   x = x + sum_k y[k, c] Z_k,
//   y = x / d[c] column by column (0 where d[c] = 0; also y32 = (float) y
//   when y32 is given),
//   out[k, c] = V_k . w over column c (fixed order; `work` needs
//   col_dots_work_size(n0, K) doubles).
void launch_cgs_update_cols(double* w, const double* V, int64_t ldv, const double* h, int nv,
                            int64_t n0, int K, hipStream_t s);
void launch_basis_combine_cols(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                               int64_t n0, int K, hipStream_t s);
void launch_basis_combine_cols(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                               int64_t n0, int K, hipStream_t s);
void launch_divide_cols(double* y, const double* x, const double* d, int64_t n0, int K,
                        hipStream_t s, float* y32 = nullptr);
size_t col_dots_work_size(int64_t n0, int K);
void launch_col_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n0, int K,
                     double* out, double* work, hipStream_t s);
// One outer process per problem of a batch (see GroupRange): work items of
// at most 1024 elements of one problem's range, and each problem's items in
// a fixed order.  Coefficient arrays hold entry (k, g) at k G + g:
//   out[k, g] = V_k . w over problem g (fixed order; `work` needs
//   group_dots_work_size(items) doubles),
//   w = w - sum_k h[k, g] V_k,  x = x + sum_k y[k, g] Z_k,
//   y = x / d[g] problem by problem (0 where d[g] = 0; also y32 = (float) y
//   when y32 is given).
struct GroupItems {
  DBuf<int64_t> start;
  DBuf<int32_t> len, grp, gptr, glist;
  int64_t n = 0;  // items
  int G = 0;      // problems
};
// chunk: the item length (1024 for the dot and update kernels, 256 for the
// fused sweeps)
void build_group_items(const std::vector<GroupRange>& ranges, int G, GroupItems& out,
                       hipStream_t s, int chunk = 1024);
size_t group_dots_work_size(const GroupItems& it);
// With `active` (one byte per problem), the items of problems whose byte is
// 0 are skipped and give zero products (callers pass it only where those
// problems' w is zero).
void launch_group_dots(const double* V, int64_t ldv, int nv, const double* w, const GroupItems& it,
                       double* out, double* work, hipStream_t s, const uint8_t* active = nullptr);
void launch_group_update(double* w, const double* V, int64_t ldv, const double* h, int nv,
                         const GroupItems& it, hipStream_t s);
void launch_group_combine(double* x, const double* Z, int64_t ldz, const double* y, int nv,
                          const GroupItems& it, hipStream_t s);
void launch_group_combine(double* x, const float* Z, int64_t ldz, const double* y, int nv,
                          const GroupItems& it, hipStream_t s);
void launch_group_divide(double* y, const double* x, const double* d, const GroupItems& it,
                         hipStream_t s, float* y32 = nullptr);
// Activity masks of a problem batch: mask[i] = 1 where any of the problems
// g0[i] .. g1[i] of 64-row group i has active[p] != 0.
void launch_group_mask(const int32_t* g0, const int32_t* g1, const uint8_t* active, int64_t n,
                       uint8_t* mask, hipStream_t s);
// Most basis vectors the fused Gram-Schmidt sweeps take (one register each).
constexpr int kFusedVecs = 32;
// The fused Gram-Schmidt sweeps per column of K interleaved columns:
// w = w - sum_k h[k K + c] V_k, then out[k K + c] = V_k . w over column c
// (update_dots, summed as launch_col_dots sums) or out[c] = w . w
// (update_norm2).  1 to 32 basis vectors; `work` needs
// col_fused_work_size(n0, K) doubles.
size_t col_fused_work_size(int64_t n0, int K);
void launch_cols_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                             int64_t n0, int K, double* out, double* work, hipStream_t s);
void launch_cols_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                              int64_t n0, int K, double* out, double* work, hipStream_t s);
// The fused Gram-Schmidt sweeps per problem, on items of at most 256
// elements (build_group_items with chunk 256): out[k, g] = V_k . w
// (fused_dots), or w = w - sum_k h[k, g] V_k and then out[k, g] = V_k . w
// (update_dots) or out[0, g] = w . w (update_norm2) over problem g, each
// summed in a fixed order.  1 to 32 basis vectors; `work` needs
// group_fused_work_size(items) doubles.
size_t group_fused_work_size(const GroupItems& it);
// `active` as in launch_group_dots (skipped items leave w unchanged: their
// w and coefficients are zero).
void launch_group_fused_dots(const double* V, int64_t ldv, int nv, const double* w,
                             const GroupItems& it, double* out, double* work, hipStream_t s,
                             const uint8_t* active = nullptr);
void launch_group_update_dots(double* w, const double* V, int64_t ldv, const double* h, int nv,
                              const GroupItems& it, double* out, double* work, hipStream_t s,
                              const uint8_t* active = nullptr);
void launch_group_update_norm2(double* w, const double* V, int64_t ldv, const double* h, int nv,
                               const GroupItems& it, double* out, double* work, hipStream_t s,
                               const uint8_t* active = nullptr);
// out[0] = sqrt(out[0]) on the device
void launch_sqrt_inplace(double* v, hipStream_t s);

// Permutations: y[perm[i]] = x[i] (scatter) and y[i] = x[perm[i]] (gather).
void launch_scatter(double* y, const double* x, const int32_t* perm, int64_t n, hipStream_t s);
// y[perm[i]] = x[i] for int32 arrays
void launch_scatter_i32(int32_t* y, const int32_t* x, const int32_t* perm, int64_t n, hipStream_t s);
void launch_gather(double* y, const double* x, const int32_t* perm, int64_t n, hipStream_t s);

// K interleaved columns: ys[pos[i] K + c] = b[c ldb + i] and x[c ldx + i] = xs[pos[i] K + c];
// columns c >= kv are padding (zero in ys, not written to x).
void launch_scatter_cols(double* ys, const double* b, int64_t ldb, const int32_t* pos, int64_t n,
                         int K, int kv, hipStream_t s);
void launch_gather_cols(double* x, int64_t ldx, const double* xs, const int32_t* pos, int64_t n,
                        int K, int kv, hipStream_t s);
// out[c] = sum_i x[i K + c]^2 in a fixed order; `work` needs col_sumsq_work_size(n, K).
size_t col_sumsq_work_size(int64_t n, int K);
void launch_col_sumsq(const double* x, int64_t n, int K, double* out, double* work, hipStream_t s);

// dst[i] = src[i] + add
void launch_offset_copy_i32(int32_t* dst, const int32_t* src, int64_t n, int64_t add,
                            hipStream_t s);

// Exclusive scan of int64 counts: out[i] = sum_{j<i} in[j], out[n] = total.
// `work` needs scan_work_size(n) int64s.  in and out may alias.
size_t scan_work_size(int64_t n);
void launch_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* work, hipStream_t s);
// rowptr (int32) from int64 offsets; sets *overflow = 1 if any exceeds int32.
void launch_offsets_to_i32(const int64_t* off, int32_t* rowptr, int64_t n1, int32_t* overflow,
                           hipStream_t s);

// ---------------------------------------------------------------- spmv.hip
// Rows-per-thread-group shape of a CSR kernel (lanes per row, power of 2).
int pick_tpr(int64_t rows, int64_t nnz);
// Launch shape of a product: lanes per row in bits 0-7 (0: row-block kernel),
// the XCD mapping in bit 8, the LDS-staged kernel in bit 9, the
// entry-staged kernel (256 consecutive rows per workgroup, one lane per row)
// in bit 10.
constexpr int kShapeXcd = 1 << 8;
constexpr int kShapeLds = 1 << 9;
constexpr int kShapeEntries = 1 << 10;
// y = A x, every row summed left to right from 0.0 by one lane (setup order).
void spmv_seq(const CSR& A, const double* x, double* y, hipStream_t s);
// y = A x with `tpr` lanes per row.
void spmv(const CSR& A, int tpr, const double* x, double* y, hipStream_t s);

// Solve-phase kernels, generic over the matrix storage (OpView::vt), the
// vector type X (double or float; rows accumulate in X) and the number K of
// interleaved columns (element (row, c) at row * K + c; K a power of two <= 64).
template <class X>
void spmv_t(const OpView& A, int tpr, int K, const X* x, X* y, hipStream_t s);
// y = A x with FP64 values and row sums, x in FP32 (widened as it is gathered).
void spmv_x32(const OpView& A, int tpr, int K, const float* x, double* y, hipStream_t s);
// Horner step of the smoother: out = (acc ? out : 0) + a (A y) + b s
template <class X>
void spmv_horner_t(const OpView& A, int tpr, int K, const X* y, const X* sv, X* out, double a,
                   double b, bool acc, hipStream_t st);
// Restriction: dst[p] = src[p] + (Z r_f)[p]   (src may alias dst)
template <class X>
void spmv_restrict_t(const OpView& Z, int tpr, int K, const X* rf, const X* src, X* dst,
                     hipStream_t s);
// F-point residual s = r_f - B e_c with B = A_fc + A_ff W (see merge_fc_ffw).
template <class X>
void spmv_residual_t(const OpView& B, int tpr, int K, const X* ec, const X* rf, X* sv,
                     hipStream_t s);
// Last Horner step fused with the one-point prolongation:
//   ef = W e_c + a (A y) + b s,  (W e_c)[i] = ec[cmap[i]] (0 where cmap[i] < 0)
template <class X>
void spmv_horner_prolong_t(const OpView& A, int tpr, int K, const X* y, const X* sv, X* ef,
                           double a, double b, const int32_t* cmap, const X* ec, hipStream_t st);
// nAIR's Neumann step out = y + D^{-1} (s - A y), the last step fused with the
// prolongation (ef = W e_c + ...), and y = D^{-1} s (ef = W e_c + D^{-1} s when
// cmap is given); D^{-1} holds one value per row.
template <class X>
void spmv_neumann_t(const OpView& A, int tpr, int K, const X* y, const X* sv, const X* dinv, X* out,
                    hipStream_t st);
template <class X>
void spmv_neumann_prolong_t(const OpView& A, int tpr, int K, const X* y, const X* sv,
                            const X* dinv, X* ef, const int32_t* cmap, const X* ec, hipStream_t st);
template <class X>
void dinv_apply_t(X* out, const X* sv, const X* dinv, const int32_t* cmap, const X* ec,
                  int64_t rows, int K, hipStream_t s);
// ef = W e_c + a s (a degree-0 smoother)
template <class X>
void prolong_axpy_t(X* ef, const X* sv, const int32_t* cmap, const X* ec, double a, int64_t rows,
                    int K, hipStream_t s);
// Newton steps of the coarse solver (see newton_apply_t).
template <class X>
void newton_real_t(const OpView& A, int tpr, int K, const X* w, X* wn, X* x, double inv,
                   bool first, double inv_last, hipStream_t s);
template <class X>
void newton_pair1_t(const OpView& A, int tpr, int K, const X* w, X* t, X* x, double c1, double c2,
                    bool first, hipStream_t s);
template <class X>
void newton_pair2_t(const OpView& A, int tpr, int K, const X* w, const X* t, X* wn, X* x,
                    double c1, double c2, double inv_last, hipStream_t s);
// x = (first ? 0 : x) + a w
template <class X>
void axpy_first_t(X* x, const X* w, double a, bool first, int64_t n, hipStream_t s);

// Precision conversions (BF16: round to nearest even of the FP32 value).
void convert_d2f(float* y, const double* x, int64_t n, hipStream_t s);
void convert_f2d(double* y, const float* x, int64_t n, hipStream_t s);
void convert_d2bf(bf16* y, const double* x, int64_t n, hipStream_t s);

// ---------------------------------------------------------------- cf.hip
// Validates CSR structure (monotone rowptr, strictly ascending in-range
// columns, finite values, nonzero diagonal present) and extracts the diagonal.
// flags: bit0 structure, bit1 nonfinite, bit2 zero/missing diagonal.
void launch_validate(const CSR& A, double* diag, int32_t* flags, hipStream_t s);
// Structural checks of constructed operators (flags bit0: CSR, bit1: map).
void launch_check_csr(const CSR& A, int32_t* flags, hipStream_t s);
void launch_check_map(const int32_t* m, int64_t n, int64_t lo, int64_t hi, int32_t* flags,
                      hipStream_t s);
// Strength: mask[p] = 1 iff entry p is a strong off-diagonal connection.
void launch_strength(const CSR& A, double theta, int8_t* mask, int64_t* row_count,
                     hipStream_t s);
// Transpose of the strong pattern: ST (rowptr/col) from mask.
void launch_pattern_transpose_count(const CSR& A, const int8_t* mask, int64_t* colcount,
                                    hipStream_t s);
void launch_pattern_transpose_fill(const CSR& A, const int8_t* mask, const int64_t* off,
                                   int64_t* cursor, int32_t* st_col, hipStream_t s);
// PMISR round on G = S + S^T (S from A/mask, S^T from st_off/st_col).
void launch_pmisr_select(const CSR& A, const int8_t* mask, const int64_t* st_off,
                         const int32_t* st_col, int8_t* state, uint64_t seed, int level,
                         hipStream_t s);
void launch_pmisr_neighbours(const CSR& A, const int8_t* mask, const int64_t* st_off,
                             const int32_t* st_col, int8_t* state, hipStream_t s);
void launch_pmisr_finalize(int8_t* state, int64_t n, int32_t* undecided, hipStream_t s);
// DDC: ratios of F rows, max and F count; histogram; conversion.
void launch_ddc_ratio(const CSR& A, const int8_t* state, const double* diag, double* r,
                      unsigned long long* rmax_bits, int32_t* nf, hipStream_t s);
void launch_ddc_hist(const double* r, const int8_t* state, int64_t n, double rmax,
                     int32_t* counts, hipStream_t s);
void launch_ddc_convert(const double* r, int8_t* state, int64_t n, double rmax, int edge,
                        hipStream_t s);
// F/C flags -> int64 flags for scanning (which: 1 = F, 2 = C)
void launch_flag(const int8_t* state, int64_t n, int which, int64_t* out, hipStream_t s);
// Sub-block extraction (rows with state rs, columns with state cs, columns
// renumbered through idx (F index or C index)).
void launch_extract_count(const CSR& A, const int8_t* state, int rs, int cs, int64_t* count,
                          const int64_t* rowidx, hipStream_t s);
void launch_extract_fill(const CSR& A, const int8_t* state, int rs, int cs,
                         const int64_t* fidx, const int64_t* cidx, const int32_t* rowptr_out,
                         int32_t* col_out, double* val_out, hipStream_t s);
// list[idx[i]] = i for the points with state == which (F or C index -> level index).
void launch_inverse_map(const int8_t* state, int64_t n, int which, const int64_t* idx,
                        int64_t* list, hipStream_t s);
// Nested positions: pos[i] = fidx[i] for F points, nF + pos_next[cidx[i]] for C points.
void launch_nested_pos(const int8_t* state, const int64_t* fidx, const int64_t* cidx, int64_t nF,
                       const int32_t* pos_next, int64_t n, int32_t* pos, hipStream_t s);
// out[f] = pos_next[cmap[f]] (or -1)
void launch_remap(const int32_t* cmap, const int32_t* pos_next, int64_t nf, int32_t* out,
                  hipStream_t s);
void launch_iota(int32_t* x, int64_t n, hipStream_t s);
// One-point prolongation: cmap[f] = coarse index of the strongest C column.
void launch_one_point(const CSR& A, const int8_t* state, const int64_t* fidx,
                      const int64_t* cidx, int32_t* cmap, hipStream_t s);

// ---------------------------------------------------------------- grid barrier
// Polls of a persistent launch's grid-barrier wait before it gives up (<= 0
// restores the default, about a second of waiting); read when such a launch
// is enqueued.
void set_grid_spin_limit(int64_t polls);
int64_t grid_spin_limit();

// ---------------------------------------------------------------- order.hip
// Breadth-first levels of the graph of A + A^T from src (level[i] >= 0 for
// every i; unreached components restart at the next level).
void bfs_levels(const CSR& A, const CSR& At, int64_t src, int32_t* level, hipStream_t s);
// The node of largest level (ties: smallest index).
int64_t far_node(const int32_t* level, int64_t n, hipStream_t s);
// rank[f] = position of F point f ordered by (key, F index).
void rank_f_points(const int8_t* state, const int64_t* fidx, const int32_t* key, int64_t n,
                   int64_t nf, int32_t* rank, hipStream_t s);
// Locality key of every node of A, from d1, the BFS distance from a far node,
// and d2, the distance from an end of d1's middle band.  With hilbert the key
// is the index of (d1, d2) along a Hilbert curve (distances below 2^15), which
// keeps 2D neighbourhoods together at every scale: the order whose keys the
// coarse levels inherit.  Otherwise, or when the distances are larger, key =
// d1 * (max d2 + 1) + d2 (d1 alone if that overflows 31 bits): on a structured
// grid, by anti-diagonal, then by position along it, which keeps the columns
// of 64 consecutive rows in one narrow window.
void locality_keys(const CSR& A, int32_t* key, hipStream_t s, bool hilbert);
// rank[i] = position of node i ordered by (key, i).
void rank_points(const int32_t* key, int64_t n, int32_t* rank, hipStream_t s);
// inv[pos[i]] = i
void invert_perm(const int32_t* pos, int64_t n, int32_t* inv, hipStream_t s);
// out[c] = key[clist[c]]
void inherit_keys(const int32_t* key, const int64_t* clist, int64_t nc, int32_t* out, hipStream_t s);
// The locality keys of a graph of independent segments (sid[i]: the segment
// of node i), computed in every segment at once.
void locality_keys_seg(const CSR& A, const int32_t* sid, int nseg, int32_t* key, hipStream_t s,
                       bool hilbert);
// The keys of every connected component at once, each component's from 0
// (not component-major; a connected graph gets locality_keys).
void locality_keys_by_component(const CSR& A, int32_t* key, hipStream_t s, bool hilbert);
// Problem-major keys of a block-diagonal batch (key = p * mult + key), by the
// row segments seg (problem p: rows seg[p] .. seg[p+1]-1) or by a problem per
// point; the problem of each key (key / mult); the number of points of each
// problem among all points, or among the F points when state is given.
int32_t max_key(const int32_t* key, int64_t n, hipStream_t s);
void problem_major_keys(int32_t* key, int64_t n, const std::vector<int64_t>& seg, int64_t mult,
                        hipStream_t s);
void problem_major_keys(int32_t* key, const int32_t* pid, int64_t n, int64_t mult, hipStream_t s);
void key_problems(const int32_t* key, int64_t n, int64_t mult, int32_t* pid, hipStream_t s);
std::vector<int32_t> count_problems(const int8_t* state, const int32_t* key, int64_t n,
                                    int64_t mult, int np, hipStream_t s);
// pos[i] = frank[fidx[i]] for F points, nF + pos_next[cidx[i]] for C points.
void launch_nested_pos_ranked(const int8_t* state, const int64_t* fidx, const int64_t* cidx,
                              const int32_t* frank, int64_t nF, const int32_t* pos_next, int64_t n,
                              int32_t* pos, hipStream_t s);
// out[frank[f]] = pos_next[cmap[f]] (or -1)
void launch_remap_ranked(const int32_t* cmap, const int32_t* pos_next, const int32_t* frank,
                         int64_t nf, int32_t* out, hipStream_t s);

// ---------------------------------------------------------------- fv.hip
int64_t fv_nnz(int64_t nx, int64_t ny, double theta);
void fv_assemble(int64_t nx, int64_t ny, double theta, const double* gw, const double* gs,
                 int32_t* rowptr, int32_t* col, double* val, double* b, double* dval, double* db,
                 hipStream_t s);
void fv_gradients(int64_t nx, int64_t ny, double theta, const int32_t* rowptr, const int32_t* col,
                  const double* dval, const double* db, const double* u, const double* lam,
                  double* dgw, double* dgs, double* dtheta, hipStream_t s);
// The same launches with r and the dot partials in the file-scope scratch
// array of fv.hip (no allocation, no wait); n = nx ny <= kFvNoallocMaxN.
constexpr int64_t kFvNoallocMaxN = int64_t(1) << 22;
void fv_gradients_noalloc(int64_t nx, int64_t ny, double theta, const int32_t* rowptr,
                          const int32_t* col, const double* dval, const double* db, const double* u,
                          const double* lam, double* dgw, double* dgs, double* dtheta, hipStream_t s);

// ---------------------------------------------------------------- probe.hip
// Average device time (ms) of one pass of a streaming read (kind 0: src only,
// dst receives nothing unless the sum is -1e300) or copy (kind 1) of `bytes`
// bytes, over `reps` back-to-back launches of `blocks` workgroups after one
// warm-up launch, timed with HIP events on s.
double stream_probe(int kind, const void* src, void* dst, int64_t bytes, int reps, int blocks,
                    hipStream_t s);

// ---------------------------------------------------------------- spgemm.hip
// C = A B with c_ij accumulated over k ascending from 0.0, exact zeros dropped.
void spgemm(const CSR& A, const CSR& B, CSR& C, hipStream_t s);
// Masked powers and the fixed-sparsity inverse on the pattern of Aff:
//   out = alpha_0 I + alpha_1 A + alpha_2 A~^2 + ..., zeros dropped.
void fixed_sparsity_inverse(const CSR& Aff, const std::vector<double>& alpha, CSR& out,
                            hipStream_t s);
// nAIR's assembled Neumann approximation (I + N~ + ... + N~^d) D^{-1} with
// N = I - D^{-1} A_ff kept on A_ff's pattern, and the diagonal inverse D^{-1}.
void neumann_fixed_sparsity(const CSR& Aff, int degree, CSR& out, hipStream_t s);
void diag_inverse(const CSR& A, DBuf<double>& dinv, hipStream_t s);
// Drop |z| < tol * max_j |z_ij| per row (no lumping), optionally negating.
void restrictor_drop(const CSR& Zin, double tol, bool negate, CSR& Z, hipStream_t s);
// Relative off-diagonal drop with lumping to the diagonal; sets *bad_diag if a
// row ends with a zero or missing diagonal.
void drop_lump(const CSR& Ain, double tol, bool lump, CSR& Aout, int32_t* bad_diag,
               hipStream_t s);
// R = [Z I] in level numbering (rows n_c, columns n).
void build_r(const CSR& Z, const int64_t* fpos, const int64_t* cpos, int64_t n, CSR& R,
             hipStream_t s);
// P = [W; I] in level numbering (rows n, columns n_c).
void build_p(const int8_t* state, const int64_t* fidx, const int64_t* cidx, const int32_t* cmap,
             int64_t n, int64_t nc, CSR& P, hipStream_t s);
// Row permutation + column renumbering: out row newrow[i] = row i of A with
// columns mapped through colmap (either map NULL: identity).  Column order within a row
// is preserved.
void permute_rows(const CSR& A, const int32_t* newrow, const int32_t* colmap, int64_t out_cols,
                  CSR& out, hipStream_t s);
// B = A_fc + A_ff W for the one-point W given by cmap (rows ascending by
// column; entries with equal columns summed A_fc first, then A_ff in order).
void merge_fc_ffw(const CSR& Afc, const CSR& Aff, const int32_t* cmap, CSR& B, hipStream_t s);
// Build A's compressed column form (see CSR::col16) if every block of rows
// spans fewer than 65536 columns; returns whether it did.
bool compress_columns(CSR& A, hipStream_t s);
// Row blocks of A for the row-block product (lanes per row 0): at most 64
// consecutive rows of one 64-row group with at most 2048 entries, or one row.
void build_row_blocks(CSR& A, hipStream_t s);
// Sort the entries of every row by column (insertion sort per row).
void sort_rows(CSR& A, hipStream_t s);
// Store A's rows in ascending order of rkey[row] (ties by row) and record the
// order in A.rmap (stored row r is row rmap[r]); columns are unchanged.
void spatial_row_order(CSR& A, const int32_t* rkey, hipStream_t s);
// Explicit transpose with ascending columns.
void transpose(const CSR& A, CSR& At, hipStream_t s);
// Deep copy of a device CSR.
void copy_csr(const CSR& A, CSR& out, hipStream_t s);

}  // namespace airg
