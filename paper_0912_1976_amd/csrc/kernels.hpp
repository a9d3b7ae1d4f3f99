// Device kernels of the PCG hot path (gfx950, wave64) and their launchers.
// All launchers enqueue on the given stream and never synchronise.
//
// Every vector kernel works on K right-hand sides at once (K in {1,2,4,8}):
// vectors are stored row-major as [n][K], so a matrix entry is read once
// for all K columns and the K values of a gathered row are contiguous.
// The vector type T is double (FP64 path) or float (inner solve of the
// mixed-precision path); reductions always accumulate in double.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vemg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kSlicesPerBlock = kBlock / kWave;
constexpr int kMaxBatch = 8;

// SELL-64 matrix: 64 consecutive rows form a slice stored column-major and
// padded to the slice's longest row, so lane t of a wavefront reads entry k
// of row 64 s + t at sptr[s] + 64 k + t (coalesced).  Only off-diagonal
// entries are stored; padding entries have value 0 and point at the row
// itself (square) or column 0 (rectangular).
//   fine A (difference form): FP64 values a_ij with the deficit d64;
//   FP32 copy: row-scaled values a_ij / a_ii with s32 = a_ii and
//   dh32 = d_i / a_ii, so (A x)_i = s_i (sum_j w_ij (x_j - x_i) + dh_i x_i).
struct Sell {
  const int64_t *sptr = nullptr;  // nslices + 1 entry offsets
  const int32_t *col = nullptr;
  const double *val64 = nullptr;
  const float *val32 = nullptr;
  const double *d64 = nullptr;
  const float *s32 = nullptr, *dh32 = nullptr;
  int64_t nrows = 0;
};

// CSR matrix processed by groups of G lanes per row (G = 4..64, a power of
// two chosen from the mean row length): the group reads consecutive entries
// of its row (coalesced) and reduces with cross-lane shuffles, so long rows
// (coarse multigrid operators, restrictions) cost a few memory round trips
// instead of one per entry.  Square operators store off-diagonals only:
// FP64 values with d64 = a_ii; FP32 values a_ij / a_ii with s32 = a_ii.
struct CsrG {
  const int32_t *ptr = nullptr;  // nrows + 1
  const int32_t *col = nullptr;
  const double *val64 = nullptr;
  const float *val32 = nullptr;
  const double *d64 = nullptr;
  const float *s32 = nullptr;
  // rectangular operators only: stored row i is output row orow[i] (the rows
  // are stored in the spatial order of the columns they gather); null: i
  const int32_t *orow = nullptr;
  int64_t nrows = 0;
  int G = 4;
};

// Device scalars of one batched PCG solve (one set per column).
struct Scal {
  double rho[kMaxBatch], alpha[kMaxBatch], beta[kMaxBatch], bnorm2[kMaxBatch], rr[kMaxBatch],
      pq[kMaxBatch];
  double tol2[kMaxBatch];  // squared relative tolerance of each column
  int done[kMaxBatch], iters[kMaxBatch], status[kMaxBatch];  // status: 0 running, 1 converged,
                                                            // 2 max_iter, -6 breakdown
  int maxit[kMaxBatch];  // iteration cap of each column
  int all_done, K;
};

// Stopping parameters of the slots that (re)start in a continuous batch:
// each column converges on its own request's tolerance and iteration cap.
struct SlotStop {
  double tol[kMaxBatch];
  int maxit[kMaxBatch];
};

inline int64_t sell_blocks(int64_t r0, int64_t r1) {
  if (r1 <= r0) return 0;
  int64_t s0 = r0 / kWave, s1 = (r1 + kWave - 1) / kWave;
  return (s1 - s0 + kSlicesPerBlock - 1) / kSlicesPerBlock;
}
inline int64_t vec_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

// ---- fine matrix (SELL, difference form) ---------------------------------
// Rows [a0, a1) and [b0, b1) whose residual is zero in exact arithmetic: the
// rows of the last colour of a forward multicolour Gauss-Seidel sweep with
// relaxation 1, whose neighbours all lie in colours swept before them.
struct ZeroRows {
  int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
};
// y = A x (mode 0) or y = g - A x (mode 1) on rows [r0, r1).  With partial,
// partial[block * K + k] = sum over the block's rows of x_ik y_ik.  order
// (optional): the range's slices in visit order (offsets from slice r0 / 64),
// so that the blocks of one XCD take one spatial region of every colour.  In
// mode 1 the rows of zr get y = 0 without reading their entries.
// Mode 1 only: with y2, the rows r >= y2_from are also stored to y2 (a copy
// of the result for a second consumer).
template <class T>
void launch_spmv(hipStream_t st, int K, const Sell &A, int mode, int64_t r0, int64_t r1, const T *x, const T *g,
                 T *y, double *partial, const int *done, const int32_t *order = nullptr, ZeroRows zr = ZeroRows(),
                 T *y2 = nullptr, int64_t y2_from = 0);
// y = g - A x (mode 1 of launch_spmv, the same arithmetic row by row) on the
// listed rows rows[0 .. nr) only, rows of zr written as zero.  A holds
// exactly those rows: its row i is the matrix's row rows[i], with the same
// entries in the same order.
template <class T>
void launch_spmv_rows(hipStream_t st, int K, const Sell &A, const int32_t *rows, int64_t nr, const T *x, const T *g,
                      T *y, const int *done, ZeroRows zr);
// One multicolour Gauss-Seidel step on the rows [a0,a1) and [b0,b1) (rows of
// one colour): x_i += (g_i - (A x)_i) / a_ii.
// Zero start (the first sweep from x = 0): of the top block (j < n_top) only
// the columns j < top_lim are read, of the rest only j < bar_lim; every other
// value (the colours not swept yet, and the row's own) is taken as zero
// without being read, so x needs no fill beforehand.
struct ZeroStart {
  bool on = false;
  int64_t n_top = 0, top_lim = 0, bar_lim = 0;
};
// With x2, the updated rows r >= x2_from are also stored to x2.
template <class T>
void launch_gs(hipStream_t st, int K, const Sell &A, int64_t a0, int64_t a1, int64_t b0, int64_t b1, const T *g,
               T *x, const int *done, ZeroStart zs = ZeroStart(), T *x2 = nullptr, int64_t x2_from = 0);
// The Gauss-Seidel step of launch_gs (the same arithmetic row by row) on the
// listed rows rows[0 .. nr) only; the rows must share no entries.  A holds
// exactly those rows, as for launch_spmv_rows.
template <class T>
void launch_gs_rows(hipStream_t st, int K, const Sell &A, const int32_t *rows, int64_t nr, const T *g, T *x,
                    const int *done, ZeroStart zs);
// y = E x (accumulate: y += E x) for a rectangular SELL matrix, rows [0, nrows).
template <class T>
void launch_rect(hipStream_t st, int K, const Sell &E, bool accumulate, const T *x, T *y, const int *done);
// z_i = (E~ y)_i + (i >= n_top ? w_i : 0); partial[block * K + k] = sum r_ik z_ik.
template <class T>
void launch_prolong_sum(hipStream_t st, int K, const Sell &E, int64_t n_top, const T *y, const T *w, const T *r,
                        T *z, double *partial, const int *done);

// ---- coarse operators and transfers (CsrG) -------------------------------
// mode 0: y = A x, 1: y = g - A x (square); rect: y = P x or y += P x.
template <class T>
void launch_csr_spmv(hipStream_t st, int K, const CsrG &A, int mode, int64_t r0, int64_t r1, const T *x,
                     const T *g, T *y, const int *done);
// Block multicolour (patch) order of a coarse level: its unknowns are stored
// patch by patch (patch colour, patch, local colour), a patch holding at most
// kPatchLdsRows unknowns.  Unknowns of patches of one colour are never
// coupled, so a forward sweep is, patch colour by patch colour, one exact
// triangular solve per patch: with h_p = g_p - A_pq x_q over the couplings
// to other patches (and to the patch's own later unknowns, with their old
// values), the patch's new values are (D_p + L_p)^{-1} h_p, L_p the strictly
// lower part of the patch's block in stored order -- the sequential SOR
// sweep in that order.  Backward: (D_p + U_p)^{-1} = ((D_p + L_p)^{-1})^T.
constexpr int kPatchLdsRows = 128;
struct PatchSweep {
  const int32_t *prow = nullptr;  // stored patch i: rows [prow[i], prow[i+1])
  const int64_t *toff = nullptr;  // its factors start at toff[i] (m (m + 1) / 2 entries each)
  // FP64: F = (D_p + L_p)^{-1} packed by rows (row r: columns 0..r) and F^T
  // packed by rows (row r: columns r..m-1); FP32 (row-scaled operator):
  // F D_p and F^T D_p, rounded
  const double *tf64 = nullptr, *tb64 = nullptr;
  const float *tf32 = nullptr, *tb32 = nullptr;
};
// One Gauss-Seidel sweep over the patches [p0, p0 + np) of one patch colour,
// one block per patch (the patch colours launched in turn, ascending for a
// forward sweep and descending for backward).  zlim >= 0: zero start
// (forward from x = 0): of the other patches only the rows j < zlim (the
// patch colours swept before) are read and the rest taken as zero, so x
// needs no fill.
template <class T>
void launch_patch_gs(hipStream_t st, int K, const CsrG &A, const PatchSweep &S, int64_t p0, int64_t np, const T *g,
                     T *x, const int *done, int64_t zlim, bool backward);
template <class T>
void launch_csr_rect(hipStream_t st, int K, const CsrG &P, bool accumulate, const T *x, T *y, const int *done);
// x = Cinv g (dense m x m FP64, symmetric, row-major), K columns; part:
// dense_chunks(m) * m * K doubles of scratch for the column chunks' partial sums.
constexpr int kDenseChunk = 512;
inline int64_t dense_chunks(int64_t m) { return (m + kDenseChunk - 1) / kDenseChunk; }
template <class T>
void launch_dense(hipStream_t st, int K, const double *Cinv, int64_t m, const T *g, T *x, double *part,
                  const int *done);

// ---- vectors ([n][K]) ----------------------------------------------------
template <class T>
void launch_fill(hipStream_t st, T *x, int64_t count, T v, const int *done);
template <class T>
void launch_copy(hipStream_t st, const T *a, T *b, int64_t count, const int *done);
// partial[block * K + k] = sum a_ik b_ik
template <class T>
void launch_dot(hipStream_t st, int K, const T *a, const T *b, int64_t n, double *partial, const int *done);
// z_i += w_i for rows i >= row0; partial[block * K + k] = sum r_ik z_ik (updated z)
template <class T>
void launch_add_dot(hipStream_t st, int K, const T *w, const T *r, T *z, int64_t row0, int64_t n, double *partial,
                    const int *done);
template <class T>
void launch_jacobi(hipStream_t st, int K, const T *r, const double *diag, T *z, int64_t n, const int *done);
// natural <-> storage order for column k of a batch (stride K)
void launch_gather(hipStream_t st, int K, int k, const double *nat, const int64_t *perm, double *sto, int64_t n);
void launch_scatter(hipStream_t st, int K, int k, const double *sto, const int64_t *perm, double *nat, int64_t n);
// mixed precision: r32 = r64 * scale[k];  x64 (+)= scale[k] * d32
void launch_demote(hipStream_t st, int K, const double *r64, const double *scale, float *r32, int64_t n,
                   const int *done);
void launch_promote(hipStream_t st, int K, const float *d32, const double *scale, double *x64, int64_t n,
                    bool accumulate, const int *done);

// ---- PCG scalars (single-block kernels sum partials in index order) ------
void launch_pcg_init(hipStream_t st, int K, Scal *s, const double *pb, int64_t npb, double tol, int maxit);
void launch_pcg_set_rho(hipStream_t st, int K, Scal *s, const double *p, int64_t np);
void launch_pcg_alpha(hipStream_t st, int K, Scal *s, const double *p, int64_t np);
template <class T>
void launch_pcg_xr(hipStream_t st, int K, Scal *s, T *x, T *r, const T *p, const T *q, int64_t n, double *partial);
void launch_pcg_conv(hipStream_t st, int K, Scal *s, const double *p, int64_t np);
void launch_pcg_beta(hipStream_t st, int K, Scal *s, const double *p, int64_t np);
template <class T>
void launch_pcg_p(hipStream_t st, int K, Scal *s, T *pvec, const T *z, int64_t n);
// out[k] = sum of the partials of column k
void launch_reduce(hipStream_t st, int K, const double *p, int64_t np, double *out);
// before a restart: clears done/status of the columns whose bit in keep is 0
void launch_pcg_resume(hipStream_t st, int K, Scal *s, unsigned keep);

// ---- extended iterate across restarts (refine.hip) ----------------------
// The solution is the unevaluated sum hi + lo ([n][K] each); a restart's
// correction x is folded in without rounding error for the columns in mask
// (hi + x rounded, its error added to lo; x = 0 afterwards).
void launch_fold(hipStream_t st, int K, unsigned mask, double *hi, double *lo, double *x, int64_t n);
// res = b - A (hi + lo) on the fine difference-form matrix, with error-free
// products and double-double sums, rounded once (K in {1,2,4,8}).
void launch_residual_ext(hipStream_t st, int K, const Sell &A, const double *b, const double *hi, const double *lo,
                         double *res);
// out = hi + lo (rounded), count entries
void launch_round(hipStream_t st, const double *hi, const double *lo, double *out, int64_t count);

// Continuous batching (K = kMaxBatch slots): columns in `mask` (re)start
// while the others keep their state.
//   join: hi_k = lo_k = x_k = 0, r_k = b_k;   restart: r_k = res_k (after a fold)
void launch_slot_vectors(hipStream_t st, unsigned mask, bool restart, const double *b, const double *res,
                         double *hi, double *lo, double *x, double *r, int64_t n);
// join: bnorm2_k from the partials of b.b, iters_k = 0; both: done_k = 0
// (1 for a zero right-hand side), status_k = 0, and the FP32 scaling of the
// preconditioner input scale_in_k = 1/||b_k||, scale_out_k = ||b_k||
void launch_slot_scalars(hipStream_t st, unsigned mask, bool restart, Scal *s, const double *pb, int64_t npb,
                         const SlotStop &stop, double *scale_in, double *scale_out);
// rho_k from the partials of r.z, for the columns in mask
void launch_slot_rho(hipStream_t st, unsigned mask, Scal *s, const double *p, int64_t np);
// p_k = z_k for the columns in mask
void launch_slot_copy(hipStream_t st, unsigned mask, const double *z, double *p, int64_t n);

}  // namespace vemg
