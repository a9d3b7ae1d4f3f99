// Device kernels of the PCG hot path (gfx950, wave64) and their launchers.
// All launchers enqueue on the given stream and never synchronise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vemg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kSlicesPerBlock = kBlock / kWave;

// SELL-64 matrix: 64 consecutive rows form a slice stored column-major and
// padded to the slice's longest row, so lane t of a wavefront reads entry k
// of row 64 s + t at sptr[s] + 64 k + t (coalesced).  Only off-diagonal
// entries are stored; `d` holds the per-row diagonal term (the deficit for
// the difference form, a_ii for the standard form).  Padding entries have
// value 0 and point at the row itself (square) or column 0 (rectangular).
struct Sell {
  const int64_t *sptr = nullptr;  // nslices + 1 entry offsets
  const int32_t *col = nullptr;
  const double *val = nullptr;
  const double *d = nullptr;
  int64_t nrows = 0;
};

// CSR matrix processed by groups of G lanes per row (G = 4..64, a power of
// two chosen from the mean row length): the group reads consecutive entries
// of its row (coalesced) and reduces with cross-lane shuffles, so long rows
// (coarse multigrid operators, restrictions) cost a few memory round trips
// instead of one per entry.  `d` as for Sell (square standard form only).
struct CsrG {
  const int32_t *ptr = nullptr;  // nrows + 1
  const int32_t *col = nullptr;
  const double *val = nullptr;
  const double *d = nullptr;
  int64_t nrows = 0;
  int G = 4;
};

// Device scalars of one PCG solve.
struct Scal {
  double rho, alpha, beta, bnorm2, tol2, rr, pq, dot;
  int done, iters, maxit, status;  // status: 0 running, 1 converged, 2 max_iter, -6 breakdown
};

// number of blocks covering rows [r0, r1)
inline int64_t sell_blocks(int64_t r0, int64_t r1) {
  if (r1 <= r0) return 0;
  int64_t s0 = r0 / kWave, s1 = (r1 + kWave - 1) / kWave;
  return (s1 - s0 + kSlicesPerBlock - 1) / kSlicesPerBlock;
}
inline int64_t vec_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

// y = A x (mode 0) or y = g - A x (mode 1) on rows [r0, r1); difference form
// y_i = sum_j a_ij (x_j - x_i) + d_i x_i when diff, else d_i x_i + sum_j a_ij x_j.
// With partial != null, partial[block] = sum over the block's rows of x_i y_i.
void launch_spmv(hipStream_t st, const Sell &A, bool diff, int mode, int64_t r0, int64_t r1,
                 const double *x, const double *g, double *y, double *partial, const int *done);
// One multicolour Gauss-Seidel step on the rows [a0,a1) and [b0,b1) (rows of
// one colour): x_i += (g_i - (A x)_i) / a_ii.
void launch_gs(hipStream_t st, const Sell &A, bool diff, int64_t a0, int64_t a1, int64_t b0, int64_t b1,
               const double *g, double *x, const int *done);
// y = P x (accumulate: y += P x) for a rectangular SELL matrix, rows [0, nrows).
void launch_rect(hipStream_t st, const Sell &P, bool accumulate, const double *x, double *y,
                 const int *done);
// z_i = (E~ y)_i + (i >= n_top ? w_i : 0); partial[block] = sum r_i z_i.
void launch_prolong_sum(hipStream_t st, const Sell &E, int64_t n_top, const double *y, const double *w,
                        const double *r, double *z, double *partial, const int *done);
// x = Cinv g (dense m x m, row-major).
void launch_dense(hipStream_t st, const double *Cinv, int64_t m, const double *g, double *x, const int *done);
void launch_fill(hipStream_t st, double *x, int64_t n, double v, const int *done);
void launch_copy(hipStream_t st, const double *a, double *b, int64_t n, const int *done);
// partial[block] = sum a_i b_i
void launch_dot(hipStream_t st, const double *a, const double *b, int64_t n, double *partial, const int *done);
// z = r / diag
void launch_jacobi(hipStream_t st, const double *r, const double *diag, double *z, int64_t n, const int *done);
// storage <-> natural order
void launch_gather(hipStream_t st, const double *nat, const int64_t *perm, double *sto, int64_t n);
void launch_scatter(hipStream_t st, const double *sto, const int64_t *perm, double *nat, int64_t n);

// CsrG versions.  mode 0: y = A x, 1: y = g - A x (square, standard form);
// rect: y = P x or y += P x over rows [0, nrows).
void launch_csr_spmv(hipStream_t st, const CsrG &A, int mode, int64_t r0, int64_t r1, const double *x,
                     const double *g, double *y, const int *done);
void launch_csr_gs(hipStream_t st, const CsrG &A, int64_t r0, int64_t r1, const double *g, double *x,
                   const int *done);
void launch_csr_rect(hipStream_t st, const CsrG &P, bool accumulate, const double *x, double *y, const int *done);

// PCG pieces (single-block scalar kernels sum the partials in index order).
void launch_pcg_init(hipStream_t st, Scal *s, const double *pb, int64_t npb, double tol, int maxit);
void launch_pcg_set_rho(hipStream_t st, Scal *s, const double *p, int64_t np);
void launch_pcg_alpha(hipStream_t st, Scal *s, const double *p, int64_t np);
void launch_pcg_xr(hipStream_t st, Scal *s, double *x, double *r, const double *p, const double *q, int64_t n,
                   double *partial);
void launch_pcg_conv(hipStream_t st, Scal *s, const double *p, int64_t np, double *hist);
void launch_pcg_beta(hipStream_t st, Scal *s, const double *p, int64_t np);
void launch_pcg_p(hipStream_t st, Scal *s, double *pvec, const double *z, int64_t n);
void launch_reduce(hipStream_t st, const double *p, int64_t np, double *out);
// clears the done flag before a restart (keeps the iteration count)
void launch_pcg_resume(hipStream_t st, Scal *s);

}  // namespace vemg
