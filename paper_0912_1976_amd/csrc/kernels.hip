// HIP kernels of the PCG hot path for gfx950 (CDNA4, wave64).
//
// The path is sparse and bandwidth-bound, so there is no MFMA here: every
// kernel streams its matrix once with coalesced SELL-64 loads, gathers the
// vector entries it needs through L2 / the Infinity Cache, and keeps
// reductions deterministic (per-block partials summed in index order by a
// single-block consumer).  Blocks are renumbered so that each of the eight
// XCDs works on a contiguous range of rows, which keeps the gathered vector
// lines in that XCD's L2.
#include "kernels.hpp"

namespace vemg {

namespace {

// Hardware dispatches block b to XCD b % 8; give every XCD a contiguous chunk.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  int64_t q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kSlicesPerBlock];
  v = wave_sum(v);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kSlicesPerBlock; ++k) t += red[k];
  }
  return t;
}

template <bool DIFF>
__device__ __forceinline__ void row_terms(const Sell &A, int64_t s, int lane, int64_t r, const double *__restrict__ x,
                                          double xr, double &acc, double &offsum) {
  const int64_t base = A.sptr[s];
  const int len = (int)((A.sptr[s + 1] - base) >> 6);
  const int32_t *__restrict__ cp = A.col + base + lane;
  const double *__restrict__ vp = A.val + base + lane;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
  int k = 0;
  // four independent entries in flight per lane
  for (; k + 3 < len; k += 4) {
    const int32_t c0 = cp[(int64_t)k * 64], c1 = cp[(int64_t)(k + 1) * 64];
    const int32_t c2 = cp[(int64_t)(k + 2) * 64], c3 = cp[(int64_t)(k + 3) * 64];
    const double v0 = vp[(int64_t)k * 64], v1 = vp[(int64_t)(k + 1) * 64];
    const double v2 = vp[(int64_t)(k + 2) * 64], v3 = vp[(int64_t)(k + 3) * 64];
    const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    if (DIFF) {
      a0 += v0 * (x0 - xr);
      a1 += v1 * (x1 - xr);
      a2 += v2 * (x2 - xr);
      a3 += v3 * (x3 - xr);
    } else {
      a0 += v0 * x0;
      a1 += v1 * x1;
      a2 += v2 * x2;
      a3 += v3 * x3;
    }
    o0 += v0;
    o1 += v1;
    o2 += v2;
    o3 += v3;
  }
  for (; k < len; ++k) {
    const int32_t c0 = cp[(int64_t)k * 64];
    const double v0 = vp[(int64_t)k * 64];
    a0 += DIFF ? v0 * (x[c0] - xr) : v0 * x[c0];
    o0 += v0;
  }
  acc = (a0 + a1) + (a2 + a3);
  offsum = (o0 + o1) + (o2 + o3);
}

// Sum of a row of a CsrG matrix by its group of G lanes (result in every lane
// of the group).
template <int G>
__device__ __forceinline__ double group_row(const CsrG &A, int64_t r, int gl, const double *__restrict__ x) {
  const int32_t b = A.ptr[r], e = A.ptr[r + 1];
  double a0 = 0.0, a1 = 0.0;
  int k = b + gl;
  for (; k + G < e; k += 2 * G) {
    a0 += A.val[k] * x[A.col[k]];
    a1 += A.val[k + G] * x[A.col[k + G]];
  }
  if (k < e) a0 += A.val[k] * x[A.col[k]];
  double t = a0 + a1;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, G);
  return t;
}

template <int G, int MODE>
__global__ __launch_bounds__(kBlock) void k_csr_spmv(CsrG A, int64_t r0, int64_t r1, const double *__restrict__ x,
                                                     const double *__restrict__ g, double *__restrict__ y,
                                                     const int *__restrict__ done) {
  if (done && *done) return;
  const int gl = threadIdx.x & (G - 1);
  const int64_t r = r0 + ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  if (r >= r1) return;
  const double t = group_row<G>(A, r, gl, x);
  if (gl == 0) {
    // MODE 0/1: square standard form; 2/3: rectangular, 3 accumulates
    if (MODE == 0) y[r] = t + A.d[r] * x[r];
    else if (MODE == 1) y[r] = g[r] - (t + A.d[r] * x[r]);
    else if (MODE == 2) y[r] = t;
    else y[r] += t;
  }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_csr_gs(CsrG A, int64_t r0, int64_t r1, const double *__restrict__ g,
                                                   double *__restrict__ x, const int *__restrict__ done) {
  if (done && *done) return;
  const int gl = threadIdx.x & (G - 1);
  const int64_t r = r0 + ((int64_t)blockIdx.x * kBlock + threadIdx.x) / G;
  if (r >= r1) return;
  const double t = group_row<G>(A, r, gl, x);  // off-diagonal part only
  if (gl == 0) {
    const double dr = A.d[r];
    x[r] = (g[r] - t) / dr;
  }
}

template <bool DIFF, int MODE, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv(Sell A, int64_t r0, int64_t r1, int64_t s_first, int64_t nb,
                                                 const double *__restrict__ x, const double *__restrict__ g,
                                                 double *__restrict__ y, double *__restrict__ partial,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int lane = threadIdx.x & 63;
  const int64_t s = s_first + blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  double prod = 0.0;
  if (r >= r0 && r < r1) {
    const double xr = x[r];
    double acc, off;
    row_terms<DIFF>(A, s, lane, r, x, xr, acc, off);
    acc += A.d[r] * xr;
    const double out = (MODE == 0) ? acc : g[r] - acc;
    y[r] = out;
    if (DOT) prod = xr * out;
  }
  if (DOT) {
    double t = block_sum(prod);
    if (threadIdx.x == 0) partial[blk] = t;
  }
}

template <bool DIFF>
__global__ __launch_bounds__(kBlock) void k_gs(Sell A, int64_t a0, int64_t a1, int64_t sa, int64_t nba, int64_t b0,
                                               int64_t b1, int64_t sb, int64_t nbt, const double *__restrict__ g,
                                               double *__restrict__ x, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t blk = xcd_block(blockIdx.x, nbt);
  int64_t r0 = a0, r1 = a1, sf = sa;
  if (blk >= nba) {
    blk -= nba;
    r0 = b0;
    r1 = b1;
    sf = sb;
  }
  const int lane = threadIdx.x & 63;
  const int64_t s = sf + blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  if (r < r0 || r >= r1) return;
  const double xr = x[r];
  double acc, off;
  row_terms<DIFF>(A, s, lane, r, x, xr, acc, off);
  const double dr = A.d[r];
  const double diag = DIFF ? dr - off : dr;
  x[r] = xr + (g[r] - (acc + dr * xr)) / diag;
}

template <bool ACC>
__global__ __launch_bounds__(kBlock) void k_rect(Sell P, int64_t nb, const double *__restrict__ x,
                                                 double *__restrict__ y, const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int lane = threadIdx.x & 63;
  const int64_t s = blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  if (r >= P.nrows) return;
  double acc, off;
  row_terms<false>(P, s, lane, r, x, 0.0, acc, off);
  y[r] = ACC ? y[r] + acc : acc;
}

__global__ __launch_bounds__(kBlock) void k_prolong_sum(Sell E, int64_t n_top, int64_t nb, const double *__restrict__ ys,
                                                        const double *__restrict__ w, const double *__restrict__ rv,
                                                        double *__restrict__ z, double *__restrict__ partial,
                                                        const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int lane = threadIdx.x & 63;
  const int64_t s = blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  double prod = 0.0;
  if (r < E.nrows) {
    double acc = 0.0, off;
    if (ys) row_terms<false>(E, s, lane, r, ys, 0.0, acc, off);
    if (r >= n_top) acc += w[r];
    z[r] = acc;
    prod = rv[r] * acc;
  }
  double t = block_sum(prod);
  if (threadIdx.x == 0) partial[blk] = t;
}

// one wavefront per row of the dense coarsest inverse
__global__ __launch_bounds__(kBlock) void k_dense(const double *__restrict__ C, int64_t m,
                                                  const double *__restrict__ g, double *__restrict__ x,
                                                  const int *__restrict__ done) {
  if (done && *done) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kSlicesPerBlock + (threadIdx.x >> 6);
  if (i >= m) return;
  double t = 0.0;
  for (int64_t j = lane; j < m; j += 64) t += C[i * m + j] * g[j];
  t = wave_sum(t);
  if (lane == 0) x[i] = t;
}

__global__ void k_fill(double *__restrict__ x, int64_t n, double v, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_copy(const double *__restrict__ a, double *__restrict__ b, int64_t n, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

__global__ __launch_bounds__(kBlock) void k_dot(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                                                double *__restrict__ partial, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double t = (i < n) ? a[i] * b[i] : 0.0;
  t = block_sum(t);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_jacobi(const double *__restrict__ r, const double *__restrict__ dg, double *__restrict__ z, int64_t n,
                         const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = r[i] / dg[i];
}

__global__ void k_gather(const double *__restrict__ nat, const int64_t *__restrict__ perm, double *__restrict__ sto,
                         int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sto[i] = nat[perm[i]];
}

__global__ void k_scatter(const double *__restrict__ sto, const int64_t *__restrict__ perm, double *__restrict__ nat,
                          int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nat[perm[i]] = sto[i];
}

// fixed-order sum of np partials by one block
__device__ __forceinline__ double sum_partials(const double *__restrict__ p, int64_t np) {
  double t = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += kBlock) t += p[k];
  __shared__ double buf[kBlock];
  buf[threadIdx.x] = t;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) buf[threadIdx.x] += buf[threadIdx.x + o];
    __syncthreads();
  }
  return buf[0];
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *p, int64_t np, double *out) {
  double t = sum_partials(p, np);
  if (threadIdx.x == 0) *out = t;
}

__global__ __launch_bounds__(kBlock) void k_pcg_init(Scal *s, const double *pb, int64_t npb, double tol, int maxit) {
  double t = sum_partials(pb, npb);
  if (threadIdx.x == 0) {
    s->bnorm2 = t;
    s->tol2 = tol * tol;
    s->maxit = maxit;
    s->iters = 0;
    s->done = 0;
    s->status = 0;
    s->rho = 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_pcg_set_rho(Scal *s, const double *p, int64_t np) {
  double t = sum_partials(p, np);
  if (threadIdx.x == 0) s->rho = t;
}

__global__ __launch_bounds__(kBlock) void k_pcg_alpha(Scal *s, const double *p, int64_t np) {
  if (s->done) return;
  double pq = sum_partials(p, np);
  if (threadIdx.x == 0) {
    s->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(s->rho)) {
      s->done = 1;
      s->status = -6;
      s->alpha = 0.0;
    } else {
      s->alpha = s->rho / pq;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_pcg_xr(const Scal *s, double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   int64_t n, double *__restrict__ partial) {
  if (s->done) return;
  const double a = s->alpha;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double t = 0.0;
  if (i < n) {
    x[i] += a * p[i];
    double ri = r[i] - a * q[i];
    r[i] = ri;
    t = ri * ri;
  }
  t = block_sum(t);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_pcg_conv(Scal *s, const double *p, int64_t np, double *hist) {
  if (s->done) return;
  double rr = sum_partials(p, np);
  if (threadIdx.x == 0) {
    int it = s->iters + 1;
    s->iters = it;
    s->rr = rr;
    if (hist) hist[it] = rr;
    if (!isfinite(rr)) {
      s->done = 1;
      s->status = -6;
    } else if (rr <= s->tol2 * s->bnorm2) {
      s->done = 1;
      s->status = 1;
    } else if (it >= s->maxit) {
      s->done = 1;
      s->status = 2;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_pcg_beta(Scal *s, const double *p, int64_t np) {
  if (s->done) return;
  double rz = sum_partials(p, np);
  if (threadIdx.x == 0) {
    s->beta = rz / s->rho;
    s->rho = rz;
  }
}

__global__ void k_pcg_p(const Scal *s, double *__restrict__ p, const double *__restrict__ z, int64_t n) {
  if (s->done) return;
  const double b = s->beta;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + b * p[i];
}

__global__ void k_pcg_resume(Scal *s) {
  if (threadIdx.x == 0) {
    s->done = 0;
    s->status = 0;
  }
}

inline dim3 grid(int64_t nb) { return dim3((unsigned)nb); }

}  // namespace

void launch_spmv(hipStream_t st, const Sell &A, bool diff, int mode, int64_t r0, int64_t r1, const double *x,
                 const double *g, double *y, double *partial, const int *done) {
  int64_t nb = sell_blocks(r0, r1);
  if (!nb) return;
  int64_t sf = r0 / kWave;
#define VEMG_SPMV(D, M, T) hipLaunchKernelGGL((k_spmv<D, M, T>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, sf, nb, x, g, y, partial, done)
  if (diff) {
    if (mode == 0) {
      if (partial) VEMG_SPMV(true, 0, true); else VEMG_SPMV(true, 0, false);
    } else {
      if (partial) VEMG_SPMV(true, 1, true); else VEMG_SPMV(true, 1, false);
    }
  } else {
    if (mode == 0) {
      if (partial) VEMG_SPMV(false, 0, true); else VEMG_SPMV(false, 0, false);
    } else {
      if (partial) VEMG_SPMV(false, 1, true); else VEMG_SPMV(false, 1, false);
    }
  }
#undef VEMG_SPMV
}

void launch_gs(hipStream_t st, const Sell &A, bool diff, int64_t a0, int64_t a1, int64_t b0, int64_t b1,
               const double *g, double *x, const int *done) {
  int64_t nba = sell_blocks(a0, a1), nbb = sell_blocks(b0, b1);
  int64_t nbt = nba + nbb;
  if (!nbt) return;
  int64_t sa = a0 / kWave, sb = b0 / kWave;
  if (diff)
    hipLaunchKernelGGL((k_gs<true>), grid(nbt), dim3(kBlock), 0, st, A, a0, a1, sa, nba, b0, b1, sb, nbt, g, x, done);
  else
    hipLaunchKernelGGL((k_gs<false>), grid(nbt), dim3(kBlock), 0, st, A, a0, a1, sa, nba, b0, b1, sb, nbt, g, x, done);
}

void launch_rect(hipStream_t st, const Sell &P, bool accumulate, const double *x, double *y, const int *done) {
  int64_t nb = sell_blocks(0, P.nrows);
  if (!nb) return;
  if (accumulate)
    hipLaunchKernelGGL((k_rect<true>), grid(nb), dim3(kBlock), 0, st, P, nb, x, y, done);
  else
    hipLaunchKernelGGL((k_rect<false>), grid(nb), dim3(kBlock), 0, st, P, nb, x, y, done);
}

void launch_prolong_sum(hipStream_t st, const Sell &E, int64_t n_top, const double *y, const double *w,
                        const double *r, double *z, double *partial, const int *done) {
  int64_t nb = sell_blocks(0, E.nrows);
  if (!nb) return;
  hipLaunchKernelGGL(k_prolong_sum, grid(nb), dim3(kBlock), 0, st, E, n_top, nb, y, w, r, z, partial, done);
}

void launch_dense(hipStream_t st, const double *Cinv, int64_t m, const double *g, double *x, const int *done) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_dense, grid((m + kSlicesPerBlock - 1) / kSlicesPerBlock), dim3(kBlock), 0, st, Cinv, m, g, x,
                     done);
}

void launch_fill(hipStream_t st, double *x, int64_t n, double v, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, grid(vec_blocks(n)), dim3(kBlock), 0, st, x, n, v, done);
}

void launch_copy(hipStream_t st, const double *a, double *b, int64_t n, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, grid(vec_blocks(n)), dim3(kBlock), 0, st, a, b, n, done);
}

void launch_dot(hipStream_t st, const double *a, const double *b, int64_t n, double *partial, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_dot, grid(vec_blocks(n)), dim3(kBlock), 0, st, a, b, n, partial, done);
}

void launch_jacobi(hipStream_t st, const double *r, const double *diag, double *z, int64_t n, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_jacobi, grid(vec_blocks(n)), dim3(kBlock), 0, st, r, diag, z, n, done);
}

void launch_gather(hipStream_t st, const double *nat, const int64_t *perm, double *sto, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather, grid(vec_blocks(n)), dim3(kBlock), 0, st, nat, perm, sto, n);
}

void launch_scatter(hipStream_t st, const double *sto, const int64_t *perm, double *nat, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter, grid(vec_blocks(n)), dim3(kBlock), 0, st, sto, perm, nat, n);
}

template <int MODE>
static void csr_dispatch(hipStream_t st, const CsrG &A, int64_t r0, int64_t r1, const double *x, const double *g,
                         double *y, const int *done) {
  int64_t rows = r1 - r0;
  if (rows <= 0) return;
  int64_t nb = (rows * A.G + kBlock - 1) / kBlock;
  switch (A.G) {
    case 4: hipLaunchKernelGGL((k_csr_spmv<4, MODE>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, x, g, y, done); break;
    case 8: hipLaunchKernelGGL((k_csr_spmv<8, MODE>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, x, g, y, done); break;
    case 16: hipLaunchKernelGGL((k_csr_spmv<16, MODE>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, x, g, y, done); break;
    case 32: hipLaunchKernelGGL((k_csr_spmv<32, MODE>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, x, g, y, done); break;
    default: hipLaunchKernelGGL((k_csr_spmv<64, MODE>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, x, g, y, done); break;
  }
}

void launch_csr_spmv(hipStream_t st, const CsrG &A, int mode, int64_t r0, int64_t r1, const double *x,
                     const double *g, double *y, const int *done) {
  if (mode == 0) csr_dispatch<0>(st, A, r0, r1, x, g, y, done);
  else csr_dispatch<1>(st, A, r0, r1, x, g, y, done);
}

void launch_csr_rect(hipStream_t st, const CsrG &P, bool accumulate, const double *x, double *y, const int *done) {
  if (accumulate) csr_dispatch<3>(st, P, 0, P.nrows, x, nullptr, y, done);
  else csr_dispatch<2>(st, P, 0, P.nrows, x, nullptr, y, done);
}

void launch_csr_gs(hipStream_t st, const CsrG &A, int64_t r0, int64_t r1, const double *g, double *x,
                   const int *done) {
  int64_t rows = r1 - r0;
  if (rows <= 0) return;
  int64_t nb = (rows * A.G + kBlock - 1) / kBlock;
  switch (A.G) {
    case 4: hipLaunchKernelGGL((k_csr_gs<4>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, g, x, done); break;
    case 8: hipLaunchKernelGGL((k_csr_gs<8>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, g, x, done); break;
    case 16: hipLaunchKernelGGL((k_csr_gs<16>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, g, x, done); break;
    case 32: hipLaunchKernelGGL((k_csr_gs<32>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, g, x, done); break;
    default: hipLaunchKernelGGL((k_csr_gs<64>), grid(nb), dim3(kBlock), 0, st, A, r0, r1, g, x, done); break;
  }
}

void launch_pcg_init(hipStream_t st, Scal *s, const double *pb, int64_t npb, double tol, int maxit) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kBlock), 0, st, s, pb, npb, tol, maxit);
}
void launch_pcg_set_rho(hipStream_t st, Scal *s, const double *p, int64_t np) {
  hipLaunchKernelGGL(k_pcg_set_rho, dim3(1), dim3(kBlock), 0, st, s, p, np);
}
void launch_pcg_alpha(hipStream_t st, Scal *s, const double *p, int64_t np) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(kBlock), 0, st, s, p, np);
}
void launch_pcg_xr(hipStream_t st, Scal *s, double *x, double *r, const double *p, const double *q, int64_t n,
                   double *partial) {
  hipLaunchKernelGGL(k_pcg_xr, grid(vec_blocks(n)), dim3(kBlock), 0, st, s, x, r, p, q, n, partial);
}
void launch_pcg_conv(hipStream_t st, Scal *s, const double *p, int64_t np, double *hist) {
  hipLaunchKernelGGL(k_pcg_conv, dim3(1), dim3(kBlock), 0, st, s, p, np, hist);
}
void launch_pcg_beta(hipStream_t st, Scal *s, const double *p, int64_t np) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(kBlock), 0, st, s, p, np);
}
void launch_pcg_p(hipStream_t st, Scal *s, double *pvec, const double *z, int64_t n) {
  hipLaunchKernelGGL(k_pcg_p, grid(vec_blocks(n)), dim3(kBlock), 0, st, s, pvec, z, n);
}
void launch_pcg_resume(hipStream_t st, Scal *s) { hipLaunchKernelGGL(k_pcg_resume, dim3(1), dim3(64), 0, st, s); }
void launch_reduce(hipStream_t st, const double *p, int64_t np, double *out) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, p, np, out);
}

}  // namespace vemg
