// Extended-precision bookkeeping of the PCG iterate across restarts.
//
// Each restart of PCG solves for a correction from zero; the solution is
// kept as the unevaluated sum hi + lo of two doubles.  Folding a correction
// in is an error-free addition (the rounding error of hi + x moves to lo),
// and the residual b - A (hi + lo) that decides the next restart is
// evaluated with error-free products and a double-double accumulator.  At
// small aspect ratio the FP64 rounding of a solution perturbs its residual
// by about eps * ||A|| ||x||, which is far above 1e-8 relative; with the
// extended iterate and residual, refinement drives the solution itself to
// FP64 accuracy and the residual test measures the iterate, not its
// rounding.
//
// This file is compiled with -ffp-contract=off: the error-free
// transformations below rely on every sum and product being rounded as
// written (the one fused operation is the explicit fma).
#include "kernels.hpp"

namespace vemg {

namespace {

struct DD {
  double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD fast_two_sum(double a, double b) {  // |a| >= |b| or a == 0
  const double s = a + b;
  return {s, b - (s - a)};
}

__device__ __forceinline__ DD two_prod(double a, double b) {
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
  const DD s = two_sum(a.hi, b.hi);
  return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

// a * (x.hi + x.lo), x.lo small
__device__ __forceinline__ DD dd_scale(double a, DD x) {
  DD p = two_prod(a, x.hi);
  p.lo += a * x.lo;
  return p;
}

__device__ __forceinline__ int64_t grid_index() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
inline dim3 grid_of(int64_t count, int block) { return dim3((unsigned)((count + block - 1) / block)); }

// res_i = b_i - (A (hi + lo))_i for every column; A in difference form:
// (A x)_i = sum_j a_ij (x_j - x_i) + d_i x_i, one thread per row.
template <int K>
__global__ __launch_bounds__(kBlock) void k_residual_ext(Sell A, const double *__restrict__ b,
                                                         const double *__restrict__ hi,
                                                         const double *__restrict__ lo,
                                                         double *__restrict__ res) {
  const int64_t r = grid_index();
  if (r >= A.nrows) return;
  const int64_t s = r >> 6;
  const int lane = (int)(r & 63);
  const int64_t base = A.sptr[s];
  const int len = (int)((A.sptr[s + 1] - base) >> 6);
  double hr[K], lr[K];
  DD acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    hr[k] = hi[r * K + k];
    lr[k] = lo[r * K + k];
    acc[k] = {0.0, 0.0};
  }
  for (int e = 0; e < len; ++e) {
    const int64_t q = base + (int64_t)e * 64 + lane;
    const int32_t c = A.col[q];
    const double v = A.val64[q];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      DD dx = two_sum(hi[(int64_t)c * K + k], -hr[k]);
      dx.lo += lo[(int64_t)c * K + k] - lr[k];
      acc[k] = dd_add(acc[k], dd_scale(v, dx));
    }
  }
  const double dr = A.d64[r];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc[k] = dd_add(acc[k], dd_scale(dr, DD{hr[k], lr[k]}));
    const DD t = two_sum(b[r * K + k], -acc[k].hi);
    res[r * K + k] = t.hi + (t.lo - acc[k].lo);
  }
}

__global__ void k_fold(unsigned mask, int K, double *__restrict__ hi, double *__restrict__ lo,
                       double *__restrict__ x, int64_t count) {
  const int64_t i = grid_index();
  if (i >= count) return;
  const int k = (int)(i % K);
  if (!((mask >> k) & 1u)) return;
  const DD s = two_sum(hi[i], x[i]);
  hi[i] = s.hi;
  lo[i] += s.lo;
  x[i] = 0.0;
}

__global__ void k_round(const double *__restrict__ hi, const double *__restrict__ lo, double *__restrict__ out,
                        int64_t count) {
  const int64_t i = grid_index();
  if (i < count) out[i] = hi[i] + lo[i];
}

}  // namespace

void launch_residual_ext(hipStream_t stm, int K, const Sell &A, const double *b, const double *hi, const double *lo,
                         double *res) {
  if (A.nrows <= 0) return;
  const dim3 g = grid_of(A.nrows, kBlock);
  switch (K) {
    case 1: hipLaunchKernelGGL(k_residual_ext<1>, g, dim3(kBlock), 0, stm, A, b, hi, lo, res); break;
    case 2: hipLaunchKernelGGL(k_residual_ext<2>, g, dim3(kBlock), 0, stm, A, b, hi, lo, res); break;
    case 4: hipLaunchKernelGGL(k_residual_ext<4>, g, dim3(kBlock), 0, stm, A, b, hi, lo, res); break;
    case 8: hipLaunchKernelGGL(k_residual_ext<8>, g, dim3(kBlock), 0, stm, A, b, hi, lo, res); break;
    default: break;
  }
}

void launch_fold(hipStream_t stm, int K, unsigned mask, double *hi, double *lo, double *x, int64_t n) {
  if (n <= 0 || !mask) return;
  hipLaunchKernelGGL(k_fold, grid_of(n * K, kBlock), dim3(kBlock), 0, stm, mask, K, hi, lo, x, n * K);
}

void launch_round(hipStream_t stm, const double *hi, const double *lo, double *out, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_round, grid_of(count, kBlock), dim3(kBlock), 0, stm, hi, lo, out, count);
}

}  // namespace vemg
