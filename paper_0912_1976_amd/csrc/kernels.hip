// HIP kernels of the PCG hot path for gfx950 (CDNA4, wave64).
//
// The path is sparse and bandwidth-bound, so there is no MFMA here: every
// kernel streams its matrix once with coalesced loads (SELL-64 for the fine
// operator, G-lanes-per-row CSR for coarse operators and transfers), reads
// each matrix entry once for all K right-hand sides of a batch, gathers the
// vector rows it needs through L2 / the Infinity Cache, and keeps
// reductions deterministic (per-block partials summed in index order by a
// single-block consumer).  Blocks are renumbered so that each of the eight
// XCDs works on a contiguous range of rows, which keeps the gathered vector
// lines in that XCD's L2.
#include <type_traits>

#include "kernels.hpp"

namespace vemg {

namespace {

// Hardware dispatches block b to XCD b % 8; give every XCD a contiguous chunk.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  int64_t q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return (x < rem) ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

template <class T, int K>
struct alignas(sizeof(T) * K) Row {
  T v[K];
};

template <class T, int K>
__device__ __forceinline__ Row<T, K> ld(const T *__restrict__ p, int64_t r) {
  return *reinterpret_cast<const Row<T, K> *>(p + r * K);
}
template <class T, int K>
__device__ __forceinline__ void st(T *__restrict__ p, int64_t r, const Row<T, K> &v) {
  *reinterpret_cast<Row<T, K> *>(p + r * K) = v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums v[0..K) over a 256-thread block in a fixed order and writes the K
// results to out[0..K) (thread 0).  Every thread of the block must call it.
template <int K>
__device__ __forceinline__ void block_sum_store(const double (&v)[K], double *out) {
  __shared__ double red[kSlicesPerBlock][kMaxBatch];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) red[w][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kSlicesPerBlock; ++q) t += red[q][k];
      out[k] = t;
    }
  }
}

template <class T>
__device__ __forceinline__ const T *sell_vals(const Sell &A);
template <>
__device__ __forceinline__ const double *sell_vals<double>(const Sell &A) {
  return A.val64;
}
template <>
__device__ __forceinline__ const float *sell_vals<float>(const Sell &A) {
  return A.val32;
}
template <class T>
__device__ __forceinline__ const T *csr_vals(const CsrG &A);
template <>
__device__ __forceinline__ const double *csr_vals<double>(const CsrG &A) {
  return A.val64;
}
template <>
__device__ __forceinline__ const float *csr_vals<float>(const CsrG &A) {
  return A.val32;
}

// Lanes that share one row of a K-column batch in the fine kernels: each
// lane holds CPL = K / LPR consecutive columns, 16 bytes at most, so that a
// gathered row is one 16-byte load per lane and the LPR lanes of a row read
// it contiguously.  Narrow rows keep one lane per row.  Spreading a wide row
// over lanes keeps the registers per lane small and several gathers in
// flight per lane, where a 64-byte row per lane allowed one.
template <class T, int K>
constexpr int row_lanes() {
  return sizeof(T) * K <= 16 ? 1 : (int)(sizeof(T) * K / 16);
}

// entries of a row kept in flight per lane
template <class T, int C>
constexpr int sell_unroll() {
  return sizeof(T) * C >= 64 ? 1 : sizeof(T) * C >= 32 ? 2 : 4;
}

// Off-diagonal terms of one SELL row (position t of slice s) for the C
// columns [q C, q C + C) of a K-column batch: acc = sum_j v_j (x_j - x_r)
// (DIFF) or sum_j v_j x_j, and off = sum_j v_j.  Every column is summed over
// the row's entries in storage order, whatever C is.
template <class T, int K, int C, bool DIFF, bool ZS = false>
__device__ __forceinline__ void sell_row(const Sell &A, int64_t s, int t, int q, const T *__restrict__ x,
                                         const Row<T, C> &xr, T (&acc)[C], T &off,
                                         const ZeroStart &z = ZeroStart()) {
  const int64_t base = A.sptr[s];
  const int len = (int)((A.sptr[s + 1] - base) >> 6);
  const int32_t *__restrict__ cp = A.col + base + t;
  const T *__restrict__ vp = sell_vals<T>(A) + base + t;
  const T *__restrict__ xq = x + q * C;
#pragma unroll
  for (int k = 0; k < C; ++k) acc[k] = T(0);
  off = T(0);
  constexpr int U = sell_unroll<T, C>();
#pragma unroll U
  for (int e = 0; e < len; ++e) {
    const int32_t c = cp[(int64_t)e * 64];
    const T v = vp[(int64_t)e * 64];
    if constexpr (ZS && K > 2) {
      // wide rows: the gathers of colours not swept yet are skipped
      if (c < (c < z.n_top ? z.top_lim : z.bar_lim)) {
        const Row<T, C> xc = *reinterpret_cast<const Row<T, C> *>(xq + (int64_t)c * K);
#pragma unroll
        for (int k = 0; k < C; ++k) acc[k] += DIFF ? v * (xc.v[k] - xr.v[k]) : v * xc.v[k];
      }
    } else {
      // narrow rows: load every entry (the loads stay pipelined) and zero
      // the ones not swept yet
      Row<T, C> xc = *reinterpret_cast<const Row<T, C> *>(xq + (int64_t)c * K);
      if constexpr (ZS) {
        const bool live = c < (c < z.n_top ? z.top_lim : z.bar_lim);
#pragma unroll
        for (int k = 0; k < C; ++k) xc.v[k] = live ? xc.v[k] : T(0);
      }
#pragma unroll
      for (int k = 0; k < C; ++k) acc[k] += DIFF ? v * (xc.v[k] - xr.v[k]) : v * xc.v[k];
    }
    off += v;
  }
}

// columns [q C, q C + C) of row r
template <class T, int K, int C>
__device__ __forceinline__ Row<T, C> ldp(const T *__restrict__ p, int64_t r, int q) {
  return *reinterpret_cast<const Row<T, C> *>(p + r * K + q * C);
}
template <class T, int K, int C>
__device__ __forceinline__ void stp(T *__restrict__ p, int64_t r, int q, const Row<T, C> &v) {
  *reinterpret_cast<Row<T, C> *>(p + r * K + q * C) = v;
}

// Block sums of per-row products when a row's K columns are spread over LPR
// lanes (blocks of kBlock * LPR threads covering kBlock rows): the products
// are first laid out one row per thread of the block's first kBlock threads,
// which then reduce exactly as block_sum_store does, so every column's sum
// has the same rounding as with one lane per row.  Every thread of the block
// must call it.
template <int K, int LPR>
__device__ __forceinline__ void block_sum_rows(const double (&v)[K / LPR], double *out) {
  constexpr int C = K / LPR;
  if constexpr (LPR == 1) {
    block_sum_store<K>(v, out);
  } else {
    __shared__ double buf[kBlock][K];
    const int rloc = threadIdx.x / LPR, q = threadIdx.x % LPR;
#pragma unroll
    for (int j = 0; j < C; ++j) buf[rloc][q * C + j] = v[j];
    __syncthreads();
    __shared__ double red[kSlicesPerBlock][kMaxBatch];
    if (threadIdx.x < kBlock) {  // whole wavefronts: wavefront w holds the rows of slice w
      const int w = threadIdx.x >> 6;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double t = wave_sum(buf[threadIdx.x][k]);
        if ((threadIdx.x & 63) == 0) red[w][k] = t;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kSlicesPerBlock; ++w) t += red[w][k];
        out[k] = t;
      }
    }
  }
}

// ------------------------------------------------------------- fine matrix
// (A x)_r in difference form (MODE 0), or g_r - (A x)_r (MODE 1), columns
// [q C, q C + C); the row's own operands are loaded before its entries
// (mi: the row's index in A, r: its index in the vectors; equal unless A
// holds a subset of the rows)
template <class T, int K, int C, int MODE>
__device__ __forceinline__ Row<T, C> fine_row(const Sell &A, int64_t s, int t, int q, int64_t mi, int64_t r,
                                              const T *__restrict__ x, const Row<T, C> &xr,
                                              const T *__restrict__ g) {
  Row<T, C> gr;
  if (MODE == 1) gr = ldp<T, K, C>(g, r, q);
  T d0, d1 = T(0);
  if constexpr (std::is_same<T, double>::value) {
    d0 = A.d64[mi];
  } else {
    d0 = A.s32[mi];
    d1 = A.dh32[mi];
  }
  T acc[C], off;
  sell_row<T, K, C, true>(A, s, t, q, x, xr, acc, off);
  Row<T, C> out;
  if constexpr (std::is_same<T, double>::value) {
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = acc[k] + d0 * xr.v[k];
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = d0 * (acc[k] + d1 * xr.v[k]);
  }
  if (MODE == 1) {
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = gr.v[k] - out.v[k];
  }
  return out;
}

// y_r = g_r - (A x)_r by lane q of row r's lanes; the rows of zr are written
// as zero without reading their entries (their residual is zero in exact
// arithmetic); with y2, a row r >= y2_from is also stored there.
template <class T, int K>
__device__ __forceinline__ void residual_row(const Sell &A, int64_t mi, int64_t r, int q, const T *__restrict__ x,
                                             const T *__restrict__ g, T *y, const ZeroRows &zr, T *y2,
                                             int64_t y2_from) {
  constexpr int LPR = row_lanes<T, K>(), C = K / LPR;
  Row<T, C> out;
  if ((r >= zr.a0 && r < zr.a1) || (r >= zr.b0 && r < zr.b1)) {
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = T(0);
  } else {
    const Row<T, C> xr = ldp<T, K, C>(x, r, q);
    out = fine_row<T, K, C, 1>(A, mi >> 6, (int)(mi & 63), q, mi, r, x, xr, g);
  }
  stp<T, K, C>(y, r, q, out);
  if (y2 && r >= y2_from) stp<T, K, C>(y2, r, q, out);
}

// The residual form on the listed rows rows[0 .. nr) only: As holds those
// rows (row i of As is row rows[i] of the matrix, its entries in the same
// order), so that its entries are read coalesced.
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_spmv_rows(Sell As, const int32_t *__restrict__ rows, int64_t nr,
                                                     const T *__restrict__ x, const T *__restrict__ g,
                                                     T *__restrict__ y, const int *__restrict__ done, ZeroRows zr) {
  constexpr int LPR = row_lanes<T, K>();
  if (done && *done) return;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / LPR;
  if (i >= nr) return;
  residual_row<T, K>(As, i, rows[i], (int)(threadIdx.x % LPR), x, g, y, zr, (T *)nullptr, 0);
}

// Blocks of kBlock rows (four slices), row_lanes<T, K>() lanes per row.
// order (may be null): the i-th slice of the range visited is s_first +
// order[i], a permutation of the range's slices; the blocks of one XCD take a
// contiguous part of it.
template <class T, int K, int MODE, bool DOT>
__global__ __launch_bounds__((kBlock * row_lanes<T, K>())) void k_spmv(
    Sell A, int64_t r0, int64_t r1, int64_t s_first, int64_t ns, int64_t nb, const int32_t *__restrict__ order,
    const T *__restrict__ x, const T *__restrict__ g, T *__restrict__ y, double *__restrict__ partial,
    const int *__restrict__ done, ZeroRows zr, T *__restrict__ y2, int64_t y2_from) {
  constexpr int LPR = row_lanes<T, K>(), C = K / LPR;
  static_assert(!(MODE == 1 && DOT), "the residual form has no block reduction");
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int rloc = threadIdx.x / LPR, q = threadIdx.x % LPR;
  const int t = rloc & 63;
  const int64_t i = blk * kSlicesPerBlock + (rloc >> 6);
  const int64_t s = s_first + (order && i < ns ? (int64_t)order[i] : i);
  const int64_t r = s * 64 + t;
  double prod[C];
#pragma unroll
  for (int k = 0; k < C; ++k) prod[k] = 0.0;
  if (i < ns && r >= r0 && r < r1) {
    if constexpr (MODE == 1) {
      // no block reduction in this form, so the lane may leave
      residual_row<T, K>(A, r, r, q, x, g, y, zr, y2, y2_from);
      return;
    }
    const Row<T, C> xr = ldp<T, K, C>(x, r, q);
    const Row<T, C> out = fine_row<T, K, C, MODE>(A, s, t, q, r, r, x, xr, g);
    stp<T, K, C>(y, r, q, out);
    if (DOT) {
#pragma unroll
      for (int k = 0; k < C; ++k) prod[k] = (double)xr.v[k] * (double)out.v[k];
    }
  }
  if (DOT) block_sum_rows<K, LPR>(prod, partial + blk * K);
}

// device form of the row ranges of one multicolour step
template <class T>
struct GsDev {
  int64_t r0[2], r1[2], sf[2], nb[2];
  T *x;
  T *x2;            // null, or a second output for the rows r >= x2_from
  int64_t x2_from;
  int n;
  int64_t nbt;
};

// one Gauss-Seidel step of row r: x_r + (g_r - (A x)_r) / a_rr, with the
// row's diagonal data d0, d1 loaded by the caller
template <class T, int C>
__device__ __forceinline__ Row<T, C> gs_apply(T d0, T d1, const Row<T, C> &xr, const Row<T, C> &gr,
                                              const T (&acc)[C], T off) {
  Row<T, C> out;
  if constexpr (std::is_same<T, double>::value) {
    const double dr = d0, diag = dr - off;
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = xr.v[k] + (gr.v[k] - (acc[k] + dr * xr.v[k])) / diag;
  } else {
    const float inv_s = 1.0f / d0, dh = d1, diag = dh - off;
#pragma unroll
    for (int k = 0; k < C; ++k) out.v[k] = xr.v[k] + (gr.v[k] * inv_s - (acc[k] + dh * xr.v[k])) / diag;
  }
  return out;
}

// One Gauss-Seidel step of row r by lane q of its row_lanes<T, K>() lanes
// (columns [q C, q C + C)); with x2, a row r >= x2_from is also stored there.
// (mi: the row's index in A, r: its index in the vectors)
template <class T, int K, bool ZS>
__device__ __forceinline__ void gs_row(const Sell &A, int64_t mi, int64_t r, int q, const T *__restrict__ g, T *x,
                                       T *x2, int64_t x2_from, const ZeroStart &z) {
  constexpr int LPR = row_lanes<T, K>(), C = K / LPR;
  const int64_t s = mi >> 6;
  const int t = (int)(mi & 63);
  Row<T, C> xr;
  if constexpr (ZS) {
#pragma unroll
    for (int k = 0; k < C; ++k) xr.v[k] = T(0);
  } else {
    xr = ldp<T, K, C>(x, r, q);
  }
  const Row<T, C> gr = ldp<T, K, C>(g, r, q);
  T d0, d1 = T(0);
  if constexpr (std::is_same<T, double>::value) {
    d0 = A.d64[mi];
  } else {
    d0 = A.s32[mi];
    d1 = A.dh32[mi];
  }
  T acc[C], off;
  sell_row<T, K, C, true, ZS>(A, s, t, q, x, xr, acc, off, z);
  const Row<T, C> out = gs_apply<T, C>(d0, d1, xr, gr, acc, off);
  stp<T, K, C>(x, r, q, out);
  if (x2 && r >= x2_from) stp<T, K, C>(x2, r, q, out);
}

// one slice per block (a colour holds few rows, so small blocks spread them
// over every CU), row_lanes<T, K>() lanes per row; up to two row ranges (the
// top and the non-top rows of one colour)
template <class T, int K, bool ZS>
__global__ __launch_bounds__((kWave * row_lanes<T, K>())) void k_gs(Sell A, GsDev<T> J, const T *__restrict__ g,
                                                                   const int *__restrict__ done, ZeroStart z) {
  constexpr int LPR = row_lanes<T, K>(), C = K / LPR;
  if (done && *done) return;
  int64_t blk = xcd_block(blockIdx.x, J.nbt);
  int j = 0;
  while (j + 1 < J.n && blk >= J.nb[j]) {
    blk -= J.nb[j];
    ++j;
  }
  const int64_t r0 = J.r0[j], r1 = J.r1[j];
  const int t = threadIdx.x / LPR, q = threadIdx.x % LPR;
  const int64_t s = J.sf[j] + blk;
  const int64_t r = s * 64 + t;
  if (r < r0 || r >= r1) return;
  gs_row<T, K, ZS>(A, r, r, q, g, J.x, J.x2, J.x2_from, z);
}

// The listed rows rows[0 .. nr) (rows that share no entries), each by its
// row_lanes<T, K>() lanes, with the arithmetic of k_gs; As holds those rows
// (row i of As is row rows[i] of the matrix, its entries in the same order).
template <class T, int K, bool ZS>
__global__ __launch_bounds__(kBlock) void k_gs_rows(Sell As, const int32_t *__restrict__ rows, int64_t nr,
                                                   const T *__restrict__ g, T *x, const int *__restrict__ done,
                                                   ZeroStart z) {
  constexpr int LPR = row_lanes<T, K>();
  if (done && *done) return;
  const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / LPR;
  if (i >= nr) return;
  gs_row<T, K, ZS>(As, i, rows[i], (int)(threadIdx.x % LPR), g, x, (T *)nullptr, 0, z);
}

template <class T, int K, bool ACC>
__global__ __launch_bounds__(kBlock) void k_rect(Sell E, int64_t nb, const T *__restrict__ x, T *__restrict__ y,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int lane = threadIdx.x & 63;
  const int64_t s = blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  if (r >= E.nrows) return;
  Row<T, K> zero;
#pragma unroll
  for (int k = 0; k < K; ++k) zero.v[k] = T(0);
  T acc[K], off;
  sell_row<T, K, K, false>(E, s, lane, 0, x, zero, acc, off);
  Row<T, K> out;
  if (ACC) out = ld<T, K>(y, r);
#pragma unroll
  for (int k = 0; k < K; ++k) out.v[k] = ACC ? out.v[k] + acc[k] : acc[k];
  st<T, K>(y, r, out);
}

template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_prolong_sum(Sell E, int64_t n_top, int64_t nb, const T *__restrict__ ys,
                                                        const T *__restrict__ w, const T *__restrict__ rv,
                                                        T *__restrict__ z, double *__restrict__ partial,
                                                        const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t blk = xcd_block(blockIdx.x, nb);
  const int lane = threadIdx.x & 63;
  const int64_t s = blk * kSlicesPerBlock + (threadIdx.x >> 6);
  const int64_t r = s * 64 + lane;
  double prod[K];
#pragma unroll
  for (int k = 0; k < K; ++k) prod[k] = 0.0;
  if (r < E.nrows) {
    Row<T, K> zero;
#pragma unroll
    for (int k = 0; k < K; ++k) zero.v[k] = T(0);
    T acc[K], off;
    sell_row<T, K, K, false>(E, s, lane, 0, ys, zero, acc, off);
    Row<T, K> out;
    if (r >= n_top) {
      const Row<T, K> wr = ld<T, K>(w, r);
#pragma unroll
      for (int k = 0; k < K; ++k) out.v[k] = acc[k] + wr.v[k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) out.v[k] = acc[k];
    }
    st<T, K>(z, r, out);
    const Row<T, K> rr = ld<T, K>(rv, r);
#pragma unroll
    for (int k = 0; k < K; ++k) prod[k] = (double)rr.v[k] * (double)out.v[k];
  }
  block_sum_store<K>(prod, partial + blk * K);
}

// ------------------------------------------------------------- CsrG
// Off-diagonal sum of one row for K columns by its group of G lanes (the
// result is valid in every lane of the group).
template <class T, int K, int G>
__device__ __forceinline__ void group_row(const CsrG &A, int64_t r, int gl, const T *__restrict__ x, T (&acc)[K]) {
  const int32_t b = A.ptr[r], e = A.ptr[r + 1];
  const T *__restrict__ vals = csr_vals<T>(A);
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
#pragma unroll 2
  for (int j = b + gl; j < e; j += G) {
    const T v = vals[j];
    const Row<T, K> xc = ld<T, K>(x, A.col[j]);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v * xc.v[k];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += __shfl_xor(acc[k], o, G);
  }
}

// Row r of a CsrG operation, by its group of G lanes (lane 0 of the group
// writes).  The kernels below renumber their blocks like the fine ones, so
// that each XCD works on a contiguous range of rows and the vector values
// those rows gather stay in that XCD's L2.  MODE 0: y = A x, 1: y = g - A x (square); 2: y = P x, 3: y += P x.
template <class T, int K, int G, int MODE>
__device__ __forceinline__ void csr_row_op(const CsrG &A, int64_t r, int gl, const T *x, const T *g, T *y) {
  // the row's own operands are loaded first, so that their latency overlaps
  // the row-pointer -> entries -> gathered values chain of group_row
  Row<T, K> gr, xr, yr;
  T dr = T(0);
  // output row of a rectangular operator (its stored rows may be permuted)
  int64_t ro = r;
  if constexpr (MODE == 2 || MODE == 3) {
    if (A.orow) ro = A.orow[r];
  }
  if (MODE == 1) gr = ld<T, K>(g, r);
  if (MODE <= 1) xr = ld<T, K>(x, r);
  if (MODE == 3) yr = ld<T, K>(y, ro);
  if (MODE <= 1) {
    if constexpr (std::is_same<T, double>::value)
      dr = A.d64[r];
    else
      dr = A.s32[r];
  }
  T acc[K];
  group_row<T, K, G>(A, r, gl, x, acc);  // off-diagonal part only
  if (gl != 0) return;
  Row<T, K> out;
  if (MODE <= 1) {
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
      for (int k = 0; k < K; ++k) out.v[k] = acc[k] + dr * xr.v[k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) out.v[k] = dr * (acc[k] + xr.v[k]);
    }
    if (MODE == 1) {
#pragma unroll
      for (int k = 0; k < K; ++k) out.v[k] = gr.v[k] - out.v[k];
    }
  } else if (MODE == 2) {
#pragma unroll
    for (int k = 0; k < K; ++k) out.v[k] = acc[k];
  } else {
    out = yr;
#pragma unroll
    for (int k = 0; k < K; ++k) out.v[k] += acc[k];
  }
  st<T, K>(y, ro, out);
}

template <class T, int K, int G, int MODE>
__global__ __launch_bounds__(kWave) void k_csr_spmv(CsrG A, int64_t r0, int64_t r1, const T *__restrict__ x,
                                                     const T *__restrict__ g, T *__restrict__ y,
                                                     const int *__restrict__ done) {
  if (done && *done) return;
  const int gl = threadIdx.x & (G - 1);
  const int64_t r = r0 + (xcd_block(blockIdx.x, gridDim.x) * kWave + threadIdx.x) / G;
  if (r >= r1) return;
  csr_row_op<T, K, G, MODE>(A, r, gl, x, g, y);
}

// Patch sweep: one block per patch, kPatchGroup lanes per unknown (a coarse
// row's few dozen couplings take a handful of loads per lane).  First every
// unknown of the patch sums the couplings whose values the sweep takes as
// they stand -- other patches (with a zero start only the patch colours swept
// before) and, without a zero start, its own patch's later unknowns (earlier
// ones backward) -- into h = g - sum (FP32: g / a_ii - sum over row-scaled
// values); then every unknown takes its row of the patch's triangular factor
// times h.  One block barrier; no sequential stages inside the patch.
constexpr int kPatchGroup = 8;
constexpr int kPatchThreads = kPatchGroup * kPatchLdsRows;

template <class T>
__device__ __forceinline__ const T *patch_factor(const PatchSweep &S, bool bwd);
template <>
__device__ __forceinline__ const double *patch_factor<double>(const PatchSweep &S, bool bwd) {
  return bwd ? S.tb64 : S.tf64;
}
template <>
__device__ __forceinline__ const float *patch_factor<float>(const PatchSweep &S, bool bwd) {
  return bwd ? S.tb32 : S.tf32;
}

template <class T, int K>
__device__ __forceinline__ void group_sum(T (&acc)[K]) {
#pragma unroll
  for (int o = kPatchGroup / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += __shfl_xor(acc[k], o, kPatchGroup);
  }
}

template <class T, int K, bool ZS, bool BWD>
__global__ __launch_bounds__(kPatchThreads) void k_patch_gs(CsrG A, PatchSweep S, int64_t p0, int64_t np,
                                                            const T *__restrict__ g, T *__restrict__ x,
                                                            const int *__restrict__ done, int64_t zlim) {
  constexpr int G = kPatchGroup;
  __shared__ Row<T, K> hs[kPatchLdsRows];
  if (done && *done) return;
  const int64_t p = p0 + xcd_block(blockIdx.x, np);
  const int32_t ps = S.prow[p], pe = S.prow[p + 1];
  const int q = threadIdx.x / G, gl = threadIdx.x % G;
  const int32_t i = ps + q;
  const bool own = i < pe;
  const T *__restrict__ vals = csr_vals<T>(A);
  // the row's part of the patch factor does not depend on the sums: load it
  // first, beside the row's own operands (kPatchLdsRows / G entries a lane at most)
  constexpr int FR = kPatchLdsRows / G;
  const int m = pe - ps;
  T fr[FR];
  {
    const T *__restrict__ f = patch_factor<T>(S, BWD) + S.toff[p];
    // forward row q: columns 0..q packed from q (q + 1) / 2; backward: columns q..m-1 from q m - q (q - 1) / 2
    const T *__restrict__ row = BWD ? f + q * m - q * (q - 1) / 2 - q : f + q * (q + 1) / 2;
#pragma unroll
    for (int t = 0; t < FR; ++t) {
      const int j = gl + t * G;
      fr[t] = (own && (BWD ? (j >= q && j < m) : j <= q)) ? row[j] : T(0);
    }
  }
  if (own) {
    const Row<T, K> gr = ld<T, K>(g, i);
    T dr = T(1);
    if constexpr (!std::is_same<T, double>::value) dr = A.s32[i];
    const int32_t b = A.ptr[i], e = A.ptr[i + 1];
    T acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = T(0);
#pragma unroll 4
    for (int32_t j = b + gl; j < e; j += G) {
      const int32_t c = A.col[j];
      const T v = vals[j];
      const bool inside = c >= ps && c < pe;
      const bool take = inside ? (!ZS && (BWD ? c < i : c > i)) : (!ZS || c < zlim);
      if (take) {
        const Row<T, K> xc = ld<T, K>(x, c);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += v * xc.v[k];
      }
    }
    group_sum<T, K>(acc);
    if (gl == 0) {
      Row<T, K> h;
      if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int k = 0; k < K; ++k) h.v[k] = gr.v[k] - acc[k];
      } else {
        const float inv_s = 1.0f / dr;
#pragma unroll
        for (int k = 0; k < K; ++k) h.v[k] = gr.v[k] * inv_s - acc[k];
      }
      hs[q] = h;
    }
  }
  __syncthreads();
  if (!own) return;
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
#pragma unroll
  for (int t = 0; t < FR; ++t) {
    const int j = gl + t * G;
    if (BWD ? (j >= q && j < m) : j <= q) {
      const Row<T, K> hj = hs[j];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] += fr[t] * hj.v[k];
    }
  }
  group_sum<T, K>(acc);
  if (gl == 0) {
    Row<T, K> out;
#pragma unroll
    for (int k = 0; k < K; ++k) out.v[k] = acc[k];
    st<T, K>(x, i, out);
  }
}

// Dense FP64 coarsest inverse applied to K columns, x = C g.  C is symmetric,
// so it is read by columns (C_ji = C_ij): the 64 lanes of a wavefront take 64
// consecutive outputs i and read 64 consecutive entries of row j of C
// together, and g_j is the same for the whole wavefront; C is streamed once,
// with several rows in flight per lane.  The columns j are cut into chunks of
// kDenseChunk (dense_chunks of them); a block of four wavefronts takes 64
// outputs over one chunk, each wavefront a quarter of it, sums the quarters
// in LDS in wavefront order and writes the chunk's partial sums, which
// k_dense_sum adds in chunk order (a single chunk is written directly).  No
// summation order depends on K.
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_dense_part(const double *__restrict__ C, int64_t m,
                                                       const T *__restrict__ g, double *__restrict__ part,
                                                       T *__restrict__ x, const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ double red[kSlicesPerBlock][K][kWave];
  __shared__ Row<T, K> gt[kDenseChunk];  // the chunk's g, read by every lane of a wavefront at once
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kWave + lane;
  const int64_t c = blockIdx.y;
  const int64_t jc = c * kDenseChunk;
  const int nj = (int)(m - jc < kDenseChunk ? m - jc : kDenseChunk);
  for (int j = threadIdx.x; j < nj; j += kBlock) gt[j] = ld<T, K>(g, jc + j);
  __syncthreads();
  constexpr int Q = kDenseChunk / kSlicesPerBlock;
  const int j0 = w * Q;
  const int j1 = j0 + Q < nj ? j0 + Q : nj;
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = 0.0;
  if (i < m) {
    const double *__restrict__ Ci = C + jc * m + i;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
      const double cji = Ci[(int64_t)j * m];
      const Row<T, K> gj = gt[j];
#pragma unroll
      for (int k = 0; k < K; ++k) t[k] += cji * (double)gj.v[k];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) red[w][k][lane] = t[k];
  __syncthreads();
  if (w != 0 || i >= m) return;
  Row<double, K> s;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = red[0][k][lane];
#pragma unroll
    for (int q = 1; q < kSlicesPerBlock; ++q) v += red[q][k][lane];
    s.v[k] = v;
  }
  if (gridDim.y == 1) {
    Row<T, K> out;
#pragma unroll
    for (int k = 0; k < K; ++k) out.v[k] = (T)s.v[k];
    st<T, K>(x, i, out);
  } else {
    st<double, K>(part + c * m * K, i, s);
  }
}

template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_dense_sum(const double *__restrict__ part, int64_t m, int64_t nc,
                                                      T *__restrict__ x, const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // output t = i K + k
  if (t >= m * K) return;
  double s = part[t];
  for (int64_t c = 1; c < nc; ++c) s += part[c * m * K + t];
  x[t] = (T)s;
}

// ------------------------------------------------------------- vectors
template <class T>
__global__ void k_fill(T *__restrict__ x, int64_t n, T v, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <class T>
__global__ void k_copy(const T *__restrict__ a, T *__restrict__ b, int64_t n, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_dot(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                double *__restrict__ partial, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = 0.0;
  if (i < n) {
    const Row<T, K> ai = ld<T, K>(a, i), bi = ld<T, K>(b, i);
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = (double)ai.v[k] * (double)bi.v[k];
  }
  block_sum_store<K>(t, partial + (int64_t)blockIdx.x * K);
}

// z_i += w_i on the rows i >= row0, then the block partials of r . z
template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_add_dot(const T *__restrict__ w, const T *__restrict__ r,
                                                    T *__restrict__ z, int64_t row0, int64_t n,
                                                    double *__restrict__ partial, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = 0.0;
  if (i < n) {
    Row<T, K> zi = ld<T, K>(z, i);
    const Row<T, K> ri = ld<T, K>(r, i);
    if (i >= row0) {
      const Row<T, K> wi = ld<T, K>(w, i);
#pragma unroll
      for (int k = 0; k < K; ++k) zi.v[k] += wi.v[k];
      st<T, K>(z, i, zi);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = (double)ri.v[k] * (double)zi.v[k];
  }
  block_sum_store<K>(t, partial + (int64_t)blockIdx.x * K);
}

template <class T, int K>
__global__ void k_jacobi(const T *__restrict__ r, const double *__restrict__ dg, T *__restrict__ z, int64_t n,
                         const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Row<T, K> ri = ld<T, K>(r, i);
  Row<T, K> out;
  const double d = dg[i];
#pragma unroll
  for (int k = 0; k < K; ++k) out.v[k] = (T)((double)ri.v[k] / d);
  st<T, K>(z, i, out);
}

__global__ void k_gather(const double *__restrict__ nat, const int64_t *__restrict__ perm, double *__restrict__ sto,
                         int64_t n, int K, int k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sto[i * K + k] = nat[perm[i]];
}

__global__ void k_scatter(const double *__restrict__ sto, const int64_t *__restrict__ perm, double *__restrict__ nat,
                          int64_t n, int K, int k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nat[perm[i]] = sto[i * K + k];
}

__global__ void k_demote(const double *__restrict__ r64, const double *__restrict__ scale, float *__restrict__ r32,
                         int64_t n, int K, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * K) r32[i] = (float)(r64[i] * scale[i % K]);
}

template <bool ACC>
__global__ void k_promote(const float *__restrict__ d32, const double *__restrict__ scale, double *__restrict__ x64,
                          int64_t n, int K, const int *__restrict__ done) {
  if (done && *done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * K) return;
  const double v = scale[i % K] * (double)d32[i];
  x64[i] = ACC ? x64[i] + v : v;
}

// ------------------------------------------------------------- PCG scalars
// Fixed-order sums of the K columns of np partials (row-major [np][K]) by one
// block, all columns at once: thread t adds rows t, t + kBlock, ... in turn,
// then a pairwise tree over the threads.  The order for column k does not
// depend on K, so a column's sum is the same alone and in a batch.
__device__ __forceinline__ void sum_partials(const double *__restrict__ p, int64_t np, int K,
                                             double (&res)[kMaxBatch]) {
  double t[kMaxBatch];
#pragma unroll
  for (int k = 0; k < kMaxBatch; ++k) t[k] = 0.0;
  // eight of each thread's partials are loaded before any is added, so that
  // a thread keeps eight loads per column in flight; the additions keep the
  // order j = tid, tid + kBlock, ...
  constexpr int U = 8;
  int64_t j = threadIdx.x;
  for (; j + (U - 1) * kBlock < np; j += U * kBlock) {
    double v[U][kMaxBatch];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < kMaxBatch; ++k) v[u][k] = (k < K) ? p[(j + u * kBlock) * K + k] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < kMaxBatch; ++k)
        if (k < K) t[k] += v[u][k];
  }
  for (; j < np; j += kBlock) {
#pragma unroll
    for (int k = 0; k < kMaxBatch; ++k)
      if (k < K) t[k] += p[j * K + k];
  }
  // then a fixed tree: xor shuffles within each wavefront, and the four
  // wavefront sums added in order (the same result in every thread)
  __shared__ double buf[kMaxBatch][kSlicesPerBlock];
#pragma unroll
  for (int k = 0; k < kMaxBatch; ++k)
    if (k < K) t[k] = wave_sum(t[k]);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < kMaxBatch; ++k)
      if (k < K) buf[k][threadIdx.x / kWave] = t[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kMaxBatch; ++k) {
    double r = 0.0;
    if (k < K) {
#pragma unroll
      for (int w = 0; w < kSlicesPerBlock; ++w) r += buf[k][w];
    }
    res[k] = r;
  }
}

// Lanes that load one partial row of K columns, 16 bytes each (one lane of 8
// bytes for K = 1), and the block size of the kernels that use
// sum_partials_wide.
template <int K>
constexpr int partial_lanes() {
  return K >= 2 ? K / 2 : 1;
}
template <int K>
constexpr int wide_block() {
  return kBlock * partial_lanes<K>();
}

// sum_partials for a K known at compile time, by a block of wide_block<K>()
// threads: the lanes of row group v (partial_lanes<K>() consecutive threads)
// load rows v, v + kBlock, ... whole, one 16-byte piece each, so that a
// wavefront reads consecutive rows and keeps several times the loads in
// flight.  Each lane adds its columns over those rows in that order, which
// is thread v's order in sum_partials, and the first kBlock threads then
// take thread v's place in its tree: the result equals sum_partials' bit for
// bit.  Every thread of the block must call it.
template <int K>
__device__ __forceinline__ void sum_partials_wide(const double *__restrict__ p, int64_t np,
                                                  double (&res)[kMaxBatch]) {
  constexpr int LP = partial_lanes<K>(), CW = K / LP;
  const int v = threadIdx.x / LP, c = threadIdx.x % LP;
  double t[CW];
#pragma unroll
  for (int k = 0; k < CW; ++k) t[k] = 0.0;
  auto load = [&](int64_t j, double(&w)[CW]) {
    if constexpr (CW == 2) {
      const double2 q = *reinterpret_cast<const double2 *>(p + j * K + c * 2);
      w[0] = q.x;
      w[1] = q.y;
    } else {
      w[0] = p[j * K + c];
    }
  };
  constexpr int U = 8;
  int64_t j = v;
  for (; j + (U - 1) * kBlock < np; j += U * kBlock) {
    double w[U][CW];
#pragma unroll
    for (int u = 0; u < U; ++u) load(j + u * kBlock, w[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < CW; ++k) t[k] += w[u][k];
  }
  for (; j < np; j += kBlock) {
    double w[CW];
    load(j, w);
#pragma unroll
    for (int k = 0; k < CW; ++k) t[k] += w[k];
  }
  __shared__ double col[K][kBlock];
#pragma unroll
  for (int k = 0; k < CW; ++k) col[c * CW + k][v] = t[k];
  __syncthreads();
  __shared__ double buf[K][kSlicesPerBlock];
  if (threadIdx.x < kBlock) {  // whole wavefronts
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double w = wave_sum(col[k][threadIdx.x]);
      if ((threadIdx.x & (kWave - 1)) == 0) buf[k][threadIdx.x / kWave] = w;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kMaxBatch; ++k) {
    double r = 0.0;
    if (k < K) {
#pragma unroll
      for (int w = 0; w < kSlicesPerBlock; ++w) r += buf[k][w];
    }
    res[k] = r;
  }
}

__device__ __forceinline__ void update_all_done(Scal *s) {
  int all = 1;
  for (int k = 0; k < s->K; ++k) all &= s->done[k];
  s->all_done = all;
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double *p, int64_t np, int K, double *out) {
  double t[kMaxBatch];
  sum_partials(p, np, K, t);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[k] = t[k];
}

__global__ __launch_bounds__(kBlock) void k_pcg_init(Scal *s, const double *pb, int64_t npb, int K, double tol,
                                                     int maxit) {
  double sums[kMaxBatch];
  sum_partials(pb, npb, K, sums);
  for (int k = 0; k < kMaxBatch; ++k) {
    const double t = sums[k];
    if (threadIdx.x == 0) {
      s->bnorm2[k] = t;
      s->iters[k] = 0;
      s->rho[k] = 0.0;
      s->alpha[k] = 0.0;
      s->beta[k] = 0.0;
      if (k >= K || t == 0.0) {
        s->done[k] = 1;
        s->status[k] = 1;
      } else if (!isfinite(t)) {
        s->done[k] = 1;
        s->status[k] = -6;
      } else {
        s->done[k] = 0;
        s->status[k] = 0;
      }
    }
  }
  if (threadIdx.x == 0) {
    s->K = K;
    for (int k = 0; k < kMaxBatch; ++k) {
      s->tol2[k] = tol * tol;
      s->maxit[k] = maxit;
    }
    update_all_done(s);
  }
}

__global__ __launch_bounds__(kBlock) void k_pcg_set_rho(Scal *s, const double *p, int64_t np) {
  double t[kMaxBatch];
  sum_partials(p, np, s->K, t);
  if (threadIdx.x == 0)
    for (int k = 0; k < s->K; ++k) s->rho[k] = t[k];
}

// The per-iteration scalar kernels handle column k in thread k, so that the
// few loads and stores of each column overlap instead of following one
// another in a single thread.
__device__ __forceinline__ double column_of(const double (&v)[kMaxBatch], int k) {
  double out = 0.0;
#pragma unroll
  for (int q = 0; q < kMaxBatch; ++q)
    if (q == k) out = v[q];
  return out;
}

// all_done from the columns' flags (thread k < K holds column k's); every
// thread of the block must call it
__device__ __forceinline__ void store_all_done(Scal *s, int K, int mine) {
  __shared__ int flags[kMaxBatch];
  if ((int)threadIdx.x < K) flags[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int all = 1;
    for (int k = 0; k < K; ++k) all &= flags[k];
    s->all_done = all;
  }
}

template <int K>
__global__ __launch_bounds__(wide_block<K>()) void k_pcg_alpha(Scal *s, const double *p, int64_t np) {
  if (s->all_done) return;
  double sums[kMaxBatch];
  sum_partials_wide<K>(p, np, sums);
  const int k = threadIdx.x;
  int done = 1;
  if (k < K) {
    done = s->done[k];
    if (!done) {
      const double pq = column_of(sums, k), rho = s->rho[k];
      s->pq[k] = pq;
      if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
        done = 1;
        s->done[k] = 1;
        s->status[k] = -6;
        s->alpha[k] = 0.0;
      } else {
        s->alpha[k] = rho / pq;
      }
    }
  }
  store_all_done(s, K, done);
}

template <class T, int K>
__global__ __launch_bounds__(kBlock) void k_pcg_xr(const Scal *s, T *__restrict__ x, T *__restrict__ r,
                                                   const T *__restrict__ p, const T *__restrict__ q, int64_t n,
                                                   double *__restrict__ partial) {
  if (s->all_done) return;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = 0.0;
  if (i < n) {
    Row<T, K> xi = ld<T, K>(x, i), ri = ld<T, K>(r, i);
    const Row<T, K> pi = ld<T, K>(p, i), qi = ld<T, K>(q, i);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!s->done[k]) {
        const T a = (T)s->alpha[k];
        xi.v[k] += a * pi.v[k];
        ri.v[k] -= a * qi.v[k];
      }
      t[k] = (double)ri.v[k] * (double)ri.v[k];
    }
    st<T, K>(x, i, xi);
    st<T, K>(r, i, ri);
  }
  block_sum_store<K>(t, partial + (int64_t)blockIdx.x * K);
}

template <int K>
__global__ __launch_bounds__(wide_block<K>()) void k_pcg_conv(Scal *s, const double *p, int64_t np) {
  if (s->all_done) return;
  double sums[kMaxBatch];
  sum_partials_wide<K>(p, np, sums);
  const int k = threadIdx.x;
  int done = 1;
  if (k < K) {
    done = s->done[k];
    if (!done) {
      const double rr = column_of(sums, k);
      const int it = s->iters[k] + 1;
      s->iters[k] = it;
      s->rr[k] = rr;
      int status = 0;
      if (!isfinite(rr))
        status = -6;
      else if (rr <= s->tol2[k] * s->bnorm2[k])
        status = 1;
      else if (it >= s->maxit[k])
        status = 2;
      if (status != 0) {
        done = 1;
        s->done[k] = 1;
        s->status[k] = status;
      }
    }
  }
  store_all_done(s, K, done);
}

template <int K>
__global__ __launch_bounds__(wide_block<K>()) void k_pcg_beta(Scal *s, const double *p, int64_t np) {
  if (s->all_done) return;
  double sums[kMaxBatch];
  sum_partials_wide<K>(p, np, sums);
  const int k = threadIdx.x;
  if (k < K && !s->done[k]) {
    const double rz = column_of(sums, k);
    s->beta[k] = rz / s->rho[k];
    s->rho[k] = rz;
  }
}

template <class T, int K>
__global__ void k_pcg_p(const Scal *s, T *__restrict__ p, const T *__restrict__ z, int64_t n) {
  if (s->all_done) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Row<T, K> pi = ld<T, K>(p, i);
  const Row<T, K> zi = ld<T, K>(z, i);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (!s->done[k]) pi.v[k] = zi.v[k] + (T)s->beta[k] * pi.v[k];
  st<T, K>(p, i, pi);
}

__global__ void k_pcg_resume(Scal *s, unsigned keep) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < s->K; ++k)
      if (!((keep >> k) & 1u)) {
        s->done[k] = 0;
        s->status[k] = 0;
      }
    update_all_done(s);
  }
}

__global__ void k_slot_vectors(unsigned mask, int restart, const double *__restrict__ b, const double *__restrict__ res,
                               double *__restrict__ hi, double *__restrict__ lo, double *__restrict__ x,
                               double *__restrict__ r, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kMaxBatch) return;
  int k = (int)(i % kMaxBatch);
  if (!((mask >> k) & 1u)) return;
  if (restart) {
    r[i] = res[i];
  } else {
    hi[i] = 0.0;
    lo[i] = 0.0;
    x[i] = 0.0;
    r[i] = b[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_slot_scalars(unsigned mask, int restart, Scal *s, const double *pb,
                                                         int64_t npb, SlotStop stop, double *scale_in,
                                                         double *scale_out) {
  double sums[kMaxBatch];
  sum_partials(pb, npb, kMaxBatch, sums);
  for (int k = 0; k < kMaxBatch; ++k) {
    if (!((mask >> k) & 1u)) continue;
    const double t = restart ? 0.0 : sums[k];
    if (threadIdx.x == 0) {
      if (!restart) {
        s->bnorm2[k] = t;
        s->iters[k] = 0;
        s->tol2[k] = stop.tol[k] * stop.tol[k];
        s->maxit[k] = stop.maxit[k];
        double nb = sqrt(t);
        bool ok = t > 0.0 && isfinite(t);
        scale_in[k] = ok ? 1.0 / nb : 0.0;
        scale_out[k] = ok ? nb : 0.0;
      }
      const double bb = s->bnorm2[k];
      if (bb == 0.0) {
        s->done[k] = 1;
        s->status[k] = 1;
      } else if (!isfinite(bb)) {
        s->done[k] = 1;
        s->status[k] = -6;
      } else {
        s->done[k] = 0;
        s->status[k] = 0;
      }
    }
  }
  if (threadIdx.x == 0) {
    s->K = kMaxBatch;
    update_all_done(s);
  }
}

__global__ __launch_bounds__(kBlock) void k_slot_rho(unsigned mask, Scal *s, const double *p, int64_t np) {
  double t[kMaxBatch];
  sum_partials(p, np, kMaxBatch, t);
  if (threadIdx.x == 0)
    for (int k = 0; k < kMaxBatch; ++k)
      if ((mask >> k) & 1u) s->rho[k] = t[k];
}

__global__ void k_slot_copy(unsigned mask, const double *__restrict__ z, double *__restrict__ p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kMaxBatch) return;
  if ((mask >> (int)(i % kMaxBatch)) & 1u) p[i] = z[i];
}

inline dim3 grid(int64_t nb) { return dim3((unsigned)nb); }

}  // namespace

void launch_slot_vectors(hipStream_t stm, unsigned mask, bool restart, const double *b, const double *res, double *hi,
                         double *lo, double *x, double *r, int64_t n) {
  if (n <= 0 || !mask) return;
  hipLaunchKernelGGL(k_slot_vectors, grid(vec_blocks(n * kMaxBatch)), dim3(kBlock), 0, stm, mask, (int)restart, b, res,
                     hi, lo, x, r, n);
}
void launch_slot_scalars(hipStream_t stm, unsigned mask, bool restart, Scal *s, const double *pb, int64_t npb,
                         const SlotStop &stop, double *scale_in, double *scale_out) {
  hipLaunchKernelGGL(k_slot_scalars, dim3(1), dim3(kBlock), 0, stm, mask, (int)restart, s, pb, npb, stop,
                     scale_in, scale_out);
}
void launch_slot_rho(hipStream_t stm, unsigned mask, Scal *s, const double *p, int64_t np) {
  hipLaunchKernelGGL(k_slot_rho, dim3(1), dim3(kBlock), 0, stm, mask, s, p, np);
}
void launch_slot_copy(hipStream_t stm, unsigned mask, const double *z, double *p, int64_t n) {
  if (n <= 0 || !mask) return;
  hipLaunchKernelGGL(k_slot_copy, grid(vec_blocks(n * kMaxBatch)), dim3(kBlock), 0, stm, mask, z, p, n);
}

#define VEMG_K_SWITCH(K, ...) \
  switch (K) {                \
    case 1: {                 \
      constexpr int KK = 1;   \
      __VA_ARGS__;            \
    } break;                  \
    case 2: {                 \
      constexpr int KK = 2;   \
      __VA_ARGS__;            \
    } break;                  \
    case 4: {                 \
      constexpr int KK = 4;   \
      __VA_ARGS__;            \
    } break;                  \
    default: {                \
      constexpr int KK = 8;   \
      __VA_ARGS__;            \
    } break;                  \
  }

#define VEMG_G_SWITCH(G, ...) \
  switch (G) {                \
    case 4: {                 \
      constexpr int GG = 4;   \
      __VA_ARGS__;            \
    } break;                  \
    case 8: {                 \
      constexpr int GG = 8;   \
      __VA_ARGS__;            \
    } break;                  \
    case 16: {                \
      constexpr int GG = 16;  \
      __VA_ARGS__;            \
    } break;                  \
    case 32: {                \
      constexpr int GG = 32;  \
      __VA_ARGS__;            \
    } break;                  \
    default: {                \
      constexpr int GG = 64;  \
      __VA_ARGS__;            \
    } break;                  \
  }

template <class T>
void launch_spmv(hipStream_t stm, int K, const Sell &A, int mode, int64_t r0, int64_t r1, const T *x, const T *g,
                 T *y, double *partial, const int *done, const int32_t *order, ZeroRows zr, T *y2, int64_t y2_from) {
  int64_t nb = sell_blocks(r0, r1);
  if (!nb) return;
  int64_t sf = r0 / kWave, ns = (r1 + kWave - 1) / kWave - sf;
  VEMG_K_SWITCH(K, {
    const dim3 blk(kBlock * row_lanes<T, KK>());
    if (mode == 0) {
      if (partial)
        hipLaunchKernelGGL((k_spmv<T, KK, 0, true>), grid(nb), blk, 0, stm, A, r0, r1, sf, ns, nb, order, x, g, y,
                           partial, done, zr, y2, y2_from);
      else
        hipLaunchKernelGGL((k_spmv<T, KK, 0, false>), grid(nb), blk, 0, stm, A, r0, r1, sf, ns, nb, order, x, g, y,
                           partial, done, zr, y2, y2_from);
    } else {
      hipLaunchKernelGGL((k_spmv<T, KK, 1, false>), grid(nb), blk, 0, stm, A, r0, r1, sf, ns, nb, order, x, g, y,
                         partial, done, zr, y2, y2_from);
    }
  })
}

static inline int64_t slices(int64_t r0, int64_t r1) {
  return r1 <= r0 ? 0 : (r1 + kWave - 1) / kWave - r0 / kWave;
}

template <class T>
void launch_spmv_rows(hipStream_t stm, int K, const Sell &A, const int32_t *rows, int64_t nr, const T *x, const T *g,
                      T *y, const int *done, ZeroRows zr) {
  if (nr <= 0) return;
  VEMG_K_SWITCH(K, {
    const int64_t nb = (nr * row_lanes<T, KK>() + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_spmv_rows<T, KK>), grid(nb), dim3(kBlock), 0, stm, A, rows, nr, x, g, y, done, zr);
  })
}

template <class T>
void launch_gs_rows(hipStream_t stm, int K, const Sell &A, const int32_t *rows, int64_t nr, const T *g, T *x,
                    const int *done, ZeroStart zs) {
  if (nr <= 0) return;
  VEMG_K_SWITCH(K, {
    const int64_t nb = (nr * row_lanes<T, KK>() + kBlock - 1) / kBlock;
    if (zs.on)
      hipLaunchKernelGGL((k_gs_rows<T, KK, true>), grid(nb), dim3(kBlock), 0, stm, A, rows, nr, g, x, done, zs);
    else
      hipLaunchKernelGGL((k_gs_rows<T, KK, false>), grid(nb), dim3(kBlock), 0, stm, A, rows, nr, g, x, done, zs);
  })
}

template <class T>
void launch_gs(hipStream_t stm, int K, const Sell &A, int64_t a0, int64_t a1, int64_t b0, int64_t b1, const T *g,
               T *x, const int *done, ZeroStart zs, T *x2, int64_t x2_from) {
  GsDev<T> J{};
  J.x = x;
  J.x2 = x2;
  J.x2_from = x2_from;
  const int64_t ra[2] = {a0, b0}, rb[2] = {a1, b1};
  for (int i = 0; i < 2; ++i) {
    const int64_t nb = slices(ra[i], rb[i]);
    if (!nb) continue;
    J.r0[J.n] = ra[i];
    J.r1[J.n] = rb[i];
    J.sf[J.n] = ra[i] / kWave;
    J.nb[J.n] = nb;
    J.nbt += nb;
    ++J.n;
  }
  if (!J.nbt) return;
  VEMG_K_SWITCH(K, {
    const dim3 blk(kWave * row_lanes<T, KK>());
    if (zs.on)
      hipLaunchKernelGGL((k_gs<T, KK, true>), grid(J.nbt), blk, 0, stm, A, J, g, done, zs);
    else
      hipLaunchKernelGGL((k_gs<T, KK, false>), grid(J.nbt), blk, 0, stm, A, J, g, done, zs);
  })
}

template <class T>
void launch_rect(hipStream_t stm, int K, const Sell &E, bool accumulate, const T *x, T *y, const int *done) {
  int64_t nb = sell_blocks(0, E.nrows);
  if (!nb) return;
  VEMG_K_SWITCH(K, {
    if (accumulate)
      hipLaunchKernelGGL((k_rect<T, KK, true>), grid(nb), dim3(kBlock), 0, stm, E, nb, x, y, done);
    else
      hipLaunchKernelGGL((k_rect<T, KK, false>), grid(nb), dim3(kBlock), 0, stm, E, nb, x, y, done);
  })
}

template <class T>
void launch_prolong_sum(hipStream_t stm, int K, const Sell &E, int64_t n_top, const T *y, const T *w, const T *r,
                        T *z, double *partial, const int *done) {
  int64_t nb = sell_blocks(0, E.nrows);
  if (!nb) return;
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_prolong_sum<T, KK>), grid(nb), dim3(kBlock), 0, stm, E, n_top, nb, y, w, r,
                                      z, partial, done))
}

template <class T>
static void csr_launch(hipStream_t stm, int K, int mode, const CsrG &A, int64_t r0, int64_t r1, const T *x,
                       const T *g, T *y, const int *done) {
  int64_t rows = r1 - r0;
  if (rows <= 0) return;
  int64_t nb = (rows * A.G + kWave - 1) / kWave;
  VEMG_K_SWITCH(K, VEMG_G_SWITCH(A.G, {
    switch (mode) {
      case 0:
        hipLaunchKernelGGL((k_csr_spmv<T, KK, GG, 0>), grid(nb), dim3(kWave), 0, stm, A, r0, r1, x, g, y, done);
        break;
      case 1:
        hipLaunchKernelGGL((k_csr_spmv<T, KK, GG, 1>), grid(nb), dim3(kWave), 0, stm, A, r0, r1, x, g, y, done);
        break;
      case 2:
        hipLaunchKernelGGL((k_csr_spmv<T, KK, GG, 2>), grid(nb), dim3(kWave), 0, stm, A, r0, r1, x, g, y, done);
        break;
      default:
        hipLaunchKernelGGL((k_csr_spmv<T, KK, GG, 3>), grid(nb), dim3(kWave), 0, stm, A, r0, r1, x, g, y, done);
        break;
    }
  }))
}

template <class T>
void launch_csr_spmv(hipStream_t stm, int K, const CsrG &A, int mode, int64_t r0, int64_t r1, const T *x,
                     const T *g, T *y, const int *done) {
  csr_launch<T>(stm, K, mode == 0 ? 0 : 1, A, r0, r1, x, g, y, done);
}

template <class T>
void launch_csr_rect(hipStream_t stm, int K, const CsrG &P, bool accumulate, const T *x, T *y, const int *done) {
  csr_launch<T>(stm, K, accumulate ? 3 : 2, P, 0, P.nrows, x, nullptr, y, done);
}

template <class T>
void launch_patch_gs(hipStream_t stm, int K, const CsrG &A, const PatchSweep &S, int64_t p0, int64_t np, const T *g,
                     T *x, const int *done, int64_t zlim, bool backward) {
  if (np <= 0) return;
  VEMG_K_SWITCH(K, {
    if (zlim >= 0)
      hipLaunchKernelGGL((k_patch_gs<T, KK, true, false>), grid(np), dim3(kPatchThreads), 0, stm, A, S, p0, np, g, x,
                         done, zlim);
    else if (backward)
      hipLaunchKernelGGL((k_patch_gs<T, KK, false, true>), grid(np), dim3(kPatchThreads), 0, stm, A, S, p0, np, g, x,
                         done, int64_t(0));
    else
      hipLaunchKernelGGL((k_patch_gs<T, KK, false, false>), grid(np), dim3(kPatchThreads), 0, stm, A, S, p0, np, g, x,
                         done, int64_t(0));
  })
}

template <class T>
void launch_dense(hipStream_t stm, int K, const double *Cinv, int64_t m, const T *g, T *x, double *part,
                  const int *done) {
  if (m <= 0) return;
  const int64_t nc = dense_chunks(m);
  const dim3 gr((unsigned)((m + kWave - 1) / kWave), (unsigned)nc);
  VEMG_K_SWITCH(K, {
    hipLaunchKernelGGL((k_dense_part<T, KK>), gr, dim3(kBlock), 0, stm, Cinv, m, g, part, x, done);
    if (nc > 1)
      hipLaunchKernelGGL((k_dense_sum<T, KK>), grid((m * KK + kBlock - 1) / kBlock), dim3(kBlock), 0, stm, part, m,
                         nc, x, done);
  })
}

template <class T>
void launch_fill(hipStream_t stm, T *x, int64_t n, T v, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fill<T>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, x, n, v, done);
}

template <class T>
void launch_copy(hipStream_t stm, const T *a, T *b, int64_t n, const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_copy<T>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, a, b, n, done);
}

template <class T>
void launch_dot(hipStream_t stm, int K, const T *a, const T *b, int64_t n, double *partial, const int *done) {
  if (n <= 0) return;
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_dot<T, KK>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, a, b, n, partial,
                                      done))
}

template <class T>
void launch_add_dot(hipStream_t stm, int K, const T *w, const T *r, T *z, int64_t row0, int64_t n, double *partial,
                    const int *done) {
  if (n <= 0) return;
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_add_dot<T, KK>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, w, r, z, row0, n,
                                      partial, done))
}

template <class T>
void launch_jacobi(hipStream_t stm, int K, const T *r, const double *diag, T *z, int64_t n, const int *done) {
  if (n <= 0) return;
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_jacobi<T, KK>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, r, diag, z, n,
                                      done))
}

void launch_gather(hipStream_t stm, int K, int k, const double *nat, const int64_t *perm, double *sto, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather, grid(vec_blocks(n)), dim3(kBlock), 0, stm, nat, perm, sto, n, K, k);
}

void launch_scatter(hipStream_t stm, int K, int k, const double *sto, const int64_t *perm, double *nat, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter, grid(vec_blocks(n)), dim3(kBlock), 0, stm, sto, perm, nat, n, K, k);
}

void launch_demote(hipStream_t stm, int K, const double *r64, const double *scale, float *r32, int64_t n,
                   const int *done) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_demote, grid(vec_blocks(n * K)), dim3(kBlock), 0, stm, r64, scale, r32, n, K, done);
}

void launch_promote(hipStream_t stm, int K, const float *d32, const double *scale, double *x64, int64_t n,
                    bool accumulate, const int *done) {
  if (n <= 0) return;
  if (accumulate)
    hipLaunchKernelGGL((k_promote<true>), grid(vec_blocks(n * K)), dim3(kBlock), 0, stm, d32, scale, x64, n, K, done);
  else
    hipLaunchKernelGGL((k_promote<false>), grid(vec_blocks(n * K)), dim3(kBlock), 0, stm, d32, scale, x64, n, K, done);
}

void launch_pcg_init(hipStream_t stm, int K, Scal *s, const double *pb, int64_t npb, double tol, int maxit) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kBlock), 0, stm, s, pb, npb, K, tol, maxit);
}
void launch_pcg_set_rho(hipStream_t stm, int, Scal *s, const double *p, int64_t np) {
  hipLaunchKernelGGL(k_pcg_set_rho, dim3(1), dim3(kBlock), 0, stm, s, p, np);
}
// the per-iteration scalar kernels take K (= s->K) at compile time
void launch_pcg_alpha(hipStream_t stm, int K, Scal *s, const double *p, int64_t np) {
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_pcg_alpha<KK>), dim3(1), dim3(wide_block<KK>()), 0, stm, s, p, np))
}
template <class T>
void launch_pcg_xr(hipStream_t stm, int K, Scal *s, T *x, T *r, const T *p, const T *q, int64_t n, double *partial) {
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_pcg_xr<T, KK>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, s, x, r, p, q, n,
                                      partial))
}
void launch_pcg_conv(hipStream_t stm, int K, Scal *s, const double *p, int64_t np) {
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_pcg_conv<KK>), dim3(1), dim3(wide_block<KK>()), 0, stm, s, p, np))
}
void launch_pcg_beta(hipStream_t stm, int K, Scal *s, const double *p, int64_t np) {
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_pcg_beta<KK>), dim3(1), dim3(wide_block<KK>()), 0, stm, s, p, np))
}
template <class T>
void launch_pcg_p(hipStream_t stm, int K, Scal *s, T *pvec, const T *z, int64_t n) {
  VEMG_K_SWITCH(K, hipLaunchKernelGGL((k_pcg_p<T, KK>), grid(vec_blocks(n)), dim3(kBlock), 0, stm, s, pvec, z, n))
}
void launch_reduce(hipStream_t stm, int K, const double *p, int64_t np, double *out) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, stm, p, np, K, out);
}
void launch_pcg_resume(hipStream_t stm, int, Scal *s, unsigned keep) {
  hipLaunchKernelGGL(k_pcg_resume, dim3(1), dim3(64), 0, stm, s, keep);
}

#define VEMG_INSTANTIATE(T)                                                                                          \
  template void launch_spmv<T>(hipStream_t, int, const Sell &, int, int64_t, int64_t, const T *, const T *, T *,      \
                               double *, const int *, const int32_t *, ZeroRows, T *, int64_t);                      \
  template void launch_spmv_rows<T>(hipStream_t, int, const Sell &, const int32_t *, int64_t, const T *, const T *,   \
                                    T *, const int *, ZeroRows);                                                     \
  template void launch_gs<T>(hipStream_t, int, const Sell &, int64_t, int64_t, int64_t, int64_t, const T *, T *,       \
                             const int *, ZeroStart, T *, int64_t);                                                  \
  template void launch_gs_rows<T>(hipStream_t, int, const Sell &, const int32_t *, int64_t, const T *, T *,           \
                                  const int *, ZeroStart);                                                           \
  template void launch_rect<T>(hipStream_t, int, const Sell &, bool, const T *, T *, const int *);                    \
  template void launch_prolong_sum<T>(hipStream_t, int, const Sell &, int64_t, const T *, const T *, const T *, T *,   \
                                      double *, const int *);                                                        \
  template void launch_csr_spmv<T>(hipStream_t, int, const CsrG &, int, int64_t, int64_t, const T *, const T *, T *,   \
                                   const int *);                                                                     \
  template void launch_patch_gs<T>(hipStream_t, int, const CsrG &, const PatchSweep &, int64_t, int64_t, const T *,  \
                                   T *, const int *, int64_t, bool);                                                 \
  template void launch_csr_rect<T>(hipStream_t, int, const CsrG &, bool, const T *, T *, const int *);                \
  template void launch_dense<T>(hipStream_t, int, const double *, int64_t, const T *, T *, double *, const int *);    \
  template void launch_fill<T>(hipStream_t, T *, int64_t, T, const int *);                                           \
  template void launch_copy<T>(hipStream_t, const T *, T *, int64_t, const int *);                                   \
  template void launch_dot<T>(hipStream_t, int, const T *, const T *, int64_t, double *, const int *);                \
  template void launch_add_dot<T>(hipStream_t, int, const T *, const T *, T *, int64_t, int64_t, double *,             \
                                  const int *);                                                                      \
  template void launch_jacobi<T>(hipStream_t, int, const T *, const double *, T *, int64_t, const int *);             \
  template void launch_pcg_xr<T>(hipStream_t, int, Scal *, T *, T *, const T *, const T *, int64_t, double *);        \
  template void launch_pcg_p<T>(hipStream_t, int, Scal *, T *, const T *, int64_t);

VEMG_INSTANTIATE(double)
VEMG_INSTANTIATE(float)

}  // namespace vemg
