// Solver handle: packs the host setup into HBM (SELL-64 fine operator,
// G-lanes-per-row CSR for coarse operators and transfers, FP64 and FP32
// copies), runs the preconditioned CG loop on the device for batches of up to
// eight right-hand sides, and exposes the C ABI of vemg.h.
//
// One PCG iteration is a fixed sequence of kernels whose scalars (alpha,
// beta, per-column convergence flags) live in device memory, so it is
// captured once per (precision, batch width) in a hipGraph and replayed;
// every kernel returns at once when all columns have converged, so the host
// only polls the flags every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/vemg.h"
#include "kernels.hpp"
#include "setup.hpp"

namespace vemg {
namespace {

struct DeviceError : std::runtime_error {
  int code;
  DeviceError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      throw ::vemg::DeviceError(e_ == hipErrorOutOfMemory ? VEMG_ERR_OOM : VEMG_ERR_DEVICE,       \
                                std::string(#expr) + ": " + hipGetErrorString(e_));               \
  } while (0)

// device allocations owned by a handle; with count_only set nothing is
// allocated or copied, only the bytes are added up (the footprint query)
struct Arena {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  bool count_only = false;
  template <class T>
  T *alloc(size_t count) {
    if (count == 0) count = 1;
    bytes += count * sizeof(T);
    if (count_only) return nullptr;
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, count * sizeof(T)));
    ptrs.push_back(p);
    return (T *)p;
  }
  template <class T>
  T *upload(const std::vector<T> &v, hipStream_t st) {
    T *p = alloc<T>(v.size());
    if (!v.empty() && !count_only) {
      // the source is a temporary host vector: finish the copy before returning
      HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    return p;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

// CSR (host) -> SELL-64 (device).  Square: the diagonal entries are taken
// out of the stored entries; the FP64 per-row term is `d` if given
// (difference form: the deficit) else a_ii.  FP32 copy: a_ij / a_ii with
// s32 = a_ii and dh32 = d / a_ii (square), or float(a_ij) (rectangular).
Sell pack_sell(Arena &ar, hipStream_t st, const Csr &A, bool square, const std::vector<double> *d,
               const std::vector<double> *diag, int64_t *stored = nullptr,
               const std::vector<int32_t> *subset = nullptr) {
  // subset: pack only these rows of A, row i of the result being A's row
  // (*subset)[i] with its entries (columns unchanged) in the same order
  int64_t n = subset ? (int64_t)subset->size() : A.nrows, ns = (n + kWave - 1) / kWave;
  auto row_of = [&](int64_t i) -> int64_t { return subset ? (int64_t)(*subset)[i] : i; };
  std::vector<int64_t> sptr(ns + 1, 0);
  std::vector<int64_t> len(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t r = row_of(i);
    int64_t c = 0;
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
      if (!(square && A.idx[k] == r)) ++c;
    len[i] = c;
  }
  for (int64_t s = 0; s < ns; ++s) {
    int64_t L = 0;
    for (int64_t r = s * kWave; r < std::min(n, (s + 1) * kWave); ++r) L = std::max(L, len[r]);
    sptr[s + 1] = sptr[s] + L * kWave;
  }
  std::vector<int32_t> col(sptr[ns]);
  std::vector<double> val(sptr[ns], 0.0);
  std::vector<float> val32(sptr[ns], 0.0f);
  std::vector<double> dv(square ? n : 0, 0.0), ad(square ? n : 0, 0.0);
  for (int64_t i = 0; square && i < n; ++i) {
    const int64_t r = row_of(i);
    if (diag) ad[i] = (*diag)[r];
    for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e)
      if (A.idx[e] == r) ad[i] = A.val[e];
    dv[i] = d ? (*d)[r] : ad[i];
  }
  for (int64_t s = 0; s < ns; ++s) {
    int64_t L = (sptr[s + 1] - sptr[s]) / kWave;
    for (int t = 0; t < kWave; ++t) {
      const int64_t i = s * kWave + t, r = i < n ? row_of(i) : -1;
      int64_t k = 0;
      if (i < n) {
        for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) {
          if (square && A.idx[e] == r) continue;
          int64_t pos = sptr[s] + k * kWave + t;
          col[pos] = A.idx[e];
          val[pos] = A.val[e];
          val32[pos] = square ? (float)(A.val[e] / ad[i]) : (float)A.val[e];
          ++k;
        }
      }
      for (; k < L; ++k) {
        int64_t pos = sptr[s] + k * kWave + t;
        col[pos] = (square && i < n) ? (int32_t)r : 0;
        val[pos] = 0.0;
        val32[pos] = 0.0f;
      }
    }
  }
  if (stored) *stored = sptr[ns];
  Sell M;
  M.nrows = n;
  M.sptr = ar.upload(sptr, st);
  M.col = ar.upload(col, st);
  M.val64 = ar.upload(val, st);
  M.val32 = ar.upload(val32, st);
  if (square) {
    std::vector<float> s32(n), dh32(n);
    for (int64_t r = 0; r < n; ++r) {
      s32[r] = (float)ad[r];
      dh32[r] = (float)(dv[r] / ad[r]);
    }
    M.d64 = ar.upload(dv, st);
    M.s32 = ar.upload(s32, st);
    M.dh32 = ar.upload(dh32, st);
  }
  return M;
}

// CSR (host) -> CsrG (device).  Square matrices keep only off-diagonals
// (FP64 values with d64 = a_ii; FP32 values a_ij / a_ii with s32 = a_ii).
// G = smallest power of two >= half the mean row length, clamped to [4, 64].
// With colkey (rectangular operators gathering from the fine level: the
// spatial rank of column c is (*colkey)[c + coloff]) the rows are stored in
// the order of their smallest column rank and orow maps them back, so that
// the rows one XCD works on gather from one region of the fine vector; each
// row keeps its entries and their order.
CsrG pack_csrg(Arena &ar, hipStream_t st, const Csr &A, bool square, int64_t *stored = nullptr,
               const std::vector<int64_t> *colkey = nullptr, int64_t coloff = 0) {
  std::vector<int32_t> ptr(A.nrows + 1, 0), col;
  std::vector<double> val, d(square ? A.nrows : 0, 0.0);
  std::vector<float> val32;
  col.reserve(A.nnz());
  val.reserve(A.nnz());
  for (int64_t r = 0; r < A.nrows && square; ++r)
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
      if (A.idx[k] == r) d[r] = A.val[k];
  std::vector<int64_t> rows(A.nrows);
  std::iota(rows.begin(), rows.end(), 0);
  const bool permute = colkey != nullptr && !square;
  if (permute) {
    std::vector<int64_t> key(A.nrows, INT64_MAX);
    for (int64_t r = 0; r < A.nrows; ++r)
      for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) key[r] = std::min(key[r], (*colkey)[A.idx[k] + coloff]);
    std::stable_sort(rows.begin(), rows.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
  }
  for (int64_t i = 0; i < A.nrows; ++i) {
    const int64_t r = rows[i];
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      if (square && A.idx[k] == r) continue;
      col.push_back(A.idx[k]);
      val.push_back(A.val[k]);
      val32.push_back(square ? (float)(A.val[k] / d[r]) : (float)A.val[k]);
    }
    ptr[i + 1] = (int32_t)col.size();
  }
  double mean = A.nrows ? (double)col.size() / (double)A.nrows : 0.0;
  int G = 4;
  while (G < 64 && G < mean / 2.0) G *= 2;
  if (stored) *stored = (int64_t)col.size();
  CsrG M;
  M.nrows = A.nrows;
  M.G = G;
  M.ptr = ar.upload(ptr, st);
  M.col = ar.upload(col, st);
  M.val64 = ar.upload(val, st);
  M.val32 = ar.upload(val32, st);
  if (permute) {
    std::vector<int32_t> orow(rows.begin(), rows.end());
    M.orow = ar.upload(orow, st);
  }
  if (square) {
    std::vector<float> s32(A.nrows);
    for (int64_t r = 0; r < A.nrows; ++r) s32[r] = (float)d[r];
    M.d64 = ar.upload(d, st);
    M.s32 = ar.upload(s32, st);
  }
  return M;
}

// per-precision work vectors, each [n][kMaxBatch]
template <class T>
struct Work {
  T *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *w = nullptr, *res = nullptr,
    *resA = nullptr, *tmp = nullptr;
  // FP64 only: the solution as the unevaluated sum xs + xl, into which each
  // restart's correction x is folded
  T *xs = nullptr, *xl = nullptr;
};

struct DLevel {
  Sell As;                      // fine A_bar level: rows [row0, row0 + n) of the fine SELL matrix
  CsrG Ac;                      // coarse levels: standard form, G lanes per row
  PatchSweep ps;                // coarse levels: the patches of the sweeps
  std::vector<int64_t> pc_start, pc_row;  // patch colour c: stored patches [pc_start[c], pc_start[c+1]), first row
  bool fine = false;
  int64_t n = 0, row0 = 0;
  int64_t n_top = 0;            // fine levels: rows of the top block in the fine matrix
  std::vector<int64_t> cstart;  // colour ranges, global row indices
  std::vector<int64_t> cstart_top;  // fine level of the whole A_UU: top-block range of each colour
  const int32_t *order = nullptr;   // fine levels: slice visit order of the residual product
  CsrG P, Pt;                   // prolongation (n x n_next) and restriction
  Sell Ps;                      // fine levels: the prolongation in SELL-64 (a few entries a row)
  double *Cinv = nullptr;       // coarsest level only: its explicit inverse
  double *dpart = nullptr;      // and the dense product's partial sums (dense_chunks(n) x n x kMaxBatch)
  bool coarsest = false;
  // vectors indexed by global row, [n][kMaxBatch], per precision
  double *x64 = nullptr, *g64 = nullptr, *r64 = nullptr;
  float *x32 = nullptr, *g32 = nullptr, *r32 = nullptr;
  template <class T>
  T *&x() {
    if constexpr (std::is_same<T, double>::value) return x64; else return x32;
  }
  template <class T>
  T *&g() {
    if constexpr (std::is_same<T, double>::value) return g64; else return g32;
  }
  template <class T>
  T *&r() {
    if constexpr (std::is_same<T, double>::value) return r64; else return r32;
  }
};

// kGraphFP32Reliable: an FP32 iteration followed by the reliable update of
// the mixed-precision solve (the last iteration of every chunk)
enum GraphKind { kGraphFP64 = 0, kGraphFP32 = 1, kGraphMixedPC = 2, kGraphFP32Reliable = 3 };

// the captured graphs of one PCG iteration: a single graph, or four segments
struct IterGraphs {
  hipGraph_t graph[7] = {};
  hipGraphExec_t exec[7] = {};
  int parts = 0;
};

}  // namespace
}  // namespace vemg

struct vemg_solver_s {
  vemg_options opt;
  int device = -1;
  hipStream_t user = nullptr, work = nullptr, work2 = nullptr;  // work2: parallel preconditioner branch
  bool own_streams = true;  // false: work and work2 belong to a server's stream pool
  size_t footprint = 0;     // device bytes of the uploaded setup (counted before the upload)
  // ev_res: the SOR cycle's residual is done (the shared forward sweep)
  hipEvent_t ev = nullptr, ev_fork = nullptr, ev_join = nullptr, ev_res = nullptr;
  std::string err;
  bool ready = false;
  vemg::Problem P;
  vemg::Arena ar;
  vemg::Sell A;                           // fine A_UU, difference form
  vemg::Sell E;
  vemg::CsrG Et;
  std::vector<vemg::DLevel> S, Ab, SA;  // SA: baseline hierarchy of the whole A_UU (may be empty)
  vemg::Work<double> v64;
  vemg::Work<float> v32;
  double *b = nullptr, *diag = nullptr, *scale_in = nullptr, *scale_out = nullptr, *dscal = nullptr;
  double *part_pq = nullptr, *part_rr = nullptr, *part_rz = nullptr, *part_b = nullptr, *part_t = nullptr;
  int64_t *perm = nullptr;
  // slice visit orders (spatial, across colours) of the products over all
  // rows and over the non-top rows
  int32_t *order_all = nullptr, *order_bar = nullptr;
  // VL + additive smoother: the smoother's fine forward sweep and residual
  // take the SOR cycle's for every non-top row they share; the rows that
  // differ, per colour for the sweep (reuse_gs[reuse_gs_start[c] ..
  // reuse_gs_start[c+1]), and for the residual (reuse_res, n_reuse_res)
  bool reuse = false;
  // the rows of reuse_gs of each colour, and those of reuse_res, packed as
  // SELL matrices of their own (entries read coalesced)
  std::vector<vemg::Sell> reuse_gs_sell;
  vemg::Sell reuse_res_sell;
  int64_t share_min_rows = 0;  // fine unknowns from which the forward sweep is shared
  bool reuse_full_res = false;  // no top surface: the smoother's residual is computed in full
  // the top block of the additive smoother's x (rows [0, n_top) of v64.w and
  // v32.w) is zero in the layout of every batch width up to w_clean
  int w_clean = vemg::kMaxBatch;
  int32_t *reuse_gs = nullptr, *reuse_res = nullptr;
  std::vector<int64_t> reuse_gs_start;
  int64_t n_reuse_res = 0;
  vemg::Scal *scal = nullptr;
  int64_t nnz_A = 0, nnz_E = 0;
  std::map<int, vemg::IterGraphs> graphs;  // key: kind * 16 + K
  // false for server lanes once the scheduler runs: a capture on one thread
  // must not coincide with device-wide synchronisation on another
  bool allow_capture = true;
};

namespace vemg {
namespace {

using Handle = vemg_solver_s;

template <class T>
Work<T> &work_of(Handle *h) {
  if constexpr (std::is_same<T, double>::value) return h->v64; else return h->v32;
}

// The patch arrays of a coarse level for its sweeps: row ranges of the stored
// patches and, per patch, F = (D_p + L_p)^{-1} of its diagonal block in stored
// order (forward substitution on the host in FP64) packed by rows, F^T packed
// by rows for the backward sweep, and both times D_p rounded to FP32 for the
// row-scaled FP32 operator.
void pack_patches(Arena &ar, hipStream_t st, const Level &L, DLevel &dl) {
  static_assert(kPatchRows == kPatchLdsRows, "the patch size of the order and of the sweep kernel differ");
  const int64_t n = L.n(), np = (int64_t)L.patch_list.size();
  if (n > INT32_MAX) throw DeviceError(hipErrorInvalidValue, "coarse level above 2^31 rows");
  std::vector<int32_t> prow(L.patch_row.begin(), L.patch_row.end());
  std::vector<int64_t> toff(np + 1, 0);
  for (int64_t p = 0; p < np; ++p) {
    const int64_t m = L.patch_row[p + 1] - L.patch_row[p];
    if (m > kPatchLdsRows) throw DeviceError(hipErrorInvalidValue, "a patch exceeds the sweep kernel's rows");
    toff[p + 1] = toff[p] + m * (m + 1) / 2;
  }
  std::vector<double> tf(toff[np]), tb(toff[np]);
  std::vector<float> tf32(toff[np]), tb32(toff[np]);
  if (!ar.count_only) {
    std::vector<double> M, F;
    for (int64_t p = 0; p < np; ++p) {
      const int64_t ps = L.patch_row[p], m = L.patch_row[p + 1] - ps;
      M.assign(m * m, 0.0);
      F.assign(m * m, 0.0);
      for (int64_t r = 0; r < m; ++r)
        for (int64_t k = L.A.ptr[ps + r]; k < L.A.ptr[ps + r + 1]; ++k) {
          const int64_t c = L.A.idx[k] - ps;
          if (c >= 0 && c <= r) M[r * m + c] = L.A.val[k];
        }
      // columns of F = (D + L)^{-1}: forward substitution on unit vectors
      for (int64_t c = 0; c < m; ++c) {
        F[c * m + c] = 1.0 / M[c * m + c];
        for (int64_t r = c + 1; r < m; ++r) {
          double t = 0.0;
          for (int64_t k = c; k < r; ++k) t += M[r * m + k] * F[k * m + c];
          F[r * m + c] = -t / M[r * m + r];
        }
      }
      double *fwd = tf.data() + toff[p], *bwd = tb.data() + toff[p];
      float *fwd32 = tf32.data() + toff[p], *bwd32 = tb32.data() + toff[p];
      for (int64_t r = 0, o = 0; r < m; ++r)
        for (int64_t c = 0; c <= r; ++c, ++o) {
          fwd[o] = F[r * m + c];
          fwd32[o] = (float)(F[r * m + c] * M[c * m + c]);
        }
      for (int64_t r = 0, o = 0; r < m; ++r)
        for (int64_t c = r; c < m; ++c, ++o) {
          bwd[o] = F[c * m + r];
          bwd32[o] = (float)(F[c * m + r] * M[c * m + c]);
        }
    }
  }
  dl.ps.prow = ar.upload(prow, st);
  dl.ps.toff = ar.upload(toff, st);
  dl.ps.tf64 = ar.upload(tf, st);
  dl.ps.tb64 = ar.upload(tb, st);
  dl.ps.tf32 = ar.upload(tf32, st);
  dl.ps.tb32 = ar.upload(tb32, st);
  dl.pc_start = L.pc_start;
  dl.pc_row.resize(L.pc_start.size());
  for (size_t c = 0; c < L.pc_start.size(); ++c) dl.pc_row[c] = L.patch_row[L.pc_start[c]];
}

enum LevelsOf { kLevelsS = 0, kLevelsAbar = 1, kLevelsSA = 2 };

void build_levels(Handle *h, std::vector<Level> &H, std::vector<DLevel> &D, int of) {
  hipStream_t st = h->work;
  D.clear();
  for (size_t l = 0; l < H.size(); ++l) {
    Level &L = H[l];
    DLevel dl;
    dl.n = L.n();
    dl.coarsest = (l + 1 == H.size());
    if (of != kLevelsS && l == 0) {
      // fine level: rows of the fine SELL matrix (non-top rows for A_bar,
      // all rows for the whole A_UU), colour ranges in global rows
      dl.fine = true;
      dl.n_top = h->P.n_top;
      dl.As = h->A;
      dl.row0 = of == kLevelsAbar ? h->P.n_top : 0;
      dl.order = of == kLevelsAbar ? h->order_bar : h->order_all;
      dl.cstart = h->P.bar_colour_start;
      if (of == kLevelsSA) {
        const int nc = std::max((int)h->P.top_colour_start.size(), (int)h->P.bar_colour_start.size()) - 1;
        dl.cstart_top = h->P.top_colour_start;
        dl.cstart_top.resize(nc + 1, dl.cstart_top.back());
        dl.cstart.resize(nc + 1, dl.cstart.back());
      }
      dl.x64 = h->v64.w;
      dl.g64 = h->v64.r;
      dl.r64 = h->v64.resA;
      dl.x32 = h->v32.w;
      dl.g32 = h->v32.r;
      dl.r32 = h->v32.resA;
    } else {
      dl.Ac = pack_csrg(h->ar, st, L.A, true);
      pack_patches(h->ar, st, L, dl);
      size_t cnt = (size_t)dl.n * kMaxBatch;
      dl.x64 = h->ar.alloc<double>(cnt);
      dl.g64 = h->ar.alloc<double>(cnt);
      dl.r64 = h->ar.alloc<double>(cnt);
      dl.x32 = h->ar.alloc<float>(cnt);
      dl.g32 = h->ar.alloc<float>(cnt);
      dl.r32 = h->ar.alloc<float>(cnt);
    }
    if (!dl.coarsest) {
      if (dl.fine)
        dl.Ps = pack_sell(h->ar, st, L.P, false, nullptr, nullptr);
      else
        dl.P = pack_csrg(h->ar, st, L.P, false);
      // the fine level's restriction gathers from fine rows row0 + c
      dl.Pt = dl.fine ? pack_csrg(h->ar, st, transpose(L.P), false, nullptr, &h->P.loc_rank, dl.row0)
                      : pack_csrg(h->ar, st, transpose(L.P), false);
    } else {
      dl.Cinv = h->ar.upload(L.Cinv, st);
      dl.dpart = h->ar.alloc<double>((size_t)dense_chunks(dl.n) * dl.n * kMaxBatch);
    }
    D.push_back(dl);
  }
}

// The rows of a fine level whose forward sweep and residual differ from the
// SOR cycle's, which has already stored its values for every other row (the
// additive smoother beside the SOR cycle).
struct Reuse {
  const int32_t *gs = nullptr;           // dirty rows, colour by colour
  const std::vector<int64_t> *gs_start = nullptr;
  const std::vector<Sell> *gs_sell = nullptr;  // those rows of each colour, packed
  const int32_t *res = nullptr;          // rows whose residual is recomputed
  int64_t nres = 0;
  const Sell *res_sell = nullptr;        // those rows, packed
  bool full_res = false;                 // recompute every row's residual (no top surface)
  int phase = 0;  // 1: the dirty rows' sweep only; 2: the residual rows and the rest of the cycle
};

template <class T>
void vcycle(hipStream_t st, int K, std::vector<DLevel> &H, size_t l, const int *done,
            const Reuse *reuse = nullptr) {
  DLevel &L = H[l];
  T *x = L.x<T>(), *g = L.g<T>(), *r = L.r<T>();
  const int64_t o = L.row0 * K;
  if (L.coarsest) {
    launch_dense<T>(st, K, L.Cinv, L.n, g + o, x + o, L.dpart, done);
    return;
  }
  const int nc = (int)(L.fine ? L.cstart.size() : L.pc_start.size()) - 1;
  // forward (zero start: x needs no fill, the colours not swept yet are not
  // read) and backward sweeps of colour c (coarse levels: patch colour c)
  auto gs = [&](int c, bool first) {
    if (L.fine) {
      // A_bar's fine level (no top range) never reads the top columns: they
      // multiply the smoother vector's top part, which is zero
      ZeroStart zs;
      zs.on = first;
      zs.n_top = L.n_top;
      zs.top_lim = L.cstart_top.empty() ? 0 : L.cstart_top[c];
      zs.bar_lim = L.cstart[c];
      if (!L.cstart_top.empty()) {
        launch_gs<T>(st, K, L.As, L.cstart_top[c], L.cstart_top[c + 1], L.cstart[c], L.cstart[c + 1], g, x, done,
                     zs);
      } else {
        launch_gs<T>(st, K, L.As, L.cstart[c], L.cstart[c + 1], 0, 0, g, x, done, zs);
      }
    } else {
      launch_patch_gs<T>(st, K, L.Ac, L.ps, L.pc_start[c], L.pc_start[c + 1] - L.pc_start[c], g, x, done,
                         first ? L.pc_row[c] : -1, !first);
    }
  };
  // the rows of the last colour have a zero residual after the forward sweep
  ZeroRows zr;
  if (L.fine && nc > 0) {
    if (!L.cstart_top.empty()) {
      zr.a0 = L.cstart_top[nc - 1];
      zr.a1 = L.cstart_top[nc];
    }
    zr.b0 = L.cstart[nc - 1];
    zr.b1 = L.cstart[nc];
  }
  if (reuse && L.fine && L.cstart_top.empty()) {
    // x and r hold the SOR cycle's values (x once its forward sweep is done,
    // r once its residual is); sweep and recompute only the rows where the
    // two differ, with the same arithmetic
    if (reuse->phase == 1) {
      for (int c = 0; c < nc; ++c) {
        ZeroStart zs;
        zs.on = true;
        zs.n_top = L.n_top;
        zs.top_lim = 0;
        zs.bar_lim = L.cstart[c];
        const int64_t a = (*reuse->gs_start)[c], b = (*reuse->gs_start)[c + 1];
        launch_gs_rows<T>(st, K, (*reuse->gs_sell)[c], reuse->gs + a, b - a, g, x, done, zs);
      }
      return;
    }
    if (reuse->full_res)
      launch_spmv<T>(st, K, L.As, 1, L.row0, L.row0 + L.n, x, g, r, nullptr, done, L.order, zr);
    else
      launch_spmv_rows<T>(st, K, *reuse->res_sell, reuse->res, reuse->nres, x, g, r, done, zr);
  } else {
    for (int c = 0; c < nc; ++c) gs(c, true);
  }
  if (L.fine) {
    if (!(reuse && L.cstart_top.empty()))
      launch_spmv<T>(st, K, L.As, 1, L.row0, L.row0 + L.n, x, g, r, nullptr, done, L.order, zr);
  } else
    launch_csr_spmv<T>(st, K, L.Ac, 1, 0, L.n, x, g, r, done);
  DLevel &C = H[l + 1];
  launch_csr_rect<T>(st, K, L.Pt, false, r + o, C.g<T>(), done);
  vcycle<T>(st, K, H, l + 1, done);
  if (L.fine)
    launch_rect<T>(st, K, L.Ps, true, C.x<T>(), x + o, done);
  else
    launch_csr_rect<T>(st, K, L.P, true, C.x<T>(), x + o, done);
  for (int c = nc - 1; c >= 0; --c) gs(c, false);
}

// One vertical-lumping multigrid cycle on stream st (Section 6, second
// preconditioner): forward multicolour SOR on A from zero, E~ coarse
// correction through one V-cycle on the surface operator, backward SOR.
// part: 0 the whole cycle, 1 the forward sweep, 3 the residual, 2 the rest;
// with share, the forward sweep's and the residual's non-top rows are also
// stored to the additive smoother's fine vectors
template <class T>
void sor_cycle(Handle *h, hipStream_t st, int K, const T *rr, T *zz, const int *done, int part = 0,
               bool share = false) {
  const Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  Work<T> &v = work_of<T>(h);
  int nct = (int)P.top_colour_start.size() - 1, ncb = (int)P.bar_colour_start.size() - 1;
  int nc = std::max(nct, ncb);
  T *x2 = share ? v.w : nullptr, *r2 = share ? v.resA : nullptr;
  // the forward sweep starts from zero: zz needs no fill, and colour c reads
  // only the colours before it (in each block)
  auto sweep = [&](int c, bool first) {
    int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (c < nct) {
      a0 = P.top_colour_start[c];
      a1 = P.top_colour_start[c + 1];
    }
    if (c < ncb) {
      b0 = P.bar_colour_start[c];
      b1 = P.bar_colour_start[c + 1];
    }
    ZeroStart zs;
    zs.on = first;
    zs.n_top = m;
    zs.top_lim = P.top_colour_start[std::min(c, nct)];
    zs.bar_lim = P.bar_colour_start[std::min(c, ncb)];
    launch_gs<T>(st, K, h->A, a0, a1, b0, b1, rr, zz, done, zs, first ? x2 : nullptr, m);
  };
  if (part == 0 || part == 1)
    for (int c = 0; c < nc; ++c) sweep(c, true);
  if (part == 0 || part == 3) {
    if (m > 0) {
      // the rows swept by the last launch have a zero residual
      ZeroRows zr;
      if (nc > 0) {
        if (nc - 1 < nct) {
          zr.a0 = P.top_colour_start[nc - 1];
          zr.a1 = P.top_colour_start[nc];
        }
        if (nc - 1 < ncb) {
          zr.b0 = P.bar_colour_start[nc - 1];
          zr.b1 = P.bar_colour_start[nc];
        }
      }
      launch_spmv<T>(st, K, h->A, 1, 0, n, zz, rr, v.res, nullptr, done, h->order_all, zr, r2, m);
    }
  }
  if (part == 1 || part == 3) return;
  if (m > 0) {
    launch_csr_rect<T>(st, K, h->Et, false, v.res, h->S[0].g<T>(), done);
    vcycle<T>(st, K, h->S, 0, done);
    launch_rect<T>(st, K, h->E, true, h->S[0].x<T>(), zz, done);
  }
  for (int c = nc - 1; c >= 0; --c) sweep(c, false);
}

// w = Z Vcyc_Abar(Z^T rr) on stream st (the additive smoother; rows of the top
// block of w stay zero)
// phase 0: the whole V-cycle; 1 and 2: its two parts beside the SOR cycle's
// shared forward sweep (see Reuse)
template <class T>
void additive_smoother(Handle *h, hipStream_t st, int K, const T *rr, const int *done, int phase = 0) {
  T *saved = h->Ab[0].g<T>();
  h->Ab[0].g<T>() = const_cast<T *>(rr);
  Reuse R;
  R.gs = h->reuse_gs;
  R.gs_start = &h->reuse_gs_start;
  R.gs_sell = &h->reuse_gs_sell;
  R.res = h->reuse_res;
  R.nres = h->n_reuse_res;
  R.res_sell = &h->reuse_res_sell;
  R.full_res = h->reuse_full_res;
  R.phase = phase;
  vcycle<T>(st, K, h->Ab, 0, done, phase ? &R : nullptr);
  h->Ab[0].g<T>() = saved;
}

// The two VL+additive forms have a second, independent branch: the additive
// smoother beside the SOR cycle (VEMG_PC_VL_ADDITIVE), or the surface branch
// beside the smoother (VEMG_PC_VL_ADDITIVE_ONLY with a non-empty surface).
bool has_branch(const Handle *h) {
  return h->opt.pc == VEMG_PC_VL_ADDITIVE || (h->opt.pc == VEMG_PC_VL_ADDITIVE_ONLY && h->P.n_top > 0);
}

// Whether the additive smoother takes the SOR cycle's forward sweep and
// residual.  The smoother then starts only after that sweep, which costs
// overlap; the sweeps it saves outweigh that only when they are long: on
// meshes of a million fine unknowns and more (any batch width), not below.
// The environment's VEMG_SHARE_MIN_ROWS, when set, replaces that bound (0:
// always), so that small meshes can exercise the shared form.
constexpr int64_t kShareMinRows = 1000000;
int64_t share_min_rows() {
  if (const char *e = std::getenv("VEMG_SHARE_MIN_ROWS")) {
    char *end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end != e && *end == '\0' && v >= 0) return (int64_t)v;
  }
  return kShareMinRows;
}
bool shares(const Handle *h, int) {
  return h->reuse && h->opt.pc == VEMG_PC_VL_ADDITIVE && h->P.n >= h->share_min_rows;
}

// second branch, on stream st2.  When shares(h, K) it comes in two phases:
// 1 after the SOR cycle's forward sweep, 2 after its residual.
template <class T>
void precond_branch(Handle *h, hipStream_t st2, int K, const T *rr, const int *done, int phase = 0) {
  if (h->opt.pc == VEMG_PC_VL_ADDITIVE) {
    additive_smoother<T>(h, st2, K, rr, done, shares(h, K) ? phase : 0);
  } else {
    launch_csr_rect<T>(st2, K, h->Et, false, rr, h->S[0].g<T>(), done);
    vcycle<T>(st2, K, h->S, 0, done);
  }
}

// first branch, on stream st.  When shares(h, K) it comes in three parts:
// 1 the SOR cycle's forward sweep and 3 its residual (both shared with the
// second branch), then 2 the rest.
template <class T>
void precond_main(Handle *h, hipStream_t st, int K, const T *rr, T *zz, const int *done, int part = 0) {
  if (h->opt.pc == VEMG_PC_VL_ADDITIVE)
    sor_cycle<T>(h, st, K, rr, zz, done, shares(h, K) ? part : 0,
                 shares(h, K) && (part == 1 || part == 3));
  else if (part == 0 || part == 2)
    additive_smoother<T>(h, st, K, rr, done);
}

// after both branches: z = sum of the two, partials of rr . z (returns their count)
template <class T>
int64_t precond_join(Handle *h, hipStream_t st, int K, const T *rr, T *zz, double *part, const int *done) {
  const int64_t n = h->P.n, m = h->P.n_top;
  Work<T> &v = work_of<T>(h);
  if (h->opt.pc == VEMG_PC_VL_ADDITIVE) {
    launch_add_dot<T>(st, K, v.w, rr, zz, m, n, part, done);
    return vec_blocks(n);
  }
  launch_prolong_sum<T>(st, K, h->E, m, h->S[0].x<T>(), v.w, rr, zz, part, done);
  return sell_blocks(0, n);
}

// z = M^{-1} rr in precision T; partial sums of rr . z go to part (blocks in *np)
template <class T>
void precond(Handle *h, int K, const T *rr, T *zz, double *part, int64_t *np, const int *done) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n;
  Work<T> &v = work_of<T>(h);
  if (has_branch(h)) {
    const bool sh = shares(h, K);
    if (sh) precond_main<T>(h, st, K, rr, zz, done, 1);
    HIPCHK(hipEventRecord(h->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(h->work2, h->ev_fork, 0));
    precond_branch<T>(h, h->work2, K, rr, done, sh ? 1 : 0);
    if (sh) {
      precond_main<T>(h, st, K, rr, zz, done, 3);
      HIPCHK(hipEventRecord(h->ev_res, st));
      HIPCHK(hipStreamWaitEvent(h->work2, h->ev_res, 0));
      precond_branch<T>(h, h->work2, K, rr, done, 2);
    }
    HIPCHK(hipEventRecord(h->ev_join, h->work2));
    precond_main<T>(h, st, K, rr, zz, done, sh ? 2 : 0);
    HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
    *np = precond_join<T>(h, st, K, rr, zz, part, done);
    return;
  }
  switch (h->opt.pc) {
    case VEMG_PC_VL_ADDITIVE_ONLY:  // empty surface: the additive smoother alone
      additive_smoother<T>(h, st, K, rr, done);
      launch_copy<T>(st, v.w, zz, n * K, done);
      launch_dot<T>(st, K, rr, zz, n, part, done);
      *np = vec_blocks(n);
      break;
    case VEMG_PC_VL_SOR:
      sor_cycle<T>(h, st, K, rr, zz, done);
      launch_dot<T>(st, K, rr, zz, n, part, done);
      *np = vec_blocks(n);
      break;
    case VEMG_PC_SA: {
      // one V-cycle of the baseline hierarchy, its fine level on rr -> zz
      DLevel &F = h->SA[0];
      T *sx = F.x<T>(), *sg = F.g<T>();
      F.x<T>() = zz;
      F.g<T>() = const_cast<T *>(rr);
      vcycle<T>(st, K, h->SA, 0, done);
      F.x<T>() = sx;
      F.g<T>() = sg;
      launch_dot<T>(st, K, rr, zz, n, part, done);
      *np = vec_blocks(n);
      break;
    }
    case VEMG_PC_JACOBI:
      launch_jacobi<T>(st, K, rr, h->diag, zz, n, done);
      launch_dot<T>(st, K, rr, zz, n, part, done);
      *np = vec_blocks(n);
      break;
    default:
      launch_copy<T>(st, rr, zz, n * K, done);
      launch_dot<T>(st, K, rr, zz, n, part, done);
      *np = vec_blocks(n);
      break;
  }
}

// The additive smoother reads the top columns of its x and takes them as
// zero, so the top block of v64.w and v32.w must be zero.  Vectors are laid
// out [n][K]: a call with K columns writes the non-top rows at [n_top K,
// n K), which a later call with more columns reads as part of its top block
// [0, n_top K).  Every call with K columns calls this first.
void batch_layout(Handle *h, int K) {
  const int64_t m = h->P.n_top;
  if (K > h->w_clean && m > 0) {
    launch_fill<double>(h->work, h->v64.w, m * K, 0.0, nullptr);
    launch_fill<float>(h->work, h->v32.w, m * K, 0.0f, nullptr);
  }
  h->w_clean = K;
}

// FP64 CG with the preconditioner applied in FP32 (columns scaled by scale_in)
int64_t precond_mixed(Handle *h, int K, const double *rr, double *zz, const int *done) {
  hipStream_t st = h->work;
  int64_t n = h->P.n, np = 0;
  launch_demote(st, K, rr, h->scale_in, h->v32.tmp, n, done);
  precond<float>(h, K, h->v32.tmp, h->v32.z, h->part_t, &np, done);
  launch_promote(st, K, h->v32.z, h->scale_out, zz, n, false, done);
  launch_dot<double>(st, K, rr, zz, n, h->part_rz, done);
  return vec_blocks(n);
}

// One PCG iteration in precision T (kind FP64/FP32) or FP64 with an FP32
// preconditioner (kind MixedPC), in four segments: the Krylov part up to the
// convergence test (and the FP32 demotion), the preconditioner's second
// branch (stream work2), its first branch, and the join plus the rest of the
// Krylov update.  Eagerly they run back to back with an event fork and join;
// as graphs each segment is captured on its own and launched on its stream,
// so that the two branches overlap on the device.
// (with the shared forward sweep also kSegMainFront, the SOR cycle's forward
// sweep; kSegMainRes, its residual; kSegBranchRest, the second branch's part
// after that residual)
enum Segment {
  kSegPre = 0,
  kSegBranch = 1,
  kSegMain = 2,
  kSegPost = 3,
  kSegMainFront = 4,
  kSegMainRes = 5,
  kSegBranchRest = 6
};

// Reliable update of the mixed-precision solve (FP32 PCG on A d = b / ||b||):
// the FP32 correction accumulated since the last update is scaled by ||b||,
// folded into the FP64 solution hi + lo without rounding error and cleared;
// the true residual b - A (hi + lo) is evaluated in extended precision
// (v64.res) and, scaled by 1 / ||b||, replaces the FP32 recurrence residual.
// The search directions are kept.  The kernels run whatever the columns'
// state, so that a chunk always ends with every correction folded.
void reliable_update(Handle *h, int K) {
  hipStream_t st = h->work;
  const int64_t n = h->P.n;
  launch_promote(st, K, h->v32.x, h->scale_out, h->v64.x, n, false, nullptr);
  launch_fold(st, K, (1u << K) - 1u, h->v64.xs, h->v64.xl, h->v64.x, n);
  launch_fill<float>(st, h->v32.x, n * K, 0.0f, nullptr);
  launch_residual_ext(st, K, h->A, h->b, h->v64.xs, h->v64.xl, h->v64.res);
  launch_demote(st, K, h->v64.res, h->scale_in, h->v32.r, n, nullptr);
}

template <class T>
void pcg_segment(Handle *h, int K, int kind, int seg) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  Work<T> &v = work_of<T>(h);
  const int *done = &h->scal->all_done;
  const bool mixed = kind == kGraphMixedPC;
  switch (seg) {
    case kSegPre:
      launch_spmv<T>(st, K, h->A, 0, 0, n, v.p, (const T *)nullptr, v.q, h->part_pq, done, h->order_all);
      launch_pcg_alpha(st, K, h->scal, h->part_pq, sell_blocks(0, n));
      launch_pcg_xr<T>(st, K, h->scal, v.x, v.r, v.p, v.q, n, h->part_rr);
      launch_pcg_conv(st, K, h->scal, h->part_rr, vec_blocks(n));
      if constexpr (std::is_same<T, double>::value)
        if (mixed) launch_demote(st, K, v.r, h->scale_in, h->v32.tmp, n, done);
      if constexpr (std::is_same<T, float>::value)
        if (kind == kGraphFP32Reliable) reliable_update(h, K);
      break;
    case kSegBranch:
    case kSegBranchRest: {
      const int phase = !shares(h, K) ? 0 : seg == kSegBranch ? 1 : 2;
      if (mixed)
        precond_branch<float>(h, h->work2, K, h->v32.tmp, done, phase);
      else
        precond_branch<T>(h, h->work2, K, v.r, done, phase);
      break;
    }
    case kSegMainFront:
    case kSegMainRes:
    case kSegMain: {
      const int part = !shares(h, K) ? 0 : seg == kSegMainFront ? 1 : seg == kSegMainRes ? 3 : 2;
      if (mixed)
        precond_main<float>(h, st, K, h->v32.tmp, h->v32.z, done, part);
      else
        precond_main<T>(h, st, K, v.r, v.z, done, part);
      break;
    }
    case kSegPost: {
      int64_t np;
      if constexpr (std::is_same<T, double>::value) {
        if (mixed) {
          precond_join<float>(h, st, K, h->v32.tmp, h->v32.z, h->part_t, done);
          launch_promote(st, K, h->v32.z, h->scale_out, v.z, n, false, done);
          launch_dot<double>(st, K, v.r, v.z, n, h->part_rz, done);
          np = vec_blocks(n);
        } else {
          np = precond_join<T>(h, st, K, v.r, v.z, h->part_rz, done);
        }
      } else {
        np = precond_join<T>(h, st, K, v.r, v.z, h->part_rz, done);
      }
      launch_pcg_beta(st, K, h->scal, h->part_rz, np);
      launch_pcg_p<T>(st, K, h->scal, v.p, v.z, n);
      break;
    }
  }
}

template <class T>
void pcg_iteration(Handle *h, int K, int kind) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  Work<T> &v = work_of<T>(h);
  const int *done = &h->scal->all_done;
  if (has_branch(h)) {
    const bool sh = shares(h, K);
    pcg_segment<T>(h, K, kind, kSegPre);
    if (sh) pcg_segment<T>(h, K, kind, kSegMainFront);
    HIPCHK(hipEventRecord(h->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(h->work2, h->ev_fork, 0));
    pcg_segment<T>(h, K, kind, kSegBranch);
    if (sh) {
      pcg_segment<T>(h, K, kind, kSegMainRes);
      HIPCHK(hipEventRecord(h->ev_res, st));
      HIPCHK(hipStreamWaitEvent(h->work2, h->ev_res, 0));
      pcg_segment<T>(h, K, kind, kSegBranchRest);
    }
    HIPCHK(hipEventRecord(h->ev_join, h->work2));
    pcg_segment<T>(h, K, kind, kSegMain);
    HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
    pcg_segment<T>(h, K, kind, kSegPost);
    return;
  }
  launch_spmv<T>(st, K, h->A, 0, 0, n, v.p, (const T *)nullptr, v.q, h->part_pq, done, h->order_all);
  launch_pcg_alpha(st, K, h->scal, h->part_pq, sell_blocks(0, n));
  launch_pcg_xr<T>(st, K, h->scal, v.x, v.r, v.p, v.q, n, h->part_rr);
  launch_pcg_conv(st, K, h->scal, h->part_rr, vec_blocks(n));
  if constexpr (std::is_same<T, float>::value)
    if (kind == kGraphFP32Reliable) reliable_update(h, K);
  int64_t np = 0;
  if (kind == kGraphMixedPC) {
    if constexpr (std::is_same<T, double>::value) np = precond_mixed(h, K, v.r, v.z, done);
  } else {
    precond<T>(h, K, v.r, v.z, h->part_rz, &np, done);
  }
  launch_pcg_beta(st, K, h->scal, h->part_rz, np);
  launch_pcg_p<T>(st, K, h->scal, v.p, v.z, n);
}

void destroy_graphs(Handle *h) {
  for (auto &kv : h->graphs)
    for (int i = 0; i < 7; ++i) {
      if (kv.second.exec[i]) (void)hipGraphExecDestroy(kv.second.exec[i]);
      if (kv.second.graph[i]) (void)hipGraphDestroy(kv.second.graph[i]);
    }
  h->graphs.clear();
}

template <class F>
void capture(hipStream_t st, hipGraph_t *g, hipGraphExec_t *ge, F &&record) {
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  record();
  HIPCHK(hipStreamEndCapture(st, g));
  HIPCHK(hipGraphInstantiate(ge, *g, nullptr, nullptr, 0));
}

// graphs of one iteration for (kind, K), captured on first use when allowed:
// one graph, or the four segments when the preconditioner has two branches
template <class T>
const IterGraphs *iteration_graphs(Handle *h, int K, int kind) {
  int key = kind * 16 + K;
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) return &it->second;
  if (!h->allow_capture) return nullptr;
  IterGraphs ig;
  if (has_branch(h)) {
    ig.parts = shares(h, K) ? 7 : 4;
    for (int seg = 0; seg < ig.parts; ++seg)
      capture(seg == kSegBranch || seg == kSegBranchRest ? h->work2 : h->work, &ig.graph[seg], &ig.exec[seg],
              [&]() { pcg_segment<T>(h, K, kind, seg); });
  } else {
    ig.parts = 1;
    capture(h->work, &ig.graph[0], &ig.exec[0], [&]() { pcg_iteration<T>(h, K, kind); });
  }
  return &h->graphs.emplace(key, ig).first->second;
}

template <class T>
void run_iteration(Handle *h, int K, int kind) {
  const IterGraphs *ig = h->opt.use_graphs ? iteration_graphs<T>(h, K, kind) : nullptr;
  if (!ig) {
    pcg_iteration<T>(h, K, kind);
  } else if (ig->parts == 1) {
    HIPCHK(hipGraphLaunch(ig->exec[0], h->work));
  } else {
    const bool sh = ig->parts == 7;
    HIPCHK(hipGraphLaunch(ig->exec[kSegPre], h->work));
    if (sh) HIPCHK(hipGraphLaunch(ig->exec[kSegMainFront], h->work));
    HIPCHK(hipEventRecord(h->ev_fork, h->work));
    HIPCHK(hipStreamWaitEvent(h->work2, h->ev_fork, 0));
    HIPCHK(hipGraphLaunch(ig->exec[kSegBranch], h->work2));
    if (sh) {
      HIPCHK(hipGraphLaunch(ig->exec[kSegMainRes], h->work));
      HIPCHK(hipEventRecord(h->ev_res, h->work));
      HIPCHK(hipStreamWaitEvent(h->work2, h->ev_res, 0));
      HIPCHK(hipGraphLaunch(ig->exec[kSegBranchRest], h->work2));
    }
    HIPCHK(hipEventRecord(h->ev_join, h->work2));
    HIPCHK(hipGraphLaunch(ig->exec[kSegMain], h->work));
    HIPCHK(hipStreamWaitEvent(h->work, h->ev_join, 0));
    HIPCHK(hipGraphLaunch(ig->exec[kSegPost], h->work));
  }
}

Scal read_scal(Handle *h) {
  Scal hs;
  HIPCHK(hipMemcpyAsync(&hs, h->scal, sizeof(Scal), hipMemcpyDeviceToHost, h->work));
  HIPCHK(hipStreamSynchronize(h->work));
  return hs;
}

// iterate until every column is done
template <class T>
Scal iterate(Handle *h, int K, int kind) {
  int poll = std::max(1, h->opt.poll_every);
  while (true) {
    for (int k = 0; k < poll; ++k) run_iteration<T>(h, K, kind);
    Scal hs = read_scal(h);
    if (hs.all_done) return hs;
  }
}

// true residual res = b - A (xs + xl) of the extended iterate, evaluated in
// extended precision, and its squared column norms (host)
void true_residual(Handle *h, int K, double *rr_host) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  launch_residual_ext(st, K, h->A, h->b, h->v64.xs, h->v64.xl, h->v64.res);
  launch_dot<double>(st, K, h->v64.res, h->v64.res, n, h->part_t, nullptr);
  launch_reduce(st, K, h->part_t, vec_blocks(n), h->dscal);
  HIPCHK(hipMemcpyAsync(rr_host, h->dscal, K * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

void upload_scales(Handle *h, int K, const double *in, const double *out) {
  HIPCHK(hipMemcpyAsync(h->scale_in, in, K * sizeof(double), hipMemcpyHostToDevice, h->work));
  HIPCHK(hipMemcpyAsync(h->scale_out, out, K * sizeof(double), hipMemcpyHostToDevice, h->work));
  HIPCHK(hipStreamSynchronize(h->work));
}

struct ColResult {
  int iters = 0;
  double rel = 0.0;
  int status = VEMG_OK;
};

// squared column norms of b (host)
void rhs_norms(Handle *h, int K, double *bb) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  launch_dot<double>(st, K, h->b, h->b, n, h->part_b, nullptr);
  launch_reduce(st, K, h->part_b, vec_blocks(n), h->dscal);
  HIPCHK(hipMemcpyAsync(bb, h->dscal, K * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

// PCG (FP64, or FP64 with FP32 preconditioner) with restarts from the true
// residual; h->b holds K columns (storage order), result in v64.x.
void solve_cg(Handle *h, int K, double rtol, int max_iter, ColResult *res) {
  batch_layout(h, K);
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  Work<double> &v = h->v64;
  bool mixed = h->opt.precision == VEMG_MIXED_PC;
  int kind = mixed ? kGraphMixedPC : kGraphFP64;
  double bb[kMaxBatch];
  rhs_norms(h, K, bb);
  if (mixed) {
    double sin[kMaxBatch], sout[kMaxBatch];
    for (int k = 0; k < K; ++k) {
      double nb = std::sqrt(bb[k]);
      sin[k] = (nb > 0.0 && std::isfinite(nb)) ? 1.0 / nb : 0.0;
      sout[k] = (nb > 0.0 && std::isfinite(nb)) ? nb : 0.0;
    }
    upload_scales(h, K, sin, sout);
  }
  launch_fill<double>(st, v.x, n * K, 0.0, nullptr);
  launch_fill<double>(st, v.xs, n * K, 0.0, nullptr);
  launch_fill<double>(st, v.xl, n * K, 0.0, nullptr);
  launch_copy<double>(st, h->b, v.r, n * K, nullptr);
  launch_dot<double>(st, K, h->b, h->b, n, h->part_b, nullptr);
  launch_pcg_init(st, K, h->scal, h->part_b, vec_blocks(n), rtol, max_iter);
  const unsigned all = (1u << K) - 1u;
  double prev[kMaxBatch];
  bool final_[kMaxBatch];
  int restarts = 0;
  for (int k = 0; k < K; ++k) {
    prev[k] = INFINITY;
    final_[k] = false;
  }
  while (true) {
    int64_t np = 0;
    if (mixed)
      np = precond_mixed(h, K, v.r, v.z, nullptr);
    else
      precond<double>(h, K, v.r, v.z, h->part_rz, &np, nullptr);
    launch_pcg_set_rho(st, K, h->scal, h->part_rz, np);
    launch_copy<double>(st, v.z, v.p, n * K, nullptr);
    Scal hs = iterate<double>(h, K, kind);
    // columns already final hold x = 0 and are not updated: folding all is exact for them
    launch_fold(st, K, all, v.xs, v.xl, v.x, n);
    double rr[kMaxBatch];
    true_residual(h, K, rr);
    unsigned keep = 0;
    bool any = false;
    for (int k = 0; k < K; ++k) {
      ColResult &c = res[k];
      c.iters = hs.iters[k];
      if (final_[k]) {
        keep |= 1u << k;
        continue;
      }
      if (bb[k] == 0.0) {
        c.rel = 0.0;
        c.status = VEMG_OK;
      } else if (hs.status[k] == -6 || !std::isfinite(bb[k])) {
        c.rel = NAN;
        c.status = VEMG_ERR_BREAKDOWN;
      } else {
        c.rel = std::sqrt(rr[k] / bb[k]);
        if (c.rel <= rtol) c.status = VEMG_OK;
        else if (hs.iters[k] >= max_iter) c.status = VEMG_WARN_MAXITER;
        else if (restarts >= h->opt.max_restarts || c.rel > 0.5 * prev[k]) c.status = VEMG_WARN_FLOOR;
        else {
          prev[k] = c.rel;
          any = true;
          continue;  // restart this column
        }
      }
      final_[k] = true;
      keep |= 1u << k;
    }
    if (!any) break;
    ++restarts;
    launch_copy<double>(st, v.res, v.r, n * K, nullptr);
    launch_pcg_resume(st, K, h->scal, keep);
  }
  launch_round(st, v.xs, v.xl, v.x, n * K);
}

// Iterates a mixed-precision solve until every column has stopped: chunks of
// poll_every FP32 iterations, the last of each chunk with the reliable update.
Scal iterate_reliable(Handle *h, int K) {
  const int poll = std::max(1, h->opt.poll_every);
  while (true) {
    for (int k = 0; k + 1 < poll; ++k) run_iteration<float>(h, K, kGraphFP32);
    run_iteration<float>(h, K, kGraphFP32Reliable);
    Scal hs = read_scal(h);
    if (hs.all_done) return hs;
  }
}

// Mixed precision (VEMG_MIXED_IR): FP64 iterative refinement whose inner FP32
// PCG keeps its Krylov space.  The inner PCG (SpMV, transfers, smoothers and
// vectors in FP32 with per-row scaled operators, inner products accumulated
// in FP64, coarsest solves in FP64) runs on A d = b / ||b||; every poll_every
// iterations a reliable update folds its correction into the FP64 solution
// hi + lo and replaces its residual with the true FP64 residual (evaluated in
// extended precision), without restarting the search directions.  A column
// whose recurrence residual meets rtol is confirmed on that true residual
// and, if it is not met, restarted from it (at most max_restarts times, while
// each restart at least halves it).  h->b holds K columns.
void solve_ir(Handle *h, int K, double rtol, int max_iter, ColResult *res) {
  batch_layout(h, K);
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  Work<float> &v = h->v32;
  double bb[kMaxBatch], sin[kMaxBatch], sout[kMaxBatch];
  rhs_norms(h, K, bb);
  for (int k = 0; k < K; ++k) {
    const double nb = std::sqrt(bb[k]);
    const bool ok = nb > 0.0 && std::isfinite(nb);
    sin[k] = ok ? 1.0 / nb : 0.0;
    sout[k] = ok ? nb : 0.0;
  }
  upload_scales(h, K, sin, sout);
  launch_fill<double>(st, h->v64.x, n * K, 0.0, nullptr);
  launch_fill<double>(st, h->v64.xs, n * K, 0.0, nullptr);
  launch_fill<double>(st, h->v64.xl, n * K, 0.0, nullptr);
  launch_fill<float>(st, v.x, n * K, 0.0f, nullptr);
  launch_demote(st, K, h->b, h->scale_in, v.r, n, nullptr);
  // bnorm2 of the scaled system (about 1); a zero b stops its column at once,
  // a non-finite one (scaled to NaN) as a breakdown
  launch_dot<float>(st, K, v.r, v.r, n, h->part_b, nullptr);
  launch_pcg_init(st, K, h->scal, h->part_b, vec_blocks(n), rtol, max_iter);
  double prev[kMaxBatch];
  bool fin[kMaxBatch];
  int restarts = 0;
  for (int k = 0; k < K; ++k) {
    prev[k] = INFINITY;
    fin[k] = false;
    res[k] = ColResult();
  }
  while (true) {
    int64_t np = 0;
    precond<float>(h, K, v.r, v.z, h->part_rz, &np, nullptr);
    launch_pcg_set_rho(st, K, h->scal, h->part_rz, np);
    launch_copy<float>(st, v.z, v.p, n * K, nullptr);
    Scal hs = iterate_reliable(h, K);
    // the last iteration folded every correction and left b - A (hi + lo) in v64.res
    launch_dot<double>(st, K, h->v64.res, h->v64.res, n, h->part_t, nullptr);
    launch_reduce(st, K, h->part_t, vec_blocks(n), h->dscal);
    double rr[kMaxBatch];
    HIPCHK(hipMemcpyAsync(rr, h->dscal, K * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    unsigned keep = 0;
    bool any = false;
    for (int k = 0; k < K; ++k) {
      ColResult &c = res[k];
      c.iters = hs.iters[k];
      if (fin[k]) {
        keep |= 1u << k;
        continue;
      }
      if (bb[k] == 0.0) {
        c.rel = 0.0;
        c.status = VEMG_OK;
      } else if (hs.status[k] == -6 || !std::isfinite(bb[k]) || !std::isfinite(rr[k])) {
        c.rel = NAN;
        c.status = VEMG_ERR_BREAKDOWN;
      } else {
        c.rel = std::sqrt(rr[k] / bb[k]);
        if (c.rel <= rtol) c.status = VEMG_OK;
        else if (hs.iters[k] >= max_iter) c.status = VEMG_WARN_MAXITER;
        else if (restarts >= h->opt.max_restarts || c.rel > 0.5 * prev[k]) c.status = VEMG_WARN_FLOOR;
        else {
          prev[k] = c.rel;
          any = true;
          continue;  // restart this column from its true residual (already in v32.r)
        }
      }
      fin[k] = true;
      keep |= 1u << k;
    }
    if (!any) break;
    ++restarts;
    launch_pcg_resume(st, K, h->scal, keep);
  }
  launch_round(st, h->v64.xs, h->v64.xl, h->v64.x, n * K);
}

// Packs the host setup into HBM.  With h->ar.count_only the same sequence
// of allocations is only counted (no device call), which gives the footprint
// of a handle before (or without) its upload.
void upload(Handle *h) {
  hipStream_t st = h->work;
  Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  const bool count = h->ar.count_only;
  h->ar.release();
  h->A = pack_sell(h->ar, st, P.Aoff, true, &P.d, &P.diag, &h->nnz_A);
  if (m > 0) {
    h->E = pack_sell(h->ar, st, P.E, false, nullptr, nullptr, &h->nnz_E);
    h->Et = pack_csrg(h->ar, st, P.Et, false, nullptr, &P.loc_rank, 0);
  }
  size_t cnt = (size_t)n * kMaxBatch;
  auto mk64 = [&](Work<double> &v) {
    v.x = h->ar.alloc<double>(cnt);
    v.r = h->ar.alloc<double>(cnt);
    v.z = h->ar.alloc<double>(cnt);
    v.p = h->ar.alloc<double>(cnt);
    v.q = h->ar.alloc<double>(cnt);
    v.w = h->ar.alloc<double>(cnt);
    v.res = h->ar.alloc<double>(cnt);
    v.resA = h->ar.alloc<double>(cnt);
    v.tmp = h->ar.alloc<double>(cnt);
    v.xs = h->ar.alloc<double>(cnt);
    v.xl = h->ar.alloc<double>(cnt);
  };
  auto mk32 = [&](Work<float> &v) {
    v.x = h->ar.alloc<float>(cnt);
    v.r = h->ar.alloc<float>(cnt);
    v.z = h->ar.alloc<float>(cnt);
    v.p = h->ar.alloc<float>(cnt);
    v.q = h->ar.alloc<float>(cnt);
    v.w = h->ar.alloc<float>(cnt);
    v.res = h->ar.alloc<float>(cnt);
    v.resA = h->ar.alloc<float>(cnt);
    v.tmp = h->ar.alloc<float>(cnt);
  };
  mk64(h->v64);
  mk32(h->v32);
  h->b = h->ar.alloc<double>(cnt);
  h->diag = h->ar.upload(P.diag, st);
  h->perm = h->ar.upload(P.perm, st);
  // The products over all rows visit their slices in spatial order across
  // the colours (a slice's key: the spatial rank of its first row in the
  // range), so that the contiguous part of the visit order one XCD takes is
  // one region of every colour, and a row's neighbours, which lie in the
  // other colours, are gathered through the same XCD's L2.
  auto slice_order = [&](int64_t r0, int64_t r1) {
    const int64_t s0 = r0 / kWave, s1 = (r1 + kWave - 1) / kWave;
    std::vector<int32_t> ord(std::max<int64_t>(s1 - s0, 0));
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      return P.loc_rank[std::max((s0 + a) * kWave, r0)] < P.loc_rank[std::max((s0 + b) * kWave, r0)];
    });
    return h->ar.upload(ord, st);
  };
  h->order_all = slice_order(0, n);
  h->order_bar = slice_order(m, n);
  // The SOR cycle and the additive smoother both start with a forward sweep
  // from zero on the same right-hand side; the smoother holds the top rows at
  // zero where the SOR cycle has swept them.  A non-top row of colour c gets
  // the same value in both, bit for bit, unless one of its neighbours of an
  // earlier colour is a top row or such a row itself ("dirty"); its residual
  // is the same unless the row, or a neighbour, is dirty or a neighbour is a
  // top row, or the two zero it differently (the smoother zeroes its last
  // colour, the SOR cycle the rows of its last launch).
  {  // for every preconditioner: a handle may be switched to VL + additive smoother
    const Csr &O = P.Aoff;
    const int ncb = (int)P.bar_colour_start.size() - 1, nct = (int)P.top_colour_start.size() - 1;
    const bool same_last = std::max(nct, ncb) == ncb;
    std::vector<uint8_t> dirty(n, 0);
    std::vector<int32_t> rows, res;
    h->reuse_gs_start.assign(1, 0);
    h->reuse_gs_sell.clear();
    for (int c = 0; c < ncb; ++c) {
      std::vector<int32_t> rc;
      for (int64_t i = P.bar_colour_start[c]; i < P.bar_colour_start[c + 1]; ++i) {
        for (int64_t k = O.ptr[i]; k < O.ptr[i + 1]; ++k) {
          const int64_t j = O.idx[k];
          if (P.colour[j] < c && (j < m || dirty[j])) {
            dirty[i] = 1;
            break;
          }
        }
        if (dirty[i]) rc.push_back((int32_t)i);
      }
      rows.insert(rows.end(), rc.begin(), rc.end());
      h->reuse_gs_start.push_back((int64_t)rows.size());
      h->reuse_gs_sell.push_back(pack_sell(h->ar, st, P.Aoff, true, &P.d, &P.diag, nullptr, &rc));
    }
    for (int64_t i = m; i < n; ++i) {
      bool d = dirty[i] || (!same_last && ncb > 0 && P.colour[i] == ncb - 1);
      for (int64_t k = O.ptr[i]; k < O.ptr[i + 1] && !d; ++k) d = O.idx[k] < m || dirty[O.idx[k]];
      if (d) res.push_back((int32_t)i);
    }
    // without a top surface no row is dirty, but the SOR cycle computes no
    // residual: the smoother computes all of its own
    h->reuse_full_res = m == 0;
    if (h->reuse_full_res) res.clear();
    h->reuse_gs = h->ar.upload(rows, st);
    h->reuse_res = h->ar.upload(res, st);
    h->reuse_res_sell = pack_sell(h->ar, st, P.Aoff, true, &P.d, &P.diag, nullptr, &res);
    h->share_min_rows = share_min_rows();
    h->n_reuse_res = (int64_t)res.size();
    h->reuse = true;
  }
  int64_t npmax = (std::max(sell_blocks(0, n), vec_blocks(n)) + 8) * kMaxBatch;
  h->part_pq = h->ar.alloc<double>(npmax);
  h->part_rr = h->ar.alloc<double>(npmax);
  h->part_rz = h->ar.alloc<double>(npmax);
  h->part_b = h->ar.alloc<double>(npmax);
  h->part_t = h->ar.alloc<double>(npmax);
  h->dscal = h->ar.alloc<double>(kMaxBatch);
  h->scale_in = h->ar.alloc<double>(kMaxBatch);
  h->scale_out = h->ar.alloc<double>(kMaxBatch);
  h->scal = h->ar.alloc<Scal>(1);
  if (!count) {
    // every column starts finished (no right-hand side yet)
    launch_fill<double>(st, h->part_b, kMaxBatch, 0.0, nullptr);
    launch_pcg_init(st, kMaxBatch, h->scal, h->part_b, 1, 1.0, 1);
    // the top block of the smoother vectors stays zero
    launch_fill<double>(st, h->v64.w, (int64_t)cnt, 0.0, nullptr);
    launch_fill<float>(st, h->v32.w, (int64_t)cnt, 0.0f, nullptr);
  }
  if (m > 0) build_levels(h, P.S, h->S, kLevelsS);
  build_levels(h, P.Abar, h->Ab, kLevelsAbar);
  h->SA.clear();
  if (!P.SA.empty()) build_levels(h, P.SA, h->SA, kLevelsSA);
  if (!count) HIPCHK(hipStreamSynchronize(st));
}

// device bytes that upload() allocates for the current host setup; the
// handle's device fields are left cleared, so upload() must follow on a
// device handle
size_t count_upload_bytes(Handle *h) {
  Arena saved = std::move(h->ar);
  h->ar = Arena();
  h->ar.count_only = true;
  upload(h);
  size_t b = h->ar.bytes;
  h->ar = std::move(saved);
  return b;
}

void sync_in(Handle *h) {
  HIPCHK(hipEventRecord(h->ev, h->user));
  HIPCHK(hipStreamWaitEvent(h->work, h->ev, 0));
}

int batch_width(int m) {
  if (m >= 8) return 8;
  if (m >= 4) return 4;
  if (m >= 2) return 2;
  return 1;
}

int do_solve(Handle *h, int nrhs, const double *b_nat, double *x_nat, double rtol, int max_iter, int *iters,
             double *relres) {
  hipStream_t st = h->work;
  int64_t n = h->P.n, N = h->P.n_nodes;
  sync_in(h);
  int worst = VEMG_OK;
  for (int first = 0; first < nrhs;) {
    int m = nrhs - first;
    int K = batch_width(m);
    if (m > 4 && m < 8) K = 8;  // pad small remainders up rather than splitting
    else if (m == 3) K = 4;
    int cols = std::min(K, m);
    if (cols < K) launch_fill<double>(st, h->b, n * K, 0.0, nullptr);
    for (int k = 0; k < cols; ++k) launch_gather(st, K, k, b_nat + (int64_t)(first + k) * N, h->perm, h->b, n);
    ColResult res[kMaxBatch];
    if (h->opt.precision == VEMG_MIXED_IR)
      solve_ir(h, K, rtol, max_iter, res);
    else
      solve_cg(h, K, rtol, max_iter, res);
    for (int k = 0; k < cols; ++k) {
      double *xk = x_nat + (int64_t)(first + k) * N;
      launch_fill<double>(st, xk, N, 0.0, nullptr);
      launch_scatter(st, K, k, h->v64.x, h->perm, xk, n);
      if (iters) iters[first + k] = res[k].iters;
      if (relres) relres[first + k] = res[k].rel;
      int s = res[k].status;
      if (s < 0 || (worst >= 0 && s > worst)) worst = s;
    }
    first += cols;
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

template <class T>
void apply_op(Handle *h, int op, const T *in, T *out) {
  batch_layout(h, 1);
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  Work<T> &v = work_of<T>(h);
  switch (op) {
    case VEMG_OP_A:
      launch_spmv<T>(st, 1, h->A, 0, 0, n, in, (const T *)nullptr, out, nullptr, nullptr, h->order_all);
      break;
    case VEMG_OP_PRECOND: {
      launch_copy<T>(st, in, v.tmp, n, nullptr);
      int64_t np = 0;
      precond<T>(h, 1, v.tmp, out, h->part_t, &np, nullptr);
      break;
    }
    case VEMG_OP_ET:
      launch_csr_rect<T>(st, 1, h->Et, false, in, out, nullptr);
      break;
    case VEMG_OP_E:
      launch_rect<T>(st, 1, h->E, false, in, out, nullptr);
      break;
    case VEMG_OP_VCYCLE_S:
      launch_copy<T>(st, in, h->S[0].g<T>(), m, nullptr);
      vcycle<T>(st, 1, h->S, 0, nullptr);
      launch_copy<T>(st, h->S[0].x<T>(), out, m, nullptr);
      break;
    case VEMG_OP_VCYCLE_ABAR: {
      launch_copy<T>(st, in, v.tmp + m, n - m, nullptr);
      T *saved = h->Ab[0].g<T>();
      h->Ab[0].g<T>() = v.tmp;
      vcycle<T>(st, 1, h->Ab, 0, nullptr);
      h->Ab[0].g<T>() = saved;
      launch_copy<T>(st, v.w + m, out, n - m, nullptr);
      break;
    }
    case VEMG_OP_GS_FWD: {
      launch_fill<T>(st, out, n, T(0), nullptr);
      int nct = (int)P.top_colour_start.size() - 1, ncb = (int)P.bar_colour_start.size() - 1;
      for (int c = 0; c < std::max(nct, ncb); ++c) {
        int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (c < nct) {
          a0 = P.top_colour_start[c];
          a1 = P.top_colour_start[c + 1];
        }
        if (c < ncb) {
          b0 = P.bar_colour_start[c];
          b1 = P.bar_colour_start[c + 1];
        }
        launch_gs<T>(st, 1, h->A, a0, a1, b0, b1, in, out, nullptr);
      }
      break;
    }
  }
}

int do_apply(Handle *h, int op, const double *in, double *out) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  if (op < VEMG_OP_A || op > VEMG_OP_GS_FWD) return VEMG_ERR_INVALID_ARG;
  if ((op == VEMG_OP_ET || op == VEMG_OP_E || op == VEMG_OP_VCYCLE_S) && m == 0) return VEMG_ERR_STATE;
  int64_t nin = (op == VEMG_OP_E || op == VEMG_OP_VCYCLE_S) ? m : (op == VEMG_OP_VCYCLE_ABAR ? n - m : n);
  int64_t nout = (op == VEMG_OP_ET || op == VEMG_OP_VCYCLE_S) ? m : (op == VEMG_OP_VCYCLE_ABAR ? n - m : n);
  sync_in(h);
  HIPCHK(hipMemsetAsync(h->scal, 0, sizeof(Scal), st));
  if (h->opt.precision == VEMG_FP64) {
    apply_op<double>(h, op, in, out);
  } else {
    double one = 1.0, ones[kMaxBatch];
    for (double &o : ones) o = one;
    upload_scales(h, 1, ones, ones);
    float *in32 = h->v32.res, *out32 = h->v32.q;
    launch_demote(st, 1, in, h->scale_in, in32, nin, nullptr);
    apply_op<float>(h, op, in32, out32);
    launch_promote(st, 1, out32, h->scale_out, out, nout, false, nullptr);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return VEMG_OK;
}

template <class T>
void time_once(Handle *h, int op, int K) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n;
  Work<T> &v = work_of<T>(h);
  if (op == VEMG_OP_A) {
    launch_spmv<T>(st, K, h->A, 0, 0, n, v.p, (const T *)nullptr, v.q, h->part_pq, nullptr, h->order_all);
    return;
  }
  if (op == VEMG_OP_ET) {
    launch_csr_rect<T>(st, K, h->Et, false, v.r, h->S[0].g<T>(), nullptr);
    return;
  }
  if (op == VEMG_OP_E) {
    launch_rect<T>(st, K, h->E, true, h->S[0].x<T>(), v.z, nullptr);
    return;
  }
  if (op == VEMG_OP_COARSEST) {
    DLevel &L = h->S.back();
    launch_dense<T>(st, K, L.Cinv, L.n, L.g<T>(), L.x<T>(), L.dpart, nullptr);
    return;
  }
  if (op == VEMG_OP_GS_COARSE) {
    DLevel &L = h->Ab[1];
    for (size_t c = 0; c + 1 < L.pc_start.size(); ++c)
      launch_patch_gs<T>(st, K, L.Ac, L.ps, L.pc_start[c], L.pc_start[c + 1] - L.pc_start[c], L.g<T>(), L.x<T>(),
                         nullptr, -1, false);
    return;
  }
  int nct = (int)P.top_colour_start.size() - 1, ncb = (int)P.bar_colour_start.size() - 1;
  for (int c = 0; c < std::max(nct, ncb); ++c) {
    int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (c < nct) {
      a0 = P.top_colour_start[c];
      a1 = P.top_colour_start[c + 1];
    }
    if (c < ncb) {
      b0 = P.bar_colour_start[c];
      b1 = P.bar_colour_start[c + 1];
    }
    launch_gs<T>(st, K, h->A, a0, a1, b0, b1, v.r, v.z, nullptr);
  }
}

int do_time(Handle *h, int op, int K, int reps, double *avg_ms, int *launches) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n;
  if (op != VEMG_OP_A && op != VEMG_OP_GS_FWD && op != VEMG_OP_GS_COARSE && op != VEMG_OP_ET && op != VEMG_OP_E &&
      op != VEMG_OP_COARSEST)
    return VEMG_ERR_INVALID_ARG;
  if (op == VEMG_OP_COARSEST && (P.n_top == 0 || h->S.empty())) return VEMG_ERR_STATE;
  if (op == VEMG_OP_GS_COARSE && (h->Ab.size() < 2 || h->Ab[1].coarsest)) return VEMG_ERR_STATE;
  if ((op == VEMG_OP_ET || op == VEMG_OP_E) && (P.n_top == 0 || h->S.empty())) return VEMG_ERR_STATE;
  if (K != 1 && K != 2 && K != 4 && K != 8) return VEMG_ERR_INVALID_ARG;
  batch_layout(h, K);
  int nc = std::max((int)P.top_colour_start.size() - 1, (int)P.bar_colour_start.size() - 1);
  if (op == VEMG_OP_GS_COARSE) {
    nc = (int)h->Ab[1].pc_start.size() - 1;
    DLevel &L = h->Ab[1];
    if (h->opt.precision == VEMG_MIXED_IR) {
      launch_fill<float>(st, L.g32, L.n * K, 1.0f, nullptr);
      launch_fill<float>(st, L.x32, L.n * K, 0.0f, nullptr);
    } else {
      launch_fill<double>(st, L.g64, L.n * K, 1.0, nullptr);
      launch_fill<double>(st, L.x64, L.n * K, 0.0, nullptr);
    }
  }
  bool f32 = h->opt.precision == VEMG_MIXED_IR;
  if (op == VEMG_OP_E) {
    if (f32)
      launch_fill<float>(st, h->S[0].x32, P.n_top * K, 1.0f, nullptr);
    else
      launch_fill<double>(st, h->S[0].x64, P.n_top * K, 1.0, nullptr);
  }
  if (f32) {
    launch_fill<float>(st, h->v32.p, n * K, 1.0f, nullptr);
    launch_fill<float>(st, h->v32.r, n * K, 1.0f, nullptr);
    launch_fill<float>(st, h->v32.z, n * K, 0.0f, nullptr);
  } else {
    launch_fill<double>(st, h->v64.p, n * K, 1.0, nullptr);
    launch_fill<double>(st, h->v64.r, n * K, 1.0, nullptr);
    launch_fill<double>(st, h->v64.z, n * K, 0.0, nullptr);
  }
  auto once = [&]() {
    if (f32) time_once<float>(h, op, K); else time_once<double>(h, op, K);
  };
  once();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k) once();
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  if (op == VEMG_OP_COARSEST) {
    DLevel &L = h->S.back();
    if (h->opt.precision == VEMG_MIXED_IR)
      launch_fill<float>(st, L.g32, L.n * K, 1.0f, nullptr);
    else
      launch_fill<double>(st, L.g64, L.n * K, 1.0, nullptr);
  }
  if (launches) *launches = (op == VEMG_OP_A || op == VEMG_OP_ET || op == VEMG_OP_E || op == VEMG_OP_COARSEST) ? 1 : nc;
  return VEMG_OK;
}

template <class T>
int export_vec(const std::vector<T> &v, void *buf, size_t *bytes) {
  size_t need = v.size() * sizeof(T);
  if (!buf) {
    *bytes = need;
    return VEMG_OK;
  }
  if (*bytes < need) return VEMG_ERR_INVALID_ARG;
  if (need) std::memcpy(buf, v.data(), need);
  *bytes = need;
  return VEMG_OK;
}

int export_csr(const Csr &A, const std::string &what, void *buf, size_t *bytes) {
  if (what == "ptr") return export_vec(A.ptr, buf, bytes);
  if (what == "idx") return export_vec(A.idx, buf, bytes);
  if (what == "val") return export_vec(A.val, buf, bytes);
  return VEMG_ERR_INVALID_ARG;
}

int do_export(Handle *h, const std::string &name, void *buf, size_t *bytes) {
  const Problem &P = h->P;
  if (name == "perm") return export_vec(P.perm, buf, bytes);
  if (name == "colour") return export_vec(P.colour, buf, bytes);
  if (name == "d") return export_vec(P.d, buf, bytes);
  if (name == "diag") return export_vec(P.diag, buf, bytes);
  if (name == "S_perm") return export_vec(P.S_perm, buf, bytes);
  auto dot = name.find('.');
  if (dot == std::string::npos) return VEMG_ERR_INVALID_ARG;
  std::string head = name.substr(0, dot), rest = name.substr(dot + 1);
  if (head == "Aoff") return export_csr(P.Aoff, rest, buf, bytes);
  if (head == "E") return export_csr(P.E, rest, buf, bytes);
  if (head == "S" || head == "Abar" || head == "SA") {
    const std::vector<Level> &H = head == "S" ? P.S : head == "Abar" ? P.Abar : P.SA;
    auto dot2 = rest.find('.');
    if (dot2 == std::string::npos) return VEMG_ERR_INVALID_ARG;
    size_t l = (size_t)std::stoul(rest.substr(0, dot2));
    std::string what = rest.substr(dot2 + 1);
    if (l >= H.size()) return VEMG_ERR_INVALID_ARG;
    const Level &L = H[l];
    if (what.rfind("A.", 0) == 0) return export_csr(L.A, what.substr(2), buf, bytes);
    if (what.rfind("P.", 0) == 0) return export_csr(L.P, what.substr(2), buf, bytes);
    if (what == "colour") return export_vec(L.colour, buf, bytes);
    if (what == "rank") return export_vec(L.rank, buf, bytes);
    if (what == "patch") return export_vec(L.patch, buf, bytes);
    if (what == "pcolour") return export_vec(L.pcolour, buf, bytes);
    if (what == "lcolour") return export_vec(L.lcolour, buf, bytes);
    if (what == "pc_start") return export_vec(L.pc_start, buf, bytes);
    if (what == "patch_row") return export_vec(L.patch_row, buf, bytes);
    if (what == "seg_ptr") return export_vec(L.seg_ptr, buf, bytes);
    if (what == "seg_row") return export_vec(L.seg_row, buf, bytes);
    if (what == "node") return export_vec(L.node, buf, bytes);
    if (what == "agg") return export_vec(L.agg, buf, bytes);
    if (what == "Cinv") return export_vec(L.Cinv, buf, bytes);
  }
  return VEMG_ERR_INVALID_ARG;
}

// A non-blocking stream with a hardware queue of its own: no implicit
// ordering with the legacy null stream (so another thread's work cannot join
// a graph being captured on it; ordering with the caller's stream is
// explicit, see sync_in), and, being created with a CU mask (every CU, so
// nothing is restricted), it does not share its queue, so the two
// preconditioner branches cannot end up serialised behind each other or
// behind another stream's work.
hipError_t create_queue_stream(int device, hipStream_t *st) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return e;
  std::vector<uint32_t> mask((prop.multiProcessorCount + 31) / 32, 0xffffffffu);
  return hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data());
}

int fail(Handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

template <class F>
int guarded(Handle *h, F &&f) {
  try {
    if (h && h->device >= 0) {
      hipError_t e = hipSetDevice(h->device);
      if (e != hipSuccess) return fail(h, VEMG_ERR_DEVICE, hipGetErrorString(e));
    }
    return f();
  } catch (const SetupError &e) {
    return fail(h, e.code, e.what());
  } catch (const DeviceError &e) {
    return fail(h, e.code, e.what());
  } catch (const std::bad_alloc &) {
    return fail(h, VEMG_ERR_OOM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(h, VEMG_ERR_DEVICE, e.what());
  }
}

}  // namespace
}  // namespace vemg


// ============================================================== static buffer
// Device memory for vemg_matvec_noalloc, which allocates nothing: a
// file-scope array that every GPU the library runs on holds until the process
// ends.  In host code its name is only a stand-in; the device address on each
// GPU comes from hipGetSymbolAddress, looked up once per device.
namespace vemg {

constexpr int64_t kScratchRows = int64_t(1) << 21;  // unknowns: two vectors of this length, 32 MiB

namespace {

__device__ __align__(256) double scratch[2 * kScratchRows];

std::mutex scratch_mu;
std::map<int, double *> scratch_addr;  // device ordinal -> address of scratch on that device

// address of the static buffer on `device` (the current device)
double *scratch_of(int device) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_addr.find(device);
  if (it != scratch_addr.end()) return it->second;
  void *p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  scratch_addr[device] = (double *)p;
  return (double *)p;
}

}  // namespace
}  // namespace vemg

// ============================================================== serving
namespace vemg {
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// One solve request.  The submitting thread fills it under the server lock;
// afterwards the scheduler thread owns iters, rel, status and cols_left
// until it sets done (under the lock), after which only readers remain.
struct SReq {
  uint64_t id = 0;
  int mesh = 0, nrhs = 0, max_iter = 0;
  const double *b = nullptr;
  double *x = nullptr;
  double rtol = 0.0, t_submit = 0.0, t_done = 0.0;
  int cols_left = 0, status = VEMG_OK;
  bool done = false;
  std::vector<int> iters;
  std::vector<double> rel;
};

// A column slot of a lane.  It points at its request directly: requests are
// owned by unique_ptr and never move, so the scheduler reaches them without
// touching the server's request list.
struct SSlot {
  SReq *req = nullptr;
  int col = 0, restarts = 0;
  double prev = INFINITY;
};

struct Lane {
  vemg_solver_s *h = nullptr;
  bool resident = false;
  size_t footprint = 0;
  std::deque<std::pair<SReq *, int>> queue;  // (request, column), scheduler thread only
  SSlot slot[kMaxBatch];
  bool launched = false;
  uint64_t last_used = 0;
  Scal *scal_host = nullptr;  // pinned copy of the lane's scalars after its last chunk
  hipEvent_t scal_ready = nullptr;
  bool busy() const {
    if (!queue.empty()) return true;
    for (auto &s : slot)
      if (s.req) return true;
    return false;
  }
};

// At most kServerStreamPairs pairs of streams serve every lane (lane i uses
// pair i mod kServerStreamPairs): a pair is the lane's Krylov stream and its
// second preconditioner branch, each created with a (full) CU mask so that it
// has a hardware queue of its own.
constexpr int kServerStreamPairs = 2;

}  // namespace
}  // namespace vemg

struct vemg_server_s {
  int device = 0;
  size_t budget = 0;
  vemg_options opt;
  hipStream_t streams[2 * vemg::kServerStreamPairs] = {};
  std::vector<std::unique_ptr<vemg::Lane>> lanes;
  std::vector<std::unique_ptr<vemg::SReq>> reqs;  // owner; appended under mu
  std::map<uint64_t, vemg::SReq *> by_id;
  std::deque<vemg::SReq *> incoming, completed;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::thread worker;
  bool stop = false, started = false;
  uint64_t next_id = 1, tick = 0;
  std::string err;
  double first_submit = -1.0, last_done = -1.0;
  // written by the scheduler thread, read by vemg_server_get_stats
  std::atomic<size_t> used{0};
  std::atomic<int64_t> chunks{0}, uploads{0}, evictions{0}, cols_done{0}, active_slots{0};
  int64_t reqs_base = 0;  // requests before the last statistics reset
};

namespace vemg {
namespace {

using Server = vemg_server_s;

void lane_release(Server *sv, Lane &L) {
  destroy_graphs(L.h);
  L.h->ar.release();
  L.resident = false;
  sv->used -= L.footprint;
  sv->evictions++;
}

// make a lane resident, evicting idle lanes (least recently used first)
bool lane_admit(Server *sv, Lane &L) {
  if (L.resident) return true;
  while (sv->budget && sv->used + L.footprint > sv->budget) {
    Lane *victim = nullptr;
    for (auto &o : sv->lanes)
      if (o->resident && !o->busy() && (!victim || o->last_used < victim->last_used)) victim = o.get();
    if (!victim) return false;
    lane_release(sv, *victim);
  }
  upload(L.h);
  if (L.h->ar.bytes != L.footprint)
    throw DeviceError(VEMG_ERR_DEVICE, "device allocations differ from the counted footprint");
  L.resident = true;
  sv->used += L.footprint;
  sv->uploads++;
  return true;
}

// each slot stops on its own request's tolerance and iteration cap
SlotStop lane_stop(const Lane &L) {
  SlotStop st;
  for (int k = 0; k < kMaxBatch; ++k) {
    const SReq *q = L.slot[k].req;
    st.tol[k] = q ? q->rtol : 1.0;
    st.maxit[k] = q ? q->max_iter : 1;
  }
  return st;
}

// (re)start the slot columns in mask: join (x = 0, r = b) or restart (r = res)
void lane_start(Lane &L, unsigned mask, bool restart) {
  Handle *h = L.h;
  batch_layout(h, kMaxBatch);
  hipStream_t st = h->work;
  int64_t n = h->P.n, N = h->P.n_nodes;
  if (!restart)
    for (int k = 0; k < kMaxBatch; ++k)
      if ((mask >> k) & 1u) {
        const SReq &q = *L.slot[k].req;
        launch_gather(st, kMaxBatch, k, q.b + (int64_t)L.slot[k].col * N, h->perm, h->b, n);
      }
  launch_slot_vectors(st, mask, restart, h->b, h->v64.res, h->v64.xs, h->v64.xl, h->v64.x, h->v64.r, n);
  launch_dot<double>(st, kMaxBatch, h->b, h->b, n, h->part_b, nullptr);
  launch_slot_scalars(st, mask, restart, h->scal, h->part_b, vec_blocks(n), lane_stop(L), h->scale_in,
                      h->scale_out);
  int64_t np = 0;
  if (h->opt.precision != VEMG_FP64)
    np = precond_mixed(h, kMaxBatch, h->v64.r, h->v64.z, nullptr);
  else
    precond<double>(h, kMaxBatch, h->v64.r, h->v64.z, h->part_rz, &np, nullptr);
  launch_slot_rho(st, mask, h->scal, h->part_rz, np);
  launch_slot_copy(st, mask, h->v64.z, h->v64.p, n);
}

void finish_request(Server *sv, SReq &q) {
  std::lock_guard<std::mutex> lk(sv->mu);
  q.done = true;
  q.t_done = now_s();
  sv->completed.push_back(&q);
  sv->last_done = q.t_done;
  sv->cv_done.notify_all();
}

// columns that finished their chunk: confirm on the FP64 true residual and
// retire them, or restart them from the true residual
void lane_collect(Server *sv, Lane &L) {
  Handle *h = L.h;
  hipStream_t st = h->work;
  HIPCHK(hipEventSynchronize(L.scal_ready));
  const Scal hs = *L.scal_host;
  unsigned fin = 0;
  for (int k = 0; k < kMaxBatch; ++k)
    if (L.slot[k].req && hs.done[k]) fin |= 1u << k;
  if (!fin) return;
  launch_fold(st, kMaxBatch, fin, h->v64.xs, h->v64.xl, h->v64.x, h->P.n);
  double rr[kMaxBatch];
  true_residual(h, kMaxBatch, rr);
  launch_round(st, h->v64.xs, h->v64.xl, h->v64.tmp, h->P.n * kMaxBatch);
  unsigned restart = 0;
  std::vector<SReq *> finished;
  int64_t n = h->P.n, N = h->P.n_nodes;
  for (int k = 0; k < kMaxBatch; ++k) {
    if (!((fin >> k) & 1u)) continue;
    SSlot &sl = L.slot[k];
    SReq &q = *sl.req;
    double bb = hs.bnorm2[k];
    double rel;
    int status;
    if (bb == 0.0) {
      rel = 0.0;
      status = VEMG_OK;
    } else if (hs.status[k] == -6 || !std::isfinite(bb)) {
      rel = NAN;
      status = VEMG_ERR_BREAKDOWN;
    } else {
      rel = std::sqrt(rr[k] / bb);
      if (rel <= q.rtol) status = VEMG_OK;
      else if (hs.iters[k] >= q.max_iter) status = VEMG_WARN_MAXITER;
      else if (sl.restarts >= h->opt.max_restarts || rel > 0.5 * sl.prev) status = VEMG_WARN_FLOOR;
      else {
        sl.prev = rel;
        sl.restarts++;
        restart |= 1u << k;
        continue;
      }
    }
    double *xk = q.x + (int64_t)sl.col * N;
    launch_fill<double>(st, xk, N, 0.0, nullptr);
    launch_scatter(st, kMaxBatch, k, h->v64.tmp, h->perm, xk, n);
    q.iters[sl.col] = hs.iters[k];
    q.rel[sl.col] = rel;
    if (status < 0 || (q.status >= 0 && status > q.status)) q.status = status;
    if (--q.cols_left == 0) finished.push_back(&q);
    sl = SSlot();
    sv->cols_done++;
  }
  if (restart) lane_start(L, restart, true);
  HIPCHK(hipStreamSynchronize(st));
  for (SReq *q : finished) finish_request(sv, *q);
}

void server_loop(Server *sv) {
  (void)hipSetDevice(sv->device);
  while (true) {
    int precision;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      auto has_work = [&]() {
        if (!sv->incoming.empty()) return true;
        for (auto &L : sv->lanes)
          if (L->busy()) return true;
        return false;
      };
      sv->cv.wait(lk, [&]() { return sv->stop || has_work(); });
      if (sv->stop && !has_work()) break;
      while (!sv->incoming.empty()) {
        SReq *q = sv->incoming.front();
        sv->incoming.pop_front();
        for (int c = 0; c < q->nrhs; ++c) sv->lanes[q->mesh]->queue.emplace_back(q, c);
      }
      precision = sv->opt.precision;
    }
    try {
      // admission, joins and launches: every lane's chunk is queued before
      // any lane is waited on, so different meshes overlap on the device
      for (auto &Lp : sv->lanes) {
        Lane &L = *Lp;
        L.launched = false;
        if (!L.busy()) continue;
        if (!lane_admit(sv, L)) continue;
        L.last_used = ++sv->tick;
        // a precision switch waits for every request to finish, so a lane
        // that takes it is idle
        L.h->opt.precision = precision;
        unsigned mask = 0;
        for (int k = 0; k < kMaxBatch && !L.queue.empty(); ++k)
          if (!L.slot[k].req) {
            L.slot[k] = SSlot();
            L.slot[k].req = L.queue.front().first;
            L.slot[k].col = L.queue.front().second;
            L.queue.pop_front();
            mask |= 1u << k;
          }
        if (mask) lane_start(L, mask, false);
        int active = 0;
        for (auto &sl : L.slot) active += sl.req != nullptr;
        if (!active) continue;
        int kind = L.h->opt.precision != VEMG_FP64 ? kGraphMixedPC : kGraphFP64;
        for (int it = 0; it < L.h->opt.poll_every; ++it) run_iteration<double>(L.h, kMaxBatch, kind);
        HIPCHK(hipMemcpyAsync(L.scal_host, L.h->scal, sizeof(Scal), hipMemcpyDeviceToHost, L.h->work));
        HIPCHK(hipEventRecord(L.scal_ready, L.h->work));
        L.launched = true;
        sv->chunks++;
        sv->active_slots += active;
      }
      for (auto &Lp : sv->lanes)
        if (Lp->launched) lane_collect(sv, *Lp);
    } catch (const std::exception &e) {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->err = e.what();
      sv->stop = true;
      // fail every pending request so that waiters return
      for (auto &q : sv->reqs)
        if (!q->done) {
          q->done = true;
          q->status = VEMG_ERR_DEVICE;
          q->t_done = now_s();
          sv->completed.push_back(q.get());
        }
      for (auto &L : sv->lanes) {
        L->queue.clear();
        for (auto &sl : L->slot) sl = SSlot();
      }
      sv->incoming.clear();
      sv->cv_done.notify_all();
      break;
    }
  }
}

}  // namespace
}  // namespace vemg

namespace vemg {
namespace {

bool valid_options(const vemg_options &opt) {
  return !(opt.top_bc < 0 || opt.top_bc > 2 ||
           (opt.top_bc == VEMG_TOP_ROBIN && !(opt.robin_alpha > 0.0 && std::isfinite(opt.robin_alpha))) ||
           opt.pc < 0 || opt.pc > 5 || opt.max_levels < 1 || opt.max_levels > 16 || opt.coarse_max < 1 ||
           opt.coarse_max > 8192 || !(opt.theta >= 0.0) || opt.poll_every < 1 || opt.precision < 0 ||
           opt.precision > 2 || !(opt.inner_rtol > 0.0 && opt.inner_rtol < 1.0) || opt.max_outer < 1 ||
           opt.extrapolation < 0 || opt.extrapolation > 1);
}

// A handle on `device`.  pool == nullptr: the handle creates its own two work
// streams; otherwise it runs on pool[0] (Krylov part, first branch) and
// pool[1] (second branch), which stay the caller's.
vemg_status create_handle(const vemg_options *o, int device, hipStream_t user, const hipStream_t *pool,
                          vemg_solver *out) {
  if (!out) return VEMG_ERR_INVALID_ARG;
  *out = nullptr;
  vemg_options opt;
  if (o)
    opt = *o;
  else
    vemg_default_options(&opt);
  if (!valid_options(opt)) return VEMG_ERR_INVALID_ARG;
  auto *h = new (std::nothrow) vemg_solver_s();
  if (!h) return VEMG_ERR_OOM;
  h->opt = opt;
  h->device = device;
  h->user = user;
  int st = guarded(h, [&]() -> int {
    if (device >= 0) {
      if (pool) {
        h->own_streams = false;
        h->work = pool[0];
        h->work2 = pool[1];
      } else {
        HIPCHK(create_queue_stream(device, &h->work));
        HIPCHK(create_queue_stream(device, &h->work2));
      }
      HIPCHK(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_res, hipEventDisableTiming));
    }
    return VEMG_OK;
  });
  if (st != VEMG_OK) {
    (void)vemg_destroy(h);  // releases whatever was created before the failure
    return (vemg_status)st;
  }
  *out = h;
  return VEMG_OK;
}

}  // namespace
}  // namespace vemg

using vemg::guarded;

extern "C" {

void vemg_default_options(vemg_options *o) {
  if (!o) return;
  o->top_bc = VEMG_TOP_PINNED;
  o->pin_node = -1;
  o->pc = VEMG_PC_VL_ADDITIVE;
  o->theta = 0.01;
  o->prolong_omega = 2.0 / 3.0;
  o->max_levels = 10;
  o->coarse_max = 8192;
  o->poll_every = 8;
  o->max_restarts = 5;
  o->use_graphs = 1;
  o->precision = VEMG_FP64;
  o->inner_rtol = 1e-4;
  o->max_outer = 30;
  o->robin_alpha = 0.0;
  o->extrapolation = VEMG_EXTRAP_PROJECTION;
}

vemg_status vemg_create(const vemg_options *o, int device, void *hip_stream, vemg_solver *out) {
  return vemg::create_handle(o, device, (hipStream_t)hip_stream, nullptr, out);
}

vemg_status vemg_setup(vemg_solver s, int64_t n_nodes, const double *xyz, int64_t n_tets, const int64_t *tets,
                       const uint8_t *top_mask) {
  if (!s) return VEMG_ERR_INVALID_ARG;
  return (vemg_status)guarded(s, [&]() -> int {
    s->ready = false;
    vemg::destroy_graphs(s);
    s->ar.release();
    vemg::SetupOptions so;
    so.top_dirichlet = s->opt.top_bc == VEMG_TOP_DIRICHLET;
    so.robin = s->opt.top_bc == VEMG_TOP_ROBIN;
    so.robin_alpha = s->opt.robin_alpha;
    so.build_sa = s->opt.pc == VEMG_PC_SA;
    so.extrapolation = s->opt.extrapolation;
    so.pin_node = s->opt.pin_node;
    so.theta = s->opt.theta;
    so.prolong_omega = s->opt.prolong_omega;
    so.max_levels = s->opt.max_levels;
    so.coarse_max = s->opt.coarse_max;
    s->P = vemg::Problem();
    vemg::build_problem(s->P, so, n_nodes, xyz, n_tets, tets, top_mask);
    s->footprint = vemg::count_upload_bytes(s);
    if (s->device >= 0) {
      vemg::upload(s);
      if (s->ar.bytes != s->footprint)
        throw vemg::DeviceError(VEMG_ERR_DEVICE, "device allocations differ from the counted footprint");
    }
    s->ready = true;
    s->err.clear();
    return VEMG_OK;
  });
}

vemg_status vemg_rhs(vemg_solver s, const double *f_host, double *b_host) {
  if (!s || !f_host || !b_host) return VEMG_ERR_INVALID_ARG;
  if (!s->ready) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int {
    vemg::mass_rhs(s->P, f_host, b_host);
    return VEMG_OK;
  });
}

vemg_status vemg_matvec(vemg_solver s, const double *x_dev, double *y_dev) {
  if (!s || !x_dev || !y_dev) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int {
    hipStream_t st = s->work;
    int64_t n = s->P.n;
    vemg::sync_in(s);
    vemg::launch_gather(st, 1, 0, x_dev, s->perm, s->v64.tmp, n);
    vemg::launch_spmv<double>(st, 1, s->A, 0, 0, n, s->v64.tmp, nullptr, s->v64.res, nullptr, nullptr, s->order_all);
    vemg::launch_fill<double>(st, y_dev, s->P.n_nodes, 0.0, nullptr);
    vemg::launch_scatter(st, 1, 0, s->v64.res, s->perm, y_dev, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return VEMG_OK;
  });
}

vemg_status vemg_matvec_noalloc(vemg_solver s, const double *x_dev, double *y_dev) {
  if (!s || !x_dev || !y_dev) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  if (s->P.n > vemg::kScratchRows) {
    s->err = "vemg_matvec_noalloc: " + std::to_string(s->P.n) + " unknowns exceed the static buffer's " +
             std::to_string(vemg::kScratchRows);
    return VEMG_ERR_INVALID_ARG;
  }
  return (vemg_status)guarded(s, [&]() -> int {
    double *buf = vemg::scratch_of(s->device);  // [0, n): x in storage order; [n, 2n): A x
    hipStream_t st = s->work;
    int64_t n = s->P.n;
    vemg::sync_in(s);
    vemg::launch_gather(st, 1, 0, x_dev, s->perm, buf, n);
    vemg::launch_spmv<double>(st, 1, s->A, 0, 0, n, buf, nullptr, buf + n, nullptr, nullptr, s->order_all);
    vemg::launch_fill<double>(st, y_dev, s->P.n_nodes, 0.0, nullptr);
    vemg::launch_scatter(st, 1, 0, buf + n, s->perm, y_dev, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return VEMG_OK;
  });
}

vemg_status vemg_solve(vemg_solver s, int nrhs, const double *b_dev, double *x_dev, double rtol, int max_iter,
                       int *iters, double *relres) {
  if (!s || !b_dev || !x_dev || nrhs < 1 || !(rtol >= 0.0) || max_iter < 1) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_solve(s, nrhs, b_dev, x_dev, rtol, max_iter, iters, relres); });
}

vemg_status vemg_apply(vemg_solver s, int op, const double *in_dev, double *out_dev) {
  if (!s || !in_dev || !out_dev) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_apply(s, op, in_dev, out_dev); });
}

vemg_status vemg_time_op(vemg_solver s, int op, int nrhs, int reps, double *avg_ms, int *launches) {
  if (!s || !avg_ms || reps < 1) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_time(s, op, nrhs, reps, avg_ms, launches); });
}

vemg_status vemg_set_preconditioner(vemg_solver s, int pc) {
  if (!s || pc < 0 || pc > 5) return VEMG_ERR_INVALID_ARG;
  if (pc == VEMG_PC_SA && s->P.SA.empty()) {
    s->err = "the smoothed aggregation baseline hierarchy is built only when the handle is set up with it";
    return VEMG_ERR_STATE;
  }
  return (vemg_status)guarded(s, [&]() -> int {
    if (s->device >= 0) {
      if (s->work) HIPCHK(hipStreamSynchronize(s->work));
      if (s->work2) HIPCHK(hipStreamSynchronize(s->work2));
    }
    vemg::destroy_graphs(s);
    s->opt.pc = pc;
    return VEMG_OK;
  });
}

vemg_status vemg_set_precision(vemg_solver s, int precision) {
  if (!s || precision < 0 || precision > 2) return VEMG_ERR_INVALID_ARG;
  s->opt.precision = precision;
  return VEMG_OK;
}

vemg_status vemg_get_info(vemg_solver s, vemg_info *info) {
  if (!s || !info) return VEMG_ERR_INVALID_ARG;
  if (!s->ready) return VEMG_ERR_STATE;
  std::memset(info, 0, sizeof(*info));
  const vemg::Problem &P = s->P;
  info->n_nodes = P.n_nodes;
  info->n = P.n;
  info->n_top = P.n_top;
  info->pin_node = P.pin;
  info->nnz_offdiag = P.Aoff.nnz();
  info->s_levels = (int)P.S.size();
  info->abar_levels = (int)P.Abar.size();
  for (size_t l = 0; l < P.S.size() && l < 16; ++l) {
    info->s_rows[l] = P.S[l].n();
    info->s_nnz[l] = P.S[l].A.nnz() - P.S[l].n();
    info->p_nnz_s[l] = P.S[l].P.nnz();
  }
  for (size_t l = 0; l < P.Abar.size() && l < 16; ++l) {
    info->abar_rows[l] = P.Abar[l].n();
    info->abar_nnz[l] = P.Abar[l].A.nnz() - P.Abar[l].n();
    info->p_nnz_abar[l] = P.Abar[l].P.nnz();
  }
  info->e_nnz = P.E.nnz();
  info->fine_colours_top = (int)P.top_colour_start.size() - 1;
  info->fine_colours_bar = (int)P.bar_colour_start.size() - 1;
  info->device_bytes = s->ar.bytes;
  return VEMG_OK;
}

vemg_status vemg_footprint(vemg_solver s, int nrhs, size_t *bytes) {
  if (!s || !bytes || nrhs < 0) return VEMG_ERR_INVALID_ARG;
  if (!s->ready) return VEMG_ERR_STATE;
  *bytes = s->footprint + (size_t)2 * (size_t)nrhs * (size_t)s->P.n_nodes * sizeof(double);
  return VEMG_OK;
}

vemg_status vemg_export(vemg_solver s, const char *name, void *buf, size_t *bytes) {
  if (!s || !name || !bytes) return VEMG_ERR_INVALID_ARG;
  if (!s->ready) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_export(s, name, buf, bytes); });
}

vemg_status vemg_destroy(vemg_solver s) {
  if (!s) return VEMG_ERR_INVALID_ARG;
  if (s->device >= 0) {
    (void)hipSetDevice(s->device);
    if (s->work) (void)hipStreamSynchronize(s->work);
    if (s->work2) (void)hipStreamSynchronize(s->work2);
    vemg::destroy_graphs(s);
    s->ar.release();
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->ev_res) (void)hipEventDestroy(s->ev_res);
    if (s->own_streams && s->work) (void)hipStreamDestroy(s->work);
    if (s->own_streams && s->work2) (void)hipStreamDestroy(s->work2);
  }
  delete s;
  return VEMG_OK;
}

const char *vemg_status_string(vemg_status st) {
  switch (st) {
    case VEMG_OK: return "ok";
    case VEMG_WARN_MAXITER: return "maximum iteration count reached";
    case VEMG_WARN_FLOOR: return "true residual stalled above the tolerance";
    case VEMG_ERR_INVALID_ARG: return "invalid argument";
    case VEMG_ERR_MESH: return "invalid mesh";
    case VEMG_ERR_PROJECTION: return "node does not project onto the top surface";
    case VEMG_ERR_OOM: return "out of memory";
    case VEMG_ERR_DEVICE: return "device error";
    case VEMG_ERR_BREAKDOWN: return "CG breakdown (p.Ap <= 0 or not finite)";
    case VEMG_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

const char *vemg_last_error(vemg_solver s) { return s ? s->err.c_str() : ""; }


vemg_status vemg_server_create(int device, size_t hbm_budget, const vemg_options *o, vemg_server *out) {
  if (!out || device < 0) return VEMG_ERR_INVALID_ARG;
  *out = nullptr;
  vemg_options opt;
  if (o)
    opt = *o;
  else
    vemg_default_options(&opt);
  if (!vemg::valid_options(opt)) return VEMG_ERR_INVALID_ARG;
  auto *sv = new (std::nothrow) vemg_server_s();
  if (!sv) return VEMG_ERR_OOM;
  sv->opt = opt;
  if (sv->opt.precision == VEMG_MIXED_IR) sv->opt.precision = VEMG_MIXED_PC;
  sv->device = device;
  sv->budget = hbm_budget;
  hipError_t e = hipSetDevice(device);
  for (int i = 0; e == hipSuccess && i < 2 * vemg::kServerStreamPairs; ++i)
    e = vemg::create_queue_stream(device, &sv->streams[i]);
  if (e != hipSuccess) {
    (void)vemg_server_destroy(sv);
    return e == hipErrorOutOfMemory ? VEMG_ERR_OOM : VEMG_ERR_DEVICE;
  }
  *out = sv;
  return VEMG_OK;
}

vemg_status vemg_server_add_mesh(vemg_server sv, int64_t n_nodes, const double *xyz, int64_t n_tets,
                                 const int64_t *tets, const uint8_t *top_mask, int *mesh_id) {
  if (!sv || !mesh_id) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->started) {
    sv->err = "meshes must be added before the first submit";
    return VEMG_ERR_STATE;
  }
  const int lane = (int)sv->lanes.size();
  const hipStream_t *pair = &sv->streams[2 * (lane % vemg::kServerStreamPairs)];
  vemg_solver h = nullptr;
  vemg_status st = vemg::create_handle(&sv->opt, sv->device, nullptr, pair, &h);
  if (st != VEMG_OK) return st;
  // a mesh that alone exceeds the budget is refused before its upload
  auto L = std::make_unique<vemg::Lane>();
  L->h = h;
  int gst = guarded(h, [&]() -> int {
    h->device = -1;  // host setup only: the footprint is counted, nothing uploaded yet
    vemg_status s2 = vemg_setup(h, n_nodes, xyz, n_tets, tets, top_mask);
    h->device = sv->device;
    if (s2 != VEMG_OK) return s2;
    HIPCHK(hipSetDevice(sv->device));
    L->footprint = h->footprint;
    if (sv->budget && L->footprint > sv->budget) {
      h->err = "mesh needs more device memory than the budget";
      return VEMG_ERR_OOM;
    }
    HIPCHK(hipHostMalloc((void **)&L->scal_host, sizeof(vemg::Scal), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&L->scal_ready, hipEventDisableTiming));
    if (sv->budget && sv->used + L->footprint > sv->budget) return VEMG_OK;  // uploaded when needed
    vemg::upload(h);
    if (h->ar.bytes != L->footprint)
      throw vemg::DeviceError(VEMG_ERR_DEVICE, "device allocations differ from the counted footprint");
    // capture both iteration graphs now, while no other thread uses the device
    if (h->opt.use_graphs) {
      vemg::iteration_graphs<double>(h, vemg::kMaxBatch, vemg::kGraphFP64);
      vemg::iteration_graphs<double>(h, vemg::kMaxBatch, vemg::kGraphMixedPC);
      HIPCHK(hipStreamSynchronize(h->work));
    }
    L->resident = true;
    sv->used += L->footprint;
    sv->uploads++;
    return VEMG_OK;
  });
  h->allow_capture = false;
  if (gst != VEMG_OK) {
    sv->err = h->err;
    if (L->scal_host) (void)hipHostFree(L->scal_host);
    if (L->scal_ready) (void)hipEventDestroy(L->scal_ready);
    vemg_destroy(h);
    return (vemg_status)gst;
  }
  *mesh_id = lane;
  sv->lanes.push_back(std::move(L));
  return VEMG_OK;
}

vemg_status vemg_server_rhs(vemg_server sv, int mesh_id, const double *f_host, double *b_host) {
  if (!sv) return VEMG_ERR_INVALID_ARG;
  vemg_solver h;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (mesh_id < 0 || mesh_id >= (int)sv->lanes.size()) return VEMG_ERR_INVALID_ARG;
    h = sv->lanes[mesh_id]->h;
  }
  return vemg_rhs(h, f_host, b_host);  // host arithmetic on the immutable host setup
}

vemg_status vemg_server_footprint(vemg_server sv, int mesh_id, int nrhs, size_t *bytes) {
  if (!sv) return VEMG_ERR_INVALID_ARG;
  vemg_solver h;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (mesh_id < 0 || mesh_id >= (int)sv->lanes.size()) return VEMG_ERR_INVALID_ARG;
    h = sv->lanes[mesh_id]->h;
  }
  return vemg_footprint(h, nrhs, bytes);  // reads the footprint fixed at setup
}

vemg_status vemg_server_submit(vemg_server sv, int mesh_id, int nrhs, const double *b_dev, double *x_dev, double rtol,
                               int max_iter, uint64_t *req_id) {
  if (!sv || !b_dev || !x_dev || nrhs < 1 || !(rtol >= 0.0) || max_iter < 1) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (mesh_id < 0 || mesh_id >= (int)sv->lanes.size()) return VEMG_ERR_INVALID_ARG;
  if (sv->stop) return VEMG_ERR_STATE;
  if (!sv->started) {
    sv->started = true;
    sv->worker = std::thread(vemg::server_loop, sv);
  }
  auto q = std::make_unique<vemg::SReq>();
  q->id = sv->next_id++;
  q->mesh = mesh_id;
  q->nrhs = nrhs;
  q->b = b_dev;
  q->x = x_dev;
  q->rtol = rtol;
  q->max_iter = std::min(max_iter, 1 << 20);
  q->t_submit = vemg::now_s();
  q->cols_left = nrhs;
  q->iters.assign(nrhs, 0);
  q->rel.assign(nrhs, 0.0);
  if (sv->first_submit < 0) sv->first_submit = q->t_submit;
  if (req_id) *req_id = q->id;
  sv->by_id[q->id] = q.get();
  sv->incoming.push_back(q.get());
  sv->reqs.push_back(std::move(q));
  sv->cv.notify_all();
  return VEMG_OK;
}

vemg_status vemg_server_poll(vemg_server sv, uint64_t *done_ids, int cap, int *n_done) {
  if (!sv || !n_done || (cap > 0 && !done_ids)) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  int k = 0;
  while (k < cap && !sv->completed.empty()) {
    done_ids[k++] = sv->completed.front()->id;
    sv->completed.pop_front();
  }
  *n_done = k;
  return sv->err.empty() ? VEMG_OK : VEMG_ERR_DEVICE;
}

vemg_status vemg_server_wait(vemg_server sv, uint64_t req_id, double timeout_s) {
  if (!sv) return VEMG_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->by_id.find(req_id);
  if (it == sv->by_id.end()) return VEMG_ERR_INVALID_ARG;
  vemg::SReq *q = it->second;
  auto pred = [&]() { return q->done; };
  if (timeout_s > 0) {
    if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return VEMG_ERR_STATE;
  } else {
    sv->cv_done.wait(lk, pred);
  }
  return sv->err.empty() ? VEMG_OK : VEMG_ERR_DEVICE;
}

vemg_status vemg_server_result(vemg_server sv, uint64_t req_id, int *status, int *iters, double *relres,
                               double *latency_ms) {
  if (!sv) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->by_id.find(req_id);
  if (it == sv->by_id.end()) return VEMG_ERR_INVALID_ARG;
  const vemg::SReq &q = *it->second;
  if (!q.done) return VEMG_ERR_STATE;
  if (status) *status = q.status;
  for (int c = 0; c < q.nrhs; ++c) {
    if (iters) iters[c] = q.iters[c];
    if (relres) relres[c] = q.rel[c];
  }
  if (latency_ms) *latency_ms = 1e3 * (q.t_done - q.t_submit);
  return VEMG_OK;
}

vemg_status vemg_server_get_stats(vemg_server sv, vemg_server_stats *st) {
  if (!sv || !st) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(st, 0, sizeof(*st));
  std::vector<double> lat;
  int64_t pending = 0;
  for (size_t i = (size_t)sv->reqs_base; i < sv->reqs.size(); ++i) {
    if (sv->reqs[i]->done) lat.push_back(1e3 * (sv->reqs[i]->t_done - sv->reqs[i]->t_submit));
    else ++pending;
  }
  std::sort(lat.begin(), lat.end());
  st->requests_done = (int64_t)lat.size();
  st->requests_queued = pending;
  st->columns_done = sv->cols_done;
  if (!lat.empty()) {
    auto pct = [&](double p) {
      double pos = p * (double)(lat.size() - 1);
      size_t i = (size_t)pos;
      double f = pos - (double)i;
      return i + 1 < lat.size() ? lat[i] * (1.0 - f) + lat[i + 1] * f : lat[i];
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    double sum = 0.0;
    for (double v : lat) sum += v;
    st->mean_ms = sum / (double)lat.size();
    st->max_ms = lat.back();
  }
  if (sv->last_done > sv->first_submit && sv->first_submit >= 0) {
    st->busy_s = sv->last_done - sv->first_submit;
    st->solves_per_s = (double)st->columns_done / st->busy_s;
  }
  const int64_t chunks = sv->chunks;
  st->mean_slot_occupancy = chunks ? (double)sv->active_slots / (double)(chunks * vemg::kMaxBatch) : 0.0;
  st->chunks = chunks;
  st->uploads = sv->uploads;
  st->evictions = sv->evictions;
  st->resident_bytes = sv->used;
  st->budget_bytes = sv->budget;
  return VEMG_OK;
}

vemg_status vemg_server_set_precision(vemg_server sv, int precision) {
  if (!sv || precision < 0 || precision > 2) return VEMG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (!sv->incoming.empty()) return VEMG_ERR_STATE;
  for (auto &q : sv->reqs)
    if (!q->done) return VEMG_ERR_STATE;
  // every request is done: the scheduler holds no slot and applies the new
  // precision to a lane before its next chunk
  sv->opt.precision = precision == VEMG_MIXED_IR ? VEMG_MIXED_PC : precision;
  sv->first_submit = sv->last_done = -1.0;
  sv->chunks = 0;
  sv->cols_done = 0;
  sv->active_slots = 0;
  for (auto &q : sv->reqs) q->t_done = q->t_submit = 0.0;
  sv->reqs_base = (int64_t)sv->reqs.size();
  return VEMG_OK;
}

vemg_status vemg_server_destroy(vemg_server sv) {
  if (!sv) return VEMG_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  (void)hipSetDevice(sv->device);
  for (auto &L : sv->lanes) {
    vemg_destroy(L->h);
    if (L->scal_host) (void)hipHostFree(L->scal_host);
    if (L->scal_ready) (void)hipEventDestroy(L->scal_ready);
  }
  for (hipStream_t st : sv->streams)
    if (st) (void)hipStreamDestroy(st);
  delete sv;
  return VEMG_OK;
}

const char *vemg_server_last_error(vemg_server sv) { return sv ? sv->err.c_str() : ""; }

}  // extern "C"
