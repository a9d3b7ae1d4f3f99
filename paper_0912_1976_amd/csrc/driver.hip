// Solver handle: packs the host setup into SELL-64 arrays in HBM, runs the
// preconditioned CG loop on the device, and exposes the C ABI of vemg.h.
//
// The PCG iteration is a fixed sequence of kernels whose scalars (alpha,
// beta, the convergence flag) live in device memory, so one iteration can be
// captured in a hipGraph and replayed; every kernel returns at once when the
// convergence flag is set, so the host only polls the flag every few
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
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
      throw ::vemg::DeviceError(e_ == hipErrorOutOfMemory ? VEMG_ERR_OOM : VEMG_ERR_DEVICE,               \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                       \
  } while (0)

// device allocations owned by a handle
struct Arena {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  template <class T>
  T *alloc(size_t count) {
    if (count == 0) count = 1;
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, count * sizeof(T)));
    ptrs.push_back(p);
    bytes += count * sizeof(T);
    return (T *)p;
  }
  template <class T>
  T *upload(const std::vector<T> &v, hipStream_t st) {
    T *p = alloc<T>(v.size());
    if (!v.empty()) {
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

// CSR (host) -> SELL-64 (device).  For a square matrix the diagonal entries
// are taken out of the stored entries: they become the per-row term `d`
// (standard form), unless `d` is given (difference form: d = deficit).
Sell pack_sell(Arena &ar, hipStream_t st, const Csr &A, bool square, const std::vector<double> *d,
               int64_t *stored = nullptr) {
  int64_t n = A.nrows, ns = (n + kWave - 1) / kWave;
  std::vector<int64_t> sptr(ns + 1, 0);
  auto offdiag_len = [&](int64_t r) {
    int64_t c = 0;
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
      if (!(square && A.idx[k] == r)) ++c;
    return c;
  };
  std::vector<int64_t> len(n);
  for (int64_t r = 0; r < n; ++r) len[r] = offdiag_len(r);
  for (int64_t s = 0; s < ns; ++s) {
    int64_t L = 0;
    for (int64_t r = s * kWave; r < std::min(n, (s + 1) * kWave); ++r) L = std::max(L, len[r]);
    sptr[s + 1] = sptr[s] + L * kWave;
  }
  std::vector<int32_t> col(sptr[ns]);
  std::vector<double> val(sptr[ns], 0.0);
  std::vector<double> dv(square ? n : 0, 0.0);
  for (int64_t s = 0; s < ns; ++s) {
    int64_t L = (sptr[s + 1] - sptr[s]) / kWave;
    for (int t = 0; t < kWave; ++t) {
      int64_t r = s * kWave + t;
      int64_t k = 0;
      if (r < n) {
        for (int64_t e = A.ptr[r]; e < A.ptr[r + 1]; ++e) {
          if (square && A.idx[e] == r) {
            if (!d) dv[r] = A.val[e];
            continue;
          }
          col[sptr[s] + k * kWave + t] = A.idx[e];
          val[sptr[s] + k * kWave + t] = A.val[e];
          ++k;
        }
      }
      for (; k < L; ++k) {
        col[sptr[s] + k * kWave + t] = (square && r < n) ? (int32_t)r : 0;
        val[sptr[s] + k * kWave + t] = 0.0;
      }
    }
  }
  if (square && d) dv = *d;
  if (stored) *stored = sptr[ns];
  Sell M;
  M.nrows = n;
  M.sptr = ar.upload(sptr, st);
  M.col = ar.upload(col, st);
  M.val = ar.upload(val, st);
  if (square) M.d = ar.upload(dv, st);
  return M;
}

// CSR (host) -> CsrG (device).  Square matrices keep only off-diagonals and
// move the diagonal into `d`.  G = smallest power of two >= half the mean
// row length, clamped to [4, 64].
CsrG pack_csrg(Arena &ar, hipStream_t st, const Csr &A, bool square, int64_t *stored = nullptr) {
  std::vector<int32_t> ptr(A.nrows + 1, 0), col;
  std::vector<double> val, d(square ? A.nrows : 0, 0.0);
  col.reserve(A.nnz());
  val.reserve(A.nnz());
  for (int64_t r = 0; r < A.nrows; ++r) {
    for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      if (square && A.idx[k] == r) {
        d[r] = A.val[k];
        continue;
      }
      col.push_back(A.idx[k]);
      val.push_back(A.val[k]);
    }
    ptr[r + 1] = (int32_t)col.size();
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
  M.val = ar.upload(val, st);
  if (square) M.d = ar.upload(d, st);
  return M;
}

struct DLevel {
  Sell As;                      // fine A_bar level: rows [row0, row0 + n) of the fine SELL matrix
  CsrG Ac;                      // coarse levels: standard form, G lanes per row
  bool fine = false;
  int64_t n = 0, row0 = 0;
  std::vector<int64_t> cstart;  // colour ranges, global row indices
  CsrG P, Pt;                   // prolongation (n x n_next) and restriction
  double *Cinv = nullptr;       // coarsest level only
  double *x = nullptr, *g = nullptr, *r = nullptr;  // indexed by global row
  bool coarsest = false;
};

}  // namespace
}  // namespace vemg

struct vemg_solver_s {
  vemg_options opt;
  int device = -1;
  hipStream_t user = nullptr, work = nullptr;
  hipEvent_t ev = nullptr;
  std::string err;
  bool ready = false;
  vemg::Problem P;
  vemg::Arena ar;
  vemg::Sell A;                           // fine A_UU, difference form
  vemg::Sell E;
  vemg::CsrG Et;
  std::vector<vemg::DLevel> S, Ab;
  hipStream_t work2 = nullptr;            // surface branch of the additive preconditioner
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr, *w = nullptr,
         *res = nullptr, *resA = nullptr, *diag = nullptr, *tmp = nullptr, *nat = nullptr;
  double *part_pq = nullptr, *part_rr = nullptr, *part_rz = nullptr, *part_b = nullptr, *part_t = nullptr,
         *hist = nullptr, *dscal = nullptr;
  int64_t *perm = nullptr;
  vemg::Scal *scal = nullptr;
  int64_t np_pq = 0, np_rr = 0, np_rz = 0, np_vec = 0;
  int64_t nnz_A = 0, nnz_E = 0;
  std::vector<int64_t> s_nnz, ab_nnz, s_pnnz, ab_pnnz;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  int max_hist = 0;
};

namespace vemg {
namespace {

using Handle = vemg_solver_s;

void build_levels(Handle *h, std::vector<Level> &H, std::vector<DLevel> &D, bool is_abar,
                  std::vector<int64_t> &nnz, std::vector<int64_t> &pnnz) {
  hipStream_t st = h->work;
  D.clear();
  nnz.clear();
  pnnz.clear();
  for (size_t l = 0; l < H.size(); ++l) {
    Level &L = H[l];
    DLevel dl;
    dl.n = L.n();
    dl.coarsest = (l + 1 == H.size());
    if (is_abar && l == 0) {
      dl.fine = true;
      dl.As = h->A;
      dl.row0 = h->P.n_top;
      dl.cstart = h->P.bar_colour_start;  // already global
      dl.x = h->w;
      dl.g = h->r;
      dl.r = h->resA;
      nnz.push_back(h->nnz_A);
    } else {
      int64_t st_nnz = 0;
      dl.Ac = pack_csrg(h->ar, st, L.A, true, &st_nnz);
      nnz.push_back(st_nnz);
      dl.cstart = L.colour_start;
      dl.x = h->ar.alloc<double>(dl.n);
      dl.g = h->ar.alloc<double>(dl.n);
      dl.r = h->ar.alloc<double>(dl.n);
    }
    if (!dl.coarsest) {
      int64_t pn = 0;
      dl.P = pack_csrg(h->ar, st, L.P, false, &pn);
      dl.Pt = pack_csrg(h->ar, st, transpose(L.P), false);
      pnnz.push_back(pn);
    } else {
      dl.Cinv = h->ar.upload(L.Cinv, st);
    }
    D.push_back(dl);
  }
}

void vcycle(hipStream_t st, std::vector<DLevel> &H, size_t l, const int *done) {
  DLevel &L = H[l];
  if (L.coarsest) {
    launch_dense(st, L.Cinv, L.n, L.g + L.row0, L.x + L.row0, done);
    return;
  }
  launch_fill(st, L.x + L.row0, L.n, 0.0, done);
  int nc = (int)L.cstart.size() - 1;
  auto gs = [&](int c) {
    if (L.fine)
      launch_gs(st, L.As, true, L.cstart[c], L.cstart[c + 1], 0, 0, L.g, L.x, done);
    else
      launch_csr_gs(st, L.Ac, L.cstart[c], L.cstart[c + 1], L.g, L.x, done);
  };
  for (int c = 0; c < nc; ++c) gs(c);
  if (L.fine)
    launch_spmv(st, L.As, true, 1, L.row0, L.row0 + L.n, L.x, L.g, L.r, nullptr, done);
  else
    launch_csr_spmv(st, L.Ac, 1, 0, L.n, L.x, L.g, L.r, done);
  DLevel &C = H[l + 1];
  launch_csr_rect(st, L.Pt, false, L.r + L.row0, C.g, done);
  vcycle(st, H, l + 1, done);
  launch_csr_rect(st, L.P, true, C.x, L.x + L.row0, done);
  for (int c = nc - 1; c >= 0; --c) gs(c);
}

// z = M^{-1} rr; partial sums of rr . z go to part_rz (count in np_rz)
void precond(Handle *h, const double *rr, double *zz, const int *done) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  switch (h->opt.pc) {
    case VEMG_PC_VL_ADDITIVE: {
      // the two terms of the additive preconditioner are independent: the
      // surface branch runs on a second stream (a parallel graph branch)
      if (m > 0) {
        HIPCHK(hipEventRecord(h->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(h->work2, h->ev_fork, 0));
        launch_csr_rect(h->work2, h->Et, false, rr, h->S[0].g, done);
        vcycle(h->work2, h->S, 0, done);
        HIPCHK(hipEventRecord(h->ev_join, h->work2));
      }
      h->Ab[0].g = const_cast<double *>(rr);
      vcycle(st, h->Ab, 0, done);
      h->Ab[0].g = h->r;
      if (m > 0) HIPCHK(hipStreamWaitEvent(st, h->ev_join, 0));
      if (m > 0) {
        launch_prolong_sum(st, h->E, m, h->S[0].x, h->w, rr, zz, h->part_rz, done);
      } else {
        launch_copy(st, h->w, zz, n, done);
        launch_dot(st, rr, zz, n, h->part_rz, done);
      }
      break;
    }
    case VEMG_PC_VL_SOR: {
      launch_fill(st, zz, n, 0.0, done);
      int nct = (int)P.top_colour_start.size() - 1, ncb = (int)P.bar_colour_start.size() - 1;
      int nc = std::max(nct, ncb);
      auto sweep = [&](int c) {
        int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (c < nct) {
          a0 = P.top_colour_start[c];
          a1 = P.top_colour_start[c + 1];
        }
        if (c < ncb) {
          b0 = P.bar_colour_start[c];
          b1 = P.bar_colour_start[c + 1];
        }
        launch_gs(st, h->A, true, a0, a1, b0, b1, rr, zz, done);
      };
      for (int c = 0; c < nc; ++c) sweep(c);
      if (m > 0) {
        launch_spmv(st, h->A, true, 1, 0, n, zz, rr, h->res, nullptr, done);
        launch_csr_rect(st, h->Et, false, h->res, h->S[0].g, done);
        vcycle(st, h->S, 0, done);
        launch_rect(st, h->E, true, h->S[0].x, zz, done);
      }
      for (int c = nc - 1; c >= 0; --c) sweep(c);
      launch_dot(st, rr, zz, n, h->part_rz, done);
      break;
    }
    case VEMG_PC_JACOBI:
      launch_jacobi(st, rr, h->diag, zz, n, done);
      launch_dot(st, rr, zz, n, h->part_rz, done);
      break;
    default:
      launch_copy(st, rr, zz, n, done);
      launch_dot(st, rr, zz, n, h->part_rz, done);
      break;
  }
}

int64_t rz_partials(Handle *h) {
  if (h->opt.pc == VEMG_PC_VL_ADDITIVE && h->P.n_top > 0) return sell_blocks(0, h->P.n);
  return vec_blocks(h->P.n);
}

void pcg_iteration(Handle *h) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  const int *done = &h->scal->done;
  launch_spmv(st, h->A, true, 0, 0, n, h->p, nullptr, h->q, h->part_pq, done);
  launch_pcg_alpha(st, h->scal, h->part_pq, h->np_pq);
  launch_pcg_xr(st, h->scal, h->x, h->r, h->p, h->q, n, h->part_rr);
  launch_pcg_conv(st, h->scal, h->part_rr, h->np_vec, h->hist);
  precond(h, h->r, h->z, done);
  launch_pcg_beta(st, h->scal, h->part_rz, h->np_rz);
  launch_pcg_p(st, h->scal, h->p, h->z, n);
}

void upload(Handle *h) {
  hipStream_t st = h->work;
  Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  h->ar.release();
  h->A = pack_sell(h->ar, st, P.Aoff, true, &P.d, &h->nnz_A);
  if (m > 0) {
    h->E = pack_sell(h->ar, st, P.E, false, nullptr, &h->nnz_E);
    h->Et = pack_csrg(h->ar, st, P.Et, false);
  }
  h->x = h->ar.alloc<double>(n);
  h->r = h->ar.alloc<double>(n);
  h->z = h->ar.alloc<double>(n);
  h->p = h->ar.alloc<double>(n);
  h->q = h->ar.alloc<double>(n);
  h->b = h->ar.alloc<double>(n);
  h->w = h->ar.alloc<double>(n);
  h->res = h->ar.alloc<double>(n);
  h->resA = h->ar.alloc<double>(n);
  h->tmp = h->ar.alloc<double>(n);
  h->nat = h->ar.alloc<double>(P.n_nodes);
  h->diag = h->ar.upload(P.diag, st);
  h->perm = h->ar.upload(P.perm, st);
  int64_t npmax = std::max(sell_blocks(0, n), vec_blocks(n)) + 8;
  h->part_pq = h->ar.alloc<double>(npmax);
  h->part_rr = h->ar.alloc<double>(npmax);
  h->part_rz = h->ar.alloc<double>(npmax);
  h->part_b = h->ar.alloc<double>(npmax);
  h->part_t = h->ar.alloc<double>(npmax);
  h->dscal = h->ar.alloc<double>(8);
  h->max_hist = 1 << 16;
  h->hist = h->ar.alloc<double>(h->max_hist + 1);
  h->scal = h->ar.alloc<Scal>(1);
  launch_fill(st, h->w, n, 0.0, nullptr);  // the top block of w stays zero
  if (m > 0) build_levels(h, P.S, h->S, false, h->s_nnz, h->s_pnnz);
  build_levels(h, P.Abar, h->Ab, true, h->ab_nnz, h->ab_pnnz);
  h->np_pq = sell_blocks(0, n);
  h->np_vec = vec_blocks(n);
  h->np_rz = rz_partials(h);
  HIPCHK(hipStreamSynchronize(st));
}

void destroy_graph(Handle *h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->graph_def) (void)hipGraphDestroy(h->graph_def);
  h->graph = nullptr;
  h->graph_def = nullptr;
}

void ensure_graph(Handle *h) {
  if (h->graph || !h->opt.use_graphs) return;
  HIPCHK(hipStreamBeginCapture(h->work, hipStreamCaptureModeThreadLocal));
  pcg_iteration(h);
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamEndCapture(h->work, &g));
  h->graph_def = g;
  HIPCHK(hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0));
}

void sync_in(Handle *h) {
  HIPCHK(hipEventRecord(h->ev, h->user));
  HIPCHK(hipStreamWaitEvent(h->work, h->ev, 0));
}

double true_residual(Handle *h) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  launch_spmv(st, h->A, true, 1, 0, n, h->x, h->b, h->res, nullptr, nullptr);
  launch_dot(st, h->res, h->res, n, h->part_t, nullptr);
  launch_reduce(st, h->part_t, vec_blocks(n), h->dscal);
  double rr = 0.0;
  HIPCHK(hipMemcpyAsync(&rr, h->dscal, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return rr;
}

// one right-hand side, storage-order vectors already in h->b
int solve_one(Handle *h, double rtol, int max_iter, int *iters_out, double *relres_out) {
  hipStream_t st = h->work;
  int64_t n = h->P.n;
  // ||b||
  launch_dot(st, h->b, h->b, n, h->part_b, nullptr);
  launch_pcg_init(st, h->scal, h->part_b, vec_blocks(n), rtol, max_iter);
  Scal hs;
  HIPCHK(hipMemcpyAsync(&hs, h->scal, sizeof(Scal), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  launch_fill(st, h->x, n, 0.0, nullptr);
  if (hs.bnorm2 == 0.0) {
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    return VEMG_OK;
  }
  if (!std::isfinite(hs.bnorm2)) {
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = NAN;
    return VEMG_ERR_BREAKDOWN;
  }
  double bnorm = std::sqrt(hs.bnorm2);
  launch_copy(st, h->b, h->r, n, nullptr);
  double prev = INFINITY;
  int restarts = 0;
  int status = VEMG_OK;
  double rel = 1.0;
  while (true) {
    // (re)start: z = M r, rho = r.z, p = z
    launch_pcg_resume(st, h->scal);
    precond(h, h->r, h->z, nullptr);
    launch_pcg_set_rho(st, h->scal, h->part_rz, h->np_rz);
    launch_copy(st, h->z, h->p, n, nullptr);
    ensure_graph(h);
    int poll = std::max(1, h->opt.poll_every);
    while (true) {
      for (int k = 0; k < poll; ++k) {
        if (h->graph)
          HIPCHK(hipGraphLaunch(h->graph, st));
        else
          pcg_iteration(h);
      }
      HIPCHK(hipMemcpyAsync(&hs, h->scal, sizeof(Scal), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hs.done) break;
    }
    if (hs.status == -6) {
      status = VEMG_ERR_BREAKDOWN;
      rel = NAN;
      break;
    }
    double rr = true_residual(h);
    rel = std::sqrt(rr) / bnorm;
    if (rel <= rtol) {
      status = VEMG_OK;
      break;
    }
    if (hs.iters >= max_iter) {
      status = VEMG_WARN_MAXITER;
      break;
    }
    if (restarts >= h->opt.max_restarts || rel > 0.5 * prev) {
      status = VEMG_WARN_FLOOR;
      break;
    }
    prev = rel;
    ++restarts;
    launch_copy(st, h->res, h->r, n, nullptr);
  }
  if (iters_out) *iters_out = hs.iters;
  if (relres_out) *relres_out = rel;
  return status;
}

int do_solve(Handle *h, int nrhs, const double *b_nat, double *x_nat, double rtol, int max_iter, int *iters,
             double *relres) {
  hipStream_t st = h->work;
  int64_t n = h->P.n, N = h->P.n_nodes;
  sync_in(h);
  int worst = VEMG_OK;
  for (int k = 0; k < nrhs; ++k) {
    launch_gather(st, b_nat + (int64_t)k * N, h->perm, h->b, n);
    int it = 0;
    double rl = 0.0;
    int s = solve_one(h, rtol, max_iter, &it, &rl);
    launch_fill(st, x_nat + (int64_t)k * N, N, 0.0, nullptr);
    launch_scatter(st, h->x, h->perm, x_nat + (int64_t)k * N, n);
    if (iters) iters[k] = it;
    if (relres) relres[k] = rl;
    if (s < 0 || (worst >= 0 && s > worst)) worst = s;
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

int do_apply(Handle *h, int op, const double *in, double *out) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n, m = P.n_top;
  sync_in(h);
  switch (op) {
    case VEMG_OP_A:
      launch_spmv(st, h->A, true, 0, 0, n, in, nullptr, out, nullptr, nullptr);
      break;
    case VEMG_OP_PRECOND:
      HIPCHK(hipMemsetAsync(h->scal, 0, sizeof(Scal), st));
      launch_copy(st, in, h->tmp, n, nullptr);
      precond(h, h->tmp, out, nullptr);
      break;
    case VEMG_OP_ET:
      if (m == 0) return VEMG_ERR_STATE;
      launch_csr_rect(st, h->Et, false, in, out, nullptr);
      break;
    case VEMG_OP_E:
      if (m == 0) return VEMG_ERR_STATE;
      launch_rect(st, h->E, false, in, out, nullptr);
      break;
    case VEMG_OP_VCYCLE_S:
      if (m == 0) return VEMG_ERR_STATE;
      launch_copy(st, in, h->S[0].g, m, nullptr);
      vcycle(st, h->S, 0, nullptr);
      launch_copy(st, h->S[0].x, out, m, nullptr);
      break;
    case VEMG_OP_VCYCLE_ABAR:
      launch_copy(st, in, h->tmp + m, n - m, nullptr);
      h->Ab[0].g = h->tmp;
      vcycle(st, h->Ab, 0, nullptr);
      h->Ab[0].g = h->r;
      launch_copy(st, h->w + m, out, n - m, nullptr);
      break;
    case VEMG_OP_GS_FWD: {
      launch_fill(st, out, n, 0.0, nullptr);
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
        launch_gs(st, h->A, true, a0, a1, b0, b1, in, out, nullptr);
      }
      break;
    }
    default:
      return VEMG_ERR_INVALID_ARG;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return VEMG_OK;
}

int do_time(Handle *h, int op, int reps, double *avg_ms, int *launches) {
  hipStream_t st = h->work;
  const Problem &P = h->P;
  int64_t n = P.n;
  int nct = (int)P.top_colour_start.size() - 1, ncb = (int)P.bar_colour_start.size() - 1;
  int nc = std::max(nct, ncb);
  launch_fill(st, h->p, n, 1.0, nullptr);
  launch_fill(st, h->r, n, 1.0, nullptr);
  auto once = [&]() {
    if (op == VEMG_OP_A) {
      launch_spmv(st, h->A, true, 0, 0, n, h->p, nullptr, h->q, h->part_pq, nullptr);
    } else {
      for (int c = 0; c < nc; ++c) {
        int64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
        if (c < nct) {
          a0 = P.top_colour_start[c];
          a1 = P.top_colour_start[c + 1];
        }
        if (c < ncb) {
          b0 = P.bar_colour_start[c];
          b1 = P.bar_colour_start[c + 1];
        }
        launch_gs(st, h->A, true, a0, a1, b0, b1, h->r, h->z, nullptr);
      }
    }
  };
  if (op != VEMG_OP_A && op != VEMG_OP_GS_FWD) return VEMG_ERR_INVALID_ARG;
  launch_fill(st, h->z, n, 0.0, nullptr);
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
  if (launches) *launches = (op == VEMG_OP_A) ? 1 : nc;
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
  if (head == "S" || head == "Abar") {
    const std::vector<Level> &H = head == "S" ? P.S : P.Abar;
    auto dot2 = rest.find('.');
    if (dot2 == std::string::npos) return VEMG_ERR_INVALID_ARG;
    size_t l = (size_t)std::stoul(rest.substr(0, dot2));
    std::string what = rest.substr(dot2 + 1);
    if (l >= H.size()) return VEMG_ERR_INVALID_ARG;
    const Level &L = H[l];
    if (what.rfind("A.", 0) == 0) return export_csr(L.A, what.substr(2), buf, bytes);
    if (what.rfind("P.", 0) == 0) return export_csr(L.P, what.substr(2), buf, bytes);
    if (what == "colour") return export_vec(L.colour, buf, bytes);
    if (what == "node") return export_vec(L.node, buf, bytes);
    if (what == "agg") return export_vec(L.agg, buf, bytes);
    if (what == "Cinv") return export_vec(L.Cinv, buf, bytes);
  }
  return VEMG_ERR_INVALID_ARG;
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
  o->coarse_max = 2048;
  o->poll_every = 8;
  o->max_restarts = 5;
  o->use_graphs = 1;
}

vemg_status vemg_create(const vemg_options *o, int device, void *hip_stream, vemg_solver *out) {
  if (!out) return VEMG_ERR_INVALID_ARG;
  *out = nullptr;
  vemg_options opt;
  if (o)
    opt = *o;
  else
    vemg_default_options(&opt);
  if (opt.top_bc < 0 || opt.top_bc > 1 || opt.pc < 0 || opt.pc > 3 || opt.max_levels < 1 || opt.max_levels > 16 ||
      opt.coarse_max < 1 || opt.coarse_max > 8192 || !(opt.theta >= 0.0) || opt.poll_every < 1)
    return VEMG_ERR_INVALID_ARG;
  auto *h = new (std::nothrow) vemg_solver_s();
  if (!h) return VEMG_ERR_OOM;
  h->opt = opt;
  h->device = device;
  h->user = (hipStream_t)hip_stream;
  int st = guarded(h, [&]() -> int {
    if (device >= 0) {
      HIPCHK(hipStreamCreate(&h->work));
      HIPCHK(hipStreamCreate(&h->work2));
      HIPCHK(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    return VEMG_OK;
  });
  if (st != VEMG_OK) {
    delete h;
    return (vemg_status)st;
  }
  *out = h;
  return VEMG_OK;
}

vemg_status vemg_setup(vemg_solver s, int64_t n_nodes, const double *xyz, int64_t n_tets, const int64_t *tets,
                       const uint8_t *top_mask) {
  if (!s) return VEMG_ERR_INVALID_ARG;
  return (vemg_status)guarded(s, [&]() -> int {
    s->ready = false;
    vemg::destroy_graph(s);
    s->ar.release();
    vemg::SetupOptions so;
    so.top_dirichlet = s->opt.top_bc;
    so.pin_node = s->opt.pin_node;
    so.theta = s->opt.theta;
    so.prolong_omega = s->opt.prolong_omega;
    so.max_levels = s->opt.max_levels;
    so.coarse_max = s->opt.coarse_max;
    s->P = vemg::Problem();
    vemg::build_problem(s->P, so, n_nodes, xyz, n_tets, tets, top_mask);
    if (s->device >= 0) vemg::upload(s);
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
    vemg::launch_gather(st, x_dev, s->perm, s->tmp, n);
    vemg::launch_spmv(st, s->A, true, 0, 0, n, s->tmp, nullptr, s->res, nullptr, nullptr);
    vemg::launch_fill(st, y_dev, s->P.n_nodes, 0.0, nullptr);
    vemg::launch_scatter(st, s->res, s->perm, y_dev, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return VEMG_OK;
  });
}

vemg_status vemg_solve(vemg_solver s, int nrhs, const double *b_dev, double *x_dev, double rtol, int max_iter,
                       int *iters, double *relres) {
  if (!s || !b_dev || !x_dev || nrhs < 1 || !(rtol >= 0.0) || max_iter < 1) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  if (max_iter > s->max_hist) max_iter = s->max_hist;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_solve(s, nrhs, b_dev, x_dev, rtol, max_iter, iters, relres); });
}

vemg_status vemg_apply(vemg_solver s, int op, const double *in_dev, double *out_dev) {
  if (!s || !in_dev || !out_dev) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_apply(s, op, in_dev, out_dev); });
}

vemg_status vemg_time_op(vemg_solver s, int op, int reps, double *avg_ms, int *launches) {
  if (!s || !avg_ms || reps < 1) return VEMG_ERR_INVALID_ARG;
  if (!s->ready || s->device < 0) return VEMG_ERR_STATE;
  return (vemg_status)guarded(s, [&]() -> int { return vemg::do_time(s, op, reps, avg_ms, launches); });
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
    vemg::destroy_graph(s);
    s->ar.release();
    if (s->work2) (void)hipStreamSynchronize(s->work2);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->work) (void)hipStreamDestroy(s->work);
    if (s->work2) (void)hipStreamDestroy(s->work2);
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

}  // extern "C"
