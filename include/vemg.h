/*
 * vemg.h -- C ABI of the vertical-extrapolation multigrid PCG solver for the
 * P1 finite-element Poisson equation on thin (small aspect ratio)
 * tetrahedral domains, after Kramer, Cotter & Pain, "Solving the Poisson
 * equation on small aspect ratio domains using unstructured meshes".
 *
 * Problem (Section 3): -Lap(phi) = f on Omega with homogeneous Neumann
 * conditions on the floor and the vertical coasts, and on the top surface
 * either
 *   VEMG_TOP_PINNED     Neumann plus the point condition phi(x_0) = 0 with
 *                       x_0 a top node (eq. point condition),
 *   VEMG_TOP_DIRICHLET  phi = 0 on the whole top surface (eq. dirichlet), or
 *   VEMG_TOP_ROBIN      the free-surface condition of Section 2 under
 *                       backward Euler, d phi/dn + alpha phi = 0 with
 *                       alpha = (n.k)/(g dt^2) > 0 (vemg_options.robin_alpha);
 *                       its weak form adds alpha times the P1 mass matrix of
 *                       the top triangles projected onto (x, y), and no node
 *                       is fixed.  Small alpha approaches the pinned
 *                       Neumann problem, large alpha the Dirichlet top.
 * The library assembles the P1 stiffness matrix A (eq. Ax=b), plus the
 * Robin term, restricted to the free nodes and solves A phi = b by
 * preconditioned conjugate gradients.
 *
 * Preconditioners (Section 6):
 *   VEMG_PC_VL_SOR       vertical lumping as the first coarsening of a
 *                        multigrid cycle: one forward multicolour SOR sweep
 *                        on A, the coarse correction E~ Vcyc_S(E~^T res)
 *                        with the vertical extrapolation E~ (Section 5.4)
 *                        and a smoothed aggregation V-cycle on the Galerkin
 *                        surface operator S = E~^T A E~, one backward sweep.
 *   VEMG_PC_VL_ADDITIVE  that cycle with the additive smoother included:
 *                        M^{-1} r = VL_SOR(r) + Z Vcyc_Abar(Z^T r), where
 *                        Vcyc_Abar is one SA V-cycle on the Dirichlet-top
 *                        block A_bar and Z = [0; I] (the combination run in
 *                        the experiments of Section 6).
 *   VEMG_PC_VL_ADDITIVE_ONLY  eq. ourpreconditioner on its own:
 *                        E~ Vcyc_S(E~^T r) + Z Vcyc_Abar(Z^T r), no SOR.
 *   VEMG_PC_SA           the paper's baseline (Section 6, first
 *                        preconditioner): one smoothed aggregation V-cycle
 *                        on the whole A, forward SOR before and backward SOR
 *                        after each coarse correction; its hierarchy is built
 *                        only when the handle is set up with this value.
 *   VEMG_PC_JACOBI, VEMG_PC_NONE  baselines.
 *
 * Conventions
 *   - Every call returns a vemg_status: 0 success, < 0 error, > 0 warning.
 *   - Vectors passed to solve/matvec are device pointers in the caller's
 *     natural node order, length n_nodes, FP64.  Entries of b at fixed nodes
 *     are ignored; x is returned as 0 there.
 *   - The library copies the mesh during setup; the caller may free it.
 *     It owns every device buffer it allocates; the caller owns b and x.
 *   - All device work is ordered on the stream given to vemg_create (the
 *     null stream if NULL); calls return after that work has finished.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef VEMG_H
#define VEMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vemg_solver_s *vemg_solver;

typedef enum {
  VEMG_OK = 0,
  VEMG_WARN_MAXITER = 1,      /* max_iter reached; x holds the last iterate */
  VEMG_WARN_FLOOR = 2,        /* true residual stalled above rtol (rounding floor) */
  VEMG_ERR_INVALID_ARG = -1,  /* null pointer, bad size or option */
  VEMG_ERR_MESH = -2,         /* inverted tetrahedron, node out of range, no top surface */
  VEMG_ERR_PROJECTION = -3,   /* a node does not project onto the top surface */
  VEMG_ERR_OOM = -4,          /* device or host allocation failed */
  VEMG_ERR_DEVICE = -5,       /* HIP runtime error */
  VEMG_ERR_BREAKDOWN = -6,    /* p.Ap <= 0 or not finite (e.g. NaN in b) */
  VEMG_ERR_STATE = -7         /* call out of order (e.g. solve before setup) */
} vemg_status;

typedef enum { VEMG_TOP_PINNED = 0, VEMG_TOP_DIRICHLET = 1, VEMG_TOP_ROBIN = 2 } vemg_top_bc;

typedef enum {
  VEMG_PC_VL_ADDITIVE = 0,
  VEMG_PC_VL_SOR = 1,
  VEMG_PC_JACOBI = 2,
  VEMG_PC_NONE = 3,
  VEMG_PC_VL_ADDITIVE_ONLY = 4,
  VEMG_PC_SA = 5
} vemg_pc;

/* Precision of the solve.
 *   VEMG_FP64        everything in FP64.
 *   VEMG_MIXED_IR    FP64 iterative refinement around an FP32 PCG that keeps
 *                    its Krylov space: the inner PCG (SpMV, transfers,
 *                    smoothers, vectors) runs in FP32 with per-row scaled
 *                    operators on A d = b / ||b||, its inner products
 *                    accumulated in FP64 and its coarsest solves in FP64;
 *                    every poll_every iterations its correction is added to
 *                    the FP64 solution and its residual replaced by the true
 *                    FP64 residual b - A x (reliable update), without
 *                    restarting the search directions.
 *   VEMG_MIXED_PC    FP64 CG (SpMV, vectors, inner products) whose
 *                    preconditioner (transfers, smoothers, V-cycles) runs in FP32. */
typedef enum { VEMG_FP64 = 0, VEMG_MIXED_IR = 1, VEMG_MIXED_PC = 2 } vemg_precision;

/* Extrapolation operator E~ = [I; F] of the surface branch (Section 5.4).
 *   VEMG_EXTRAP_PROJECTION  each node below the top takes the linear
 *                           interpolant of the surface triangle its vertical
 *                           projection lands in (at most three entries a row).
 *   VEMG_EXTRAP_SSPAI       the same pattern, F refitted from the operator
 *                           (the sparse approximate inverse alternative of
 *                           Section 5.4): column i of F solves the exact
 *                           extrapolation's column system A_bar f = -C^T e_i
 *                           restricted to its pattern, one dense Cholesky
 *                           solve per surface unknown at setup.  With
 *                           vertical columns it tends to the projection as
 *                           eps^2; on meshes with broken columns it loses the
 *                           constants and converges far more slowly at small
 *                           eps. */
typedef enum { VEMG_EXTRAP_PROJECTION = 0, VEMG_EXTRAP_SSPAI = 1 } vemg_extrapolation;

typedef struct {
  int top_bc;          /* vemg_top_bc */
  int64_t pin_node;    /* pinned top node (natural index); -1: top node closest to the origin */
  int pc;              /* vemg_pc */
  double theta;        /* strength threshold, 0.01 (Section 6) */
  double prolong_omega;/* prolongator smoothing, 2/3 (Section 6) */
  int max_levels;      /* per hierarchy, 10 */
  int64_t coarse_max;  /* unknowns on the coarsest level (solved exactly through an explicit
                          FP64 inverse), 8192 (at most 8192) */
  int poll_every;      /* PCG iterations per host poll of the convergence flag, 8 */
  int max_restarts;    /* restarts from the true residual, 5 */
  int use_graphs;      /* capture one PCG iteration in a hipGraph, 1 */
  int precision;       /* vemg_precision, VEMG_FP64 */
  double inner_rtol;   /* in (0, 1); not used by the solver (kept for the layout), 1e-4 */
  int max_outer;       /* >= 1; not used by the solver (kept for the layout), 30 */
  double robin_alpha;  /* VEMG_TOP_ROBIN: alpha > 0 (ignored otherwise), 0 */
  int extrapolation;   /* vemg_extrapolation, VEMG_EXTRAP_PROJECTION */
} vemg_options;

typedef struct {
  int64_t n_nodes;     /* mesh nodes */
  int64_t n;           /* free unknowns */
  int64_t n_top;       /* free top unknowns m' (0 with a Dirichlet top) */
  int64_t pin_node;    /* pinned node, -1 with a Dirichlet top */
  int64_t nnz_offdiag; /* stored off-diagonals of A */
  int s_levels, abar_levels;
  int64_t s_rows[16], abar_rows[16];     /* unknowns per level */
  int64_t s_nnz[16], abar_nnz[16];       /* stored entries per level (off-diagonal) */
  int64_t p_nnz_s[16], p_nnz_abar[16];   /* prolongator entries per level */
  int64_t e_nnz;       /* entries of E~ */
  int fine_colours_top, fine_colours_bar;
  size_t device_bytes; /* device memory held by the handle */
} vemg_info;

/* Fills o with the paper's parameters and the defaults above. */
void vemg_default_options(vemg_options *o);

/* Creates a handle on `device` (HIP ordinal; -1 = host-only setup, for
 * inspecting the setup without a GPU) using `hip_stream` (a hipStream_t, may
 * be NULL).  *out is NULL on error. */
vemg_status vemg_create(const vemg_options *o, int device, void *hip_stream, vemg_solver *out);

/* Setup (Sections 3, 5.4, 6): assembly of A on the free nodes, node order
 * (top block first, eq. phi_decomposition), colouring, E~, both SA
 * hierarchies, upload to HBM.  xyz: host [n_nodes][3]; tets: host
 * [n_tets][4], 0-based, positively oriented; top_mask: host [n_nodes],
 * nonzero for nodes on the top surface.  Errors: VEMG_ERR_MESH (first bad
 * tetrahedron in vemg_last_error), VEMG_ERR_PROJECTION, VEMG_ERR_INVALID_ARG. */
vemg_status vemg_setup(vemg_solver s, int64_t n_nodes, const double *xyz, int64_t n_tets,
                       const int64_t *tets, const uint8_t *top_mask);

/* Right-hand side of eq. Ax=b from nodal source values: b = M f with the
 * consistent P1 mass matrix; with the pinned top, b is first made
 * orthogonal to constants (the Neumann problem needs int f = 0).  Host
 * arrays, natural order, length n_nodes; fixed nodes get 0. */
vemg_status vemg_rhs(vemg_solver s, const double *f_host, double *b_host);

/* y = A x on the free nodes (difference form), device pointers, natural
 * order; y is 0 at fixed nodes. */
vemg_status vemg_matvec(vemg_solver s, const double *x_dev, double *y_dev);

/* vemg_matvec for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, with the two storage-order work vectors taken from a
 * static buffer of the library (32 MiB, held on every GPU the library runs on
 * until the process ends) instead of the handle, so the call itself
 * allocates nothing.  Limit: n (free unknowns, vemg_info.n) <= 2^21 =
 * 2,097,152; larger handles get VEMG_ERR_INVALID_ARG with the sizes in
 * vemg_last_error.  Every call on one GPU shares that GPU's buffer: calls
 * that overlap on one GPU (from several threads or handles) race.  Result
 * and errors otherwise as vemg_matvec. */
vemg_status vemg_matvec_noalloc(vemg_solver s, const double *x_dev, double *y_dev);

/* Solves A x = b for nrhs right-hand sides stored one after another
 * ([nrhs][n_nodes], device).  Right-hand sides are solved in batches of up
 * to 8 that share every matrix read (SpMM-style launches); each column
 * converges on its own.  PCG restarts from the true residual: each restart
 * solves for a correction from zero, and the solution is kept on the device
 * as an unevaluated sum hi + lo of two doubles into which every correction
 * is added without rounding error.  The true residual b - A (hi + lo) is
 * evaluated with error-free products and double-double sums, so the FP64
 * accuracy floor that grows with the condition number (Section 6) does not
 * stop the refinement.  Stops when ||b - A (hi + lo)||_2 <= rtol ||b||_2 or
 * after max_iter iterations (products with A; for VEMG_MIXED_IR the inner
 * FP32 iterations summed over refinement steps).  x receives hi + lo rounded
 * to FP64, which changes each residual entry by at most u (|A| |x|)_i,
 * u = 2^-53.  iters and relres (host, length nrhs, may be NULL) receive the
 * iteration count and that final relative residual of each right-hand side.
 * Returns the worst status: VEMG_WARN_MAXITER / VEMG_WARN_FLOOR with the
 * last iterate when rtol was not reached, VEMG_ERR_BREAKDOWN on p.Ap <= 0 or
 * NaN (that column only; the others are still solved). */
vemg_status vemg_solve(vemg_solver s, int nrhs, const double *b_dev, double *x_dev, double rtol,
                       int max_iter, int *iters, double *relres);

/* Operators of the hot path, for testing one step at a time.  Vectors are
 * device FP64 in the library's storage order (see vemg_export "perm"); with
 * a mixed-precision handle the operator runs in FP32 (input rounded to FP32,
 * output widened to FP64):
 *   VEMG_OP_A          out[n]  = A in[n]           (difference form)
 *   VEMG_OP_PRECOND    out[n]  = M^{-1} in[n]      (the handle's preconditioner)
 *   VEMG_OP_ET         out[m'] = E~^T in[n]
 *   VEMG_OP_E          out[n]  = E~ in[m']
 *   VEMG_OP_VCYCLE_S   out[m'] = Vcyc_S(in[m'])    (zero initial guess)
 *   VEMG_OP_VCYCLE_ABAR out[n-m'] = Vcyc_Abar(in[n-m'])
 *   VEMG_OP_GS_FWD     out[n]  = one forward multicolour SOR sweep on A x = in, x0 = 0 */
typedef enum {
  VEMG_OP_A = 0,
  VEMG_OP_PRECOND = 1,
  VEMG_OP_ET = 2,
  VEMG_OP_E = 3,
  VEMG_OP_VCYCLE_S = 4,
  VEMG_OP_VCYCLE_ABAR = 5,
  VEMG_OP_GS_FWD = 6,
  VEMG_OP_GS_COARSE = 7, /* vemg_time_op only: one forward sweep on the first coarse level of A_bar */
  VEMG_OP_COARSEST = 8   /* vemg_time_op only: the coarsest surface level's dense inverse times a vector */
} vemg_op;
vemg_status vemg_apply(vemg_solver s, int op, const double *in_dev, double *out_dev);

/* Benchmark support: average device time in milliseconds of one
 * application of VEMG_OP_A (one SpMV launch), VEMG_OP_GS_FWD (one forward
 * multicolour sweep over all rows, one launch per colour),
 * VEMG_OP_GS_COARSE (the same on A_bar's first coarse level, one launch per
 * patch colour), VEMG_OP_COARSEST (the explicit inverse of the surface
 * hierarchy's coarsest level times a vector, one launch), VEMG_OP_ET
 * (the restriction E~^T, one launch) or VEMG_OP_E (the prolongation E~
 * added into an n-vector, as the SOR cycle applies it, one launch) to nrhs (1..8)
 * columns, in the handle's inner precision (FP32 for VEMG_MIXED_IR, FP64
 * otherwise), measured with HIP events on the handle's own stream around
 * `reps` back-to-back applications on internal buffers, after one untimed
 * application.  *launches receives the kernel launches per application. */
vemg_status vemg_time_op(vemg_solver s, int op, int nrhs, int reps, double *avg_ms, int *launches);

vemg_status vemg_get_info(vemg_solver s, vemg_info *info);

/* Device memory needed to solve nrhs right-hand sides on this mesh, for
 * admission by memory footprint: the bytes the handle holds in HBM from
 * setup to destroy (fine operator in FP64 and row-scaled FP32, E~ and its
 * transpose, both smoothed aggregation hierarchies with their coarsest
 * inverses, the Krylov work space for batches of up to 8 columns) plus the
 * caller's b and x arrays, 2 * nrhs * n_nodes doubles.  nrhs = 0 gives the
 * handle alone; its part does not depend on nrhs, since larger requests run
 * in batches of 8 on the same work space.  Counted at setup from the same
 * allocation sequence as the upload, so it is exact and is also available
 * for a host-only handle (device -1) before any device is touched.
 * Errors: VEMG_ERR_INVALID_ARG (null pointer, nrhs < 0), VEMG_ERR_STATE
 * (no setup). */
vemg_status vemg_footprint(vemg_solver s, int nrhs, size_t *bytes);

/* Switches the preconditioner (vemg_pc) of a set-up handle; the setup (E~,
 * both hierarchies, packed operators) serves every preconditioner, so only
 * the captured iteration graphs are dropped.  Waits for the handle's pending
 * work.  VEMG_ERR_INVALID_ARG for an unknown value; VEMG_ERR_STATE for
 * VEMG_PC_SA on a handle set up without that hierarchy. */
vemg_status vemg_set_preconditioner(vemg_solver s, int pc);

/* Switches the precision (vemg_precision) of later solves; the FP32 operator
 * copies are built at setup, so nothing is rebuilt.  VEMG_ERR_INVALID_ARG
 * for an unknown value. */
vemg_status vemg_set_precision(vemg_solver s, int precision);

/* Copies a setup array to host memory for inspection (bit-exact tests).
 * name: "perm" (int64 [n], storage -> natural), "colour" (int32 [n]),
 * "Aoff.ptr" (int64), "Aoff.idx" (int32), "Aoff.val", "d", "diag" (double),
 * "E.ptr", "E.idx", "E.val", "S_perm" (int64),
 * "<h>.<level>.<what>" with h in {S, Abar, SA} and what in {A.ptr, A.idx, A.val,
 * P.ptr, P.idx, P.val, colour, node, agg, Cinv, rank (int64)}; levels in the
 * block multicolour order of the coarse SOR sweeps (all but the fine levels
 * of Abar and SA) also export patch, pcolour, lcolour (int32 per row) and
 * pc_start, patch_row, seg_ptr, seg_row (int64 ranges).  With buf == NULL
 * only *bytes is set; otherwise *bytes must hold the buffer size. */
vemg_status vemg_export(vemg_solver s, const char *name, void *buf, size_t *bytes);

vemg_status vemg_destroy(vemg_solver s);

const char *vemg_status_string(vemg_status st);

/* Message of the last error on this handle ("" if none). */
const char *vemg_last_error(vemg_solver s);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of solve requests over several resident
 * meshes.  A scheduler thread owns one lane per mesh with 8 right-hand-side
 * slots whose Krylov state stays in HBM.  Queued right-hand sides join free
 * slots whenever the lane's current chunk of PCG iterations ends, converged
 * columns retire after an FP64 true-residual check (so a column's result
 * does not depend on what else shares its batch), and the chunks of
 * different meshes run concurrently on their own streams.  Meshes are made
 * resident (uploaded) against an HBM budget; idle meshes are evicted
 * least-recently-used first.  Solves use the handle options given at
 * creation (VEMG_MIXED_IR is served as VEMG_MIXED_PC: its FP64 CG keeps
 * per-column state that can join and retire at any chunk boundary).
 * ------------------------------------------------------------------------ */
typedef struct vemg_server_s *vemg_server;

typedef struct {
  int64_t requests_done, columns_done, requests_queued;
  double p50_ms, p99_ms, mean_ms, max_ms;  /* request latency, submit -> result written */
  double solves_per_s;                     /* right-hand sides completed per second of busy time */
  double busy_s;                           /* first submit -> last completion */
  double mean_slot_occupancy;              /* active slots / 8, averaged over chunks */
  int64_t chunks, uploads, evictions;
  size_t resident_bytes, budget_bytes;
} vemg_server_stats;

/* hbm_budget: device bytes the resident meshes may use (0 = no limit); a
 * mesh is admitted when its vemg_footprint (nrhs = 0) fits beside the other
 * resident meshes.  All lanes share two pairs of streams (four hardware
 * queues in all): lane i runs on pair i mod 2. */
vemg_status vemg_server_create(int device, size_t hbm_budget, const vemg_options *o, vemg_server *out);
/* Registers a mesh (host setup now; same arguments as vemg_setup).  Fails
 * with VEMG_ERR_OOM if the mesh alone exceeds the budget. */
vemg_status vemg_server_add_mesh(vemg_server s, int64_t n_nodes, const double *xyz, int64_t n_tets,
                                 const int64_t *tets, const uint8_t *top_mask, int *mesh_id);
/* vemg_rhs for a registered mesh (host arrays). */
vemg_status vemg_server_rhs(vemg_server s, int mesh_id, const double *f_host, double *b_host);
/* vemg_footprint of a registered mesh: what admission compares against the
 * budget (nrhs = 0) and what a request of nrhs columns adds for its own b and
 * x arrays, which the caller allocates. */
vemg_status vemg_server_footprint(vemg_server s, int mesh_id, int nrhs, size_t *bytes);
/* Queues nrhs right-hand sides ([nrhs][n_nodes], device, natural order,
 * fully written before the call) and returns at once.  Each column stops on
 * this request's rtol and max_iter, whatever shares its batch.  x ([nrhs][n_nodes],
 * device) is written when the request completes; both buffers must stay
 * valid until then. */
vemg_status vemg_server_submit(vemg_server s, int mesh_id, int nrhs, const double *b_dev, double *x_dev,
                               double rtol, int max_iter, uint64_t *req_id);
/* Ids of requests completed since the last poll (at most cap). */
vemg_status vemg_server_poll(vemg_server s, uint64_t *done_ids, int cap, int *n_done);
/* Blocks until the request is complete (timeout_s <= 0: no timeout). */
vemg_status vemg_server_wait(vemg_server s, uint64_t req_id, double timeout_s);
/* Result of a completed request: worst column status, and per column the
 * iterations and true relative residual (arrays of nrhs, may be NULL). */
vemg_status vemg_server_result(vemg_server s, uint64_t req_id, int *status, int *iters, double *relres,
                               double *latency_ms);
vemg_status vemg_server_get_stats(vemg_server s, vemg_server_stats *st);
/* Switches the precision of later solves (VEMG_FP64 or VEMG_MIXED_PC) and
 * resets the statistics; only while no request is queued or running
 * (VEMG_ERR_STATE otherwise). */
vemg_status vemg_server_set_precision(vemg_server s, int precision);
/* Finishes queued work, stops the scheduler and frees every mesh. */
vemg_status vemg_server_destroy(vemg_server s);
/* Message of the last server error ("" if none). */
const char *vemg_server_last_error(vemg_server s);

#ifdef __cplusplus
}
#endif

#endif /* VEMG_H */
