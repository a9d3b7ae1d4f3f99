"""Smoothed aggregation multigrid (paper Sections 5.1 and 6), oracle version.

Test infrastructure only: plain NumPy/SciPy with pure-Python loops for the
greedy phases.

Paper facts used:
* Galerkin coarse operator P^T A P (eq. reduced AMG) and the V-cycle with a
  forward SOR sweep before restriction and a backward sweep after
  prolongation (Section 5.1, V-cycle diagram);
* smoothed aggregation after Vanek et al. (1996); strength of connection
  |a_ij| > theta sqrt(a_ii a_jj) with theta = 0.01; prolongator smoothing
  with omega = 2/3; SOR with omega = 1 (Section 6, first preconditioner).

Readings where the paper is silent (all stated in the design notes):
* aggregation in three passes over the level's index order
  (P1) i and all its strong neighbours unaggregated -> new aggregate
       {i} + strong neighbours;
  (P2) a node left over joins the P1 aggregate of its strongest strong
       neighbour (ties within a relative 1e-10 of the maximum go to the
       smallest neighbour index);
  (P3) a node still left starts a new aggregate with its still
       unaggregated strong neighbours;
  coarse nodes are numbered in order of creation;
* the near-kernel of each hierarchy is given as a set of vectors (the
  constant for A_bar; the constant and the horizontal coordinates for the
  vertically lumped operator); the tentative prolongator orthonormalises them
  aggregate by aggregate (Vanek et al.);
* prolongator smoothing uses A itself (no filtering):
  P = (I - omega D^{-1} A) P^, D = diag(A), so P keeps A's near-kernel;
* the sparsity pattern of every product is structural (entries that cancel
  to zero are kept);
* SOR sweeps are multicolour.  The coarse levels are stored in the block
  multicolour (patch) order of ordering.patch_order: patches of unknowns
  consecutive in the spatial order, patch colour, patch, local colour; the
  sweep takes the composite colours (patch colour, local colour) ascending
  (forward) or descending (backward).  The spatial order of a coarse level
  ranks its aggregates by their first member in the finer level's spatial
  order (the unknowns of one aggregate in creation order);
* coarsening stops at <= coarse_max unknowns, when a level would keep more
  than 0.8 of its unknowns, or at max_levels; the coarsest level is solved
  exactly (dense Cholesky).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import ordering

THETA = 0.01
OMEGA_P = 2.0 / 3.0
TIE_RTOL = 1e-10


# ---------------------------------------------------------------------------
# sparse helpers with structural patterns
# ---------------------------------------------------------------------------

def _pattern(M):
    P = M.tocsr().copy()
    P.data = np.ones_like(P.data)
    return P


def on_pattern(pattern, values):
    """CSR with the structure of ``pattern`` and the entries of ``values``
    (zero where ``values`` has none)."""
    pattern = pattern.tocsr()
    pattern.sort_indices()
    values = values.tocsr()
    values.sum_duplicates()
    values.sort_indices()
    n = pattern.shape[1]
    pr = np.repeat(np.arange(pattern.shape[0]), np.diff(pattern.indptr))
    vr = np.repeat(np.arange(values.shape[0]), np.diff(values.indptr))
    kp = pr.astype(np.int64) * n + pattern.indices
    kv = vr.astype(np.int64) * n + values.indices
    if kv.size == 0:
        data = np.zeros(kp.size)
    else:
        idx = np.minimum(np.searchsorted(kv, kp), kv.size - 1)
        data = np.where(kv[idx] == kp, values.data[idx], 0.0)
    out = sp.csr_matrix((data, pattern.indices.copy(), pattern.indptr.copy()), shape=pattern.shape)
    return out


def structural_product(*mats):
    """Product of sparse matrices on the structural pattern of the product
    of their patterns."""
    val = mats[0].tocsr()
    pat = _pattern(mats[0])
    for M in mats[1:]:
        val = (val @ M).tocsr()
        pat = (pat @ _pattern(M)).tocsr()
    pat.data[:] = 1.0
    return on_pattern(pat, val)


# ---------------------------------------------------------------------------
# strength, aggregation, prolongator
# ---------------------------------------------------------------------------

def strong_connections(A):
    """Boolean mask over A's stored entries: off-diagonal and
    |a_ij| > theta * sqrt(a_ii a_jj) (Section 6)."""
    A = A.tocsr()
    diag = A.diagonal()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    off = rows != cols
    thr = THETA * np.sqrt(diag[rows] * diag[cols])
    return off & (np.abs(A.data) > thr)


def aggregate(A):
    """Aggregates of a scalar level matrix A (one unknown per node)."""
    G = node_strength_graph(A, np.arange(A.shape[0]), A.shape[0])
    return aggregate_graph(G)


def tentative_prolongator(agg):
    n = agg.size
    nc = int(agg.max()) + 1 if n else 0
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nc))


@dataclass
class Level:
    A: sp.csr_matrix                 # standard form, storage order
    colour: np.ndarray               # sweep colour of each row (composite on patch-ordered levels)
    node: np.ndarray                 # aggregation node of each row (dof)
    B: np.ndarray                    # near-kernel vectors restricted to this level [n, k]
    rank: np.ndarray | None = None   # position of each row in the level's spatial order
    patch: np.ndarray | None = None  # patch-ordered levels: patch, patch colour, local colour
    pcolour: np.ndarray | None = None
    lcolour: np.ndarray | None = None
    P: sp.csr_matrix | None = None   # prolongator to this level from the next
    chol: tuple | None = None        # Cholesky factor on the coarsest level
    agg: np.ndarray | None = None    # aggregate of each node
    diag: np.ndarray = field(default=None)

    @property
    def n(self):
        return self.A.shape[0]


def patch_level(A, rank):
    """Block multicolour (patch) order of a level whose unknowns have the
    spatial ranks `rank` (ordering.patch_order).  Returns (permutation
    new->old, dict of the per-row arrays in the new order: colour (the
    composite sweep colour), patch, pcolour, lcolour, rank)."""
    perm, patch, pcol, lcol = ordering.patch_order(A, rank)
    return perm, dict(colour=ordering.composite_colour(pcol, lcol), patch=patch, pcolour=pcol,
                      lcolour=lcol, rank=np.asarray(rank)[perm])


def coarse_rank(L, agg, cnode):
    """Spatial rank of the coarse unknowns (creation order): aggregates are
    ranked by their member of smallest rank in the finer level L, and the
    unknowns of one aggregate follow their creation order."""
    nagg = int(agg.max()) + 1
    first = np.full(nagg, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, agg[L.node], np.asarray(L.rank, dtype=np.int64))
    order = np.lexsort((np.arange(cnode.size), first[cnode]))
    rank = np.empty(cnode.size, dtype=np.int64)
    rank[order] = np.arange(cnode.size)
    return rank


def permute(A, perm):
    A = A.tocsr()[perm][:, perm].tocsr()
    A.sort_indices()
    return A


def node_strength_graph(A, node, nnodes, theta=THETA):
    """Strong node graph: nodes I != J are strongly connected when
    ||A_IJ||_F > theta sqrt(||A_II||_F ||A_JJ||_F), with A_IJ the block of
    entries whose row belongs to I and column to J.  For one unknown per
    node this is the scalar test of Section 6.  Returns a CSR matrix whose
    entries are ||A_IJ||_F on the strong connections (sorted indices)."""
    C = A.tocoo()
    I = node[C.row]
    J = node[C.col]
    F = sp.csr_matrix((C.data * C.data, (I, J)), shape=(nnodes, nnodes))
    F.sum_duplicates()
    F.data = np.sqrt(F.data)
    d = F.diagonal()
    rows = np.repeat(np.arange(nnodes), np.diff(F.indptr))
    off = rows != F.indices
    st = off & (F.data > theta * np.sqrt(d[rows] * d[F.indices]))
    G = sp.csr_matrix((F.data[st], (rows[st], F.indices[st])), shape=(nnodes, nnodes))
    G.sort_indices()
    return G


def aggregate_graph(G):
    """The three aggregation passes on a strong graph G (entries = strength).
    Returns the aggregate (creation order) of every node."""
    n = G.shape[0]
    indptr = G.indptr.tolist()
    indices = G.indices.tolist()
    w = G.data.tolist()
    nbrs = [[(indices[k], w[k]) for k in range(indptr[i], indptr[i + 1])] for i in range(n)]
    agg = [-1] * n
    nagg = 0
    for i in range(n):                                   # P1
        if agg[i] >= 0:
            continue
        if all(agg[j] < 0 for j, _ in nbrs[i]):
            agg[i] = nagg
            for j, _ in nbrs[i]:
                agg[j] = nagg
            nagg += 1
    after_p1 = list(agg)
    for i in range(n):                                   # P2
        if agg[i] >= 0:
            continue
        cand = [(j, x) for j, x in nbrs[i] if after_p1[j] >= 0]
        if not cand:
            continue
        wmax = max(x for _, x in cand)
        best = min(j for j, x in cand if x >= wmax * (1.0 - TIE_RTOL))
        agg[i] = after_p1[best]
    for i in range(n):                                   # P3
        if agg[i] >= 0:
            continue
        agg[i] = nagg
        for j, _ in nbrs[i]:
            if agg[j] < 0:
                agg[j] = nagg
        nagg += 1
    return np.array(agg, dtype=np.int64)


GS_DROP = 1e-10


def tentative_from_kernel(B, node, agg):
    """Tentative prolongator of Vanek et al.: on every aggregate the
    near-kernel vectors (columns of B restricted to the aggregate's unknowns)
    are orthonormalised by modified Gram-Schmidt in column order; a vector
    whose norm falls to GS_DROP times its original norm is dropped.  The
    kept vectors are the aggregate's coarse unknowns (aggregate by
    aggregate, then in column order) and the coefficients R = Q^T B give the
    near-kernel vectors of the coarse level.
    Returns (P^ CSR, B_coarse, node of every coarse unknown)."""
    dof_agg = agg[node]
    order = np.argsort(dof_agg, kind="stable")
    starts = np.searchsorted(dof_agg[order], np.arange(int(agg.max()) + 2))
    rows, cols, vals, Bc, cnode = [], [], [], [], []
    nc = 0
    k = B.shape[1]
    for a in range(int(agg.max()) + 1):
        idx = order[starts[a]:starts[a + 1]]
        Q = []
        for c in range(k):
            v = B[idx, c].copy()
            n0 = float(np.sqrt(v @ v))
            for q in Q:
                v = v - (q @ v) * q
            nv = float(np.sqrt(v @ v))
            if n0 > 0.0 and nv > GS_DROP * n0:
                Q.append(v / nv)
        for q in Q:
            rows.append(idx)
            cols.append(np.full(idx.size, nc))
            vals.append(q)
            Bc.append(np.array([q @ B[idx, c] for c in range(k)]))
            cnode.append(a)
            nc += 1
    P0 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(B.shape[0], nc))
    P0.sort_indices()
    return P0, np.array(Bc).reshape(nc, k), np.array(cnode, dtype=np.int64)


def smoothed_prolongator_from(A, P0):
    """P = (I - omega D^{-1} A) P^, D = diag(A), on the structural pattern
    (Jacobi smoothing of the tentative prolongator with omega = 2/3)."""
    n = A.shape[0]
    S = (sp.identity(n, format="csr") - OMEGA_P * sp.diags(1.0 / A.diagonal()) @ A).tocsr()
    pat = (_pattern(A) + sp.identity(n, format="csr")).tocsr()
    pat.data[:] = 1.0
    return structural_product(on_pattern(pat, S), P0)


def build_hierarchy(A0, colour0, B0=None, coarse_max=8192, max_levels=10, stall=0.8, rank0=None, first=None):
    """SA hierarchy on A0 (in storage order, with the sweep colour colour0 of
    every row; the sweeps select rows by colour), one unknown per node on
    the finest level, near-kernel vectors B0 (default: the constant vector),
    spatial rank rank0 of every row (default: the storage order).  first:
    optional dict of the first level's patch arrays (patch, pcolour,
    lcolour) when it is patch-ordered itself.  Every coarser level is stored
    in its patch order (patch_level).

    Coarsening stops at coarse_max unknowns, at max_levels, or when a level
    would keep more than `stall` of its unknowns.  Reading: Section 6 fixes
    the strength threshold (0.01) but not what happens when too few
    couplings pass it, as on meshes with vertical columns at small eps,
    where only the vertical couplings are strong and, once the columns are
    aggregated, no coupling is: such a level is aggregated again with every
    coupling counted as strong (threshold 0) before coarsening gives up, so
    that the coarsest level stays small enough for its dense solve."""
    n0 = A0.shape[0]
    if B0 is None:
        B0 = np.ones((n0, 1))
    levels = [Level(A=A0.tocsr(), colour=np.asarray(colour0), node=np.arange(n0),
                    B=np.asarray(B0, dtype=np.float64),
                    rank=np.arange(n0) if rank0 is None else np.asarray(rank0), **(first or {}))]
    nnodes = n0
    while True:
        L = levels[-1]
        L.diag = L.A.diagonal().copy()
        if L.n <= coarse_max or len(levels) >= max_levels:
            break
        G = node_strength_graph(L.A, L.node, nnodes)
        agg = aggregate_graph(G)
        P0, Bc, cnode = tentative_from_kernel(L.B, L.node, agg)
        nc = P0.shape[1]
        if nc > stall * L.n:
            G = node_strength_graph(L.A, L.node, nnodes, 0.0)
            agg = aggregate_graph(G)
            P0, Bc, cnode = tentative_from_kernel(L.B, L.node, agg)
            nc = P0.shape[1]
            if nc > stall * L.n:
                break
        P = smoothed_prolongator_from(L.A, P0)
        Ac = structural_product(P.T.tocsr(), L.A, P)
        perm, arrs = patch_level(Ac, coarse_rank(L, agg, cnode))
        L.P = P[:, perm].tocsr()
        L.P.sort_indices()
        L.agg = agg
        nnodes = int(agg.max()) + 1
        levels.append(Level(A=permute(Ac, perm), node=cnode[perm], B=Bc[perm], **arrs))
    last = levels[-1]
    last.chol = sla.cho_factor(last.A.toarray(), lower=True)
    return levels


def operator_complexity(levels):
    return sum(L.A.nnz for L in levels) / levels[0].A.nnz


# ---------------------------------------------------------------------------
# smoothing and the V-cycle
# ---------------------------------------------------------------------------

def gs_sweep(A, diag, colour, g, x, forward=True):
    """One multicolour Gauss-Seidel (SOR, omega = 1) sweep for A x = g:
    the rows of one colour share no entries, so updating them together is
    the sequential sweep taken in colour order."""
    x = x.copy()
    cols = np.unique(colour).tolist()
    seq = cols if forward else cols[::-1]
    for c in seq:
        rows = np.nonzero(colour == c)[0]
        if rows.size == 0:
            continue
        x[rows] = x[rows] + (g[rows] - A[rows] @ x) / diag[rows]
    return x


def vcycle(levels, g, lvl=0):
    """One V(1,1)-cycle with zero initial guess (Section 5.1):
    forward SOR, restrict the residual, recurse, prolongate, backward SOR."""
    L = levels[lvl]
    if lvl == len(levels) - 1:
        return sla.cho_solve(L.chol, g)
    x = gs_sweep(L.A, L.diag, L.colour, g, np.zeros_like(g), forward=True)
    r = g - L.A @ x
    e = vcycle(levels, L.P.T @ r, lvl + 1)
    x = x + L.P @ e
    x = gs_sweep(L.A, L.diag, L.colour, g, x, forward=False)
    return x
