"""Node ordering and greedy colouring (oracle).

Test infrastructure only.

The paper orders the unknowns top block first, phi = (phi'; phi_bar)
(eqs. phi_decomposition / equation_decomposition).  Within each block the
order used here is a locality order followed by a colour sort, so that the
symmetric Gauss-Seidel (SOR, omega = 1) sweeps of Section 6 can update one
colour class at a time.  Colours are greedy in smallest-last vertex order,
which keeps the number of colour classes (sequential sweep stages) small:
four on a Kuhn-split box, whose tetrahedra are 4-cliques.  These are
readings of the paper (it does not fix an order); they are pinned by the
validity tests (permutation, valid colouring, the smallest-last property)
and, for the GPU library, by bit-exact comparison.  The coarse multigrid
levels are swept in a block multicolour order (patches of unknowns, see
patch_order below).

Locality key of a free node (x, y, z):
  T = max(1, round(sqrt(m_top / 64)))   tiles per side, m_top = #top nodes
  F = 8 T                               fine cells per side
  fx = min(F-1, floor((x - xmin)/(xmax - xmin) * F)), likewise fy
  key = (block, (fy // 8) * T + fx // 8, (fy % 8) * 8 + fx % 8, -z, node)
with block 0 for top nodes and 1 otherwise; the bounding box is over all
mesh nodes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def locality_order(xyz, top, free):
    """Free node indices sorted by the locality key described above."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    m_top = int(np.count_nonzero(top))
    T = max(1, int(round(math.sqrt(m_top / 64.0))))
    F = 8 * T
    xmin, xmax = x.min(), x.max()
    ymin, ymax = y.min(), y.max()
    fx = np.minimum(F - 1, np.floor((x - xmin) / (xmax - xmin) * F).astype(np.int64))
    fy = np.minimum(F - 1, np.floor((y - ymin) / (ymax - ymin) * F).astype(np.int64))
    tile = (fy // 8) * T + fx // 8
    fine = (fy % 8) * 8 + fx % 8
    block = np.where(top, 0, 1)
    idx = np.nonzero(free)[0]
    order = np.lexsort((idx, -z[idx], fine[idx], tile[idx], block[idx]))
    return idx[order]


def smallest_last_order(A):
    """Smallest-last vertex order of the off-diagonal pattern of the square
    CSR matrix A (Matula and Beck): repeatedly remove the vertex of smallest
    degree among the vertices not yet removed (degree counted over those
    vertices only; ties to the smallest index), and return the removal
    sequence reversed.  Greedy colouring in this order uses at most one more
    colour than the graph's degeneracy.  Plain Python with a lazy heap."""
    import heapq
    n = A.shape[0]
    indptr = A.indptr.tolist()
    indices = A.indices.tolist()
    deg = [0] * n
    for i in range(n):
        deg[i] = sum(1 for jj in range(indptr[i], indptr[i + 1]) if indices[jj] != i)
    heap = [(deg[i], i) for i in range(n)]
    heapq.heapify(heap)
    removed = [False] * n
    seq = []
    while heap:
        d, i = heapq.heappop(heap)
        if removed[i] or d != deg[i]:
            continue            # stale entry: i was removed or its degree has dropped
        removed[i] = True
        seq.append(i)
        for jj in range(indptr[i], indptr[i + 1]):
            j = indices[jj]
            if j != i and not removed[j]:
                deg[j] -= 1
                heapq.heappush(heap, (deg[j], j))
    seq.reverse()
    return np.array(seq, dtype=np.int64)


def colouring(A):
    """The colouring used for every SOR sweep: greedy in smallest-last order."""
    return greedy_colouring(A, smallest_last_order(A))


def greedy_colouring(A, order=None):
    """Greedy colouring of the off-diagonal pattern of the square CSR matrix
    A: visiting nodes in ``order`` (default 0..n-1), each takes the smallest
    colour not used by an already coloured neighbour.  Plain Python loop."""
    n = A.shape[0]
    indptr = A.indptr.tolist()
    indices = A.indices.tolist()
    colour = [-1] * n
    seq = range(n) if order is None else [int(v) for v in order]
    for i in seq:
        used = set()
        for jj in range(indptr[i], indptr[i + 1]):
            j = indices[jj]
            if j != i and colour[j] >= 0:
                used.add(colour[j])
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return np.array(colour, dtype=np.int64)


def colour_sorted(order, colour, block=None):
    """Stable sort of ``order`` by (block, colour of the node)."""
    c = colour[order]
    if block is None:
        keys = (np.arange(len(order)), c)
    else:
        keys = (np.arange(len(order)), c, block[order])
    return order[np.lexsort(keys)]


def colour_ranges(colour_sorted_colours):
    """[start, end) of each colour in a colour-sorted colour array."""
    c = np.asarray(colour_sorted_colours)
    if c.size == 0:
        return np.zeros((0, 2), dtype=np.int64)
    nc = int(c.max()) + 1
    starts = np.searchsorted(c, np.arange(nc), side="left")
    ends = np.searchsorted(c, np.arange(nc), side="right")
    return np.stack([starts, ends], axis=1)


def is_valid_colouring(A, colour):
    """No two neighbours (off-diagonal entries) share a colour."""
    A = A.tocoo()
    off = A.row != A.col
    return bool(np.all(colour[A.row[off]] != colour[A.col[off]]))


# ---------------------------------------------------------------------------
# Patch ordering of the coarse multigrid levels
# ---------------------------------------------------------------------------
# Reading (the paper fixes no SOR order): the sweeps of the coarse levels
# visit their unknowns in a block multicolour order.  The unknowns, taken in
# their spatial order (a rank per unknown), are cut into consecutive patches
# of at most PATCH_ROWS unknowns whose rows hold at most PATCH_ENTRIES
# off-diagonal entries together (a patch always takes at least one unknown).
# Two patches are neighbours when an entry of the level's matrix couples
# them.  The patches are coloured (greedy in smallest-last order on the patch
# graph), and the unknowns of every patch are coloured on the patch's own
# couplings (greedy in smallest-last order, unknowns in rank order).  The
# sweep order is: patch colour, then patch, then local colour, then rank.
# Unknowns of equal (patch colour, local colour) are never coupled (within a
# patch by the local colouring, across patches by the patch colouring), so a
# sweep in this order is the multicolour sweep over the composite colours
# (patch colour, local colour) in lexicographic order, and that is a plain
# sequential forward (or, reversed, backward) SOR sweep.
PATCH_ROWS = 128
PATCH_ENTRIES = 4096


def _pattern_csr(A):
    """Off-diagonal structural pattern of a square matrix (CSR, sorted)."""
    A = A.tocoo()
    off = A.row != A.col
    n = A.shape[0]
    P = sp.csr_matrix((np.ones(int(off.sum())), (A.row[off], A.col[off])), shape=(n, n))
    P.sum_duplicates()
    P.sort_indices()
    return P


def patches_of(A, rank, rows_max=PATCH_ROWS, entries_max=PATCH_ENTRIES):
    """Patch of every unknown (patches numbered in rank order): the unknowns
    in rank order are appended to the current patch until it holds rows_max
    unknowns or the next unknown's off-diagonal count would take the patch's
    total above entries_max; then a new patch starts."""
    A = _pattern_csr(A)
    n = A.shape[0]
    length = np.diff(A.indptr)
    patch = np.empty(n, dtype=np.int64)
    p, rows, ents = -1, 0, 0
    for i in np.argsort(rank, kind="stable").tolist():
        L = int(length[i])
        if p < 0 or rows == rows_max or ents + L > entries_max:
            p, rows, ents = p + 1, 0, 0
        patch[i] = p
        rows += 1
        ents += L
    return patch


def patch_graph(A, patch):
    """Patch adjacency: patches p != q are neighbours when some entry a_ij has
    i in p and j in q.  CSR pattern over the patches."""
    A = _pattern_csr(A).tocoo()
    npatch = int(patch.max()) + 1 if patch.size else 0
    pi, pj = patch[A.row], patch[A.col]
    cross = pi != pj
    G = sp.csr_matrix((np.ones(int(cross.sum())), (pi[cross], pj[cross])), shape=(npatch, npatch))
    G.sum_duplicates()
    G.sort_indices()
    return G


def patch_order(A, rank, rows_max=PATCH_ROWS, entries_max=PATCH_ENTRIES):
    """The block multicolour order described above.  Returns (perm, patch,
    pcolour, lcolour): perm[new] = old, and the patch, patch colour and local
    colour of every unknown in the new order."""
    A = _pattern_csr(A)
    n = A.shape[0]
    rank = np.asarray(rank)
    patch = patches_of(A, rank, rows_max, entries_max)
    pcol = colouring(patch_graph(A, patch)) if n else np.zeros(0, dtype=np.int64)
    lcol = np.zeros(n, dtype=np.int64)
    by_patch = np.lexsort((rank, patch))          # rows of each patch in rank order
    starts = np.searchsorted(patch[by_patch], np.arange(int(patch.max()) + 2 if n else 1))
    for p in range(starts.size - 1):
        rows = by_patch[starts[p]:starts[p + 1]]
        lcol[rows] = colouring(A[rows][:, rows].tocsr())
    perm = np.lexsort((rank, lcol, patch, pcol[patch]))
    return perm, patch[perm], pcol[patch][perm], lcol[perm]


def composite_colour(pcolour, lcolour, rows_max=PATCH_ROWS):
    """One integer per (patch colour, local colour) pair, in the pairs'
    lexicographic order (a local colour is below the patch's row count)."""
    return np.asarray(pcolour) * rows_max + np.asarray(lcolour)
