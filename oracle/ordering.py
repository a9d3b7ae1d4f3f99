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
and, for the GPU library, by bit-exact comparison.

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
