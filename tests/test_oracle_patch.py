"""Pins of the block multicolour (patch) order of the coarse levels (oracle):
the patches, both colourings and the sweep order against their definitions
by brute force, and the sweep against the sequential Gauss-Seidel sweep in
the stored order (a triangular solve)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from inputs import box_mesh
from oracle import amg, ordering, solver


def _random_spd(n, density, seed):
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=density, random_state=rng, format="csr")
    A = (R + R.T).tocsr()
    A.data[:] = -np.abs(A.data)
    A = (A + sp.diags(np.asarray(-A.sum(axis=1)).ravel() + 1.0)).tocsr()
    A.sort_indices()
    return A


def _offdiag_counts(A):
    A = A.tocoo()
    return np.bincount(A.row[A.row != A.col], minlength=A.shape[0])


@pytest.mark.parametrize("seed,rows_max,entries_max", [(0, 7, 40), (1, 64, 4096), (2, 5, 12), (3, 16, 1)])
def test_patches_follow_their_definition(seed, rows_max, entries_max):
    A = _random_spd(150, 0.04, seed)
    rank = np.random.default_rng(seed + 10).permutation(150)
    patch = ordering.patches_of(A, rank, rows_max, entries_max)
    length = _offdiag_counts(A)
    seq = np.argsort(rank)
    # brute force: walk the rank order and start a patch whenever the limits say so
    expect, p, rows, ents = {}, -1, 0, 0
    for i in seq:
        if p < 0 or rows == rows_max or ents + length[i] > entries_max:
            p, rows, ents = p + 1, 0, 0
        expect[i] = p
        rows += 1
        ents += length[i]
    assert all(patch[i] == expect[i] for i in range(150))
    # consecutive in rank order, limits kept (a single unknown may exceed entries_max)
    assert np.all(np.diff(patch[seq]) >= 0) and np.all(np.diff(patch[seq]) <= 1)
    for q in range(patch.max() + 1):
        rows_q = np.nonzero(patch == q)[0]
        assert 1 <= rows_q.size <= rows_max
        assert rows_q.size == 1 or length[rows_q].sum() <= entries_max


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_patch_order_colourings_and_order_by_brute_force(seed):
    n = 300
    A = _random_spd(n, 0.02, seed)
    rank = np.random.default_rng(seed + 20).permutation(n)
    perm, patch, pcol, lcol = ordering.patch_order(A, rank, 16, 200)
    assert np.array_equal(np.sort(perm), np.arange(n))
    old_patch = ordering.patches_of(A, rank, 16, 200)
    assert np.array_equal(patch, old_patch[perm])
    C = A.tocoo()
    off = C.row != C.col
    i, j = C.row[off], C.col[off]
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    pi, pj = patch[inv[i]], patch[inv[j]]
    # patch colouring: coupled unknowns of different patches never share a patch colour
    assert np.all(pcol[inv[i]][pi != pj] != pcol[inv[j]][pi != pj])
    # every unknown of a patch has its patch's colour
    for q in range(patch.max() + 1):
        assert np.unique(pcol[patch == q]).size == 1
    # local colouring: coupled unknowns of one patch never share a local colour
    assert np.all(lcol[inv[i]][pi == pj] != lcol[inv[j]][pi == pj])
    # the composite colour is a valid colouring of the whole matrix
    comp = ordering.composite_colour(pcol, lcol, 16)
    Ap = A[perm][:, perm]
    assert ordering.is_valid_colouring(Ap, comp)
    # the order: patch colour, patch, local colour, rank
    keys = [(pcol[k], patch[k], lcol[k], rank[perm[k]]) for k in range(n)]
    assert keys == sorted(keys)
    # each colouring is the smallest-last greedy one of its graph
    G = ordering.patch_graph(A, old_patch)
    pc_by_patch = np.array([pcol[patch == q][0] for q in range(patch.max() + 1)])
    assert np.array_equal(pc_by_patch, ordering.colouring(G))
    for q in range(patch.max() + 1):
        rows_new = np.nonzero(patch == q)[0]          # already in rank order within (patch, lcol)
        rows_old = perm[rows_new]
        by_rank = rows_old[np.argsort(rank[rows_old])]
        sub = A[by_rank][:, by_rank].tocsr()
        lc = ordering.colouring(sub)
        pos = {r: k for k, r in enumerate(by_rank)}
        assert all(lcol[inv[r]] == lc[pos[r]] for r in rows_old)


@pytest.mark.parametrize("forward", [True, False])
def test_patch_sweep_is_the_sequential_sweep_in_stored_order(forward):
    # a coupled pair has the same relative order in the composite colour order
    # and in the stored order, so the multicolour sweep from zero is the
    # triangular solve of the stored matrix
    n = 400
    A = _random_spd(n, 0.015, 5)
    rank = np.random.default_rng(6).permutation(n)
    perm, patch, pcol, lcol = ordering.patch_order(A, rank, 12, 80)
    assert patch.max() > 10 and pcol.max() > 1
    Ap = amg.permute(A, perm)
    comp = ordering.composite_colour(pcol, lcol, 12)
    g = np.random.default_rng(7).standard_normal(n)
    x = amg.gs_sweep(Ap, Ap.diagonal(), comp, g, np.zeros(n), forward=forward)
    tri = sp.tril(Ap, format="csr") if forward else sp.triu(Ap, format="csr")
    ref = spla.spsolve_triangular(tri, g, lower=forward)
    assert np.max(np.abs(x - ref)) < 1e-12 * np.max(np.abs(ref))


def test_coarse_rank_orders_aggregates_by_their_first_member():
    # five fine rows with ranks 3 1 4 0 2, aggregates {0,1} {2,4} {3}; the
    # coarse unknowns are created as aggregate 0, 1 (two unknowns), 2
    L = amg.Level(A=sp.identity(5, format="csr"), colour=np.zeros(5, dtype=int), node=np.arange(5),
                  B=np.ones((5, 1)), rank=np.array([3, 1, 4, 0, 2]))
    agg = np.array([0, 0, 1, 2, 1])
    cnode = np.array([0, 1, 1, 2])
    # first members: aggregate 0 -> rank 1, aggregate 1 -> rank 2, aggregate 2 -> rank 0
    assert amg.coarse_rank(L, agg, cnode).tolist() == [1, 2, 3, 0]


def test_hierarchy_levels_are_patch_ordered():
    m = box_mesh(33, 33, 9, 1e-2, jitter=0.3, seed=2, bathymetry=True)
    s = solver.setup(m, "N", coarse_max=300)
    checked = 0
    for levels, first_patched in ((s.S_levels, True), (s.Abar_levels, False)):
        for li, L in enumerate(levels):
            if li == 0 and not first_patched:
                continue
            assert L.patch is not None
            checked += L.patch.max() > 0
            assert ordering.is_valid_colouring(L.A, L.colour)
            assert np.array_equal(L.colour, ordering.composite_colour(L.pcolour, L.lcolour))
            assert np.array_equal(np.sort(L.rank), np.arange(L.n))
            # stored by (patch colour, patch, local colour, rank); patches contiguous
            keys = list(zip(L.pcolour.tolist(), L.patch.tolist(), L.lcolour.tolist(), L.rank.tolist()))
            assert keys == sorted(keys)
            assert np.all(np.diff(L.patch[np.argsort(L.rank, kind="stable")]) >= 0)
            # the stored order re-derives from the level's own matrix and ranks
            inv_rank = np.argsort(L.rank)
            perm, patch, pcol, lcol = ordering.patch_order(L.A[inv_rank][:, inv_rank], np.arange(L.n))
            assert np.array_equal(inv_rank[perm], np.arange(L.n))
    assert checked >= 2
