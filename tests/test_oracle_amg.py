"""Pins of the oracle's smoothed aggregation and smoothing (Sections 5.1, 6)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from inputs import box_mesh
from oracle import amg, ordering, solver


def chain(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def test_aggregation_of_a_chain_by_hand():
    # 1-D Laplacian on 9 nodes, every neighbour strong.
    # P1: 0 -> {0,1}; 1 taken; 2 has aggregated neighbour 1; 3 -> {2,3,4};
    #     5 has 4 taken; 6 -> {5,6,7}; 8 has 7 taken.
    # P2: none left except 8 -> joins aggregate of 7 (its only strong neighbour).
    agg = amg.aggregate(chain(9))
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2, 2, 2]


def test_aggregation_pass2_strongest_then_smallest():
    # P1: 0 -> {0,1}; 2 -> {2,3}; node 4 (linked to 1 and 3) is left over.
    # P2: it joins the aggregate of its strongest aggregated neighbour; on a
    # tie the smaller neighbour index (1) wins.
    def mat(w43):
        return sp.csr_matrix(np.array([[2., -1, 0, 0, 0],
                                       [-1, 3, 0, 0, -1],
                                       [0, 0, 2, -1, 0],
                                       [0, 0, -1, 3, -w43],
                                       [0, -1, 0, -w43, 2]]))
    assert amg.aggregate(mat(1.0)).tolist() == [0, 0, 1, 1, 0]
    assert amg.aggregate(mat(1.1)).tolist() == [0, 0, 1, 1, 1]


def test_weak_links_do_not_aggregate():
    # strength |a_ij| > 0.01 sqrt(a_ii a_jj): a 1e-5 link is weak
    A = sp.csr_matrix(np.array([[1.0, -1e-5], [-1e-5, 1.0]]))
    assert amg.aggregate(A).tolist() == [0, 1]
    A = sp.csr_matrix(np.array([[1.0, -0.02], [-0.02, 1.0]]))
    assert amg.aggregate(A).tolist() == [0, 0]


def test_smoothed_prolongator_keeps_near_kernel():
    # P = (I - 2/3 D^{-1} A) P^ with P^ B_c = B gives P B_c = B - 2/3 D^{-1} A B,
    # so a kernel vector of A is still reproduced exactly by the coarse space
    A = chain(12).tolil()
    A[0, 0] = 1.0
    A[11, 11] = 1.0          # Neumann chain: A 1 = 0
    A = A.tocsr()
    agg = np.repeat(np.arange(4), 3)
    P0, Bc, _ = amg.tentative_from_kernel(np.ones((12, 1)), np.arange(12), agg)
    P = amg.smoothed_prolongator_from(A, P0)
    assert np.allclose(P @ Bc, np.ones((12, 1)), atol=1e-14)
    dense = (np.eye(12) - (2.0 / 3.0) * np.diag(1.0 / A.diagonal()) @ A.toarray()) @ P0.toarray()
    assert np.allclose(P.toarray(), dense, atol=1e-15)


def test_tentative_prolongator_orthonormal_and_exact_on_kernel():
    rng = np.random.default_rng(0)
    n = 40
    agg = rng.integers(0, 7, n)
    agg = np.unique(agg, return_inverse=True)[1]
    B = np.column_stack([np.ones(n), rng.random(n), rng.random(n)])
    P0, Bc, cnode = amg.tentative_from_kernel(B, np.arange(n), agg)
    G = (P0.T @ P0).toarray()
    assert np.allclose(G, np.eye(G.shape[0]), atol=1e-13)
    assert np.allclose(P0 @ Bc, B, atol=1e-13)     # kernel vectors reproduced exactly


def _hier(mode="N"):
    m = box_mesh(9, 9, 5, 0.01, jitter=0.2, seed=3, bathymetry=True)
    return m, solver.setup(m, mode, coarse_max=24)


def test_colourings_and_aggregates_valid():
    m, s = _hier()
    assert ordering.is_valid_colouring(s.A, s.colour)
    for levels in (s.S_levels, s.Abar_levels):
        for L in levels:
            assert np.all(np.diff(L.colour) >= 0)
            assert ordering.is_valid_colouring(L.A, L.colour)
            assert (L.A - L.A.T).count_nonzero() == 0 or abs(L.A - L.A.T).max() < 1e-12 * abs(L.A).max()
        for L in levels[:-1]:
            # every node belongs to exactly one aggregate, aggregates are contiguous ids
            assert L.agg.min() == 0 and np.unique(L.agg).size == L.agg.max() + 1


def _brute_smallest_last(A):
    # the definition, by recomputation from scratch at every step
    n = A.shape[0]
    Ad = (A.tocsr() != 0).astype(int).tolil()
    Ad.setdiag(0)
    G = sp.csr_matrix(Ad)
    G = ((G + G.T) > 0).astype(int)
    alive = np.ones(n, bool)
    seq = []
    for _ in range(n):
        deg = np.asarray(G[:, alive].sum(axis=1)).ravel()
        cand = np.nonzero(alive)[0]
        i = cand[np.argmin(deg[cand])]      # first minimum = smallest index
        seq.append(i)
        alive[i] = False
    return np.array(seq[::-1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_smallest_last_order_matches_definition(seed):
    rng = np.random.default_rng(seed)
    n = 60
    R = sp.random(n, n, density=0.08, random_state=rng, format="csr")
    A = (R + R.T + sp.eye(n)).tocsr()
    A.sort_indices()
    assert np.array_equal(ordering.smallest_last_order(A), _brute_smallest_last(A))
    col = ordering.colouring(A)
    assert ordering.is_valid_colouring(A, col)


def test_kuhn_box_needs_exactly_four_colours():
    # every tetrahedron is a 4-clique of the matrix graph, so four colours are
    # the minimum; the Kuhn split admits four ((i + j + k) mod 4 differs along
    # every edge), and the smallest-last greedy colouring finds that minimum
    m = box_mesh(9, 8, 6, 1e-3, jitter=0.3, seed=4, bathymetry=True)
    s = solver.setup(m, "N", coarse_max=256)
    assert ordering.is_valid_colouring(s.A, s.colour)
    assert int(s.colour.max()) + 1 == 4


def test_multicolour_gs_equals_sequential_gs():
    # forward sweep with zero initial guess = (D + L)^{-1} g in colour-sorted order
    m, s = _hier()
    L = s.Abar_levels[0]
    g = np.random.default_rng(1).standard_normal(L.n)
    x = amg.gs_sweep(L.A, L.diag, L.colour, g, np.zeros(L.n), forward=True)
    lower = sp.tril(L.A, format="csr")
    ref = spla.spsolve_triangular(lower, g, lower=True)
    assert np.max(np.abs(x - ref)) < 1e-12 * np.max(np.abs(ref))
    upper = sp.triu(L.A, format="csr")
    y = amg.gs_sweep(L.A, L.diag, L.colour, g, np.zeros(L.n), forward=False)
    ref = spla.spsolve_triangular(upper, g, lower=False)
    assert np.max(np.abs(y - ref)) < 1e-12 * np.max(np.abs(ref))


def test_last_colour_residual_vanishes_after_forward_sweep():
    # with relaxation 1 the rows of the last colour are solved exactly from
    # neighbours that no later colour changes: their residual g - A x is zero
    # up to rounding (the library writes it as zero); the other colours' is not
    m, s = _hier()
    for A, diag, colour in ((s.A, s.diag, s.colour), (s.Abar_levels[0].A, s.Abar_levels[0].diag,
                                                      s.Abar_levels[0].colour)):
        n = A.shape[0]
        g = np.random.default_rng(2).standard_normal(n)
        for x0 in (np.zeros(n), np.random.default_rng(3).standard_normal(n)):
            x = amg.gs_sweep(A, diag, colour, g, x0, forward=True)
            r = g - A @ x
            scale = np.abs(g) + abs(A) @ np.abs(x)
            last = colour == colour.max()
            assert last.any() and (~last).any()
            assert np.max(np.abs(r[last]) / scale[last]) < 1e-13
            assert np.max(np.abs(r[~last]) / scale[~last]) > 1e-3


@pytest.mark.parametrize("which", ["S", "Abar"])
def test_vcycle_is_symmetric_positive_definite(which):
    m, s = _hier()
    levels = s.S_levels if which == "S" else s.Abar_levels
    n = levels[0].n
    V = np.column_stack([amg.vcycle(levels, e) for e in np.eye(n)])
    assert np.abs(V - V.T).max() < 1e-10 * np.abs(V).max()
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_two_level_with_complete_coarse_space_is_exact():
    # if the coarse space is everything (P = I, exact coarse solve), the V-cycle is A^{-1}
    A = chain(6) + 0.1 * sp.identity(6)
    perm = np.array([0, 2, 4, 1, 3, 5])
    A = A.tocsr()[perm][:, perm].tocsr()
    L0 = amg.Level(A=A, colour=np.array([0, 0, 0, 1, 1, 1]), node=np.arange(6), B=np.ones((6, 1)))
    L0.diag = A.diagonal()
    L0.P = sp.identity(6, format="csr")
    L1 = amg.Level(A=A, colour=np.zeros(6, dtype=int), node=np.arange(6), B=np.ones((6, 1)))
    L1.diag = A.diagonal()
    L1.chol = sla.cho_factor(A.toarray(), lower=True)
    g = np.arange(6.0)
    x = amg.vcycle([L0, L1], g)
    assert np.allclose(A @ x, g, atol=1e-12)


def test_stalled_level_is_aggregated_with_every_coupling():
    # a chain whose links are all weak (1e-5 against a unit diagonal) does
    # not coarsen at the threshold 0.01; the level is then aggregated with
    # every coupling strong, which for a chain is the aggregation of the
    # same chain with strong links
    n = 60
    weak = sp.diags([-1e-5 * np.ones(n - 1), np.ones(n), -1e-5 * np.ones(n - 1)], [-1, 0, 1], format="csr")
    assert amg.aggregate(weak).tolist() == list(range(n))
    levels = amg.build_hierarchy(weak, np.zeros(n, dtype=np.int64), None, coarse_max=10, max_levels=3)
    assert len(levels) >= 2
    assert levels[0].agg.tolist() == amg.aggregate(chain(n)).tolist()
    assert levels[1].n < n // 2


def test_vertical_columns_coarsen_below_coarse_max():
    # aligned columns at eps = 1e-3: only vertical couplings are strong; once
    # the columns are aggregated the coarsening continues through the
    # stall rule, and the preconditioned solve still converges
    m = box_mesh(13, 13, 7, 1e-3, jitter=0.0, seed=1, bathymetry=False)
    o = solver.setup(m, "N", coarse_max=30)
    assert o.Abar_levels[-1].n <= 30
    rng = np.random.default_rng(4)
    b = rng.standard_normal(o.n)
    x, it, rel, ok = solver.solve(o, b, 1e-10, "vl_as")
    xd = spla.spsolve(o.A.tocsc(), b)
    assert ok and np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
