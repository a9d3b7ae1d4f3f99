"""Pins of the oracle's remaining choices, each against something other than
its own formula:

* the point condition's node x_0 (eq. point condition, reading: the top node
  closest to the origin, ties to the smallest index) against the mesh's
  known geometry and a brute-force search;
* the mode-N right-hand side (the Neumann problem needs a source of zero
  mean, Section 3) against invariance under constant shifts of f and against
  the element-volume quadrature of the mean of f;
* the block strength of connection used on levels with several unknowns per
  node (the near-kernel {1, x, y} of the surface operator) against a
  hand-computed 2-node x 3-unknown matrix.
"""
import numpy as np
import scipy.sparse as sp

from inputs import box_mesh, fourier_field
from oracle import amg, fem, solver as osolver


def test_pin_node_is_the_origin_corner_of_a_box():
    # natural numbering v = i + nx (j + ny k), k = nz - 1 on top: the corner
    # (0, 0, 0) is node nx * ny * (nz - 1); the side walls are not jittered
    for jit, seed in ((0.0, 0), (0.3, 5)):
        nx, ny, nz = 9, 7, 4
        m = box_mesh(nx, ny, nz, 1e-3, jitter=jit, seed=seed, bathymetry=True)
        p = fem.pin_node(m.xyz, m.top)
        assert p == nx * ny * (nz - 1)
        assert np.all(m.xyz[p] == 0.0) and m.top[p]


def test_pin_node_brute_force_and_ties():
    rng = np.random.default_rng(3)
    for _ in range(20):
        xyz = rng.uniform(-1, 1, (40, 3))
        top = rng.uniform(size=40) < 0.4
        top[rng.integers(40)] = True
        best = None
        for i in range(40):
            if top[i]:
                d = xyz[i] @ xyz[i]
                if best is None or d < best[0]:
                    best = (d, i)
        assert fem.pin_node(xyz, top) == best[1]
    # an exact tie goes to the smaller index; a closer node off the top is ignored
    xyz = np.array([[0.0, 0.0, -0.1], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0], [0.5, 0.5, -1.0]])
    top = np.array([False, True, True, False])
    assert fem.pin_node(xyz, top) == 1
    assert fem.pin_node(xyz[[0, 2, 1, 3]], top[[0, 2, 1, 3]]) == 1


def _element_mean_of(xyz, tets, f):
    """int f_h / |Omega| by the exact quadrature of a P1 field on each
    tetrahedron: its volume times the mean of its four vertex values."""
    p = xyz[tets]
    vol = np.abs(np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))) / 6.0
    return float(np.sum(vol * f[tets].mean(axis=1)) / np.sum(vol))


def test_mode_n_rhs_has_zero_mean_source():
    m = box_mesh(9, 8, 5, 1e-2, jitter=0.3, seed=4, bathymetry=True)
    o = osolver.setup(m, "N", coarse_max=16)
    f = fourier_field(m.xyz, 1e-2, 7) + 3.0
    b = osolver.rhs_from_field(o, f)
    scale = np.abs(o.mass @ np.abs(f)).max()
    # a constant source is all mean: nothing is left
    c = osolver.rhs_from_field(o, np.full(m.n, 2.5))
    assert np.max(np.abs(c)) <= 1e-14 * 2.5 * np.abs(o.mass @ np.ones(m.n)).max()
    # shifting f by a constant leaves b unchanged (a wrong weight vector or
    # sign would leave c (M 1 - w) or 2 c w behind)
    b2 = osolver.rhs_from_field(o, f - 7.0)
    assert np.max(np.abs(b2 - b)) <= 1e-13 * scale
    # b is M (f - fbar) with fbar the mean of f_h over the domain, computed
    # here by element quadrature instead of from the mass matrix
    fbar = _element_mean_of(m.xyz, m.tets, f)
    ref = (o.mass @ (f - fbar))[o.perm]
    assert np.max(np.abs(b - ref)) <= 1e-12 * scale
    # the full vector (with the pinned entry) integrates to zero
    full = o.mass @ (f - fbar)
    assert abs(full.sum()) <= 1e-12 * np.abs(full).sum()


def test_mode_d_rhs_is_not_projected():
    m = box_mesh(7, 7, 4, 1e-2, jitter=0.2, seed=2)
    o = osolver.setup(m, "D", coarse_max=16)
    f = fourier_field(m.xyz, 1e-2, 3) + 1.0
    assert np.array_equal(osolver.rhs_from_field(o, f), (o.mass @ f)[o.perm])


def test_block_strength_of_two_nodes_with_three_unknowns():
    # unknowns 0, 2, 4 belong to node 0 and 1, 3, 5 to node 1 (interleaved,
    # so that a transposed or dof-indexed lookup fails)
    node = np.array([0, 1, 0, 1, 0, 1])
    A = np.zeros((6, 6))
    d0 = [[4.0, 1.0, 0.0], [1.0, 5.0, 2.0], [0.0, 2.0, 6.0]]    # block (0, 0)
    d1 = [[3.0, 0.0, 1.0], [0.0, 2.0, 0.0], [1.0, 0.0, 7.0]]    # block (1, 1)
    c = [[0.03, -0.02, 0.05], [0.0, 0.03, -0.05], [0.04, 0.0, 0.06]]  # block (0, 1)
    i0, i1 = [0, 2, 4], [1, 3, 5]
    for a in range(3):
        for b in range(3):
            A[i0[a], i0[b]] = d0[a][b]
            A[i1[a], i1[b]] = d1[a][b]
            A[i0[a], i1[b]] = c[a][b]
            A[i1[b], i0[a]] = c[a][b]
    # by hand: ||C||_F^2 = 9 + 4 + 25 + 9 + 25 + 16 + 36 = 124 (x 1e-4); ||D0||_F^2 = 16 + 2 + 25 + 8 + 36 = 87;
    # ||D1||_F^2 = 9 + 2 + 4 + 49 = 64
    fc, f0, f1 = np.sqrt(124e-4), np.sqrt(87.0), np.sqrt(64.0)
    thr = 0.01 * np.sqrt(f0 * f1)
    assert fc > thr  # strong as blocks, although every single entry is weak:
    diag = np.diag(A)
    assert all(abs(c[a][b]) <= 0.01 * np.sqrt(diag[i0[a]] * diag[i1[b]]) for a in range(3) for b in range(3))
    G = amg.node_strength_graph(sp.csr_matrix(A), node, 2)
    assert G.shape == (2, 2) and G.nnz == 2
    assert abs(G[0, 1] - fc) <= 1e-15 * fc and abs(G[1, 0] - fc) <= 1e-15 * fc
    # a threshold just above the block ratio makes the pair weak
    G2 = amg.node_strength_graph(sp.csr_matrix(A), node, 2, theta=1.001 * fc / np.sqrt(f0 * f1))
    assert G2.nnz == 0
    # the scalar test (one unknown per node) sees no strong entry at all
    G3 = amg.node_strength_graph(sp.csr_matrix(A), np.arange(6), 6)
    assert not any(G3[i, j] for i in i0 for j in i1)
