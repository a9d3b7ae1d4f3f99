"""Pins of the oracle's P1 assembly (Section 3) against closed forms and
invariants that do not reuse the oracle's own formulas."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from inputs import box_mesh, manufactured_u, manufactured_f
from oracle import fem


def test_unit_right_tet_stiffness_closed_form():
    # textbook P1 stiffness of the reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1)
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    K = fem.element_stiffness(xyz, np.array([[0, 1, 2, 3]]))[0]
    ref = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6.0
    assert np.allclose(K, ref, rtol=0, atol=1e-15)


def test_unit_right_tet_mass_closed_form():
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    M = fem.element_mass(xyz, np.array([[0, 1, 2, 3]]))[0]
    ref = (np.ones((4, 4)) + np.eye(4)) / 120.0
    assert np.allclose(M, ref, rtol=0, atol=1e-17)


def test_orientation_error():
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    with pytest.raises(ValueError):
        fem.element_stiffness(xyz, np.array([[0, 2, 1, 3]]))


@pytest.fixture(scope="module")
def small():
    return box_mesh(7, 6, 5, 0.05, jitter=0.25, seed=3, bathymetry=True)


def test_mass_sums_to_volume():
    H = 0.02
    m = box_mesh(6, 5, 4, H, jitter=0.2, seed=1)
    M = fem.assemble_mass(m.xyz, m.tets)
    assert abs(M.sum() - H) < 1e-15 * 10


def test_symmetry_and_zero_row_sums(small):
    A, Aoff = fem.assemble_stiffness(small.xyz, small.tets)
    assert (A - A.T).count_nonzero() == 0          # bitwise symmetric
    scale = abs(A).sum(axis=1).A.ravel()
    assert np.max(np.abs(A @ np.ones(small.n)) / scale) < 1e-14


def test_row_sum_diagonal_equals_direct_diagonal(small):
    A, _ = fem.assemble_stiffness(small.xyz, small.tets)
    d = fem.assemble_diagonal_direct(small.xyz, small.tets)
    assert np.max(np.abs(A.diagonal() - d) / np.abs(d)) < 1e-12


def test_patch_test_linear_field(small):
    # P1 reproduces linear fields: (A u)_i = 0 at every node not on the boundary
    A, _ = fem.assemble_stiffness(small.xyz, small.tets)
    u = 0.3 + 1.7 * small.xyz[:, 0] - 0.4 * small.xyz[:, 1] + 25.0 * small.xyz[:, 2]
    nx, ny, nz = small.meta["nx"], small.meta["ny"], small.meta["nz"]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    interior = ((i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    r = A @ u
    scale = abs(A).sum(axis=1).A.ravel() * np.abs(u).max()
    assert np.max(np.abs(r[interior]) / scale[interior]) < 1e-13


def test_vertical_horizontal_split_and_scaling():
    # A = A_0 + A_H; stretching z by s scales A_H by s and A_0 by 1/s (Section 4)
    m = box_mesh(5, 5, 4, 1.0, jitter=0.2, seed=5)
    A, _ = fem.assemble_stiffness(m.xyz, m.tets)
    A0, _ = fem.assemble_stiffness(m.xyz, m.tets, weights=(0.0, 0.0, 1.0))
    AH, _ = fem.assemble_stiffness(m.xyz, m.tets, weights=(1.0, 1.0, 0.0))
    assert abs(A - A0 - AH).max() < 1e-13 * abs(A).max()
    s = 1e-3
    xyz2 = m.xyz * np.array([1.0, 1.0, s])
    A2, _ = fem.assemble_stiffness(xyz2, m.tets)
    assert abs(A2 - (A0 / s + AH * s)).max() < 1e-12 * abs(A2).max()


def _solve_mode_D(m, H):
    """Nodal max error and discrete L2 error (M-norm) of the Dirichlet-top
    problem with the manufactured solution."""
    A, Aoff = fem.assemble_stiffness(m.xyz, m.tets)
    M = fem.assemble_mass(m.xyz, m.tets)
    D = fem.dirichlet_set(m.xyz, m.top, "D")
    U, Auu, d = fem.reduce_to_unknowns(Aoff, D)
    Af = fem.full_matrix(Auu, d).tocsc()
    b = (M @ manufactured_f(m.xyz, H))[U]
    x = spla.spsolve(Af, b)
    e = np.zeros(m.n)
    e[U] = x - manufactured_u(m.xyz, H)[U]
    return np.max(np.abs(e)), np.sqrt(e @ (M @ e) / H)


@pytest.mark.parametrize("H,jit,min_rate_max,min_rate_l2", [(1.0, 0.15, 1.8, 1.9), (0.1, 0.0, 1.75, 1.9)])
def test_manufactured_solution_second_order(H, jit, min_rate_max, min_rate_l2):
    # nodal errors decay like h^2 under uniform refinement (thin domains are
    # pre-asymptotic for the max norm, whose P1 rate also carries a log h)
    emax, el2 = [], []
    for n in (9, 17, 33):
        m = box_mesh(n, n, n, H, jitter=jit, seed=7)
        a, b = _solve_mode_D(m, H)
        emax.append(a)
        el2.append(b)
    rmax = np.log2(np.array(emax[:-1]) / np.array(emax[1:]))
    rl2 = np.log2(np.array(el2[:-1]) / np.array(el2[1:]))
    assert rmax[-1] >= min_rate_max, (emax, rmax)
    assert rl2[-1] >= min_rate_l2, (el2, rl2)


def _eigs(m, mode):
    _, Aoff = fem.assemble_stiffness(m.xyz, m.tets)
    D = fem.dirichlet_set(m.xyz, m.top, mode)
    _, Auu, d = fem.reduce_to_unknowns(Aoff, D)
    return np.linalg.eigvalsh(fem.full_matrix(Auu, d).toarray())


def test_condition_number_scaling():
    # Section 4: with the Neumann top (point condition) lambda_min ~ eps^2 and
    # cond ~ eps^-2; with a Dirichlet top cond(A_bar) stays bounded.
    lam_n, cond_n, cond_d = [], [], []
    for H in (1e-2, 1e-3):
        m = box_mesh(6, 6, 4, H, jitter=0.2, seed=2)
        en = _eigs(m, "N") / (1.0 / H)       # remove the physical-coordinate factor L^2/H
        ed = _eigs(m, "D")
        lam_n.append(en[0])
        cond_n.append(en[-1] / en[0])
        cond_d.append(ed[-1] / ed[0])
    assert 70 < lam_n[0] / lam_n[1] < 130
    assert 70 < cond_n[1] / cond_n[0] < 130
    assert cond_d[1] / cond_d[0] < 1.5
