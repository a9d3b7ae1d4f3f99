"""Pins of the Robin (free-surface) top condition, Section 2: the weak form
adds alpha times the P1 mass matrix of the horizontally projected top
triangles to A; nothing is fixed."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from inputs import box_mesh, fourier_field
from oracle import extrap, fem, precond, solver


def _full_top_mass(m):
    Moff, L = fem.top_surface_mass(m.xyz, extrap.top_triangles(m.tets, m.top))
    diag = L - np.asarray(Moff.sum(axis=1)).ravel()
    return (Moff + sp.diags(diag)).tocsr()


def test_top_mass_integrates_exactly():
    # P1 reproduces linear functions, so the surface mass matrix integrates
    # products of linear functions over the unit square exactly
    m = box_mesh(7, 6, 4, 0.01, jitter=0.3, seed=5, bathymetry=True)
    M = _full_top_mass(m)
    one = np.ones(m.n)
    x, y = m.xyz[:, 0], m.xyz[:, 1]
    assert abs(one @ M @ one - 1.0) < 1e-14
    assert abs(one @ M @ x - 0.5) < 1e-14
    assert abs(x @ M @ x - 1.0 / 3.0) < 1e-14
    assert abs(x @ M @ y - 0.25) < 1e-14
    assert np.all(M[~m.top][:, ~m.top].data == 0) if M[~m.top][:, ~m.top].nnz else True


def test_robin_matrix_is_spd_with_the_robin_deficit():
    m = box_mesh(6, 5, 4, 0.01, jitter=0.2, seed=2)
    alpha = 3.0
    s = solver.setup(m, "R", coarse_max=10, alpha=alpha)
    A = s.A.toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() > 0
    # A applied to a constant is alpha M_top 1 (rows of the top block only)
    M = _full_top_mass(m)
    ones = np.ones(s.n)
    ref = alpha * (M @ np.ones(m.n))[s.perm]
    assert np.abs(solver.apply_A(s, ones) - ref).max() < 1e-12 * np.abs(ref).max()


def test_robin_tends_to_dirichlet_for_large_alpha():
    m = box_mesh(7, 7, 5, 0.01, jitter=0.2, seed=4)
    f = fourier_field(m.xyz, 0.01, 6)
    sD = solver.setup(m, "D", coarse_max=20)
    xD = solver.to_natural(sD, spla.spsolve(sD.A.tocsc(), solver.rhs_from_field(sD, f)))
    errs = []
    for alpha in (1e4, 1e6):
        sR = solver.setup(m, "R", coarse_max=20, alpha=alpha)
        xR = solver.to_natural(sR, spla.spsolve(sR.A.tocsc(), solver.rhs_from_field(sR, f)))
        errs.append(np.linalg.norm(xR - xD) / np.linalg.norm(xD))
    # the difference decays like 1/alpha
    assert 0.008 * errs[0] < errs[1] < 0.012 * errs[0] and errs[1] < 1e-3, errs


def test_robin_manufactured_solution_converges_at_second_order():
    # u = cos(k (z + H)) solves -Lap u = k^2 u, has zero normal derivative on
    # the floor and the sides, and satisfies du/dn + alpha u = 0 on the top
    # for alpha = k tan(k H)
    # (uniform refinement of a unit cube: the horizontal jitter makes the
    # elements tilted, so all directions are refined together)
    H = 1.0
    k = 1.5
    alpha = k * np.tan(k * H)
    errs = []
    for nz in (5, 9, 17):
        m = box_mesh(nz, nz, nz, H, jitter=0.2, seed=3)
        u = np.cos(k * (m.xyz[:, 2] + H))
        s = solver.setup(m, "R", coarse_max=20, alpha=alpha)
        b = solver.rhs_from_field(s, k * k * u)
        x = solver.to_natural(s, spla.spsolve(s.A.tocsc(), b))
        errs.append(np.max(np.abs(x - u)) / np.max(np.abs(u)))
    # max-norm ratios 3.1 and 3.3 on these jittered meshes (second order, still
    # pre-asymptotic); a wrong sign or scale of the Robin term leaves an O(1) error
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert errs[2] < 5e-3, errs


@pytest.mark.parametrize("pc", ["vl_as", "vl_sor", "vl_add"])
def test_robin_preconditioners_spd_and_pcg_matches_direct(pc):
    m = box_mesh(8, 7, 5, 0.01, jitter=0.25, seed=21, bathymetry=True)
    s = solver.setup(m, "R", coarse_max=20, alpha=10.0)
    M = precond.make(s, pc)
    Bm = np.column_stack([M(e) for e in np.eye(s.n)])
    assert np.abs(Bm - Bm.T).max() < 1e-10 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0
    b = solver.rhs_from_field(s, fourier_field(m.xyz, 0.01, 3))
    x, it, rel, ok = solver.solve(s, b, 1e-11, pc, max_iter=5000)
    assert ok
    xd = spla.spsolve(s.A.tocsc(), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
