"""Pins of the vertical extrapolation operator E~ (Section 5.4)."""
import numpy as np
import pytest

from inputs import box_mesh
from oracle import extrap, fem, solver


@pytest.fixture(scope="module")
def setup_n():
    m = box_mesh(9, 8, 5, 0.01, jitter=0.3, seed=11, bathymetry=True)
    return m, solver.setup(m, "N", coarse_max=16)


def test_rows_nonnegative_at_most_three_and_sum_to_one(setup_n):
    m, s = setup_n
    E = s.E.tocsr()
    assert E.data.min() >= 0.0
    assert np.diff(E.indptr).max() <= 3
    sums = np.asarray(E.sum(axis=1)).ravel()
    # a row sums to one unless its surface triangle contains the pinned node,
    # whose weight is dropped
    tri = extrap.top_triangles(m.tets, m.top)
    _, tri_of_row = extrap.vertical_extrapolation(m.xyz, m.tets, m.top, s.perm,
                                                  fem.dirichlet_set(m.xyz, m.top, "N"))
    near_pin = np.array([t >= 0 and s.pin in tri[t] for t in tri_of_row])
    assert np.all(np.abs(sums[~near_pin] - 1.0) < 1e-14)
    assert np.all(sums[near_pin] < 1.0 + 1e-14)


def test_top_rows_are_identity(setup_n):
    m, s = setup_n
    E = s.E.tocsr()
    top_rows = E[: s.n_top]
    assert np.all(np.diff(top_rows.indptr) == 1)
    assert np.all(top_rows.data == 1.0)
    # S storage column of every top row is a permutation
    assert np.array_equal(np.sort(top_rows.indices), np.arange(s.n_top))


def test_reproduces_linear_functions(setup_n):
    # P1 interpolation on the surface reproduces a + b x + c y; with the point
    # condition the field must vanish at x_0
    m, s = setup_n
    x0 = m.xyz[s.pin]
    f = 0.7 * (m.xyz[:, 0] - x0[0]) - 1.3 * (m.xyz[:, 1] - x0[1])
    top_nodes = s.perm[: s.n_top][s.S_perm]
    got = s.E @ f[top_nodes]
    assert np.max(np.abs(got - f[s.perm])) < 1e-13


def test_locate_matches_brute_force():
    m = box_mesh(7, 7, 4, 0.01, jitter=0.3, seed=4)
    tri = extrap.top_triangles(m.tets, m.top)
    pts = m.xyz[~m.top][:, :2]
    which, lam = extrap.locate(pts, tri, m.xyz)
    txy = m.xyz[tri][:, :, :2]
    for p, w in zip(pts, which):
        inside = [t for t in range(tri.shape[0])
                  if (extrap.barycentric(p[None], txy[t][None])[0] >= -extrap.TOL_INSIDE).all()]
        assert w == min(inside)


def test_projection_error_outside_surface():
    m = box_mesh(5, 5, 3, 0.01)
    m.xyz[0, 0] = -0.5          # a floor node outside the top surface's shadow
    D = fem.dirichlet_set(m.xyz, m.top, "N")
    order = np.nonzero(~D)[0]
    order = np.concatenate([order[m.top[order]], order[~m.top[order]]])
    with pytest.raises(ValueError):
        extrap.vertical_extrapolation(m.xyz, m.tets, m.top, order, D)


def test_exact_extrapolation_tends_to_vertical_extrapolation():
    # Section 5.3: E = [I; -A_bar^{-1} C^T] is the discrete harmonic extension;
    # as eps -> 0 it becomes the vertical extrapolation.  On aligned columns
    # (no jitter, flat floor) E~ is exactly that limit, and E - E~ = O(eps^2).
    errs = []
    for H in (1e-2, 1e-3):
        m = box_mesh(6, 6, 4, H)
        s = solver.setup(m, "N", coarse_max=16)
        A = s.A.toarray()
        nt = s.n_top
        C = A[:nt, nt:]
        Abar = A[nt:, nt:]
        Eex = np.vstack([np.eye(nt), -np.linalg.solve(Abar, C.T)])
        Et = s.E.toarray()[:, np.argsort(s.S_perm)]
        errs.append(np.abs(Eex - Et).max())
    assert errs[1] < 1e-3
    assert 80 < errs[0] / errs[1] < 120
