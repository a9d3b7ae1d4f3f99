"""Pins of the oracle's sparse-approximate-inverse extrapolation (Section 5.4,
second approach): E~ = [I; F] on the projection's pattern, column i of F
solving the exact extrapolation's column system restricted to its pattern.

* With a full pattern the restriction is void and E~ is the exact
  extrapolation E = [I; -A_bar^{-1} C^T]: then eq. (E multigrid) with exact
  solves reproduces A^{-1}, checked against a dense inverse of A.
* With vertical columns the exact E tends to the vertical extrapolation as
  eps -> 0 (Section 5.3), which the projection's E~ represents exactly on
  its own pattern, so the refitted F approaches it; the gap shrinks as eps^2.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from inputs import box_mesh
from oracle import extrap, solver as osolver


def _full_pattern_identity(mode, alpha):
    m = box_mesh(5, 4, 3, 0.1, jitter=0.2, seed=3, bathymetry=True)
    o = osolver.setup(m, mode, coarse_max=4, alpha=alpha)
    n, mt = o.n, o.n_top
    # a full non-top block (any stored values; the refit overwrites them)
    pattern = sp.csr_matrix(np.vstack([np.eye(mt), np.full((n - mt, mt), 0.5)]))
    E = extrap.sspai_refit(pattern, o.A, mt).toarray()
    A = o.A.toarray()
    Z = np.vstack([np.zeros((mt, n - mt)), np.eye(n - mt)])
    M = E @ np.linalg.solve(E.T @ A @ E, E.T) + Z @ np.linalg.solve(Z.T @ A @ Z, Z.T)
    Ainv = np.linalg.inv(A)
    return np.abs(M - Ainv).max() / np.abs(Ainv).max()


@pytest.mark.parametrize("mode,alpha", [("N", 0.0), ("R", 3.0)])
def test_full_pattern_gives_exact_inverse(mode, alpha):
    assert _full_pattern_identity(mode, alpha) < 1e-11


def _gap(H, jitter):
    m = box_mesh(9, 9, 5, H, jitter=jitter, seed=3, bathymetry=False)
    proj = osolver.setup(m, "N", coarse_max=40)
    fit = osolver.setup(m, "N", coarse_max=40, extrapolation="sspai")
    assert np.array_equal(proj.E.indptr, fit.E.indptr)
    assert np.array_equal(proj.E.indices, fit.E.indices)
    mt = proj.n_top
    top = fit.E[:mt].toarray()
    assert np.array_equal(top, proj.E[:mt].toarray())   # top rows stay the identity (permuted)
    return np.abs((fit.E - proj.E).toarray()).max()


def test_vertical_columns_tend_to_projection_as_eps_squared():
    g2, g3, g4 = _gap(1e-2, 0.0), _gap(1e-3, 0.0), _gap(1e-4, 0.0)
    assert g4 < 1e-5
    assert 80.0 < g2 / g3 < 125.0
    assert 80.0 < g3 / g4 < 125.0


def test_columns_solve_their_restricted_systems():
    # each fitted column satisfies its own restricted system; no column of
    # the pattern is left at the projection's values
    m = box_mesh(7, 6, 4, 1e-2, jitter=0.3, seed=2, bathymetry=True)
    o = osolver.setup(m, "N", coarse_max=40, extrapolation="sspai")
    proj = osolver.setup(m, "N", coarse_max=40)
    mt = o.n_top
    A = o.A.tocsr()
    Ec = o.E.tocsc()
    Pc = proj.E.tocsc()
    changed = 0
    for i in range(Ec.shape[1]):
        rows = Ec.indices[Ec.indptr[i]:Ec.indptr[i + 1]]
        vals = Ec.data[Ec.indptr[i]:Ec.indptr[i + 1]]
        J = rows[rows >= mt]
        v = vals[rows >= mt]
        if J.size == 0:
            continue
        # column of S storage -> top-block position of the surface node
        ti = o.S_perm[i]
        res = A[J][:, J] @ v + A[J, ti].toarray().ravel()
        assert np.abs(res).max() <= 1e-12 * np.abs(A[J][:, J]).max() * max(np.abs(v).max(), 1.0)
        changed += not np.allclose(v, Pc.data[Pc.indptr[i]:Pc.indptr[i + 1]][rows >= mt])
    assert changed > 0


def test_unknown_extrapolation_rejected():
    m = box_mesh(5, 4, 3, 0.1, jitter=0.0, seed=1)
    with pytest.raises(ValueError):
        osolver.setup(m, "N", extrapolation="harmonic")
