"""Pins of the preconditioners (Sections 5.2-5.5, 6) and of PCG."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from inputs import box_mesh, fourier_field, manufactured_u
from oracle import pcg, precond, solver


@pytest.fixture(scope="module", params=["N", "D"])
def small(request):
    m = box_mesh(8, 7, 5, 0.01, jitter=0.25, seed=21, bathymetry=True)
    return m, solver.setup(m, request.param, coarse_max=20)


def test_schur_and_exact_inverse_decomposition():
    # eq. E equation: E^T A E = B - C A_bar^{-1} C^T, and eq. E multigrid:
    # A^{-1} = E (E^T A E)^{-1} E^T + Z A_bar^{-1} Z^T, with E = [I; -A_bar^{-1} C^T]
    m = box_mesh(6, 5, 4, 0.05, jitter=0.2, seed=2)
    s = solver.setup(m, "N", coarse_max=10)
    A = s.A.toarray()
    nt = s.n_top
    B, C, Abar = A[:nt, :nt], A[:nt, nt:], A[nt:, nt:]
    Ai = np.linalg.inv(Abar)
    E = np.vstack([np.eye(nt), -Ai @ C.T])
    schur = B - C @ Ai @ C.T
    assert np.abs(E.T @ A @ E - schur).max() < 1e-10 * np.abs(schur).max()
    Z = np.vstack([np.zeros((nt, A.shape[0] - nt)), np.eye(A.shape[0] - nt)])
    Minv = E @ np.linalg.inv(E.T @ A @ E) @ E.T + Z @ Ai @ Z.T
    Ainv = np.linalg.inv(A)
    assert np.abs(Minv - Ainv).max() < 1e-8 * np.abs(Ainv).max()


@pytest.mark.parametrize("pc", ["vl_as", "vl_sor", "vl_add", "jacobi"])
def test_preconditioners_symmetric_positive_definite(small, pc):
    m, s = small
    M = precond.make(s, pc)
    Bm = np.column_stack([M(e) for e in np.eye(s.n)])
    assert np.abs(Bm - Bm.T).max() < 1e-10 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0


@pytest.mark.parametrize("pc", ["vl_as", "vl_sor", "vl_add", "jacobi", "none"])
def test_pcg_matches_direct_solve(small, pc):
    m, s = small
    b = solver.rhs_from_field(s, fourier_field(m.xyz, 0.01, 3))
    x, it, rel, ok = solver.solve(s, b, 1e-11, pc, max_iter=5000)
    assert ok
    xd = spla.spsolve(s.A.tocsc(), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9


def test_manufactured_discrete_solution_recovered():
    # the paper's protocol: choose x*, set b = A x*, so the error is known exactly
    m = box_mesh(9, 9, 5, 0.01, jitter=0.2, seed=1)
    s = solver.setup(m, "N", coarse_max=20)
    xs = manufactured_u(m.xyz, 0.01)
    b = solver.rhs_from_solution(s, xs)
    x, it, rel, ok = solver.solve(s, b, 1e-11, "vl_as")
    assert ok
    ref = xs[s.perm]
    assert np.max(np.abs(x - ref)) / np.max(np.abs(ref)) < 1e-9


def test_cg_error_decreases_in_energy_norm(small):
    m, s = small
    b = solver.rhs_from_field(s, fourier_field(m.xyz, 0.01, 4))
    xd = spla.spsolve(s.A.tocsc(), b)
    M = precond.make(s, "vl_as")
    errs = []
    for k in range(1, 15):
        x, it, _, _ = pcg.pcg(lambda v: solver.apply_A(s, v), M, b, 0.0, max_iter=k)
        e = x - xd
        errs.append(e @ (s.A @ e))
    assert all(b2 <= b1 * (1 + 1e-9) for b1, b2 in zip(errs, errs[1:]))


def test_zero_rhs_and_breakdown():
    x, it, hist, ok = pcg.pcg(lambda v: v, lambda r: r, np.zeros(5), 1e-8)
    assert it == 0 and ok and not x.any()
    with pytest.raises(pcg.Breakdown):
        pcg.pcg(lambda v: -v, lambda r: r, np.ones(5), 1e-8)


@pytest.mark.parametrize("jitter", [0.0, 0.3])
def test_vertical_lumping_iterations_flat_in_aspect_ratio(jitter):
    # Section 6: with vertical lumping the iteration count stops depending on
    # eps for small eps.  Plain smoothed aggregation on A also copes with
    # aligned columns, but on broken columns (the paper's vertically
    # unstructured case) it develops eps-dependent plateaus.
    its = {pc: [] for pc in ("vl_as", "vl_sor", "vl_add", "sa")}
    for H in (1e-2, 1e-3, 1e-4):
        m = box_mesh(17, 17, 9, H, jitter=jitter, seed=1, bathymetry=True)
        s = solver.setup(m, "N", coarse_max=256)
        b = solver.rhs_from_field(s, fourier_field(m.xyz, H, 9))
        for pc in its:
            _, it, _, ok = solver.solve(s, b, 1e-8, pc, max_iter=20000)
            its[pc].append(it)
    for pc in ("vl_as", "vl_sor", "vl_add"):
        assert its[pc][2] <= 1.3 * its[pc][0], its
    if jitter > 0:
        assert its["sa"][2] >= 1.5 * its["sa"][0], its
        assert its["sa"][2] >= 2 * its["vl_sor"][2], its


def test_additive_smoother_pays_off_on_multiscale_mesh():
    # Section 6, Mesh B: on a centre-refined mesh the vertical-lumping cycle
    # alone converges slowly (small elements leave small eigenvalues that the
    # surface correction does not touch); including the additive smoother,
    # a V-cycle over all scales of A_bar, cuts the iteration count sharply.
    from inputs import graded_mesh
    m = graded_mesh(1 / 40, 1e-3, jitter=0.25, seed=3)
    s = solver.setup(m, "N", coarse_max=256)
    b = solver.rhs_from_field(s, fourier_field(m.xyz, 1e-3, 100))
    its = {}
    for pc in ("vl_as", "vl_sor"):
        _, its[pc], _, ok = solver.solve(s, b, 1e-8, pc, max_iter=5000)
        assert ok
    assert its["vl_as"] <= 0.75 * its["vl_sor"], its


def _exact_residual(Aoff, d, b, x_parts):
    """b - A_UU sum(x_parts) in exact rational arithmetic (difference form)."""
    from fractions import Fraction as F
    A = Aoff.tocsr()
    x = [sum((F(float(p[i])) for p in x_parts), F(0)) for i in range(A.shape[0])]
    out = []
    for i in range(A.shape[0]):
        acc = F(float(d[i])) * x[i]
        for k in range(A.indptr[i], A.indptr[i + 1]):
            acc += F(float(A.data[k])) * (x[A.indices[k]] - x[i])
        out.append(F(float(b[i])) - acc)
    return out


def test_two_sum_is_error_free():
    from fractions import Fraction as F
    rng = np.random.default_rng(5)
    a = rng.standard_normal(200) * 10.0 ** rng.integers(-20, 20, 200)
    b = rng.standard_normal(200) * 10.0 ** rng.integers(-20, 20, 200)
    s, e = pcg.two_sum(a, b)
    for ai, bi, si, ei in zip(a, b, s, e):
        assert F(float(si)) + F(float(ei)) == F(float(ai)) + F(float(bi))
        assert si == ai + bi


@pytest.mark.parametrize("smooth", [False, True])
def test_extended_residual_matches_exact_arithmetic(smooth):
    # brute force in rationals on a tiny thin mesh; the smooth case is a
    # nearly constant iterate, where the FP64 difference form cancels
    from oracle import fem
    m = box_mesh(6, 5, 4, 1e-4, jitter=0.3, seed=3, bathymetry=True)
    s = solver.setup(m, "N", coarse_max=10)
    rng = np.random.default_rng(6)
    n = s.n
    hi = 1.0 + 1e-3 * rng.standard_normal(n) if smooth else rng.standard_normal(n)
    lo = hi * 2.0 ** -53 * rng.uniform(-1, 1, n)
    b = solver.apply_A(s, hi) * (1 + 1e-9 * rng.standard_normal(n))
    got = fem.residual_extended(s.Aoff, s.d, b, hi, lo)
    exact = _exact_residual(s.Aoff, s.d, b, [hi, lo])
    A = s.Aoff.tocsr()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    x = hi + lo
    scale = np.abs(b) + np.abs(s.d * x) + np.bincount(rows, np.abs(A.data * (x[A.indices] - x[rows])), n)
    for i in range(n):
        err = abs(float(exact[i] - type(exact[i])(float(got[i]))))
        assert err <= 2.0 ** -53 * abs(float(exact[i])) + 2.0 ** -60 * scale[i], i
    # the plain FP64 residual of the rounded sum is visibly worse here
    plain = b - solver.apply_A(s, x)
    ex = np.array([float(v) for v in exact])
    assert np.linalg.norm(got - ex) <= 1e-3 * np.linalg.norm(plain - ex) + 1e-300


def test_extended_refinement_goes_below_the_fp64_floor():
    # Section 6: the FP64 accuracy floor grows as eps decreases.  With the
    # plain FP64 residual PCG stalls there; with the extended iterate and
    # residual the same preconditioned iteration reaches far lower.
    from oracle import fem
    m = box_mesh(17, 17, 9, 1e-4, jitter=0.3, seed=1, bathymetry=True)
    s = solver.setup(m, "N", coarse_max=256)
    b = solver.rhs_from_field(s, fourier_field(m.xyz, 1e-4, 9))
    M = precond.make(s, "vl_as")
    A = lambda v: solver.apply_A(s, v)
    _, _, rel_plain, ok_plain, _ = pcg.pcg_restarted(A, M, b, 1e-11, 5000)
    x, _, rel_ext, ok_ext, _ = pcg.pcg_restarted(
        A, M, b, 1e-11, 5000, residual=lambda h, l: fem.residual_extended(s.Aoff, s.d, b, h, l))
    assert not ok_plain and ok_ext, (rel_plain, rel_ext)
    assert rel_ext <= 1e-11 and rel_plain > 1e-10
