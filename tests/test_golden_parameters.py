"""The paper's printed parameters (tests/golden/paper_parameters.txt, each
line cited) against the oracle, the library's defaults and the benchmark's
comparison: no test value here comes from the code under test."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import amg

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_parameters.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            name, value, cite = line.rstrip("\n").split("\t")
            assert cite.startswith("Section"), name
            out[name] = [float(v) for v in value.split(",")]
    return out


G = _golden()


def test_oracle_uses_the_papers_sa_parameters():
    assert amg.THETA == G["sa_strength_threshold"][0]
    assert amg.OMEGA_P == pytest.approx(G["sa_prolongator_omega"][0], rel=1e-15)


def _textbook_sor(A, g, x, omega, order):
    x = x.copy()
    for i in order:
        s = g[i] - A[i] @ x + A[i, i] * x[i]
        x[i] = (1.0 - omega) * x[i] + omega * s / A[i, i]
    return x


@pytest.mark.parametrize("forward", [True, False])
def test_oracle_sweep_is_sor_with_the_papers_omega(forward):
    """With one colour per row the multicolour sweep is the sequential sweep;
    it must equal the textbook SOR update with the paper's relaxation
    factor, in natural order (forward) or reversed (backward)."""
    rng = np.random.default_rng(4)
    n = 9
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    g = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    got = amg.gs_sweep(A, np.diag(A).copy(), np.arange(n), g, x0, forward=forward)
    order = range(n) if forward else range(n - 1, -1, -1)
    ref = _textbook_sor(A, g, x0, G["sor_omega"][0], order)
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_library_defaults_are_the_papers_parameters():
    lib_mod = pytest.importorskip("paper_0912_1976_amd")
    lib = lib_mod.load_library()
    o = lib_mod._lib.Options()
    lib.vemg_default_options(C.byref(o))
    assert o.theta == G["sa_strength_threshold"][0]
    assert o.prolong_omega == pytest.approx(G["sa_prolongator_omega"][0], rel=1e-15)


def test_benchmark_compares_at_the_papers_aspect_ratios():
    import bench

    assert list(bench.SA_COMPARISON_EPS) == G["aspect_ratios"]
