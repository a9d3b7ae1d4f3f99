"""The allocation-free entry point vemg_matvec_noalloc against vemg_matvec,
through the C ABI: bit for bit the same product (same kernels) on two calls
in a row, the second on a smaller mesh, and a handle beyond the static
buffer's limit is refused with an error.  Run in a fresh process or after the
other tests, it must pass either way."""
import ctypes as C

import numpy as np
import pytest

from inputs import box_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0912_1976_amd as lib  # noqa: E402  (a missing package fails, never skips)


def _noalloc(s, x):
    y = torch.empty_like(x)
    st = s._lib.vemg_matvec_noalloc(s._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    return st, y


def test_noalloc_matvec_equals_matvec_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    big = box_mesh(129, 129, 33, 1e-3, bathymetry=True, jitter=0.3, seed=2)
    small = box_mesh(21, 17, 6, 1e-2, jitter=0.2, seed=9)
    for m in (big, small):  # the second call has a smaller input
        print("case noalloc matvec", m.n, flush=True)
        s = lib.Solver(m.xyz, m.tets, m.top, device=0)
        x = torch.as_tensor(np.random.default_rng(m.n).standard_normal(m.n), device=dev)
        ref = s.matvec(x)
        st, y = _noalloc(s, x)
        assert st == 0
        assert torch.equal(y, ref)
        st, y2 = _noalloc(s, 2.0 * x)
        assert st == 0 and torch.equal(y2, s.matvec(2.0 * x))
        s.close()


def test_noalloc_matvec_refuses_handles_beyond_its_buffer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # 257 x 257 x 33 has 2,179,616 unknowns, above the 2^21 the buffer holds
    m = box_mesh(257, 257, 33, 1e-4, bathymetry=True, jitter=0.3, seed=4)
    s = lib.Solver(m.xyz, m.tets, m.top, device=0)
    assert s.info()["n"] > 1 << 21
    x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    st, _ = _noalloc(s, x)
    assert st == -1
    assert "exceed" in s._lib.vemg_last_error(s._h).decode()
    # the handle still works, and so does the other entry point
    assert s.matvec(x).abs().max().item() == 0.0
    s.close()
