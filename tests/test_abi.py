"""The C ABI (include/vemg.h) without a GPU: every declared function is
exported, options and status strings behave, and host-only handles reject
compute calls."""
import ctypes as C
import os
import re

import numpy as np
import pytest

lib_mod = pytest.importorskip("paper_0912_1976_amd")

from inputs import box_mesh  # noqa: E402

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vemg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vemg_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = lib_mod.load_library()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options_are_the_papers_parameters():
    lib = lib_mod.load_library()
    o = lib_mod._lib.Options()
    lib.vemg_default_options(C.byref(o))
    assert o.theta == 0.01 and abs(o.prolong_omega - 2.0 / 3.0) < 1e-15
    assert o.pc == 0 and o.top_bc == 0 and o.precision == 0


def test_status_strings_and_invalid_arguments():
    lib = lib_mod.load_library()
    for st in range(-7, 3):
        assert lib.vemg_status_string(st)
    o = lib_mod._lib.Options()
    lib.vemg_default_options(C.byref(o))
    o.theta = -1.0
    h = C.c_void_p()
    assert lib.vemg_create(C.byref(o), -1, None, C.byref(h)) == -1
    assert lib.vemg_create(None, -1, None, None) == -1
    lib.vemg_default_options(C.byref(o))
    assert o.extrapolation == 0
    o.extrapolation = 2
    assert lib.vemg_create(C.byref(o), -1, None, C.byref(h)) == -1


def test_host_only_handle_rejects_compute():
    m = box_mesh(5, 5, 3, 0.01)
    s = lib_mod.Solver(m.xyz, m.tets, m.top, device=-1)
    lib = s._lib
    dummy = C.c_void_p(16)
    assert lib.vemg_solve(s._h, 1, dummy, dummy, 1e-8, 10, None, None) == -7
    assert lib.vemg_matvec(s._h, dummy, dummy) == -7
    assert lib.vemg_apply(s._h, 0, dummy, dummy) == -7
    # rhs is host-side and works
    b = s.rhs(np.ones(m.n))
    assert np.isfinite(b).all()


def test_plain_c_consumer(tmp_path):
    # the header compiles as strict C99 and a C program drives the library
    # through it; its results match the binding's
    import shutil
    import subprocess

    import numpy as np

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.join(root, "paper_0912_1976_amd")
    exe = tmp_path / "consumer"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(root, "include"), os.path.join(root, "tests", "abi_c", "consumer.c"),
                    "-L", libdir, "-lvemg", "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    m = box_mesh(9, 8, 5, 0.01, jitter=0.3, seed=11, bathymetry=True)
    mesh = tmp_path / "mesh.bin"
    with open(mesh, "wb") as f:
        np.array([m.n, m.tets.shape[0]], dtype=np.int64).tofile(f)
        np.ascontiguousarray(m.xyz, dtype=np.float64).tofile(f)
        np.ascontiguousarray(m.tets, dtype=np.int64).tofile(f)
        np.ascontiguousarray(m.top, dtype=np.uint8).tofile(f)
    out = subprocess.run([str(exe), str(mesh)], check=True, capture_output=True, text=True).stdout.split()
    got = dict(kv.split("=") for kv in out)
    s = lib_mod.Solver(m.xyz, m.tets, m.top, device=-1, coarse_max=16)
    info = s.info()
    perm = s.export("perm", np.int64)
    assert int(got["n"]) == info["n"] and int(got["n_top"]) == info["n_top"]
    assert int(got["nnz_offdiag"]) == info["nnz_offdiag"]
    assert int(got["s_levels"]) == info["s_levels"] and int(got["abar_levels"]) == info["abar_levels"]
    assert int(got["perm_checksum"]) == int(np.sum(perm * np.arange(1, perm.size + 1)))
    assert int(got["solve"]) == -7  # VEMG_ERR_STATE: no device
    # footprint of a host-only handle: counted without a device; b and x of
    # three columns add 2 * 3 * n_nodes doubles
    fp0, fp3 = int(got["footprint0"]), int(got["footprint3"])
    assert fp0 > 0 and int(got["device_bytes"]) == 0
    assert fp3 - fp0 == 2 * 3 * m.n * 8
    assert s.footprint(0) == fp0


def build_consumer(tmp_path):
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.join(root, "paper_0912_1976_amd")
    exe = tmp_path / "consumer"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(root, "include"), os.path.join(root, "tests", "abi_c", "consumer.c"),
                    "-L", libdir, "-lvemg", "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    return exe


def write_mesh(path, m):
    with open(path, "wb") as f:
        np.array([m.n, m.tets.shape[0]], dtype=np.int64).tofile(f)
        np.ascontiguousarray(m.xyz, dtype=np.float64).tofile(f)
        np.ascontiguousarray(m.tets, dtype=np.int64).tofile(f)
        np.ascontiguousarray(m.top, dtype=np.uint8).tofile(f)


def test_footprint_arguments():
    m = box_mesh(6, 5, 4, 0.01, jitter=0.2, seed=3)
    s = lib_mod.Solver(m.xyz, m.tets, m.top, device=-1)
    lib = s._lib
    nb = C.c_size_t(0)
    assert lib.vemg_footprint(s._h, -1, C.byref(nb)) == -1
    assert lib.vemg_footprint(s._h, 0, None) == -1
    assert lib.vemg_footprint(None, 0, C.byref(nb)) == -1
    # a larger problem holds more
    big = box_mesh(12, 11, 6, 0.01, jitter=0.2, seed=3)
    sb = lib_mod.Solver(big.xyz, big.tets, big.top, device=-1)
    assert sb.footprint(0) > s.footprint(0) > 0


def test_missing_library_fails_loudly(monkeypatch):
    """Without libvemg.so a Solver cannot be made: ImportError, no fallback."""
    from paper_0912_1976_amd import _lib

    monkeypatch.setattr(_lib, "_LIB", None)
    monkeypatch.setattr(_lib, "library_path", lambda: os.path.join(os.path.dirname(_lib.__file__), "absent.so"))
    m = box_mesh(5, 5, 3, 0.01)
    with pytest.raises(ImportError, match="absent.so"):
        lib_mod.Solver(m.xyz, m.tets, m.top, device=-1)
