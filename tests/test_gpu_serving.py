"""GPU tests of the continuous-batching server: each result equals the same
right-hand side solved alone, admission under a tight HBM budget evicts and
re-uploads meshes without changing results, and the statistics are sane."""
import time

import numpy as np
import pytest

from inputs import box_mesh, fourier_field

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_0912_1976_amd as lib  # noqa: E402  (a missing package fails, never skips)

MESHES = [dict(nx=13, nz=6, H=1e-2, seed=5), dict(nx=23, nz=9, H=4e-3, seed=6), dict(nx=33, nz=9, H=1e-3, seed=7)]


def _meshes():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [box_mesh(c["nx"], c["nx"], c["nz"], c["H"], jitter=0.3, seed=c["seed"], bathymetry=True) for c in MESHES]


def _run_stream(server, meshes, ids, plan, rtol):
    dev = torch.device("cuda", 0)
    subs = []
    for (mi, nrhs, seed, delay) in plan:
        B = np.stack([server.rhs(ids[mi], fourier_field(meshes[mi].xyz, MESHES[mi]["H"], seed + k))
                      for k in range(nrhs)])
        time.sleep(delay)
        rid = server.submit(ids[mi], torch.as_tensor(B, device=dev), rtol=rtol)
        subs.append((rid, mi, B))
    out = []
    for rid, mi, B in subs:
        server.wait(rid, timeout=120.0)
        x, st, its, rel, lat = server.result(rid)
        out.append((mi, B, x.cpu().numpy(), st, its, rel, lat))
    return out


PLAN = [(0, 3, 10, 0.0), (2, 1, 20, 0.001), (1, 8, 30, 0.0), (0, 1, 40, 0.002), (2, 4, 50, 0.0),
        (1, 2, 60, 0.001), (2, 6, 70, 0.0), (0, 5, 80, 0.0), (1, 1, 90, 0.003), (2, 2, 100, 0.0)]


@pytest.mark.parametrize("precision", ["mixed_pc", "fp64"])
def test_results_alone_equal_results_in_the_mix(precision):
    meshes = _meshes()
    print("case serving", precision, flush=True)
    srv = lib.Server(device=0, precision=precision)
    ids = [srv.add_mesh(m.xyz, m.tets, m.top) for m in meshes]
    res = _run_stream(srv, meshes, ids, PLAN, 1e-8)
    st = srv.stats()
    srv.close()
    for mi, B, x, status, its, rel, lat in res:
        print("mesh", mi, "status", status, "iters", its, "relres", ["%.2e" % r for r in rel],
              "latency %.1f ms" % lat, flush=True)
    print("stats", st, flush=True)
    assert st["requests_done"] == len(PLAN)
    assert st["columns_done"] == sum(p[1] for p in PLAN)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"] + 1e-9
    assert st["solves_per_s"] > 0 and 0 < st["mean_slot_occupancy"] <= 1
    alone = {mi: lib.Solver(m.xyz, m.tets, m.top, device=0, precision=precision) for mi, m in enumerate(meshes)}
    worst = 0.0
    for mi, B, x, status, its, rel, lat in res:
        assert status == 0 and max(rel) <= 1e-8
        xa, ita, rela, sta = alone[mi].solve(B, rtol=1e-8)
        xa = xa.cpu().numpy()
        for k in range(B.shape[0]):
            d = np.linalg.norm(x[k] - xa[k]) / np.linalg.norm(xa[k])
            worst = max(worst, d)
    print("max relative difference alone vs mix", worst, flush=True)
    assert worst <= 1e-6


def test_admission_under_tight_budget_evicts_and_reuploads():
    meshes = _meshes()
    foot = sorted(lib.Solver(m.xyz, m.tets, m.top, device=0).info()["device_bytes"] for m in meshes)
    # room for the largest and the smallest mesh, never for all three at once
    budget = int(foot[2] + foot[0] + 0.5 * (foot[1] - foot[0]))
    srv = lib.Server(device=0, hbm_budget=budget)
    ids = [srv.add_mesh(m.xyz, m.tets, m.top) for m in meshes]
    res = _run_stream(srv, meshes, ids, PLAN[:6], 1e-8)
    st = srv.stats()
    srv.close()
    print("stats", st, flush=True)
    assert st["evictions"] > 0 and st["resident_bytes"] <= budget
    for mi, B, x, status, its, rel, lat in res:
        assert status == 0 and max(rel) <= 1e-8


@pytest.mark.parametrize("precision", ["mixed_pc", "fp64"])
def test_served_results_match_the_oracle(precision):
    """Each served column against the CPU oracle's FP64 solution of the same
    right-hand side (both solved far below 1e-8, so that the comparison
    measures the solvers, not the conditioning of the small-eps meshes)."""
    from oracle import solver as osolver

    meshes = _meshes()
    print("case serving vs oracle", precision, flush=True)
    srv = lib.Server(device=0, precision=precision)
    ids = [srv.add_mesh(m.xyz, m.tets, m.top) for m in meshes]
    plan = [(0, 2, 110, 0.0), (2, 3, 120, 0.0), (1, 1, 130, 0.001), (2, 1, 140, 0.0), (0, 3, 150, 0.0)]
    res = _run_stream(srv, meshes, ids, plan, 1e-11)
    srv.close()
    orc = {mi: osolver.setup(m, "N") for mi, m in enumerate(meshes)}
    tol = 1e-8 if precision == "fp64" else 1e-6
    worst = 0.0
    for mi, B, x, status, its, rel, lat in res:
        assert status == 0 and max(rel) <= 1e-11
        o = orc[mi]
        for k in range(B.shape[0]):
            xo, ito, relo, ok = osolver.solve(o, B[k][o.perm], 1e-12, "vl_as", 3000)
            assert ok
            err = np.linalg.norm(x[k][o.perm] - xo) / np.linalg.norm(xo)
            worst = max(worst, err)
            fixed = np.ones(meshes[mi].n, bool)
            fixed[o.perm] = False
            assert np.all(x[k][fixed] == 0.0)
    print("max relative L2 error of served columns against the oracle", worst, flush=True)
    assert worst <= tol


def test_each_column_stops_on_its_own_request():
    """A loose-tolerance request and a request with a small iteration cap
    share a lane with tight requests: each stops on its own rtol and
    max_iter, with the iteration count it has when solved alone."""
    meshes = _meshes()
    dev = torch.device("cuda", 0)
    m = meshes[2]
    srv = lib.Server(device=0, precision="fp64")
    mid = [srv.add_mesh(mm.xyz, mm.tets, mm.top) for mm in meshes][2]
    B = np.stack([srv.rhs(mid, fourier_field(m.xyz, MESHES[2]["H"], 300 + k)) for k in range(4)])
    Bt = torch.as_tensor(B, device=dev)
    r_tight = srv.submit(mid, Bt[0:2], rtol=1e-10)
    r_loose = srv.submit(mid, Bt[2:3], rtol=1e-4)
    r_cap = srv.submit(mid, Bt[3:4], rtol=1e-10, max_iter=5)
    for r in (r_tight, r_loose, r_cap):
        srv.wait(r, timeout=120.0)
    _, st_t, it_t, rel_t, _ = srv.result(r_tight)
    _, st_l, it_l, rel_l, _ = srv.result(r_loose)
    _, st_c, it_c, rel_c, _ = srv.result(r_cap)
    srv.close()
    alone = lib.Solver(m.xyz, m.tets, m.top, device=0)
    _, it_la, rel_la, st_la = alone.solve(B[2], rtol=1e-4)
    _, it_ta, _, _ = alone.solve(B[0], rtol=1e-10)
    print("tight", st_t, it_t, "loose", st_l, it_l, rel_l, "alone", it_la, "cap", st_c, it_c, rel_c, flush=True)
    assert st_t == 0 and max(rel_t) <= 1e-10 and it_t[0] == it_ta[0]
    assert st_l == 0 and rel_l[0] <= 1e-4 and it_l[0] == it_la[0] < it_t[0]
    assert st_c == 1 and it_c[0] == 5


def test_footprint_is_the_uploaded_size():
    """vemg_footprint (counted at setup without the device) equals the
    device memory the handle holds after its upload, for the solver and for
    the server's lanes; the C consumer sees the same on the device."""
    import subprocess

    from test_abi import build_consumer, write_mesh

    meshes = _meshes()
    srv = lib.Server(device=0)
    for m in meshes:
        s = lib.Solver(m.xyz, m.tets, m.top, device=0)
        info = s.info()
        assert s.footprint(0) == info["device_bytes"] > 0
        assert s.footprint(2) == info["device_bytes"] + 2 * 2 * m.n * 8
        mid = srv.add_mesh(m.xyz, m.tets, m.top)
        assert srv.footprint(mid, 0) == s.footprint(0)
        s.close()
    assert srv.stats()["resident_bytes"] == sum(srv.footprint(i, 0) for i in range(len(meshes)))
    srv.close()
    import pathlib
    import tempfile

    with tempfile.TemporaryDirectory() as d:
        d = pathlib.Path(d)
        exe = build_consumer(d)
        write_mesh(d / "mesh.bin", meshes[0])
        out = subprocess.run([str(exe), str(d / "mesh.bin"), "0"], check=True, capture_output=True,
                             text=True).stdout.split()
    got = dict(kv.split("=") for kv in out)
    print("consumer on the device:", got, flush=True)
    assert int(got["footprint0"]) == int(got["device_bytes"]) > 0
