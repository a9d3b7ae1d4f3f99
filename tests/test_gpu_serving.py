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
