"""Writes the oracle's FP64 solutions of the full-size workloads, sampled,
as text fixtures for the GPU parity tests and the benchmark's error report.

Only oracle/ and inputs/ are called: the mesh and right-hand side come from
the seeded generators, the oracle assembles, sets up the vertical
extrapolation, both smoothed aggregation hierarchies and solves with PCG
(VL + additive smoother) to the stated tolerance, confirming on its
extended-precision true residual.  Each fixture holds, per right-hand side,
the unknown count, the iterations, the relative residual, the 2-norm of the
solution and its values at seeded sample nodes (natural numbering).

    python tests/golden/make_oracle_samples.py WORKLOAD [--cols 0,1] [--rtol 1e-11] [--mode N|D]
    (several parts: --out PART for each, then --merge PART...)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs import box_mesh, fourier_field, graded_mesh, manufactured_u  # noqa: E402
from oracle import solver as osolver  # noqa: E402

# the full-size workloads (mesh, aspect ratio, right-hand-side seeds)
WORKLOADS = {
    "thinbox-257x257x33-eps1e-4": dict(kind="box", nx=257, nz=33, H=1e-4, jitter=0.3, seed=4, rhs_seed=200),
    "thinbox-129x129x33-eps1e-3": dict(kind="box", nx=129, nz=33, H=1e-3, jitter=0.3, seed=2, rhs_seed=100),
    "graded-hmin1/960-eps1e-3": dict(kind="graded", h_min=1 / 960, H=1e-3, jitter=0.25, seed=3),
}
SAMPLES = 1024


def fixture_path(workload, mode="N"):
    tag = workload.replace("/", "_")
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_samples_{tag}_{mode}.txt")


def build_mesh(wl):
    if wl["kind"] == "box":
        return box_mesh(wl["nx"], wl["nx"], wl["nz"], wl["H"], jitter=wl["jitter"], seed=wl["seed"],
                        bathymetry=True)
    return graded_mesh(wl["h_min"], wl["H"], jitter=wl["jitter"], seed=wl["seed"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--cols", default="0")
    ap.add_argument("--rtol", type=float, default=1e-11)
    ap.add_argument("--mode", default="N", choices=("N", "D"))
    ap.add_argument("--out", help="write here instead of the fixture (to merge later with --merge)")
    ap.add_argument("--merge", nargs="+", metavar="PART", help="merge partial outputs into the fixture and exit")
    args = ap.parse_args()
    if args.merge:
        merged = None
        for part in args.merge:
            with open(part) as fh:
                rec = json.load(fh)
            if merged is None:
                merged = rec
            else:
                assert rec["sample_nodes"] == merged["sample_nodes"] and rec["rtol"] == merged["rtol"]
                merged["columns"].update(rec["columns"])
        merged["columns"] = {k: merged["columns"][k] for k in sorted(merged["columns"], key=int)}
        with open(fixture_path(args.workload, merged["mode"]), "w") as fh:
            json.dump(merged, fh, indent=0)
        return
    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    mesh = build_mesh(wl)
    o = osolver.setup(mesh, args.mode)
    print(f"setup {time.perf_counter() - t0:.1f} s, n = {o.n}", flush=True)
    rng = np.random.default_rng(12345)
    nodes = np.sort(rng.choice(o.perm, size=min(SAMPLES, o.n), replace=False))
    out = {"workload": args.workload, "mode": args.mode, "rtol": args.rtol, "pc": "vl_as", "n": int(o.n),
           "n_nodes": int(mesh.n), "sample_nodes": nodes.tolist(), "columns": {}}
    for c in (int(v) for v in args.cols.split(",")):
        if wl["kind"] == "box":
            f = fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"] + c)
            b = osolver.rhs_from_field(o, f)
            rhs = {"field": "fourier", "seed": wl["rhs_seed"] + c}
        else:
            # manufactured nodal solution: b = A x* (the paper's error protocol)
            b = osolver.rhs_from_solution(o, manufactured_u(mesh.xyz, wl["H"]))
            rhs = {"field": "manufactured", "b": "A x*"}
        t = time.perf_counter()
        x, it, rel, ok = osolver.solve(o, b, args.rtol, "vl_as", 5000)
        xn = osolver.to_natural(o, x)
        print(f"column {c}: {it} iterations, relres {rel:.3e}, {time.perf_counter() - t:.1f} s", flush=True)
        out["columns"][str(c)] = dict(rhs, iterations=int(it), relres=float(rel), converged=bool(ok),
                                      norm2=float(np.linalg.norm(x)),
                                      values=[float.hex(float(v)) for v in xn[nodes]])
    path = args.out or fixture_path(args.workload, args.mode)
    old = {}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
    if old.get("sample_nodes") == out["sample_nodes"] and old.get("rtol") == out["rtol"]:
        old["columns"].update(out["columns"])
        out = old
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
