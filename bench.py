"""Benchmark: FP64 vertical-extrapolation multigrid PCG on one MI355X.

Workload (default): thin box 129 x 129 x 33 vertices (549,152 free unknowns),
aspect ratio 1e-3, bathymetric floor z = -H(1 + 0.3 sin 2 pi x sin 2 pi y),
+-0.3 h seeded horizontal jitter of every interior vertex on every layer,
6 P1 tetrahedra per cell, point condition on the top (Neumann elsewhere),
right-hand side b = M f for a seeded 16-mode smooth random field, relative
residual tolerance 1e-8, preconditioner = vertical lumping + additive
smoother.  One step = one complete solve (setup excluded), inputs resident
in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "thinbox-129x129x33-eps1e-3": dict(nx=129, nz=33, H=1e-3, jitter=0.3, seed=2, bathymetry=True, rhs_seed=100),
    "thinbox-257x257x33-eps1e-4": dict(nx=257, nz=33, H=1e-4, jitter=0.3, seed=4, bathymetry=True, rhs_seed=200),
    "thinbox-17x17x9-eps1e-2": dict(nx=17, nz=9, H=1e-2, jitter=0.2, seed=1, bathymetry=False, rhs_seed=100),
}
HBM_PEAK_GBS = 8000.0


def spmv_bytes(info):
    """Algorithmic bytes of one difference-form SpMV over all rows: every
    stored off-diagonal (8-byte value, 4-byte column), and per row the
    deficit d_i, x_i, y_i and one read of x_j (gathers counted once)."""
    return info["nnz_offdiag"] * 12 + info["n"] * 32


def gs_sweep_bytes(info):
    """One forward multicolour sweep: every off-diagonal once (12 B), and
    per row d_i, g_i, the read and write of x_i and one gathered x_j."""
    return info["nnz_offdiag"] * 12 + info["n"] * 40


def cpu_baseline(mesh, wl, iters):
    """The oracle as it stands, single-threaded, timed over `iters` PCG
    iterations of the same solve (setup untimed)."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import numpy as np

    from inputs import fourier_field
    from oracle import pcg, precond, solver as osolver

    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        o = osolver.setup(mesh, "N")
        t_setup = time.perf_counter() - t0
        b = osolver.rhs_from_field(o, fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"]))
        M = precond.make(o, "vl_as")
        t0 = time.perf_counter()
        _, it, _, _ = pcg.pcg(lambda v: osolver.apply_A(o, v), M, b, 0.0, max_iter=iters)
        t = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    return {"value": o.n * it / t, "unit": "DOF*iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{it} PCG iterations of the same solve (oracle setup {t_setup:.1f} s untimed)",
            "seconds": round(t, 3), "cpu": _cpu_model(), "host_cpus": os.cpu_count()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="thinbox-129x129x33-eps1e-3", choices=sorted(WORKLOADS))
    ap.add_argument("--pc", default="vl_as", choices=["vl_as", "vl_sor", "jacobi", "none"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU decomposition is described in DESIGN.md, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    print(f"[bench] workload {args.workload}: building mesh", file=sys.stderr, flush=True)
    mesh = box_mesh(wl["nx"], wl["nx"], wl["nz"], wl["H"], jitter=wl["jitter"], seed=wl["seed"],
                    bathymetry=wl["bathymetry"])
    t0 = time.perf_counter()
    s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc=args.pc, device=0)
    t_setup = time.perf_counter() - t0
    info = s.info()
    b = torch.as_tensor(s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"])), device=dev)
    print(f"[bench] setup {t_setup:.2f} s, n={info['n']}; warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        x, its, rel, st = s.solve(b, rtol=args.rtol, max_iter=5000)
    torch.cuda.synchronize()
    times, iters, rels = [], [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, its, rel, st = s.solve(b, rtol=args.rtol, max_iter=5000)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        iters.append(its[0])
        rels.append(rel[0])
    total = sum(times)
    n = info["n"]
    value = n * sum(iters) / total
    print(f"[bench] {args.steps} solves, iters {iters[0]}, {1e3 * total / args.steps:.2f} ms/solve",
          file=sys.stderr, flush=True)

    # live per-kernel timing (HIP events on the library's stream)
    ms_spmv, _ = s.time_op(vemg.OP_A, reps=50)
    ms_gs, nl_gs = s.time_op(vemg.OP_GS_FWD, reps=20)
    bw_spmv = spmv_bytes(info) / (ms_spmv * 1e-3) / 1e9
    bw_gs = gs_sweep_bytes(info) / (ms_gs * 1e-3) / 1e9
    # per iteration the fine A is swept twice by SOR (pre and post smoothing)
    # and applied twice as SpMV (CG product and smoother residual)
    if 2 * ms_gs >= 2 * ms_spmv:
        dom = {"kernel": "k_gs<true> (fine multicolour SOR sweep)", "bytes": gs_sweep_bytes(info) / nl_gs,
               "ms": ms_gs / nl_gs, "launches_per_sweep": nl_gs}
    else:
        dom = {"kernel": "k_spmv<true,*> (fine difference-form SpMV)", "bytes": spmv_bytes(info), "ms": ms_spmv}
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(mesh, wl, args.cpu_iters)

    line = {
        "metric": "DOF-iters/s, time to 1e-8 rel residual; solves/s + p50/p99 (mixed vs FP64)",
        "value": value,
        "unit": "DOF*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_dof": n, "rtol": args.rtol, "precond": args.pc,
                   "top": "point condition (Neumann elsewhere)", "precision": "fp64"},
        "iterations": iters[0],
        "time_to_tol_ms": 1e3 * float(np.median(times)),
        "solves_per_s": args.steps / total,
        "relres": max(rels),
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom["kernel"],
                     "bytes_per_launch": dom["bytes"], "ms_per_launch": dom["ms"]},
        "kernels": {"spmv_ms": ms_spmv, "spmv_GBs": bw_spmv, "gs_sweep_ms": ms_gs, "gs_sweep_GBs": bw_gs,
                    "gs_launches": nl_gs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
