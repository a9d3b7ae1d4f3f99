"""Benchmark of the vertical-extrapolation multigrid PCG on one MI355X.

Headline workload: thin box 129 x 129 x 33 vertices (549,152 free unknowns),
aspect ratio 1e-3, bathymetric floor z = -H(1 + 0.3 sin 2 pi x sin 2 pi y),
+-0.3 h seeded horizontal jitter of every interior vertex on every layer,
6 P1 tetrahedra per cell, point condition on the top (Neumann elsewhere),
right-hand side b = M f for a seeded 16-mode smooth random field, relative
residual tolerance 1e-8, vertical lumping + additive smoother, FP64.  One
step = one complete solve (setup excluded), inputs resident in HBM.

Also measured (reported beside the headline in the same JSON line): eight
right-hand sides per launch, the two mixed-precision forms, the serving
stream over six resident meshes (continuous batching; saturated and Poisson
arrivals; mixed precision vs FP64), the free-surface (Robin) top, plain
smoothed aggregation against the lumping method at three aspect ratios, the
projected vs SSPAI-refitted extrapolation, the 257 x 257 x 33 and graded
multiscale configurations, live kernel timings for the roofline, and the
CPU oracle on a bounded sample of the headline solve.

Profiling helpers (no GPU): --pmc-summary and --pmc-traffic read rocprofv3
counter passes (FETCH_SIZE, WRITE_SIZE) of --profile-kernels runs;
--trace-timed reads a kernel trace of a bench run and averages the hot
kernels' dispatches over the live timing after the solves.
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
# serving meshes: (n, layers, H), seeds 5..10 -> 10,625 ... 2,179,617 nodes
SERVE_MESHES = [(25, 17, 1e-2), (49, 21, 4e-3), (97, 21, 1.6e-3), (129, 33, 6.3e-4), (177, 33, 2.5e-4),
                (257, 33, 1e-4)]
HBM_PEAK_GBS = 8000.0
# aspect ratios of the paper's comparison of smoothed aggregation against the
# lumping method (Section 6, Figs. iso_no_vl_eps and iso_vl_eps)
SA_COMPARISON_EPS = (1e-2, 1e-3, 1e-4)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def spmv_bytes(info, K=1, elt=8, val=8):
    """Algorithmic bytes of one difference-form SpMV over all rows: every
    stored off-diagonal (value + 4-byte column), per row the deficit (or the
    two FP32 row factors) and, per column of the batch, x_i, y_i and one
    gathered x_j."""
    return info["nnz_offdiag"] * (val + 4) + info["n"] * (8 + 3 * elt * K)


def gs_sweep_bytes(info, K=1, elt=8, val=8):
    """One forward multicolour sweep: every off-diagonal once, per row the
    row factors and, per column, g_i, the read and write of x_i and one
    gathered x_j."""
    return info["nnz_offdiag"] * (val + 4) + info["n"] * (8 + 4 * elt * K)


def coarse_gs_bytes(info, level=1, K=1, elt=8, val=8):
    """One forward multicolour sweep on a coarse A_bar level (CSR, standard
    form without the diagonal): every off-diagonal once (value + column), per
    row the row pointer, the diagonal and, per column, g_i, the read and
    write of x_i and one gathered x_j."""
    off = info["abar_nnz"][level] - info["abar_rows"][level]
    return off * (val + 4) + info["abar_rows"][level] * (4 + 8 + 4 * elt * K)


def restrict_bytes(info, K=1, elt=8, val=8):
    """The restriction g = E~^T r (CSR of E~^T): every stored entry (value +
    column), r read once, per surface row the row pointer and the output."""
    return info["e_nnz"] * (val + 4) + info["n"] * elt * K + info["n_top"] * (4 + elt * K)


def prolong_bytes(info, K=1, elt=8, val=8):
    """The prolongation z += E~ y: every stored entry (value + column), z read
    and written once, y read once."""
    return info["e_nnz"] * (val + 4) + 2 * info["n"] * elt * K + info["n_top"] * elt * K


def kernel_rates(s, info, vemg, K=1, reps=20):
    """Live per-application times of the hot operators of one iteration
    (HIP events on the library's stream) and their algorithmic rates."""
    out = {}
    for name, op, nbytes in (("spmv", vemg.OP_A, spmv_bytes(info, K)),
                             ("fine_sweep", vemg.OP_GS_FWD, gs_sweep_bytes(info, K)),
                             ("coarse_sweep", vemg.OP_GS_COARSE, coarse_gs_bytes(info, K=K)),
                             ("restrict_Et", vemg.OP_ET, restrict_bytes(info, K)),
                             ("prolong_E", vemg.OP_E, prolong_bytes(info, K))):
        try:
            ms, nl = s.time_op(op, reps=reps, nrhs=K)
        except vemg.VemgError:
            continue
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "launches": nl, "bytes": nbytes, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


# Fine-level sweeps, fine SpMVs and coarse (first coarse level of A_bar and
# the surface operator) sweeps per PCG iteration, by preconditioner:
#   vl_as:  SOR cycle (2 fine sweeps, 1 residual SpMV, 2 sweeps on S) and the
#           A_bar V-cycle (2 fine sweeps over the non-top rows, 1 residual
#           SpMV, 2 sweeps on A_bar level 1), plus the CG product
#   vl_sor: the SOR cycle alone plus the CG product
#   vl_add: both V-cycles without the SOR cycle plus the CG product
PER_ITERATION = {"vl_as": (4, 3, 4), "vl_sor": (2, 2, 2), "vl_add": (2, 2, 4), "jacobi": (0, 1, 0),
                 "none": (0, 1, 0)}
KERNEL_NAMES = {"gs": "k_gs<double, 1, false> (fine multicolour SOR, one colour per launch)",
                "spmv": "k_spmv<double, 1, 0, true> (fine difference-form SpMV fused with p.q)",
                "cgs": "k_csr_gs<double, 1, 32, false> (coarse multicolour SOR, one colour per launch)",
                "et": "k_csr_spmv<double, 1, 64, 2> (restriction E~^T, CSR, 64 lanes per surface row)",
                "e": "k_rect<double, 1, true> (prolongation z += E~ y, SELL, one thread per fine row)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_0912_1976_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel's reading),
    or None when there is none for this kernel and workload or the kernel
    sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != _kernel_source_hash() or rec.get("workload") != workload:
        return None
    k = rec.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("hbm_bytes_per_launch")


def profile_kernels(workload, K=1):
    """The hot kernels of one PCG iteration for K right-hand sides, each
    repeated, plus a plain copy of known size (the calibration of the PMC
    byte counters): the command profiled by the rocprofv3 --pmc passes."""
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh

    wl = WORKLOADS[workload]
    mesh = box_mesh(wl["nx"], wl["nx"], wl["nz"], wl["H"], jitter=wl["jitter"], seed=wl["seed"],
                    bathymetry=wl["bathymetry"])
    s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc="vl_as", device=0)
    info = s.info()
    for name, op in (("fine sweep", vemg.OP_GS_FWD), ("fine spmv", vemg.OP_A), ("coarse sweep", vemg.OP_GS_COARSE),
                     ("restriction E~^T", vemg.OP_ET), ("prolongation E~", vemg.OP_E)):
        ms, nl = s.time_op(op, reps=10, nrhs=K)
        print(f"[profile] {name} (K={K}): {ms:.4f} ms per application, {nl} launches", flush=True)
    a = torch.ones(CALIBRATION_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(f"[profile] calibration: 3 elementwise products reading and writing {CALIBRATION_BYTES} bytes each; "
          f"n={info['n']} nnz_offdiag={info['nnz_offdiag']}", flush=True)


CALIBRATION_BYTES = 512 << 20
PMC_KERNELS = {"gs": "k_gs<double, 1, false>", "spmv": "k_spmv<double, 1, 0, true>",
               "cgs": "k_csr_gs<double, 1, 32, false>", "et": "k_csr_spmv<double, 1, 64, 2>",
               "e": "k_rect<double, 1, true>", "calibration": "MulFunctor"}


def _pmc_means(path, counter):
    import csv
    import glob
    files = [path] if path.endswith(".csv") else glob.glob(os.path.join(path, "**", "*counter_collection.csv"),
                                                          recursive=True)
    out = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                for key, pat in PMC_KERNELS.items():
                    if pat in row["Kernel_Name"]:
                        t = out.setdefault(key, [0.0, 0])
                        t[0] += float(row["Counter_Value"])
                        t[1] += 1
    return {k: v[0] / v[1] for k, v in out.items()}


def pmc_traffic(fetch_dir, write_dir, workload):
    """HBM-side bytes per launch of the hot kernels from the two PMC passes:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each divided by what the
    same counter reads for the calibration product (CALIBRATION_BYTES read
    and written once) relative to its true size."""
    fetch = _pmc_means(fetch_dir, "FETCH_SIZE")
    write = _pmc_means(write_dir, "WRITE_SIZE")
    kib = CALIBRATION_BYTES / 1024.0
    ff, wf = fetch["calibration"] / kib, write["calibration"] / kib
    rec = {"workload": workload, "source_hash": _kernel_source_hash(),
           "calibration": {"bytes": CALIBRATION_BYTES, "fetch_factor": ff, "write_factor": wf},
           "commands": [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fetch_dir} -o run -- "
                        f"python3 -u bench.py --profile-kernels --workload {workload}",
                        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {write_dir} -o run -- "
                        f"python3 -u bench.py --profile-kernels --workload {workload}",
                        f"python3 bench.py --pmc-traffic {fetch_dir} {write_dir} --workload {workload}"],
           "kernels": {}}
    for key in ("gs", "spmv", "cgs", "et", "e"):
        if key in fetch and key in write:
            rec["kernels"][key] = {"kernel": KERNEL_NAMES[key], "fetch_kib": fetch[key], "write_kib": write[key],
                                   "hbm_bytes_per_launch": 1024.0 * (fetch[key] / ff + write[key] / wf)}
    print(json.dumps(rec, indent=1))


def trace_timed(path):
    """Mean dispatch duration of each hot kernel over the live timing that
    follows the solves (its last run of consecutive dispatches, fills between
    them allowed), from a rocprofv3 kernel-trace CSV: the figure to set beside
    the per-launch times bench.py measures with HIP events."""
    import csv
    import glob
    files = [path] if path.endswith(".csv") else glob.glob(os.path.join(path, "**", "*kernel_trace.csv"),
                                                          recursive=True)
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows += [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in csv.DictReader(fh)]
    rows.sort()
    out = {}
    for key in ("spmv", "gs", "cgs"):
        pat = PMC_KERNELS[key]
        run, last = [], []
        for t0, t1, name in rows:
            if pat in name:
                run.append(t1 - t0)
            elif "k_fill<" not in name:
                if run:
                    last = run
                run = []
        if run:
            last = run
        if last:
            out[key] = {"kernel": KERNEL_NAMES[key], "dispatches": len(last),
                        "mean_us": sum(last) / len(last) / 1e3}
    print(json.dumps(out, indent=1))


def pmc_summary(paths):
    """Mean of each PMC counter per kernel over the dispatches of rocprofv3
    counter-collection CSV files (values as the counters report them)."""
    import csv
    import glob
    from collections import defaultdict

    acc = defaultdict(lambda: [0.0, 0])
    for p in paths:
        files = [p] if p.endswith(".csv") else glob.glob(os.path.join(p, "**", "*counter_collection.csv"),
                                                        recursive=True)
        for f in files:
            with open(f, newline="") as fh:
                for row in csv.DictReader(fh):
                    key = (row["Kernel_Name"], row["Counter_Name"])
                    acc[key][0] += float(row["Counter_Value"])
                    acc[key][1] += 1
    print("| dispatches | mean value | counter | kernel |")
    print("|---:|---:|---|---|")
    for (kern, ctr), (tot, cnt) in sorted(acc.items(), key=lambda kv: -kv[1][0]):
        print(f"| {cnt} | {tot / cnt:.1f} | {ctr} | `{kern[:110]}` |")


def timed_solves(s, b, steps, warmup, rtol):
    import torch
    for _ in range(warmup):
        s.solve(b, rtol=rtol, max_iter=5000)
    torch.cuda.synchronize()
    times, iters, rels, sts = [], [], [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, its, rel, st = s.solve(b, rtol=rtol, max_iter=5000)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        iters.append(its)
        rels.append(rel)
        sts.append(st)
    return x, times, iters, rels, sts


def cpu_baseline(mesh, wl, iters):
    """The oracle as it stands, single-threaded, timed over `iters` PCG
    iterations of the headline solve (its setup untimed)."""
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_limits

    from inputs import fourier_field
    from oracle import pcg, precond, solver as osolver

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = osolver.setup(mesh, "N")
        t_setup = time.perf_counter() - t0
        b = osolver.rhs_from_field(o, fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"]))
        M = precond.make(o, "vl_as")
        t0 = time.perf_counter()
        _, it, _, _ = pcg.pcg(lambda v: osolver.apply_A(o, v), M, b, 0.0, max_iter=iters)
        t = time.perf_counter() - t0
    return {"value": o.n * it / t, "unit": "DOF*iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{it} PCG iterations (VL + additive smoother) of the headline solve, oracle setup "
                      f"{t_setup:.1f} s untimed",
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


def serving(nreq, seed, rtol, dev):
    """Stream of solve requests over six resident meshes: each request picks a
    mesh uniformly and 1..8 right-hand sides (seeded).  Run saturated (all
    submitted at once) and with Poisson arrivals at 0.8x the saturated
    request rate, in mixed precision and in FP64."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field

    rng = np.random.default_rng(seed)
    srv = vemg.Server(device=0, precision="mixed_pc")
    meshes, pools, sizes = [], [], []
    t0 = time.perf_counter()
    for i, (nx, nz, H) in enumerate(SERVE_MESHES):
        m = box_mesh(nx, nx, nz, H, jitter=0.3, seed=5 + i, bathymetry=True)
        mid = srv.add_mesh(m.xyz, m.tets, m.top)
        pool = np.stack([srv.rhs(mid, fourier_field(m.xyz, H, 1000 + 16 * i + k)) for k in range(8)])
        pools.append(torch.as_tensor(pool, device=dev))
        meshes.append(mid)
        sizes.append(m.n)
        log(f"serving mesh {i}: {m.n} nodes")
    t_setup = time.perf_counter() - t0
    plan = [(int(rng.integers(0, len(meshes))), int(rng.integers(1, 9))) for _ in range(nreq)]
    cols = [rng.permutation(8)[:k] for _, k in plan]

    def run(rate):
        rids = []
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, nreq) if rate else np.zeros(nreq)
        t_start = time.perf_counter()
        t_next = t_start
        for (mi, k), c, gap in zip(plan, cols, gaps):
            t_next += gap
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            rids.append(srv.submit(meshes[mi], pools[mi][torch.as_tensor(c, device=dev)], rtol=rtol))
        worst, floor = 0, 0
        for rid in rids:
            srv.wait(rid, timeout=600.0)
            x, st, its, rel, lat = srv.result(rid)
            worst = min(worst, st) if st < 0 else max(worst, st)
            floor += int(st == 2)
        s = srv.stats()
        return {"requests": nreq, "columns": int(s["columns_done"]), "solves_per_s": s["solves_per_s"],
                "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"], "mean_ms": s["mean_ms"], "max_ms": s["max_ms"],
                "busy_s": s["busy_s"], "slot_occupancy": s["mean_slot_occupancy"], "worst_status": worst,
                "requests_at_floor": floor, "arrival_rate_per_s": rate}

    out = {"meshes_nodes": sizes, "setup_s": t_setup, "rtol": rtol}
    for prec in ("mixed_pc", "fp64"):
        srv.set_precision(prec)
        sat = run(0.0)
        log(f"serving {prec} saturated: {sat['solves_per_s']:.1f} solves/s p50 {sat['p50_ms']:.1f} ms")
        rate = 0.8 * sat["requests"] / sat["busy_s"]
        srv.set_precision(prec)
        poi = run(rate)
        log(f"serving {prec} poisson {rate:.1f}/s: p50 {poi['p50_ms']:.1f} ms p99 {poi['p99_ms']:.1f} ms")
        out[prec] = {"saturated": sat, "poisson": poi}
    srv.close()
    return out


def config_runs(dev, rtol):
    """The two other single-GPU configurations at full size.
    * 257 x 257 x 33 thin box, eps 1e-4 (2.18M unknowns), eight seeded smooth
      right-hand sides per solve: FP64, FP32 inner PCG inside FP64 iterative
      refinement, and FP32 preconditioner in FP64 CG; solves/s and the error
      of every column against the FP64 solution.
    * Centre-refined multiscale thin box (h_min 1/900, 16-64 layers, eps 1e-3,
      about 3.5M unknowns), b = A x* for the manufactured x*: VL + additive
      smoother against VL + SOR (the paper's Mesh B comparison), iterations,
      time to tolerance and the relative max-norm error against x*."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field, graded_mesh, manufactured_u

    out = {}
    t0 = time.perf_counter()
    m = box_mesh(257, 257, 33, 1e-4, jitter=0.3, seed=4, bathymetry=True)
    s = vemg.Solver(m.xyz, m.tets, m.top, top_bc="pinned", pc="vl_as", device=0)
    B = torch.as_tensor(np.stack([s.rhs(fourier_field(m.xyz, 1e-4, 200 + k)) for k in range(8)]), device=dev)
    rec = {"workload": "thinbox-257x257x33-eps1e-4", "n_dof": s.info()["n"], "rhs_per_solve": 8,
           "setup_s": time.perf_counter() - t0}
    rec["kernels"] = {"K1": kernel_rates(s, s.info(), vemg, 1), "K8": kernel_rates(s, s.info(), vemg, 8, reps=10)}
    x64 = None
    for prec in ("fp64", "mixed_ir", "mixed_pc"):
        s.set_precision(prec)
        x, t, it, rel, st = timed_solves(s, B, 2, 1, rtol)
        r = {"ms_per_batch": 1e3 * float(np.median(t)), "solves_per_s": 8 / float(np.median(t)),
             "iterations": it[0], "max_relres": max(rel[0]), "status": st[0]}
        if x64 is None:
            x64 = x
        else:
            r["max_rel_err_vs_fp64"] = max(float(torch.linalg.norm(x[k] - x64[k]) / torch.linalg.norm(x64[k]))
                                           for k in range(8))
        rec[prec] = r
        log(f"config 4 {prec}: {r['solves_per_s']:.1f} solves/s, iterations {max(r['iterations'])}")
    s.close()
    out["thinbox_257_eps1e-4_batch8"] = rec

    t0 = time.perf_counter()
    m = graded_mesh(1 / 900, 1e-3, jitter=0.25, seed=3)
    s = vemg.Solver(m.xyz, m.tets, m.top, top_bc="pinned", pc="vl_as", device=0)
    info = s.info()
    rec = {"workload": "graded-hmin1/900-eps1e-3", "n_dof": info["n"], "setup_s": time.perf_counter() - t0}
    xs = manufactured_u(m.xyz, 1e-3)
    b = s.matvec(xs)
    free = np.zeros(m.n, bool)
    free[s.export("perm", np.int64)] = True
    for pc in ("vl_as", "vl_sor"):
        s.set_preconditioner(pc)
        x, t, it, rel, st = timed_solves(s, b, 2, 1, rtol)
        xh = x.cpu().numpy()
        err = float(np.max(np.abs(xh[free] - xs[free])) / np.max(np.abs(xs[free])))
        rec[pc] = {"time_to_tol_ms": 1e3 * float(np.median(t)), "iterations": it[0][0], "relres": rel[0][0],
                   "status": st[0], "dof_iters_per_s": info["n"] * it[0][0] / float(np.median(t)),
                   "max_rel_err_vs_manufactured": err}
        log(f"config 3 {pc}: {rec[pc]['iterations']} iterations, {rec[pc]['time_to_tol_ms']:.1f} ms")
    s.close()
    out["graded_multiscale"] = rec
    return out


def sa_baseline_runs(dev, rtol):
    """The paper's comparison (Section 6, Figs. iso_no_vl_eps and iso_vl_eps)
    at the headline size: plain smoothed aggregation PCG against the
    VL + additive smoother preconditioner on the 129 x 129 x 33 box at aspect
    ratios 1e-2, 1e-3 and 1e-4 (same seeds and field as the headline)."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field

    out = {}
    for H in SA_COMPARISON_EPS:
        m = box_mesh(129, 129, 33, H, jitter=0.3, seed=2, bathymetry=True)
        s = vemg.Solver(m.xyz, m.tets, m.top, top_bc="pinned", pc="sa", device=0)
        b = torch.as_tensor(s.rhs(fourier_field(m.xyz, H, 100)), device=dev)
        rec = {}
        for pc in ("sa", "vl_as"):
            s.set_preconditioner(pc)
            x, t, it, rel, st = timed_solves(s, b, 2, 1, rtol)
            rec[pc] = {"iterations": it[0][0], "time_to_tol_ms": 1e3 * float(np.median(t)), "relres": rel[0][0],
                       "status": st[0]}
        out[f"eps={H:g}"] = rec
        log(f"eps {H:g}: SA {rec['sa']['iterations']} iterations ({rec['sa']['time_to_tol_ms']:.0f} ms), "
            f"VL+AS {rec['vl_as']['iterations']} ({rec['vl_as']['time_to_tol_ms']:.0f} ms)")
        s.close()
    return out


def sspai_runs(dev, rtol):
    """The two extrapolations of Section 5.4 side by side: the vertical
    projection and its pattern refitted from the operator (sparse approximate
    inverse), VL + additive smoother, on a 65 x 65 x 17 box of the headline
    kind (jittered columns, bathymetry) at aspect ratios 1 to 1e-3, and on
    vertical columns (no jitter, flat floor) at 1e-3."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field

    out = {}
    cases = [(H, 0.3, True) for H in (1.0, 1e-1, 1e-2, 1e-3)] + [(1e-3, 0.0, False)]
    for H, jit, bat in cases:
        m = box_mesh(65, 65, 17, H, jitter=jit, seed=2, bathymetry=bat)
        rec = {}
        for ex in ("projection", "sspai"):
            t0 = time.perf_counter()
            s = vemg.Solver(m.xyz, m.tets, m.top, top_bc="pinned", pc="vl_as", device=0, extrapolation=ex)
            setup_s = time.perf_counter() - t0
            b = torch.as_tensor(s.rhs(fourier_field(m.xyz, H, 100)), device=dev)
            x, t, it, rel, st = timed_solves(s, b, 2, 1, rtol)
            rec[ex] = {"iterations": it[0][0], "time_to_tol_ms": 1e3 * float(np.median(t)), "relres": rel[0][0],
                       "status": st[0], "setup_s": setup_s}
            s.close()
        key = f"eps={H:g}" + ("" if jit else ",vertical-columns")
        out[key] = rec
        log(f"{key}: projection {rec['projection']['iterations']} iterations, "
            f"SSPAI {rec['sspai']['iterations']} (setup {rec['sspai']['setup_s']:.2f} s vs "
            f"{rec['projection']['setup_s']:.2f} s)")
    return out


def robin_runs(mesh, wl, dev, rtol):
    """The headline mesh with the free-surface (Robin) top instead of the point
    condition: alpha H = H / (g dt^2) of 3e-5 (a 4 km ocean and a one-hour
    step: close to the Neumann limit) and 3e-2 (a step of a few minutes)."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import fourier_field

    out = {}
    for aH in (3e-5, 3e-2):
        alpha = aH / wl["H"]
        s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="robin", robin_alpha=alpha, pc="vl_as", device=0)
        b = torch.as_tensor(s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"])), device=dev)
        x, t, it, rel, st = timed_solves(s, b, 3, 1, rtol)
        out[f"alphaH={aH:g}"] = {"alpha": alpha, "iterations": it[0][0], "time_to_tol_ms": 1e3 * float(np.median(t)),
                                 "relres": rel[0][0], "status": st[0]}
        log(f"robin alpha H = {aH:g}: {it[0][0]} iterations, {1e3 * float(np.median(t)):.1f} ms")
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="thinbox-129x129x33-eps1e-3", choices=sorted(WORKLOADS))
    ap.add_argument("--pc", default="vl_as", choices=sorted(PER_ITERATION))
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline solve and roofline only")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests per serving stream (four streams: mixed and FP64, saturated and Poisson); "
                         "the full serving configuration is 512, about seven minutes more than the default")
    ap.add_argument("--no-configs", action="store_true", help="skip the full-size 257^2 and graded configurations")
    ap.add_argument("--profile-batch", type=int, default=1, choices=(1, 2, 4, 8),
                    help="right-hand sides per launch for --profile-kernels")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="run only the hot kernels and a copy calibration (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-summary", nargs="+", metavar="DIR_OR_CSV",
                    help="summarise rocprofv3 counter-collection output and exit (no GPU)")
    ap.add_argument("--trace-timed", metavar="DIR_OR_CSV",
                    help="mean trace duration of the hot kernels over the live timing after the solves (no GPU)")
    ap.add_argument("--pmc-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="per-launch HBM bytes of the hot kernels from the two PMC passes, as JSON (no GPU)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.trace_timed:
        trace_timed(args.trace_timed)
        return
    if args.pmc_traffic:
        pmc_traffic(*args.pmc_traffic, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the decomposition over several GPUs is designed, not built).", file=sys.stderr)
        sys.exit(2)

    if args.profile_kernels:
        profile_kernels(args.workload, args.profile_batch)
        return

    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import box_mesh, fourier_field

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    log(f"workload {args.workload}: building mesh")
    mesh = box_mesh(wl["nx"], wl["nx"], wl["nz"], wl["H"], jitter=wl["jitter"], seed=wl["seed"],
                    bathymetry=wl["bathymetry"])
    t0 = time.perf_counter()
    s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc=args.pc, device=0)
    t_setup = time.perf_counter() - t0
    info = s.info()
    n = info["n"]
    b1 = torch.as_tensor(s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"])), device=dev)
    log(f"setup {t_setup:.2f} s, n={n}; timing {args.steps} FP64 solves")
    x64, times, iters, rels, sts = timed_solves(s, b1, args.steps, args.warmup, args.rtol)
    total = sum(times)
    its = iters[0][0]
    value = n * sum(i[0] for i in iters) / total
    log(f"FP64: {its} iterations, {1e3 * total / args.steps:.2f} ms/solve, relres {rels[0][0]:.2e}")

    # live per-kernel timing (HIP events on the library's stream)
    ms_spmv, _ = s.time_op(vemg.OP_A, reps=50)
    ms_gs, nl_gs = s.time_op(vemg.OP_GS_FWD, reps=20)
    try:
        ms_cgs, nl_cgs = s.time_op(vemg.OP_GS_COARSE, reps=20)
    except vemg.VemgError:  # A_bar has no coarse level above the coarsest
        ms_cgs, nl_cgs = 0.0, 1
    n_gs, n_spmv, n_cgs = PER_ITERATION[args.pc]
    share = {"gs": n_gs * ms_gs, "spmv": n_spmv * ms_spmv, "cgs": n_cgs * ms_cgs}
    dom_key = max(share, key=share.get)
    dom = {"gs": (gs_sweep_bytes(info) / nl_gs, ms_gs / nl_gs),
           "spmv": (spmv_bytes(info), ms_spmv),
           "cgs": (coarse_gs_bytes(info) / nl_cgs, ms_cgs / nl_cgs)}[dom_key]
    achieved = dom[0] / (dom[1] * 1e-3) / 1e9
    traffic = measured_traffic(dom_key, args.workload)

    extras = {}
    if not args.no_extras:
        B8 = torch.as_tensor(np.stack([s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"] + k))
                                       for k in range(8)]), device=dev)
        xb, tb, ib, rb, _ = timed_solves(s, B8, 3, 1, args.rtol)
        extras["fp64_batch8"] = {"solves_per_s": 8 * 3 / sum(tb), "ms_per_batch": 1e3 * sum(tb) / 3,
                                 "iterations": ib[0], "max_relres": max(rb[0])}
        extras["kernels_batch8"] = kernel_rates(s, info, vemg, 8, reps=10)
        extras["transfers"] = {k: v for k, v in kernel_rates(s, info, vemg, 1).items()
                               if k in ("restrict_Et", "prolong_E")}
        log(f"FP64 x8: {extras['fp64_batch8']['solves_per_s']:.1f} solves/s")
        for prec in ("mixed_ir", "mixed_pc"):
            sm = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc=args.pc, device=0, precision=prec)
            xm, tm, im, rm, stm = timed_solves(sm, b1, max(3, args.steps // 2), 1, args.rtol)
            err = float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))
            xmb, tmb, imb, rmb, _ = timed_solves(sm, B8, 3, 1, args.rtol)
            errb = float(torch.linalg.norm(xmb - xb) / torch.linalg.norm(xb))
            rec = {"time_to_tol_ms": 1e3 * float(np.median(tm)), "iterations": im[0][0], "relres": rm[0][0],
                   "status": stm[0], "rel_err_vs_fp64": err, "batch8_solves_per_s": 8 * 3 / sum(tmb),
                   "batch8_rel_err_vs_fp64": errb}
            if prec == "mixed_ir":
                ms32, _ = sm.time_op(vemg.OP_A, reps=50)
                rec["spmv32_ms"] = ms32
                rec["spmv32_GBs"] = spmv_bytes(info, 1, 4, 4) / (ms32 * 1e-3) / 1e9
            extras[prec] = rec
            log(f"{prec}: {rec['time_to_tol_ms']:.1f} ms, iters {rec['iterations']}, err {err:.1e}")
            sm.close()
        log("serving stream")
        extras["serving"] = serving(args.serve_requests, 11, args.rtol, dev)
        extras["robin_top"] = robin_runs(mesh, wl, dev, args.rtol)
        extras["sa_baseline"] = sa_baseline_runs(dev, args.rtol)
        extras["sspai_extrapolation"] = sspai_runs(dev, args.rtol)
        if not args.no_configs:
            extras["configs"] = config_runs(dev, args.rtol)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
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
                   "top": "point condition (Neumann elsewhere)", "precision": "fp64", "rhs_per_solve": 1},
        "iterations": its,
        "time_to_tol_ms": 1e3 * float(np.median(times)),
        "solves_per_s": args.steps / total,
        "relres": max(r[0] for r in rels),
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": KERNEL_NAMES[dom_key],
                     "bytes_per_launch": dom[0], "ms_per_launch": dom[1]},
        "kernels": {"spmv_ms": ms_spmv, "spmv_GBs": spmv_bytes(info) / (ms_spmv * 1e-3) / 1e9,
                    "gs_sweep_ms": ms_gs, "gs_sweep_GBs": gs_sweep_bytes(info) / (ms_gs * 1e-3) / 1e9,
                    "gs_launches": nl_gs, "coarse_sweep_ms": ms_cgs,
                    "coarse_sweep_GBs": coarse_gs_bytes(info) / (ms_cgs * 1e-3) / 1e9 if ms_cgs else None,
                    "coarse_launches": nl_cgs,
                    "ms_per_iteration_estimate": share},
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
