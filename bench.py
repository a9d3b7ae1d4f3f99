"""Benchmark of the vertical-extrapolation multigrid PCG on one MI355X.

Headline workload (one step = one solve of a batch of right-hand sides,
setup excluded, inputs resident in HBM): the thin box of 257 x 257 x 33
vertices (2,179,616 free unknowns), aspect ratio 1e-4, bathymetric floor
z = -H(1 + 0.3 sin 2 pi x sin 2 pi y), +-0.3 h seeded horizontal jitter of
every interior vertex on every layer, 6 P1 tetrahedra per cell, point
condition on the top (Neumann elsewhere), eight right-hand sides b = M f of
seeded 16-mode smooth random fields solved together (one SpMM-style batch),
relative residual 1e-8 for every column, vertical lumping + additive
smoother, FP64.  value = unknowns x iterations summed over the columns, per
second.

Beside it in the same JSON line: the mixed-precision forms on the same batch
with every column's error against the FP64 oracle (sampled fixture), the
dominant kernel's roofline and the whole iteration's algorithmic bytes
against its time, the other configurations (17 x 17 x 9 at 1e-10 and the
129 x 129 x 33 box, each with the point condition and the Dirichlet top;
the 4.0M-unknown graded multiscale mesh; the 512-request serving stream over
six resident meshes, mixed precision against FP64), and the CPU oracle
timed on a bounded sample of the headline workload in a child process on
one host core (it runs while the GPU is measured), then on the 17x17x9 box
(a whole solve) and a sample of the 129x129x33 box, reported per
configuration beside the headline's.  --paper-comparisons adds
the comparisons of Section 6 (smoothed aggregation against the lumping
method, VL + SOR), the free-surface top and the SSPAI extrapolation.

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
    "thinbox-257x257x33-eps1e-4": dict(kind="box", nx=257, nz=33, H=1e-4, jitter=0.3, seed=4, bathymetry=True,
                                       rhs_seed=200, nrhs=8, rtol=1e-8),
    "thinbox-129x129x33-eps1e-3": dict(kind="box", nx=129, nz=33, H=1e-3, jitter=0.3, seed=2, bathymetry=True,
                                       rhs_seed=100, nrhs=1, rtol=1e-8),
    "thinbox-17x17x9-eps1e-2": dict(kind="box", nx=17, nz=9, H=1e-2, jitter=0.2, seed=1, bathymetry=False,
                                    rhs_seed=100, nrhs=1, rtol=1e-10),
    "graded-hmin1/960-eps1e-3": dict(kind="graded", h_min=1 / 960, H=1e-3, jitter=0.25, seed=3, nrhs=1,
                                     rtol=1e-8),
}
HEADLINE = "thinbox-257x257x33-eps1e-4"
# serving meshes: (n, layers, H), seeds 5..10 -> 10,625 ... 2,179,617 nodes
SERVE_MESHES = [(25, 17, 1e-2), (49, 21, 4e-3), (97, 21, 1.6e-3), (129, 33, 6.3e-4), (177, 33, 2.5e-4),
                (257, 33, 1e-4)]
HBM_PEAK_GBS = 8000.0
# aspect ratios of the paper's comparison of smoothed aggregation against the
# lumping method (Section 6, Figs. iso_no_vl_eps and iso_vl_eps)
SA_COMPARISON_EPS = (1e-2, 1e-3, 1e-4)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_mesh(wl):
    from inputs import box_mesh, graded_mesh
    if wl["kind"] == "graded":
        return graded_mesh(wl["h_min"], wl["H"], jitter=wl["jitter"], seed=wl["seed"])
    return box_mesh(wl["nx"], wl["nx"], wl["nz"], wl["H"], jitter=wl["jitter"], seed=wl["seed"],
                    bathymetry=wl["bathymetry"])


# ---------------------------------------------------------------------------
# Algorithmic bytes: what each kernel must move at least, every stored array
# (without padding) and every vector read or written once per pass, from the
# sizes of the built arrays (vemg_info).  T = bytes per vector value, V = per
# matrix value, K = columns of the batch; column indices and row pointers are
# 4 bytes.  Fine rows carry one 8-byte row datum (the deficit in FP64, the two
# FP32 row factors in mixed precision).
# ---------------------------------------------------------------------------

def spmv_bytes(info, K=1, elt=8, val=8, residual=False, rows=None, nnz=None):
    """Difference-form SpMV y = A x (or y = g - A x): the off-diagonals and
    the row datum, x read and y written (and g read)."""
    n = info["n"] if rows is None else rows
    nnz = info["nnz_offdiag"] if nnz is None else nnz
    return nnz * (val + 4) + n * 8 + (3 if residual else 2) * n * elt * K


def gs_sweep_bytes(info, K=1, elt=8, val=8, rows=None, nnz=None):
    """One multicolour sweep (all colours): the off-diagonals and row datum,
    g read, x read and written once."""
    n = info["n"] if rows is None else rows
    nnz = info["nnz_offdiag"] if nnz is None else nnz
    return nnz * (val + 4) + n * 8 + 3 * n * elt * K


def csr_level_bytes(rows, off, K, elt, val):
    """Coarse square level (CSR, diagonal apart): one sweep, and one residual."""
    sweep = off * (val + 4) + rows * (4 + 8) + 3 * rows * elt * K
    return sweep, sweep


def transfer_bytes(p_nnz, rows, rows_c, K, elt, val):
    """Restriction (CSR of P^T: rows_c rows) and prolongation added into the
    fine vector (P: rows rows)."""
    restrict = p_nnz * (val + 4) + rows_c * 4 + rows * elt * K + rows_c * elt * K
    prolong = p_nnz * (val + 4) + rows * 4 + rows_c * elt * K + 2 * rows * elt * K
    return restrict, prolong


def coarse_gs_bytes(info, level=1, K=1, elt=8, val=8):
    """One forward sweep on A_bar level `level` (all its colours)."""
    return csr_level_bytes(info["abar_rows"][level], info["abar_nnz"][level], K, elt, val)[0]


def restrict_bytes(info, K=1, elt=8, val=8):
    """g = E~^T r (CSR of E~^T, rows in spatial order with a map back)."""
    m = info["n_top"]
    return info["e_nnz"] * (val + 4) + m * (4 + 4) + info["n"] * elt * K + m * elt * K


def prolong_bytes(info, K=1, elt=8, val=8):
    """z += E~ y: the entries, y read, z read and written."""
    return info["e_nnz"] * (val + 4) + info["n_top"] * elt * K + 2 * info["n"] * elt * K


def vcycle_bytes(rows, off, pnnz, K, elt, val, fine_rows=None, fine_nnz=None):
    """One V(1,1)-cycle: per level two sweeps, the residual, the restriction
    and the prolongation; the coarsest level's dense inverse.  The finest
    level of A_bar is the fine SELL operator's non-top rows."""
    total = 0
    L = len(rows)
    for l in range(L):
        m = rows[l]
        if l == L - 1:
            total += m * m * 8 + 2 * m * elt * K
            break
        if l == 0 and fine_rows is not None:
            sw = gs_sweep_bytes(None, K, elt, val, rows=fine_rows, nnz=fine_nnz)
            res = spmv_bytes(None, K, elt, val, residual=True, rows=fine_rows, nnz=fine_nnz)
        else:
            sw, res = csr_level_bytes(m, off[l], K, elt, val)
        r, p = transfer_bytes(pnnz[l], m, rows[l + 1], K, elt, val)
        total += 2 * sw + res + r + p
    return total


# The library's additive smoother takes the SOR cycle's fine forward sweep and
# residual on meshes of this many fine unknowns or more (the rows where the
# two differ, a few per cent, are swept again; their bytes are not counted).
SHARE_MIN_ROWS = 1000000


def iteration_bytes(info, K=1, pc="vl_as", precision="fp64"):
    """Algorithmic bytes of one PCG iteration (preconditioner included) for a
    batch of K columns, from the built arrays' sizes.  Mixed precision: the
    preconditioner in FP32 (values and vectors), the Krylov part in FP64, plus
    the demotion of r and promotion of z.  With the shared forward sweep the
    additive smoother's fine sweep and residual are replaced by the SOR
    cycle's stores of x and r into the smoother's vectors."""
    n = info["n"]
    pe, pv = (4, 4) if precision != "fp64" else (8, 8)
    krylov = spmv_bytes(info, K) + 6 * n * 8 * K + 3 * n * 8 * K   # q = A p with p.q; x, r update; p = z + beta p
    sor = (2 * gs_sweep_bytes(info, K, pe, pv) + spmv_bytes(info, K, pe, pv, residual=True)
           + restrict_bytes(info, K, pe, pv) + prolong_bytes(info, K, pe, pv)) if info["n_top"] else 0
    s_cycle = vcycle_bytes(info["s_rows"], info["s_nnz"], info["p_nnz_s"], K, pe, pv) if info["n_top"] else 0
    nbar = info["n"] - info["n_top"]
    a_cycle = vcycle_bytes(info["abar_rows"], info["abar_nnz"], info["p_nnz_abar"], K, pe, pv,
                           fine_rows=nbar, fine_nnz=info["abar_nnz"][0])
    if pc == "vl_as" and info["n_top"] and n >= SHARE_MIN_ROWS:
        a_cycle -= (gs_sweep_bytes(None, K, pe, pv, rows=nbar, nnz=info["abar_nnz"][0])
                    + spmv_bytes(None, K, pe, pv, residual=True, rows=nbar, nnz=info["abar_nnz"][0]))
        a_cycle += 2 * nbar * pe * K
    join = 4 * n * pe * K + n * 8 * K  # z += w over the non-top rows with r.z; (mixed) r read for the dot
    mixed = (n * 8 * K + n * 4 * K) * 2 if precision != "fp64" else 0
    if pc == "vl_sor":
        return krylov + sor + s_cycle + n * pe * K * 2 + mixed
    if pc == "vl_add":
        return (krylov + restrict_bytes(info, K, pe, pv) + s_cycle + a_cycle + prolong_bytes(info, K, pe, pv)
                + join + mixed)
    return krylov + sor + s_cycle + a_cycle + join + mixed


def coarsest_bytes(info, K=1, elt=8):
    """The surface hierarchy's coarsest dense inverse times a vector: the FP64
    inverse streamed once, g read and x written."""
    m = info["s_rows"][info["s_levels"] - 1] if info["s_levels"] else 0
    return m * m * 8 + 2 * m * elt * K


def kernel_rates(s, info, vemg, K=1, reps=20, precision="fp64"):
    """Live per-application times of the hot operators of one iteration
    (HIP events on the library's stream) and their algorithmic rates."""
    pe, pv = (4, 4) if precision == "mixed_ir" else (8, 8)
    out = {}
    for name, op, nbytes in (("spmv", vemg.OP_A, spmv_bytes(info, K, pe, pv)),
                             ("fine_sweep", vemg.OP_GS_FWD, gs_sweep_bytes(info, K, pe, pv)),
                             ("coarse_sweep", vemg.OP_GS_COARSE, coarse_gs_bytes(info, 1, K, pe, pv)),
                             ("coarsest_dense", vemg.OP_COARSEST, coarsest_bytes(info, K, pe)),
                             ("restrict_Et", vemg.OP_ET, restrict_bytes(info, K, pe, pv)),
                             ("prolong_E", vemg.OP_E, prolong_bytes(info, K, pe, pv))):
        try:
            ms, nl = s.time_op(op, reps=reps, nrhs=K)
        except vemg.VemgError:
            continue
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "launches": nl, "bytes": nbytes, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


# Fine-level sweeps, fine SpMVs and sweeps on A_bar's first coarse level per
# PCG iteration, by preconditioner (the surface levels are not timed apart):
#   vl_as:  SOR cycle (2 fine sweeps, 1 residual SpMV) and the A_bar V-cycle
#           (2 fine sweeps over the non-top rows, 1 residual SpMV, 2 sweeps on
#           A_bar level 1), plus the CG product
#   vl_sor: the SOR cycle alone plus the CG product
#   vl_add: the A_bar V-cycle plus the CG product
# (vl_as on meshes of SHARE_MIN_ROWS fine unknowns or more: the A_bar
# V-cycle's forward sweep and residual come from the SOR cycle, so 3 full
# sweeps and 2 SpMVs)
PER_ITERATION = {"vl_as": (4, 3, 2), "vl_sor": (2, 2, 0), "vl_add": (2, 2, 2), "jacobi": (0, 1, 0),
                 "none": (0, 1, 0)}
PER_ITERATION_SHARED = {"vl_as": (3, 2, 2)}
KERNEL_NAMES = {
    "gs": "k_gs<double, {K}, false> (fine multicolour SOR, one colour per launch)",
    "spmv": "k_spmv<double, {K}, 0, true> (fine difference-form SpMV fused with p.q)",
    "cgs": "k_patch_gs<double, {K}, false, false> (coarse block multicolour SOR, one patch colour per launch)",
    "et": "k_csr_spmv<double, {K}, 64, 2> (restriction E~^T, CSR, 64 lanes per surface row)",
    "e": "k_rect<double, {K}, true> (prolongation z += E~ y, SELL, one thread per fine row)",
    "dense": "k_dense_part<double, {K}> (the surface coarsest level's explicit inverse streamed by columns)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def dominant_kernel(rates, pc, K, n):
    """The hot kernel with the largest share of one iteration's time: its
    algorithmic bytes and average duration per launch (the roofline entry);
    n: the fine unknowns (whether the forward sweep is shared)."""
    n_gs, n_spmv, n_cgs = (PER_ITERATION_SHARED[pc] if pc in PER_ITERATION_SHARED and n >= SHARE_MIN_ROWS
                           else PER_ITERATION[pc])
    share = {"gs": n_gs * rates["fine_sweep"]["ms"], "spmv": n_spmv * rates["spmv"]["ms"],
             "cgs": n_cgs * rates.get("coarse_sweep", {"ms": 0.0})["ms"]}
    key = max(share, key=share.get)
    r = rates[{"gs": "fine_sweep", "spmv": "spmv", "cgs": "coarse_sweep"}[key]]
    return key, {"kernel": KERNEL_NAMES[key].format(K=K), "bytes_per_launch": r["bytes"] / r["launches"],
                 "ms_per_launch": r["ms"] / r["launches"], "launches_per_application": r["launches"],
                 "ms_per_iteration_estimate": share}


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_0912_1976_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key, workload, K):
    """HBM bytes per launch of a kernel from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel's reading),
    or None when there is none for this kernel, workload and batch width, or
    the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("source_hash") != _kernel_source_hash() or rec.get("workload") != workload
            or rec.get("K", 1) != K):
        return None
    k = rec.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("hbm_bytes_per_launch")


def profile_kernels(workload, K=1):
    """The hot kernels of one PCG iteration for K right-hand sides, each
    repeated, plus a plain copy of known size (the calibration of the PMC
    byte counters): the command profiled by the rocprofv3 --pmc passes."""
    import torch

    import paper_0912_1976_amd as vemg

    mesh = build_mesh(WORKLOADS[workload])
    s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc="vl_as", device=0)
    info = s.info()
    for name, op in (("fine sweep", vemg.OP_GS_FWD), ("fine spmv", vemg.OP_A), ("coarse sweep", vemg.OP_GS_COARSE),
                     ("coarsest dense product", vemg.OP_COARSEST), ("restriction E~^T", vemg.OP_ET),
                     ("prolongation E~", vemg.OP_E)):
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


def pmc_kernels(K):
    """Kernel-name patterns of the hot kernels with K columns (and of the
    calibration copy) in rocprofv3 output."""
    return {"gs": f"k_gs<double, {K}, false>", "spmv": f"k_spmv<double, {K}, 0, true>",
            "cgs": f"k_patch_gs<double, {K}, false, false>", "et": f"k_csr_spmv<double, {K}, 64, 2>",
            "e": f"k_rect<double, {K}, true>", "dense": f"k_dense_part<double, {K}>", "calibration": "MulFunctor"}


def _pmc_means(path, counter, K):
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
                for key, pat in pmc_kernels(K).items():
                    if pat in row["Kernel_Name"]:
                        t = out.setdefault(key, [0.0, 0])
                        t[0] += float(row["Counter_Value"])
                        t[1] += 1
    return {k: v[0] / v[1] for k, v in out.items()}


def pmc_traffic(fetch_dir, write_dir, workload, K):
    """HBM-side bytes per launch of the hot kernels from the two PMC passes:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each divided by what the
    same counter reads for the calibration product (CALIBRATION_BYTES read
    and written once) relative to its true size."""
    fetch = _pmc_means(fetch_dir, "FETCH_SIZE", K)
    write = _pmc_means(write_dir, "WRITE_SIZE", K)
    kib = CALIBRATION_BYTES / 1024.0
    ff, wf = fetch["calibration"] / kib, write["calibration"] / kib
    cmd = f"python3 -u bench.py --profile-kernels --workload {workload} --profile-batch {K}"
    rec = {"workload": workload, "K": K, "source_hash": _kernel_source_hash(),
           "calibration": {"bytes": CALIBRATION_BYTES, "fetch_factor": ff, "write_factor": wf},
           "commands": [f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {fetch_dir} -o run -- {cmd}",
                        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {write_dir} -o run -- {cmd}",
                        f"python3 bench.py --pmc-traffic {fetch_dir} {write_dir} --workload {workload} "
                        f"--profile-batch {K}"],
           "kernels": {}}
    for key in ("gs", "spmv", "cgs", "et", "e", "dense"):
        if key in fetch and key in write:
            rec["kernels"][key] = {"kernel": KERNEL_NAMES[key].format(K=K), "fetch_kib": fetch[key],
                                   "write_kib": write[key],
                                   "hbm_bytes_per_launch": 1024.0 * (fetch[key] / ff + write[key] / wf)}
    print(json.dumps(rec, indent=1))


def trace_timed(path, K):
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
    pats = pmc_kernels(K)
    for key in ("spmv", "gs", "cgs"):
        pat = pats[key]
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
            out[key] = {"kernel": KERNEL_NAMES[key].format(K=K), "dispatches": len(last),
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


def _oracle_sample(workload, iters, core, tol=0.0):
    """The oracle as it stands on one host core, its setup untimed, then
    PCG (VL + additive smoother) on column 0 of the workload timed: `iters`
    iterations, or fewer when the relative residual reaches `tol` first."""
    from inputs import fourier_field, manufactured_u
    from oracle import pcg, precond, solver as osolver

    wl = WORKLOADS[workload]
    mesh = build_mesh(wl)
    t0 = time.perf_counter()
    o = osolver.setup(mesh, "N")
    t_setup = time.perf_counter() - t0
    if wl["kind"] == "graded":
        b = osolver.rhs_from_solution(o, manufactured_u(mesh.xyz, wl["H"]))
    else:
        b = osolver.rhs_from_field(o, fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"]))
    M = precond.make(o, "vl_as")
    t0 = time.perf_counter()
    _, it, hist, _ = pcg.pcg(lambda v: osolver.apply_A(o, v), M, b, tol, max_iter=iters)
    t = time.perf_counter() - t0
    what = f"{it} PCG iterations" if tol == 0.0 else f"the whole solve ({it} PCG iterations to {hist[-1]:.1e})"
    return {"value": o.n * it / t, "unit": "DOF*iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} (VL + additive smoother) of column 0 of the {workload} "
                      f"workload (full mesh, {o.n} unknowns), oracle setup {t_setup:.1f} s untimed, "
                      f"run in a child process pinned to host core {core} while the GPU was measured",
            "seconds": round(t, 3), "setup_s": round(t_setup, 1), "cpu": _cpu_model(),
            "host_cpus": os.cpu_count()}


# the other configurations whose oracle is timed too, with the relative
# residual that ends the sample early (0: the fixed iteration count); the
# graded mesh's oracle setup alone takes minutes, the serving stream is a mix
# of the box meshes
CPU_BASELINE_CONFIGS = {"thinbox-17x17x9-eps1e-2": 1e-8, "thinbox-129x129x33-eps1e-3": 0.0}


def _cpu_baseline_child(workloads, iters, core, queue):
    """Child process: the oracle samples of the workloads in turn, each put on
    the queue as (workload, result) when done."""
    try:
        os.sched_setaffinity(0, {core})
    except (AttributeError, OSError):
        pass
    from threadpoolctl import threadpool_limits

    with threadpool_limits(limits=1):
        for w in workloads:
            tol = CPU_BASELINE_CONFIGS.get(w, 0.0)
            queue.put((w, _oracle_sample(w, 1000 if tol > 0.0 else iters, core, tol)))


def start_cpu_baseline(workloads, iters):
    """Starts the oracle's timed samples of the workloads (the headline first)
    in a child process on one host core (the last one this process may use)
    and returns (process, queue)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    try:
        core = max(os.sched_getaffinity(0))
    except AttributeError:
        core = 0
    p = ctx.Process(target=_cpu_baseline_child, args=(list(workloads), iters, core, q), daemon=True)
    p.start()
    return p, q


def finish_cpu_baseline(handle, count, timeout):
    """{workload: result} of the first `count` samples that finish within
    `timeout` seconds in all; the child is then stopped."""
    import queue as _queue
    p, q = handle
    out = {}
    deadline = time.perf_counter() + timeout
    while len(out) < count and time.perf_counter() < deadline:
        try:
            w, r = q.get(timeout=2.0)
        except _queue.Empty:
            if not p.is_alive() and q.empty():
                break  # the child ended (or failed) without another result
            continue
        out[w] = r
    p.join(5)
    if p.is_alive():
        p.terminate()
    return out


def oracle_fixture(workload, mode="N"):
    """The oracle's sampled FP64 solution of a workload (tests/golden), or
    None: {column: (sample node array, values, norm2)}."""
    import numpy as np
    tag = workload.replace("/", "_")
    path = os.path.join(ROOT, "tests", "golden", f"oracle_samples_{tag}_{mode}.txt")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    nodes = np.asarray(rec["sample_nodes"], dtype=np.int64)
    return {int(c): (nodes, np.array([float.fromhex(v) for v in col["values"]]), col["norm2"], col["iterations"])
            for c, col in rec["columns"].items()}


def error_vs_oracle(x_nat, fixture, col):
    """Relative error of a solution against the oracle's on the fixture's
    sample nodes: ||x - x_o||_S / ||x_o||_S (None without a fixture)."""
    import numpy as np
    if fixture is None or col not in fixture:
        return None
    nodes, vals, _, _ = fixture[col]
    xs = x_nat[nodes]
    return float(np.linalg.norm(xs - vals) / np.linalg.norm(vals))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def serving(nreq, seed, rtol, dev, calib=64):
    """Stream of solve requests over six resident meshes: each request picks a
    mesh uniformly and 1..8 right-hand sides (seeded).  Per precision (mixed
    first, the configuration's solver, then FP64 on the same plan): the first
    `calib` requests submitted at once measure the saturated request rate,
    then all `nreq` requests arrive as a Poisson stream at 0.8 times that
    rate.  Every request is checked for status and relative residual, and
    each column's mixed result against its FP64 result."""
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

    def run(count, rate, keep):
        rids = []
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, count) if rate else np.zeros(count)
        t_next = time.perf_counter()
        for (mi, k), c, gap in zip(plan[:count], cols[:count], gaps):
            t_next += gap
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            rids.append(srv.submit(meshes[mi], pools[mi][torch.as_tensor(c, device=dev)], rtol=rtol))
        worst, floor, relmax, xs = 0, 0, 0.0, []
        for rid in rids:
            srv.wait(rid, timeout=900.0)
            x, st, its, rel, lat = srv.result(rid)
            worst = min(worst, st) if st < 0 else max(worst, st)
            floor += int(st == 2)
            relmax = max(relmax, max(rel))
            if keep:
                xs.append(x)
        s = srv.stats()
        out = {"requests": count, "columns": int(s["columns_done"]), "solves_per_s": s["solves_per_s"],
               "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"], "mean_ms": s["mean_ms"], "max_ms": s["max_ms"],
               "busy_s": s["busy_s"], "slot_occupancy": s["mean_slot_occupancy"], "worst_status": worst,
               "requests_at_floor": floor, "max_relres": relmax, "arrival_rate_per_s": rate}
        return out, xs

    out = {"meshes_nodes": sizes, "setup_s": t_setup, "rtol": rtol, "requests": nreq,
           "stream_pairs": 2}
    results = {}
    for prec in ("mixed_pc", "fp64"):
        srv.set_precision(prec)
        sat, _ = run(min(calib, nreq), 0.0, False)
        rate = 0.8 * sat["requests"] / sat["busy_s"]
        log(f"serving {prec} saturated ({sat['requests']} requests): {sat['solves_per_s']:.1f} solves/s")
        srv.set_precision(prec)
        poi, xs = run(nreq, rate, True)
        results[prec] = xs
        log(f"serving {prec} poisson {rate:.2f}/s, {nreq} requests: {poi['solves_per_s']:.1f} solves/s, "
            f"p50 {poi['p50_ms']:.1f} ms p99 {poi['p99_ms']:.1f} ms")
        out[prec] = {"saturated_calibration": sat, "poisson": poi}
    diffs = [float(torch.linalg.norm(a[k] - b[k]) / torch.linalg.norm(b[k]))
             for a, b in zip(results["mixed_pc"], results["fp64"]) for k in range(a.shape[0])]
    out["max_rel_diff_mixed_vs_fp64"] = max(diffs)
    srv.close()
    return out


def timed_config(s, B, steps, warmup, rtol, info, fixture=None):
    """Median time to tolerance of one solve of the batch B, with iterations,
    statuses, relative residuals and errors against the oracle's fixture."""
    import numpy as np
    x, t, it, rel, st = timed_solves(s, B, steps, warmup, rtol)
    med = float(np.median(t))
    X = x.cpu().numpy().reshape(-1, x.shape[-1])
    out = {"time_to_tol_ms": 1e3 * med, "iterations": it[0], "max_relres": max(rel[0]), "status": st[0],
           "dof_iters_per_s": info["n"] * sum(it[0]) / med, "solves_per_s": X.shape[0] / med}
    if fixture is not None:
        errs = [error_vs_oracle(X[k], fixture, k) for k in range(X.shape[0])]
        out["rel_err_vs_oracle_sampled"] = [e for e in errs]
    return x, out


def config_runs(dev, steps):
    """The other configurations at full size, each with the point condition
    (mode N) and the Dirichlet top (mode D):
    * 17 x 17 x 9 box, eps 1e-2, tolerance 1e-10;
    * 129 x 129 x 33 bathymetric box, eps 1e-3, tolerance 1e-8;
    * centre-refined multiscale box (h_min 1/960, 16-64 layers, eps 1e-3,
      3,974,225 nodes), b = A x* for the manufactured x* (the paper's error
      protocol): VL + additive smoother and VL + SOR (the paper's Mesh B
      comparison), iterations, time to tolerance and the error against x*."""
    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import fourier_field, manufactured_u

    out = {}
    for name in ("thinbox-17x17x9-eps1e-2", "thinbox-129x129x33-eps1e-3", "graded-hmin1/960-eps1e-3"):
        wl = WORKLOADS[name]
        t0 = time.perf_counter()
        mesh = build_mesh(wl)
        t_mesh = time.perf_counter() - t0
        rec = {"mesh_nodes": mesh.n, "mesh_s": t_mesh, "rtol": wl["rtol"]}
        for mode in ("N", "D"):
            t0 = time.perf_counter()
            s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc=mode, pc="vl_as", device=0)
            info = s.info()
            r = {"n_dof": info["n"], "setup_s": time.perf_counter() - t0}
            if wl["kind"] == "graded":
                xs = manufactured_u(mesh.xyz, wl["H"])
                b = s.matvec(xs)
                free = np.zeros(mesh.n, bool)
                free[s.export("perm", np.int64)] = True
                for pc in ("vl_as", "vl_sor"):
                    s.set_preconditioner(pc)
                    x, rr = timed_config(s, b, 2, 1, wl["rtol"], info)
                    xh = x.cpu().numpy()
                    rr["max_rel_err_vs_manufactured"] = float(np.max(np.abs(xh[free] - xs[free]))
                                                              / np.max(np.abs(xs[free])))
                    rr["rel_l2_err_vs_manufactured"] = float(np.linalg.norm(xh[free] - xs[free])
                                                             / np.linalg.norm(xs[free]))
                    r[pc] = rr
                    log(f"{name} {mode} {pc}: {rr['iterations']} iterations, {rr['time_to_tol_ms']:.1f} ms")
            else:
                b = torch.as_tensor(s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"])), device=dev)
                x, rr = timed_config(s, b, steps, 2, wl["rtol"], info, oracle_fixture(name, mode))
                r.update(rr)
                log(f"{name} {mode}: {rr['iterations']} iterations, {rr['time_to_tol_ms']:.2f} ms")
            s.close()
            rec[mode] = r
        out[name] = rec
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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=HEADLINE, choices=sorted(WORKLOADS))
    ap.add_argument("--pc", default="vl_as", choices=sorted(PER_ITERATION))
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline solve and roofline only")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream (the serving configuration's 512 by default)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other full-size configurations")
    ap.add_argument("--paper-comparisons", action="store_true",
                    help="also run Section 6's comparisons (SA, VL + SOR), the Robin top and SSPAI")
    ap.add_argument("--profile-batch", type=int, default=8, choices=(1, 2, 4, 8),
                    help="right-hand sides per launch for --profile-kernels / --pmc-traffic / --trace-timed")
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
        trace_timed(args.trace_timed, args.profile_batch)
        return
    if args.pmc_traffic:
        pmc_traffic(*args.pmc_traffic, args.workload, args.profile_batch)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the decomposition over several GPUs is designed, not built).", file=sys.stderr)
        sys.exit(2)

    if args.profile_kernels:
        profile_kernels(args.workload, args.profile_batch)
        return

    wl = WORKLOADS[args.workload]
    # the oracle's timed sample runs on one host core while the GPU is measured
    cpu_workloads = [args.workload] + [w for w in CPU_BASELINE_CONFIGS if w != args.workload]
    if args.no_extras or args.no_configs:
        cpu_workloads = cpu_workloads[:1]
    cpu_job = None if args.no_cpu_baseline else start_cpu_baseline(cpu_workloads, args.cpu_iters)

    import numpy as np
    import torch

    import paper_0912_1976_amd as vemg
    from inputs import fourier_field, manufactured_u

    dev = torch.device("cuda", 0)
    log(f"workload {args.workload}: building mesh")
    mesh = build_mesh(wl)
    t0 = time.perf_counter()
    s = vemg.Solver(mesh.xyz, mesh.tets, mesh.top, top_bc="pinned", pc=args.pc, device=0)
    t_setup = time.perf_counter() - t0
    info = s.info()
    n, K = info["n"], wl["nrhs"]
    if wl["kind"] == "graded":
        B = s.matvec(manufactured_u(mesh.xyz, wl["H"]))
    else:
        B = torch.as_tensor(np.stack([s.rhs(fourier_field(mesh.xyz, wl["H"], wl["rhs_seed"] + k))
                                      for k in range(K)]), device=dev)
        if K == 1:
            B = B[0]
    rtol = wl["rtol"]
    log(f"setup {t_setup:.2f} s, n={n}; timing {args.steps} FP64 solves of {K} right-hand side(s)")
    x64, times, iters, rels, sts = timed_solves(s, B, args.steps, args.warmup, rtol)
    total = sum(times)
    col_iters = sum(sum(i) for i in iters)
    value = n * col_iters / total
    max_it = max(iters[0])
    log(f"FP64: iterations {iters[0]}, {1e3 * total / args.steps:.2f} ms/solve, relres {max(rels[0]):.2e}")
    fixture = oracle_fixture(args.workload)
    X64 = x64.cpu().numpy().reshape(K, -1)
    err64 = [error_vs_oracle(X64[k], fixture, k) for k in range(K)]

    # live per-kernel timing (HIP events on the library's stream) and the roofline
    rates = kernel_rates(s, info, vemg, K, reps=20)
    dom_key, dom = dominant_kernel(rates, args.pc, K, info["n"])
    achieved = dom["bytes_per_launch"] / (dom["ms_per_launch"] * 1e-3) / 1e9
    traffic = measured_traffic(dom_key, args.workload, K)
    it_bytes = iteration_bytes(info, K, args.pc)
    ms_iter = 1e3 * float(np.median(times)) / max_it
    whole = {"bytes_per_iteration": it_bytes, "ms_per_iteration": ms_iter,
             "GBs": it_bytes / (ms_iter * 1e-3) / 1e9,
             "frac": it_bytes / (ms_iter * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "note": "algorithmic bytes of one PCG iteration from the built arrays' sizes over the solve's "
                     "time per iteration (the slowest column's count)"}
    log(f"dominant kernel {dom['kernel']}: {achieved:.0f} GB/s; whole iteration {whole['GBs']:.0f} GB/s")

    extras = {"kernels": rates, "whole_iteration": whole, "fp64_rel_err_vs_oracle_sampled": err64}
    if not args.no_extras:
        # mixed precision on the same handle and batch
        for prec in ("mixed_pc", "mixed_ir"):
            s.set_precision(prec)
            xm, tm, im, rm, stm = timed_solves(s, B, max(2, args.steps // 2), 1, rtol)
            Xm = xm.cpu().numpy().reshape(K, -1)
            med = float(np.median(tm))
            rec = {"ms_per_solve": 1e3 * med, "solves_per_s": K / med, "iterations": im[0],
                   "max_relres": max(rm[0]), "status": stm[0],
                   "dof_iters_per_s": n * sum(im[0]) / med,
                   "rel_err_vs_oracle_sampled": [error_vs_oracle(Xm[k], fixture, k) for k in range(K)],
                   "max_rel_err_vs_fp64": max(float(np.linalg.norm(Xm[k] - X64[k]) / np.linalg.norm(X64[k]))
                                              for k in range(K)),
                   "iteration_bytes": iteration_bytes(info, K, args.pc, prec)}
            extras[prec] = rec
            log(f"{prec}: {rec['solves_per_s']:.2f} solves/s, iterations {im[0]}")
        s.set_precision("fp64")
        if K > 1:
            x1, t1, i1, r1, st1 = timed_solves(s, B[0], max(2, args.steps // 2), 1, rtol)
            extras["fp64_one_rhs"] = {"time_to_tol_ms": 1e3 * float(np.median(t1)), "iterations": i1[0][0],
                                      "dof_iters_per_s": n * i1[0][0] / float(np.median(t1))}
            extras["kernels_one_rhs"] = kernel_rates(s, info, vemg, 1, reps=20)
        s.close()
        if not args.no_configs:
            extras["configs"] = config_runs(dev, max(3, args.steps))
        if not args.no_serving:
            log("serving stream")
            extras["serving"] = serving(args.serve_requests, 11, 1e-8, dev)
        if args.paper_comparisons:
            extras["sa_baseline"] = sa_baseline_runs(dev, 1e-8)
            m2 = build_mesh(WORKLOADS["thinbox-129x129x33-eps1e-3"])
            extras["robin_top"] = robin_runs(m2, WORKLOADS["thinbox-129x129x33-eps1e-3"], dev, 1e-8)
            extras["sspai_extrapolation"] = sspai_runs(dev, 1e-8)

    cpu = None
    if cpu_job is not None:
        log("waiting for the cpu baseline (oracle)")
        samples = finish_cpu_baseline(cpu_job, len(cpu_workloads), timeout=600)
        cpu = samples.get(args.workload)
        others = {w: r for w, r in samples.items() if w != args.workload}
        if others:
            extras["cpu_baseline_configs"] = others

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
        "config": {"workload": args.workload, "n_dof": n, "rhs_per_step": K, "rtol": rtol, "precond": args.pc,
                   "top": "point condition (Neumann elsewhere)", "precision": "fp64",
                   "value_definition": "unknowns x iterations summed over the batch's columns per second"},
        "iterations": iters[0],
        "time_to_tol_ms": 1e3 * float(np.median(times)),
        "solves_per_s": K * args.steps / total,
        "relres": max(max(r) for r in rels),
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, **dom},
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
