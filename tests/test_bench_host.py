"""Host-side logic of bench.py: the one-GPU guard, the PMC traffic arithmetic,
the trace summary on small synthetic rocprofv3 CSV files, and the oracle
baseline child on the smallest box (no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          cwd=ROOT, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for name, value in rows:
            w.writerow([name, counter, value])


def test_pmc_traffic_divides_each_counter_by_its_calibration(tmp_path, capsys):
    kib = bench.CALIBRATION_BYTES / 1024.0
    cal = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<double> >"
    gs = "void vemg::(anonymous namespace)::k_gs<double, 1, false>(vemg::Sell, ...)"
    gs_zero = "void vemg::(anonymous namespace)::k_gs<double, 1, true>(vemg::Sell, ...)"
    spmv = "void vemg::(anonymous namespace)::k_spmv<double, 1, 0, true>(vemg::Sell, ...)"
    # FETCH reads half the true bytes, WRITE all of them; two dispatches per kernel
    _counter_csv(str(tmp_path / "f"), "FETCH_SIZE",
                 [(cal, 0.5 * kib), (cal, 0.5 * kib), (gs, 100.0), (gs, 300.0), (gs_zero, 1e6), (spmv, 50.0)])
    _counter_csv(str(tmp_path / "w"), "WRITE_SIZE",
                 [(cal, kib), (gs, 10.0), (gs, 30.0), (gs_zero, 1e6), (spmv, 5.0)])
    bench.pmc_traffic(str(tmp_path / "f"), str(tmp_path / "w"), "thinbox-129x129x33-eps1e-3", 1)
    rec = json.loads(capsys.readouterr().out)
    assert rec["K"] == 1
    assert rec["source_hash"] == bench._kernel_source_hash()
    assert rec["calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]
    # the zero-start sweep is not the general form and is not counted
    assert k["gs"]["fetch_kib"] == pytest.approx(200.0)
    assert k["gs"]["hbm_bytes_per_launch"] == pytest.approx(1024.0 * (200.0 / 0.5 + 20.0))
    assert k["spmv"]["hbm_bytes_per_launch"] == pytest.approx(1024.0 * (100.0 + 5.0))
    assert "cgs" not in k


def test_trace_timed_takes_the_last_run_of_each_kernel(tmp_path, capsys):
    cgs = "void vemg::(anonymous namespace)::k_patch_gs<double, 1, false, false>(vemg::CsrG, ...)"
    cgs_zero = "void vemg::(anonymous namespace)::k_patch_gs<double, 1, true, false>(vemg::CsrG, ...)"
    fill = "void vemg::(anonymous namespace)::k_fill<double>(double*, long, double, int const*)"
    other = "vemg::(anonymous namespace)::k_pcg_alpha(...)"
    rows, t = [], 0

    def add(name, dur):
        nonlocal t
        rows.append((name, t, t + dur))
        t += dur + 1000

    # the solve: sweeps interleaved with other kernels
    for _ in range(3):
        add(cgs_zero, 9000)
        add(cgs, 7000)
        add(other, 2000)
    # the live timing: a fill, then back-to-back general sweeps
    add(fill, 500)
    for d in (3000, 3200, 3400):
        add(cgs, d)
    add(fill, 500)
    add(cgs, 3400)
    path = tmp_path / "run_kernel_trace.csv"
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        # rows out of order on purpose: the summary sorts by start time
        for name, t0, t1 in reversed(rows):
            w.writerow([name, t0, t1])
    bench.trace_timed(str(tmp_path), 1)
    out = json.loads(capsys.readouterr().out)
    assert set(out) == {"cgs"}
    assert out["cgs"]["dispatches"] == 4
    assert out["cgs"]["mean_us"] == pytest.approx(3.25)


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    """The roofline's traffic comes from the committed PMC record only while
    the kernel sources hash to the recorded value and the workload matches;
    otherwise it is null."""
    rec = {"workload": "thinbox-129x129x33-eps1e-3", "K": 8, "source_hash": bench._kernel_source_hash(),
           "kernels": {"cgs": {"hbm_bytes_per_launch": 1234.0}}}
    f = tmp_path / "pmc_traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("cgs", "thinbox-129x129x33-eps1e-3", 8) == 1234.0
    assert bench.measured_traffic("cgs", "thinbox-129x129x33-eps1e-3", 1) is None
    assert bench.measured_traffic("gs", "thinbox-129x129x33-eps1e-3", 8) is None
    assert bench.measured_traffic("cgs", "thinbox-257x257x33-eps1e-4", 8) is None
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("cgs", "thinbox-129x129x33-eps1e-3", 8) is None
    f.write_text("not json")
    assert bench.measured_traffic("cgs", "thinbox-129x129x33-eps1e-3", 8) is None


def _info():
    # sizes of a small made-up setup: 100 unknowns, 10 on top, 2 surface levels, 3 A_bar levels
    return {"n": 100, "n_top": 10, "nnz_offdiag": 1300, "e_nnz": 280,
            "s_rows": [10, 3], "s_nnz": [40, 6], "p_nnz_s": [20, 0],
            "abar_rows": [90, 20, 4], "abar_nnz": [1150, 160, 12], "p_nnz_abar": [300, 60, 0]}


def test_byte_model_counts_each_array_once():
    info = _info()
    # SpMV: 12 bytes per off-diagonal, the row datum, x read and y written
    assert bench.spmv_bytes(info, 1) == 1300 * 12 + 100 * 8 + 2 * 100 * 8
    assert bench.spmv_bytes(info, 8) == 1300 * 12 + 100 * 8 + 2 * 100 * 64
    assert bench.spmv_bytes(info, 8, 4, 4, residual=True) == 1300 * 8 + 100 * 8 + 3 * 100 * 32
    # E~^T: entries, row pointer and row map per surface row, r read, g written
    assert bench.restrict_bytes(info, 2) == 280 * 12 + 10 * 8 + 100 * 16 + 10 * 16
    assert bench.prolong_bytes(info, 1) == 280 * 12 + 10 * 8 + 2 * 100 * 8
    # a two-level cycle: two sweeps, residual and both transfers on level 0, the dense coarsest
    sw = 40 * 12 + 10 * 12 + 3 * 10 * 8
    r, p = 20 * 12 + 3 * 4 + 10 * 8 + 3 * 8, 20 * 12 + 10 * 4 + 3 * 8 + 2 * 10 * 8
    assert bench.vcycle_bytes([10, 3], [40, 6], [20, 0], 1, 8, 8) == 3 * sw + r + p + 9 * 8 + 2 * 3 * 8


def test_iteration_bytes_add_up_the_preconditioner_branches():
    info = _info()
    full = bench.iteration_bytes(info, 1, "vl_as")
    sor = bench.iteration_bytes(info, 1, "vl_sor")
    # the additive smoother's V-cycle on A_bar is the difference (plus the join)
    a_cycle = bench.vcycle_bytes(info["abar_rows"], info["abar_nnz"], info["p_nnz_abar"], 1, 8, 8,
                                 fine_rows=90, fine_nnz=1150)
    join = 4 * 100 * 8 + 100 * 8
    assert bench.SHARE_MIN_ROWS > 100
    assert full - sor == a_cycle + join - 2 * 100 * 8
    # on a mesh large enough to share the forward sweep, the smoother's fine
    # forward sweep and residual are the SOR cycle's, which stores x and r of
    # the 90 non-top rows once more
    shared = (bench.gs_sweep_bytes(None, 1, 8, 8, rows=90, nnz=1150)
              + bench.spmv_bytes(None, 1, 8, 8, residual=True, rows=90, nnz=1150))
    saved = bench.SHARE_MIN_ROWS
    try:
        bench.SHARE_MIN_ROWS = 100
        assert bench.iteration_bytes(info, 1, "vl_as") == full - shared + 2 * 90 * 8
    finally:
        bench.SHARE_MIN_ROWS = saved
    # batches and FP32 preconditioners scale the vector traffic, not the matrices
    assert bench.iteration_bytes(info, 8, "vl_as") > full
    assert bench.iteration_bytes(info, 1, "vl_as", "mixed_pc") < full + 4 * 100 * 12


def test_cpu_baseline_child_reports_each_config():
    """The oracle's samples run in a child process on one core and come back
    per workload; the small box is timed over its whole solve."""
    h = bench.start_cpu_baseline(["thinbox-17x17x9-eps1e-2"], 5)
    out = bench.finish_cpu_baseline(h, 1, 120)
    r = out["thinbox-17x17x9-eps1e-2"]
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "DOF*iters/s"
    assert r["value"] > 0.0
    assert "whole solve" in r["sample"]
    assert not h[0].is_alive()
