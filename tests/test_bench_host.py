"""Host-side logic of bench.py (no GPU): the one-GPU guard, the counter
summary's arithmetic on synthetic rocprofv3 CSVs, and the rule that the
roofline's traffic figure is only taken from a summary of the current kernel
source."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_batch_counter_summary_scales_and_selects(tmp_path):
    copy_bytes = 1 << 20
    A = "void pfk::k_zmarch_batch<3, double, false, 2, true, 512, 1, false, 1>(pfk::ZArgs<double> const*, int const*, int)"
    B = "void pfk::k_zmarch_batch<4, double, false, 2, true, 512, 1, false, 1>(pfk::ZArgs<double> const*, int const*, int)"
    single = "void pfk::k_zmarch<3, double, false, 0, true, 512, 1, false, 1>(pfk::ZArgs<double>)"
    copy = "__amd_rocclr_copyBuffer"
    # FETCH reads half the copied bytes (scale 2), WRITE all of them (scale 1);
    # the WRITE run did one dispatch fewer (its own algorithmic count)
    f_rows = [(copy, copy_bytes / 2 / 1024)]
    w_rows = [(copy, copy_bytes / 1024)]
    alg_f = [9000.0, 6000.0, 3000.0]               # members drop out: fewer bytes per launch
    alg_w = [9000.0, 6000.0]
    for a in alg_f:
        f_rows.append((A, 0.40 * a / 1024))        # 0.80 of the algorithmic bytes once scaled
    for a in alg_w:
        w_rows.append((A, 0.30 * a / 1024))        # 0.30
    f_rows += [(B, 99.0), (single, 77.0)]          # other kernels are not counted
    w_rows += [(B, 99.0), (single, 77.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    flog, wlog = tmp_path / "f.log", tmp_path / "w.log"
    _write_csv(fp, "FETCH_SIZE", f_rows)
    _write_csv(wp, "WRITE_SIZE", w_rows)
    for path, alg in ((flog, alg_f), (wlog, alg_w)):
        path.write_text("[bench] noise\n" + json.dumps({"pmc_run": {"launches_timed": len(alg),
                                                                     "bytes_timed": sum(alg),
                                                                     "mean_us": 1.0}}) + "\n")
    out = bench.pmc_summary_batch(str(fp), str(wp), copy_bytes, str(flog), str(wlog))
    assert out["FETCH_SIZE_scale"] == pytest.approx(2.0) and out["WRITE_SIZE_scale"] == pytest.approx(1.0)
    assert out["FETCH_SIZE_dispatches"] == 3 and out["WRITE_SIZE_dispatches"] == 2
    assert out["FETCH_SIZE_bytes_per_launch"] == pytest.approx(0.8 * sum(alg_f) / 3)
    assert out["counter_over_algorithmic"] == pytest.approx(1.1)
    # a run whose dispatch count does not match its own log gives no ratio
    wlog.write_text(json.dumps({"pmc_run": {"launches_timed": 3, "bytes_timed": 1.0, "mean_us": 1.0}}) + "\n")
    assert "counter_over_algorithmic" not in bench.pmc_summary_batch(str(fp), str(wp), copy_bytes, str(flog),
                                                                     str(wlog))


def test_193_counter_summary_counts_whole_steps(tmp_path):
    copy_bytes = 1 << 20
    n = 5
    N = n ** 3
    name, per = bench.PMC_193_KERNELS["step_a_fp64"]
    A = f"void pfk::{name}(pfk::ZArgs<double>)"
    alg = per * N
    copy = "__amd_rocclr_copyBuffer"
    f_rows = [(copy, copy_bytes / 2 / 1024)]       # FETCH scale 2, WRITE scale 1
    w_rows = [(copy, copy_bytes / 1024)]
    for frac in (0.6, 0.6, 0.001):                 # two whole steps, one exit after convergence
        f_rows.append((A, 0.5 * frac * alg / 1024))
        w_rows.append((A, 0.5 * frac * alg / 1024))
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fp, "FETCH_SIZE", f_rows)
    _write_csv(wp, "WRITE_SIZE", w_rows)
    out = bench.pmc_summary_193(str(fp), str(wp), copy_bytes, n=n)
    e = out["kernels"]["step_a_fp64"]
    assert e["dispatches"] == 3 and e["runs_aligned"] and e["dispatches_counted"] == 2
    assert e["FETCH_SIZE"] == pytest.approx(0.6 * alg) and e["WRITE_SIZE"] == pytest.approx(0.3 * alg)
    assert e["counter_over_algorithmic"] == pytest.approx(0.9)
    assert out["kernels"]["step_b_fp64"]["dispatches"] == 0


def test_traffic_only_from_current_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "PMC_BATCH_FILE", str(prof / "pmc_batch64_step_a.json"))
    assert bench.traffic_from_profiles(1000.0) is None                      # no summary
    csrc = tmp_path / "paper_1711_04060_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "pf_kernels.h").write_text("// kernel source\n")
    h = bench.kernel_source_hash()
    (prof / "pmc_batch64_step_a.json").write_text(json.dumps({"source_hash": h, "counter_over_algorithmic": 1.25}))
    assert bench.traffic_from_profiles(1000.0) == pytest.approx(1250.0)
    (csrc / "pf_kernels.h").write_text("// kernel source, changed\n")
    assert bench.traffic_from_profiles(1000.0) is None                      # kernel changed


def test_trace_summary_busy_idle_and_gaps(tmp_path):
    path = tmp_path / "k.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # A [0, 10 us), B [12, 20), overlapping C [15, 30), A [40, 50)
        for name, s0, e0 in (("void pfk::k_a<1>(x)", 0, 10_000), ("void pfk::k_b(x)", 12_000, 20_000),
                             ("void pfk::k_c(x)", 15_000, 30_000), ("void pfk::k_a<1>(x)", 40_000, 50_000)):
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s0, "End_Timestamp": e0})
    out = bench.trace_summary([str(path)])
    assert out["events"] == 4
    assert out["span_s"] == pytest.approx(50e-6)
    assert out["busy_s"] == pytest.approx(38e-6)     # [0, 10) + [12, 30) + [40, 50)
    assert out["idle_s"] == pytest.approx(12e-6)
    pairs = {g["pair"]: g for g in out["top_gaps"]}
    assert pairs["pfk::k_a<1> -> pfk::k_b"]["mean_us"] == pytest.approx(2.0)
    assert pairs["pfk::k_c -> pfk::k_a<1>"]["mean_us"] == pytest.approx(10.0)
    busy = {k["kernel"]: k for k in out["busy_by_kernel"]}
    assert busy["pfk::k_a<1>"]["count"] == 2 and busy["pfk::k_a<1>"]["seconds"] == pytest.approx(20e-6)
    assert busy["pfk::k_a<1>"]["mean_us_full"] == pytest.approx(10.0)
    # early exits (a few percent of a full launch) are left out of the full-launch mean
    assert bench._full_launches([1000, 20_000, 21_000, 900, 19_000]) == {"count_full": 3,
                                                                        "mean_us_full": pytest.approx(20.0)}
