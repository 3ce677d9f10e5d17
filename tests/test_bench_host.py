"""Host-side logic of bench.py (no GPU): the one-GPU guard, the counter
summary's arithmetic on synthetic rocprofv3 CSVs, and the rule that the
roofline's traffic figure is only taken from a summary of the current kernel
source and workload."""
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


def test_counter_summary_scales_selects_and_filters(tmp_path):
    n = 1000
    alg_a, alg_b = 12 * n * 8, 7 * n * 8
    copy_bytes = 1 << 20
    A = "void pfk::k_zmarch<3, double, false, 512, 1, false, 1>(pfk::ZArgs<double>)"
    A_other = "void pfk::k_zmarch<3, double, false, 256, 2, false, 1>(pfk::ZArgs<double>)"
    B = "void pfk::k_zmarch<4, double, false, 512, 1, false, 1>(pfk::ZArgs<double>)"
    copy = "__amd_rocclr_copyBuffer"
    # FETCH reads half the copied bytes (scale 2), WRITE all of them (scale 1)
    f_rows = [(copy, copy_bytes / 2 / 1024)]
    w_rows = [(copy, copy_bytes / 1024)]
    # step A: three launches that ran (raw fetch 0.40-0.44 of the algorithmic bytes, 0.80-0.88 scaled)
    for fa, wa in ((0.40, 0.25), (0.42, 0.26), (0.44, 0.27)):
        f_rows.append((A, fa * alg_a / 1024))
        w_rows.append((A, wa * alg_a / 1024))
    # one launch that exited early: excluded by the half-the-bytes filter
    f_rows.append((A, 0.01 * alg_a / 1024))
    w_rows.append((A, 0.0))
    # a tuner candidate with one launch: not the most frequent instance
    f_rows.append((A_other, 5.0 * alg_a / 1024))
    w_rows.append((A_other, 5.0 * alg_a / 1024))
    f_rows.append((B, 0.45 * alg_b / 1024))
    w_rows.append((B, 0.3 * alg_b / 1024))
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fp, "FETCH_SIZE", f_rows)
    _write_csv(wp, "WRITE_SIZE", w_rows)
    out = bench.pmc_summary_families(str(fp), str(wp), "synthetic", copy_bytes, n)
    a = out["kernels"]["step_a_fp64"]
    assert a["kernel"] == "pfk::k_zmarch<3, double, false, 512, 1, false, 1>"
    assert a["dispatches"] == 4 and a["dispatches_counted"] == 3 and a["runs_aligned"]
    assert a["FETCH_SIZE_scale"] == pytest.approx(2.0) and a["WRITE_SIZE_scale"] == pytest.approx(1.0)
    assert a["FETCH_SIZE"] == pytest.approx(2.0 * 0.42 * alg_a)
    assert a["WRITE_SIZE"] == pytest.approx(0.26 * alg_a)
    assert a["counter_over_algorithmic"] == pytest.approx(0.84 + 0.26)
    assert out["hbm_bytes_per_launch"] == pytest.approx(a["counter_bytes"])
    b = out["kernels"]["step_b_fp64"]
    assert b["counter_bytes"] == pytest.approx((0.9 + 0.3) * alg_b)
    assert "step_a_fp32" not in out["kernels"]


def test_traffic_only_from_current_source_and_workload(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("membrane_pore_97") is None          # no summary
    csrc = tmp_path / "paper_1711_04060_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "pf_kernels.h").write_text("// kernel source\n")
    h = bench.kernel_source_hash()
    (prof / "pmc_bicg_step_a.json").write_text(json.dumps(
        {"workload": "membrane_pore_97", "source_hash": h, "hbm_bytes_per_launch": 123.0}))
    assert bench.traffic_from_profiles("membrane_pore_97") == 123.0
    assert bench.traffic_from_profiles("membrane_pore_49") is None          # other workload
    (csrc / "pf_kernels.h").write_text("// kernel source, changed\n")
    assert bench.traffic_from_profiles("membrane_pore_97") is None          # kernel changed


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
