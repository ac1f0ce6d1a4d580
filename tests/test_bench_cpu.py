"""Host-side logic of bench.py (no GPU): the one-GPU contract, the kernel
source hash that guards committed counter runs, and the conversion of
rocprofv3 byte counters into HBM bytes per launch."""
import csv
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def _copy_sources(dst):
    for s in bench.KERNEL_SOURCES:
        os.makedirs(os.path.dirname(os.path.join(dst, s)), exist_ok=True)
        shutil.copy(os.path.join(ROOT, s), os.path.join(dst, s))


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_hash()
    assert h0 == bench.kernel_hash()
    p = tmp_path / "paper_1608_04118_amd" / "csrc" / "step2_kernel.hpp"
    text = p.read_text()
    # a new comment line and a changed trailing comment: same kernel, same hash
    p.write_text("// a remark\n\n" + text.replace("#pragma once", "#pragma once  // guard", 1))
    assert bench.kernel_hash() == h0
    # a code change: different hash
    p.write_text(text.replace("#pragma once", "#pragma once\nstatic const int unused_probe = 1;", 1))
    assert bench.kernel_hash() != h0


def test_measured_traffic_only_for_current_sources(tmp_path, monkeypatch):
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    rec = {"f32": {"kernel_hash": bench.kernel_hash(), "bytes_per_launch": 11.5e9}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("f32") == 11.5e9
    assert bench.measured_traffic("f64") is None
    rec["f32"]["kernel_hash"] = "0" * 16
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("f32") is None


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_ingest_counters_calibrates_by_the_copy(tmp_path, capsys):
    copy, step2, other = "__amd_rocclr_copyBuffer", "void ltne::step2_kernel<float, 1>(float const*, ...)", \
        "void ltne::step_kernel<float, float, 5>(...)"
    gib = 2 ** 30
    # FETCH_SIZE reads half the copy's bytes (scale 2), WRITE_SIZE all of them
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(copy, gib / 2048), (copy, 3.0), (step2, 2.8e6), (step2, 2.9e6), (step2, 3.0e6), (other, 9e9)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(copy, gib / 1024), (step2, 5.0e6), (step2, 5.2e6), (step2, 5.1e6)])
    out = tmp_path / "traffic.json"
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), gib, str(out))
    capsys.readouterr()
    rec = json.loads(out.read_text())["f32"]
    c = rec["counters"]
    assert c["FETCH_SIZE"]["scale"] == pytest.approx(2.0) and c["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    # medians of the step kernel's dispatches only (the small copy and other kernels are ignored)
    assert c["FETCH_SIZE"]["step_bytes"] == pytest.approx(2.9e6 * 1024 * 2)
    assert c["WRITE_SIZE"]["step_bytes"] == pytest.approx(5.1e6 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(2.9e6 * 2048 + 5.1e6 * 1024)
    assert rec["must_move_bytes_per_launch"] == 156 * 8192 * 8192
    assert rec["one_step_equivalent_bytes_per_launch"] == 156 * 8192 * 8192 * 2
    assert rec["kernel_hash"] == bench.kernel_hash()


def test_ingest_counters_needs_both_kernels(tmp_path):
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 2 ** 19)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 2 ** 20)])
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 2 ** 30,
                              str(tmp_path / "traffic.json"))


def test_sq_ingest_and_roofline_block(tmp_path, monkeypatch):
    """SQ_INSTS_VALU of the two-step kernel becomes instructions per launch
    (median), valid only for the current kernel sources; the roofline block
    divides the bytes a launch must move by its time, and restates the
    two-step launch against vector issue and as the one-step equivalent."""
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "sq.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for v in (1.0e9, 1.2e9, 1.1e9):
            w.writerow({"Kernel_Name": "void ltne::step2_kernel<float, 1>(float const*, ...)",
                        "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": v})
        w.writerow({"Kernel_Name": "void ltne::step_kernel<float, float, 5>(...)",
                    "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 5.0})
    bench.ingest_sq(str(path), str(tmp_path / "profiles" / "sq.json"))
    assert bench.measured_valu("f32") == 1.1e9
    r = {"launch_ms": 2.5, "steps_per_launch": 2}
    out = bench.roofline("f32", r, 11.0e9)
    n = bench.N * bench.N
    assert out["bytes_per_launch"] == 156 * n
    assert abs(out["achieved"] - 156 * n / 2.5e-3 / 1e9) < 0.1
    assert abs(out["frac"] - out["achieved"] / 8000.0) < 1e-4
    assert abs(out["one_step_equivalent"]["gbs"] - 2 * out["achieved"]) < 0.2
    assert abs(out["valu_issue"]["issue_floor_ms"] - 1.1e9 / (256 * 2.4e9) * 1e3) < 1e-3
    assert abs(out["traffic_gbs"] - 11.0e9 / 2.5e-3 / 1e9) < 0.1
    single = bench.roofline("f64", {"launch_ms": 3.6, "steps_per_launch": 1}, None)
    assert single["bytes_per_launch"] == 312 * n and "valu_issue" not in single


def test_counter_runs_of_both_two_step_forms(tmp_path, monkeypatch, capsys):
    """Counter runs of the FP32 and the FP64 two-step kernels land in one
    summary, each under its form, picked out by the kernel's element type;
    the bench line's per-form figures then divide them by the launch time."""
    _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    out = tmp_path / "profiles" / "traffic.json"
    copy = "__amd_rocclr_copyBuffer"
    f32k = "void ltne::step2_kernel<float, 1>(float const*, ...)"
    f64k = "void ltne::step2_kernel<double, 1>(double const*, ...)"
    gib = 2 ** 30
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", [(copy, gib / 2048), (f32k, 1.0e6), (f64k, 5.0e6)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", [(copy, gib / 1024), (f32k, 2.0e6), (f64k, 7.0e6)])
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), gib, str(out), "f32")
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), gib, str(out), "f64")
    capsys.readouterr()
    t = json.loads(out.read_text())
    assert t["f32"]["bytes_per_launch"] == pytest.approx(1.0e6 * 2048 + 2.0e6 * 1024)
    assert t["f64"]["bytes_per_launch"] == pytest.approx(5.0e6 * 2048 + 7.0e6 * 1024)
    assert t["f64"]["must_move_bytes_per_launch"] == 312 * 8192 * 8192
    fig = bench.counter_figures("f64", {"launch_ms": 5.0})
    assert fig["traffic_bytes_per_launch"] == t["f64"]["bytes_per_launch"]
    assert abs(fig["traffic_frac"] - t["f64"]["bytes_per_launch"] / 5e-3 / 1e9 / 8000.0) < 1e-4
    assert "valu_issue_frac" not in fig
    assert bench.counter_figures("f16s", {"launch_ms": 1.0}) == {}
