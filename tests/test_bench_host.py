"""Host-side logic of bench.py (no device work): the one-GPU guard, the
source hash that keys measured traffic, and the scaling of the HBM
counters into bytes per launch."""
import argparse
import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""          # no JSON line


def test_code_text_ignores_comments_and_blank_lines(bench):
    a = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    b = "/* header\n   comment */\nint f(int x) {\n\n  // a note\n  return x + 1;\n}\n"
    assert bench.code_text(a) == bench.code_text(b)
    # a change of code is seen
    assert bench.code_text(a) != bench.code_text(a.replace("+ 1", "+ 2"))


def _counter_csv(path, counter, rows):
    cols = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scaled_by_the_copy_reading(bench, tmp_path, monkeypatch):
    """FETCH_SIZE reading half of a 1 GiB copy's bytes doubles the kernel's
    reading; WRITE_SIZE reading all of them keeps it; other kernels and
    small copies are ignored; the result is keyed by the source hash."""
    step = "void cuba::k_step<true, false, 512u>(cuba::Cells, long)"
    other = "void cuba::k_step<false, false, 512u>(cuba::Cells, long)"
    copy = "__amd_rocclr_copyBuffer"
    gib_kib = float(1 << 20)
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(step, 10000, 1000.0), (step, 10000, 3000.0),
                                       (other, 10000, 9e9), (copy, 65536, gib_kib / 2),
                                       (copy, 256, 1.0)])
    _counter_csv(write, "WRITE_SIZE", [(step, 10000, 5000.0), (copy, 65536, gib_kib)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_path", lambda workload: str(out))
    a = argparse.Namespace(pmc_csv=[str(fetch), str(write)], workload="unit", pmc_sq=None,
                           pmc_fp64=None)
    bench.write_traffic(a)
    t = json.load(open(out))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert t["write_bytes_per_launch"] == pytest.approx(5000.0 * 1024)
    assert t["bytes_per_launch"] == pytest.approx(t["fetch_bytes_per_launch"]
                                                  + t["write_bytes_per_launch"])
    assert t["kernel_source_hash"] == bench.kernel_source_hash()
    # read back only while the sources still hash to the stored key
    assert bench.measured_profile("unit")["bytes_per_launch"] == pytest.approx(
        t["bytes_per_launch"])
    t["kernel_source_hash"] = "0" * 16
    json.dump(t, open(out, "w"))
    assert bench.measured_profile("unit") is None


def test_valu_busy_from_sq_counter_and_trace(bench, tmp_path):
    """4 SQ_ACTIVE_INST_VALU quad-cycles per SIMD-cycle of the kernel's
    average trace duration: a kernel keeping all 1024 SIMDs busy for its
    whole 100 us reads 1024 x 240000 / 4 quad-cycles, i.e. busy 1."""
    step = "void cuba::k_step<true, false, 512u>(cuba::Cells, long)"
    sq = tmp_path / "sq.csv"
    full = 1024 * 240000 / 4
    _counter_csv(sq, "SQ_ACTIVE_INST_VALU", [(step, 10000, full), (step, 10000, full / 2)])
    stats = tmp_path / "stats.csv"
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": "__amd_rocclr_copyBuffer", "Calls": 3, "AverageNs": 5.0})
        w.writerow({"Name": step, "Calls": 2, "AverageNs": 100000.0})
    v = bench.valu_busy(str(sq), str(stats))
    assert v["valu_busy"] == pytest.approx(0.75)
    assert v["trace_avg_ns"] == 100000.0


def test_usable_cores_reports_affinity_and_count(bench):
    c = bench.usable_cores()
    assert 1 <= c["usable"] <= c["affinity"] <= (c["cpu_count"] or c["affinity"])


def test_fp64_executed_from_counters(bench, tmp_path):
    """Executed FP64 operations per launch: 64 lanes x (add + mul +
    transcendental + 2 fma) wave-instructions, averaged over the dominant
    kernel's dispatches; other kernels are ignored."""
    step = "void cuba::k_step<true, false, 512u>(cuba::Cells, long)"
    other = "void cuba::k_stream_bin<64u>(cuba::Cells)"
    path = tmp_path / "fp64.csv"
    cols = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    rows = [(step, "SQ_INSTS_VALU_ADD_F64", 10.0), (step, "SQ_INSTS_VALU_ADD_F64", 30.0),
            (step, "SQ_INSTS_VALU_MUL_F64", 5.0), (step, "SQ_INSTS_VALU_FMA_F64", 7.0),
            (step, "SQ_INSTS_VALU_TRANS_F64", 1.0), (other, "SQ_INSTS_VALU_FMA_F64", 1e9)]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (name, ctr, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Grid_Size": 64, "Kernel_Name": name,
                        "Counter_Name": ctr, "Counter_Value": v})
    out = bench.fp64_executed(str(path))
    assert out["fp64_executed_flops_per_launch"] == pytest.approx(64 * (20 + 5 + 2 * 7 + 1))
