"""Host logic of bench.py (no GPU): the rocprofv3 summary (durations, HBM
traffic scaled by the calibration copy, further counter passes) and the
reading of committed summaries back into the JSON line, which must ignore a
summary made for another kernel source."""
import csv
import io
import json
import os
import subprocess
import sys
from contextlib import redirect_stdout
from types import SimpleNamespace

import pytest

import bench

KERNEL = "dfr_kernel<6, double, double, true, true, 0, double>"


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def _fake_run(tmp_path):
    trace = tmp_path / "trace"
    trace.mkdir()
    _write_csv(trace / "run_kernel_stats.csv", [
        {"Name": f"void dfrsw::{KERNEL}(args)", "Calls": "4", "AverageNs": "20000", "TotalDurationNs": "80000",
         "Percentage": "80.0"},
        {"Name": "__amd_rocclr_copyBuffer", "Calls": "1", "AverageNs": "20000", "TotalDurationNs": "20000",
         "Percentage": "20.0"}])
    # launches of 30, 10, 20 and 12 us; the last two are the timed region
    t, rows = 0, []
    for d in (30, 10, 20, 12):
        rows.append({"Kernel_Name": f"void dfrsw::{KERNEL}(args)", "Start_Timestamp": str(t),
                     "End_Timestamp": str(t + d * 1000)})
        t += 100000
    _write_csv(trace / "run_kernel_trace.csv", rows)

    def counters(name, values, cal=None):
        d = tmp_path / name
        d.mkdir()
        rows = []
        for i, (cn, v) in enumerate(values):
            rows.append({"Dispatch_Id": str(i + 1), "Kernel_Name": f"void dfrsw::{KERNEL}(args)",
                         "Counter_Name": cn, "Counter_Value": str(v)})
        if cal:
            rows.append({"Dispatch_Id": "99", "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": cal[0],
                         "Counter_Value": str(cal[1])})
        _write_csv(d / "run_counter_collection.csv", rows)
        return str(d)
    # FETCH_SIZE reads half the bytes of the 256 MiB copy (factor 2), WRITE_SIZE all of them
    fetch = counters("fetch", [("FETCH_SIZE", 1000.0), ("FETCH_SIZE", 3000.0)], ("FETCH_SIZE", 131072.0))
    write = counters("write", [("WRITE_SIZE", 500.0), ("WRITE_SIZE", 700.0)], ("WRITE_SIZE", 262144.0))
    u1 = counters("u1", [("VALUBusy", 10.0), ("VALUBusy", 30.0), ("LdsUtil", 5.0), ("LdsUtil", 7.0)])
    u2 = counters("u2", [("SQ_INSTS_VALU_FLOPS_FP64", 1.0e6), ("SQ_INSTS_VALU_FLOPS_FP64", 3.0e6)])
    return str(trace), fetch, write, [u1, u2]


def _summary(tmp_path, last=0):
    trace, fetch, write, util = _fake_run(tmp_path)
    args = SimpleNamespace(summarize_profile=trace, fetch=fetch, write=write, counters=util,
                           kernel="true, true, 0, double>", last=last)
    buf = io.StringIO()
    with redirect_stdout(buf):
        assert bench.summarize_profile(args) == 0
    return buf.getvalue()


def test_summary_durations_traffic_and_counters(tmp_path):
    out = _summary(tmp_path)
    assert "timed_region_avg_us: 18.000 over the last 4 launches" in out
    lines = {l.split(":")[0]: l for l in out.splitlines()}
    # mean FETCH 2000 KiB x 2 and mean WRITE 600 KiB x 1, in bytes
    t = lines["traffic_bytes_per_launch"].split()
    assert float(t[1]) == pytest.approx((2000 * 2 + 600) * 1024.0)
    assert t[-1] == bench.kernel_source_digest()
    u = dict(p.split("=") for p in lines["utilisation"].split()[1:-2])
    assert float(u["VALUBusy"]) == pytest.approx(20.0) and float(u["LdsUtil"]) == pytest.approx(6.0)
    assert float(u["SQ_INSTS_VALU_FLOPS_FP64"]) == pytest.approx(2.0e6)


def test_summary_last_n_takes_the_latest_launches(tmp_path):
    out = _summary(tmp_path, last=2)
    assert "timed_region_avg_us: 16.000 over the last 2 launches" in out
    again = tmp_path / "again"
    again.mkdir()
    out = _summary(again, last=1)
    assert "timed_region_avg_us: 12.000 over the last 1 launches" in out
    u = dict(p.split("=") for p in out.splitlines()[-1].split()[1:-2])
    assert float(u["VALUBusy"]) == pytest.approx(30.0) and float(u["LdsUtil"]) == pytest.approx(7.0)


def test_committed_summary_read_back_only_for_the_current_source(tmp_path, monkeypatch):
    out = _summary(tmp_path)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.txt").write_text("# header\n" + out)
    (prof / "old.txt").write_text(out.replace(bench.kernel_source_digest(), "0123456789abcdef"))
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    assert bench.profiled_traffic("k.txt") == pytest.approx((2000 * 2 + 600) * 1024.0)
    assert bench.profiled_traffic("old.txt") is None
    assert bench.profiled_utilisation("old.txt") is None
    assert bench.profiled_traffic("missing.txt") is None
    s = bench.utilisation_summary("k.txt", 10.0)
    assert s["valu_busy_pct"] == pytest.approx(20.0) and s["lds_util_pct"] == pytest.approx(6.0)
    # 2e6 flops per wave instruction count x 64 lanes over 10 us
    assert s["valu_fp64_tflops"] == pytest.approx(2.0e6 * 64 / 10e-6 / 1e12)
    assert s["valu_fp64_frac_of_peak"] == pytest.approx(s["valu_fp64_tflops"] / bench.FP64_VECTOR_PEAK_TFLOPS)
    # without a live duration the profile's own timed average is used
    assert bench.utilisation_summary("k.txt", None)["valu_fp64_tflops"] == pytest.approx(2.0e6 * 64 / 18e-6 / 1e12)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "--gpus 1" in r.stderr
    assert not r.stdout.strip() or "value" not in json.loads(r.stdout.strip().splitlines()[-1])
