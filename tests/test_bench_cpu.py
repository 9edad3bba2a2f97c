"""Host logic of bench.py's profile summaries (no GPU): the early-exit split
of per-dispatch figures, the counter summary's scaling by the calibration
copy, and the traffic read-back with its source-hash check, on small
synthetic rocprofv3-style CSV files."""
import csv
import os

import pytest

import bench


def _write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, val in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_early_exit_cut_separates_speculative_dispatches():
    work = [15.8, 16.1, 16.0, 15.9]
    early = [3.9, 4.1, 1.7]
    vals = early * 3 + work      # more early exits than working dispatches
    cut = bench.early_exit_cut(vals)
    assert max(early) < cut < min(work)
    vals = work * 5 + early      # mostly working dispatches
    cut = bench.early_exit_cut(vals)
    assert max(early) < cut < min(work)
    # a short run where fewer than a quarter of the column passes work: two
    # working, one skipped apply (the step's last iteration) and six early
    # exits per step, as in a counter run from the ground state
    col = ([20923.0] * 2 + [16.0] + [10.0] * 6) * 12
    cut = bench.early_exit_cut(col)
    assert 16.0 < cut < 20923.0
    assert sum(1 for x in col if x >= cut) == 24


def test_counter_summary_scales_by_copy_and_drops_early_exits(tmp_path, monkeypatch):
    row, col = (f"void hub::dev::{bench.DOMINANT_KERNELS[0]}(hub::dev::KArgs)",
                f"void hub::dev::{bench.DOMINANT_KERNELS[1]}(hub::dev::ColArgs)")
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>"
    copy_kib = bench.COPY_BYTES / 1024.0 / 2.0   # a counter that reads half the bytes: scale 2
    fetch = [(copy, copy_kib)] + [(row, 1000.0)] * 3 + [(row, 2.0)] * 6 + [(col, 3000.0)] * 3 + [(col, 1.0)] * 6
    write = [(copy, bench.COPY_BYTES / 1024.0)] + [(row, 500.0)] * 3 + [(row, 0.5)] * 6 + [(col, 250.0)] * 3
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = tmp_path / "summary.txt"
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(out), command="synthetic")
    txt = out.read_text()
    kv = dict(line.split(": ", 1) for line in txt.splitlines() if ": " in line and not line.startswith("#"))
    assert float(kv["hbm_fetch_bytes_per_launch"]) == pytest.approx((1000.0 + 3000.0) * 1024 * 2.0)
    assert float(kv["hbm_write_bytes_per_launch"]) == pytest.approx((500.0 + 250.0) * 1024 * 1.0)
    assert "plus 6 early exits" in txt
    # the traffic read-back honours the source hash
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(out))
    assert bench.measured_traffic() == pytest.approx((1000.0 + 3000.0) * 2048 + 750.0 * 1024)
    out.write_text(txt.replace(bench.kernel_source_hash(), "0000000000000000"))
    assert bench.measured_traffic() is None



def test_stats_summary_and_traced_pair_time(tmp_path, monkeypatch):
    row, col = (f"void hub::dev::{bench.DOMINANT_KERNELS[0]}(hub::dev::KArgs)",
                f"void hub::dev::{bench.DOMINANT_KERNELS[1]}(hub::dev::ColArgs)")
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": row, "Calls": 6, "AverageNs": 12000, "TotalDurationNs": 72000, "Percentage": 60})
        w.writerow({"Name": col, "Calls": 6, "AverageNs": 8000, "TotalDurationNs": 48000, "Percentage": 40})
    # per step: two working pairs, the last column pass skipped, one early-exit pair
    durs = [(row, 16000), (col, 14000), (row, 16000), (col, 14000), (row, 16000), (col, 3500),
            (row, 3000), (col, 3000)] * 2
    t = 0
    with open(d / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, ns in durs:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + ns})
            t += ns + 500
    out = tmp_path / "stats.txt"
    bench.summarize_stats(str(d), str(out), command="synthetic", note="one|two")
    txt = out.read_text()
    assert "# one" in txt and "# two" in txt
    assert "working 6 avg_us 16.00" in txt and "working 4 avg_us 14.00" in txt
    monkeypatch.setattr(bench, "STATS_FILE", str(out))
    assert bench.traced_pair_us() == pytest.approx(30.0)
    assert bench.trace_figure(4 * 853776 * 16)["avg_launch_us"] == pytest.approx(30.0)
    out.write_text(txt.replace(bench.kernel_source_hash(), "0000000000000000"))
    assert bench.traced_pair_us() is None and bench.trace_figure(1.0) is None
