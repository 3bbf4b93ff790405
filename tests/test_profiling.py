"""The rocprofv3 summaries the measured figures come from: counter scaling by
the calibration copy, the LDS ratios, kernel statistics, and the bench's
rule that a traffic summary counts only for the kernel sources it was taken
from.  Synthetic counter files, on the CPU."""
from __future__ import annotations

import csv
import json
import math
import os

import pytest

import bench
from paper_2010_08695_amd import profiling as P

KNAME = "tip::(anonymous namespace)::{}(tip::DevGraph, int)"


def _counters(d, rows):
    """rows: (dispatch, kernel, counter, value); two per-XCD halves each."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for disp, k, c, v in rows:
            w.writerow([disp, KNAME.format(k), c, v / 2])
            w.writerow([disp, KNAME.format(k), c, v / 2])
    return str(d)


def _stats(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_kernel_stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"])
        for k, calls, tot in rows:
            w.writerow([KNAME.format(k), calls, tot, tot / calls, 50.0, tot / calls / 2, tot / calls * 2])
    return str(d)


def test_kernel_stats_parse_and_sort(tmp_path):
    d = _stats(tmp_path / "s", [("k_small", 10, 1e6), ("k_peel_dense", 4, 8e6)])
    rows = P.kernel_stats(d)
    assert [r["name"] for r in rows] == ["k_peel_dense", "k_small"]
    assert rows[0]["calls"] == 4 and rows[0]["avg_ns"] == 2e6


def test_counter_values_summed_per_dispatch(tmp_path):
    d = _counters(tmp_path / "c", [(1, "k_a", "FETCH_SIZE", 100.0), (2, "k_a", "FETCH_SIZE", 300.0),
                                   (3, "k_b", "FETCH_SIZE", 7.0), (3, "k_b", "WRITE_SIZE", 9.0)])
    assert sorted(P.counter_per_dispatch(d, "FETCH_SIZE")["k_a"]) == [100.0, 300.0]
    assert P.counter_per_dispatch(d, "WRITE_SIZE") == {"k_b": [9.0]}


def test_traffic_scaled_by_the_copy_and_gated_by_source(tmp_path, monkeypatch):
    mib = 1024
    # the 1 GiB copy reads half its bytes in FETCH_SIZE and all in WRITE_SIZE
    cf = _counters(tmp_path / "cf", [(1, "copy", "FETCH_SIZE", mib * 1024 / 2)])
    cw = _counters(tmp_path / "cw", [(1, "copy", "WRITE_SIZE", mib * 1024)])
    kf = _counters(tmp_path / "kf", [(5, "k_peel_dense", "FETCH_SIZE", 1000.0), (6, "k_peel_dense", "FETCH_SIZE", 3000.0)])
    kw = _counters(tmp_path / "kw", [(5, "k_peel_dense", "WRITE_SIZE", 500.0), (6, "k_peel_dense", "WRITE_SIZE", 500.0)])
    out = tmp_path / "profiles" / "k_peel_dense.wl.traffic.txt"
    os.makedirs(out.parent)

    class A:
        fetch, write, calib_fetch, calib_write = kf, kw, cf, cw
        calib_mib, kernel, workload, cmd = mib, "k_peel_dense", "wl", "cmd"
    A.out = str(out)
    assert P.cmd_traffic(A) == 0
    rec = json.loads(out.read_text().split("\n---\n")[0])
    assert math.isclose(rec["fetch_scale"], 2.0) and math.isclose(rec["write_scale"], 1.0)
    # mean 2000 KiB fetched x 2 + mean 500 KiB written x 1
    assert math.isclose(rec["bytes_per_launch"], (2000 * 2 + 500) * 1024)
    sha = bench.kernel_source_sha()   # of the real sources, before ROOT moves
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: sha)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert math.isclose(bench.load_traffic("wl"), rec["bytes_per_launch"])
    rec["kernel_sha"] = "0" * 16
    out.write_text(json.dumps(rec) + "\n---\n")
    assert bench.load_traffic("wl") is None
    assert bench.load_traffic("other") is None


def test_lds_ratios_and_bandwidth(tmp_path, capsys):
    a = _counters(tmp_path / "a", [
        (1, "k_peel_dense", "SQ_LDS_BANK_CONFLICT", 200.0), (1, "k_peel_dense", "SQ_LDS_IDX_ACTIVE", 1200.0),
        (1, "k_peel_dense", "SQ_INSTS_LDS", 64.0), (1, "k_peel_dense", "SQ_ACTIVE_INST_LDS", 30.0),
        (1, "k_peel_dense", "SQ_WAVE_CYCLES", 600.0), (1, "k_peel_dense", "SQ_BUSY_CU_CYCLES", 1.0),
        (1, "k_peel_dense", "GRBM_GUI_ACTIVE", 1.0)])
    b = _counters(tmp_path / "b", [
        (1, "k_peel_dense", "SQ_INSTS_LDS_LOAD_BANDWIDTH", 6e9), (1, "k_peel_dense", "SQ_INSTS_LDS_STORE_BANDWIDTH", 3e9),
        (1, "k_peel_dense", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH", 1e9), (1, "k_peel_dense", "SQ_INSTS_LDS_ATOMIC", 1.0)])
    t = _stats(tmp_path / "t", [("k_peel_dense", 1, 80e6)])   # 80 ms

    class A:
        conflicts, bytes, trace, kernels, workload, cmd, out = a, b, t, "k_peel_dense,k_absent", "wl", "c", ""
    assert P.cmd_lds(A) == 0
    row = [l for l in capsys.readouterr().out.splitlines() if l.startswith("k_peel_dense")][0].split()
    # conflicts / conflict-free cycles = 200 / 1000; LDS share 30 / 600;
    # 64 B x 1e10 over 80 ms = 8 TB/s of the 78.6 TB/s peak
    assert float(row[3]) == pytest.approx(0.2) and float(row[4]) == pytest.approx(0.05)
    assert float(row[5]) == pytest.approx(640.0) and float(row[7]) == pytest.approx(8.0)
    assert P.LDS_PEAK_TBS == pytest.approx(78.6432)


def test_wave_state_shares(tmp_path, capsys):
    d = _counters(tmp_path / "w", [
        (1, "k_peel_dense", "SQ_WAVE_CYCLES", 1000.0), (1, "k_peel_dense", "SQ_WAIT_ANY", 550.0),
        (1, "k_peel_dense", "SQ_WAIT_INST_ANY", 150.0), (1, "k_peel_dense", "SQ_ACTIVE_INST_ANY", 300.0),
        (1, "k_peel_dense", "SQ_ACTIVE_INST_VALU", 160.0), (1, "k_peel_dense", "SQ_ACTIVE_INST_LDS", 30.0),
        (1, "k_peel_dense", "SQ_WAVES", 16.0), (1, "k_peel_dense", "SQ_BUSY_CYCLES", 10.0),
        (2, "k_peel_dense", "SQ_WAVE_CYCLES", 1000.0), (2, "k_peel_dense", "SQ_WAIT_ANY", 650.0),
        (2, "k_peel_dense", "SQ_WAIT_INST_ANY", 50.0), (2, "k_peel_dense", "SQ_ACTIVE_INST_ANY", 300.0),
        (2, "k_peel_dense", "SQ_ACTIVE_INST_VALU", 140.0), (2, "k_peel_dense", "SQ_ACTIVE_INST_LDS", 30.0),
        (2, "k_peel_dense", "SQ_WAVES", 16.0), (2, "k_peel_dense", "SQ_BUSY_CYCLES", 10.0)])

    class A:
        dir, kernels, workload, cmd, out = d, "k_peel_dense,k_absent", "wl", "c", ""
    assert P.cmd_waves(A) == 0
    row = [l for l in capsys.readouterr().out.splitlines() if l.startswith("k_peel_dense")][0].split()
    # summed over both dispatches: 1200 / 2000 waiting, 200 / 2000 ready, 600 / 2000 issuing
    assert int(row[1]) == 2
    assert [float(x) for x in row[3:]] == pytest.approx([0.6, 0.1, 0.3, 0.15, 0.03])


def test_launch_summary_pairs_rocprof_with_the_bench_line(tmp_path, capsys):
    t = _stats(tmp_path / "t", [("k_peel_dense", 4, 800e3)])   # 200 us per launch
    log = tmp_path / "bench.log"
    line = {"metric": "m", "roofline": {"achieved": 1000.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.125,
                                        "mean_launch_ms": 0.25, "alg_bytes_per_launch": 250e6}}
    log.write_text("[bench] noise\n" + json.dumps(line) + "\n")

    class A:
        dir, bench_log, kernel, workload, cmd, out = t, str(log), "k_peel_dense", "wl", "c", ""
    assert P.cmd_launch(A) == 0
    out = capsys.readouterr().out
    assert "average 200.0 us" in out and "mean 250.0 us per launch" in out
    # 250 MB over rocprofv3's 200 us: 1250 GB/s
    assert "1250.0 GB/s" in out and "15.6% of 8 TB/s" in out


def test_fd_trace_critical_path(tmp_path, capsys):
    log = tmp_path / "fd.log"
    lines = ["tip-fd-task task=0 n=10 levels=5 start_us=0.0 end_us=50.0",   # an earlier run: superseded
             "tip-fd-task task=0 n=100 levels=10 start_us=0.0 end_us=200.0",
             "tip-fd-task task=1 n=3000 levels=100 start_us=1.0 end_us=901.0",
             "tip-fd-task task=2 n=40 levels=4 start_us=0.5 end_us=40.5"]
    # the first line starts a run that the second (task 0 again) ends
    log.write_text("\n".join(lines) + "\n")

    class A:
        workload, top, cmd, out = "wl", 2, "c", ""
    A.log = str(log)
    assert P.cmd_fdtrace(A) == 0
    out = capsys.readouterr().out
    assert "3 tasks" in out and "launch span 0.90 ms" in out and "at most 100 in one subset" in out
    tops = [l for l in out.splitlines() if l.strip().startswith("task ") and "n_i" in l]
    assert len(tops) == 2 and "n_i    3000" in tops[0] and "9.0 us/level" in tops[0]


def test_traffic_record_matches_the_dense_kernel_source():
    """The committed HBM-traffic record of the dominant kernel was taken with
    its current source (otherwise the bench line reports traffic null): after
    a change to that kernel the counter runs must be repeated."""
    assert bench.load_traffic("cl-10m") is not None, bench.kernel_source_sha()
