"""rocprof_summary.py on small synthetic rocprofv3 CSV directories: the trace-timed average, the traffic
per launch (calibrated on the 1 GiB copy of the same process) and the per-stage table come out of the
counter and trace rows as defined."""
import csv
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STAGED = "void hiccl::hiccl_staged<256, false>(hiccl::ExecArgs, unsigned int, unsigned int)"
PERSIST = "void hiccl::hiccl_persistent<256, false>(hiccl::ExecArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _trace(d, dispatches):
    rows = [["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 7, name, i + 1, start, end]
            for i, (name, start, end) in enumerate(dispatches)]
    _write(os.path.join(d, "kt_kernel_trace.csv"),
           ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
            "Correlation_Id", "Start_Timestamp", "End_Timestamp"], rows)
    _write(os.path.join(d, "kt_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [[STAGED, 1, 1, 1.0, 100.0, 1, 1, 0.0]])


def _counters(d, counter, per_dispatch):
    rows = [[i + 1, i + 1, "Agent 1", 1, 1, 1, 256, 7, name, 256, 0, 0, 128, 0, 64, counter, value, 0, 1]
            for i, (name, value) in enumerate(per_dispatch)]
    _write(os.path.join(d, "p_counter_collection.csv"),
           ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"],
           rows)


def test_summary_from_synthetic_csv(tmp_path, monkeypatch):
    import sys
    sys.path.insert(0, ROOT)
    try:
        import rocprof_summary as RS
        plans = RS.plans()
    except ImportError as e:
        pytest.skip(str(e))
    L = sum(len(plans[n]["stages"]) for n in RS.bench.SIX)
    # trace: staged 12 steps of L stage launches (stage i of every step lasts 1000 + i ns; the 2 warm-up
    # steps last longer), then the persistent executor's 7 steps of 6 launches of 5000 ns
    disp, t = [], 0
    for step in range(12):
        for i in range(L):
            dur = (1000 + i) if step >= 2 else 99999
            disp.append((STAGED, t, t + dur))
            t += dur + 10
    for step in range(7):
        for i in range(6):
            disp.append((PERSIST, t, t + 5000))
            t += 5010
    _trace(str(tmp_path / "kt"), disp)
    # counters: three steps of each executor; the last timed step's dispatches read 100 KiB fetched and
    # 50 KiB written each; the 1 GiB copy reads 2^19 KiB (factor 2) and writes 2^20 KiB (factor 1)
    dirs = {}
    for mode, kern, n in (("staged", STAGED, L), ("persistent", PERSIST, 6)):
        for counter, last, cal in (("FETCH_SIZE", 100.0, 2.0 ** 19), ("WRITE_SIZE", 50.0, 2.0 ** 20)):
            rows = [(kern, 1.0)] * (2 * n) + [(kern, last)] * n + [(COPY, 3.0), (COPY, cal)]
            d = tmp_path / f"{counter}_{mode}"
            _counters(str(d), counter, rows)
            dirs[(counter, mode)] = str(d)
    out = tmp_path / "profiles"
    out.mkdir()
    monkeypatch.setattr(sys, "argv", ["rocprof_summary.py", "--trace", str(tmp_path / "kt"),
                                      "--fetch-staged", dirs[("FETCH_SIZE", "staged")],
                                      "--write-staged", dirs[("WRITE_SIZE", "staged")],
                                      "--fetch-persistent", dirs[("FETCH_SIZE", "persistent")],
                                      "--write-persistent", dirs[("WRITE_SIZE", "persistent")],
                                      "--out", str(out)])
    RS.main()
    rec = json.load(open(out / "traffic_hiccl_staged_six_collectives_16r_64MiB.json"))
    # per launch: 100 KiB x factor 2 fetched + 50 KiB x factor 1 written
    assert rec["launches_per_step"] == L
    assert abs(rec["traffic_bytes_per_launch"] - (100 * 1024 * 2 + 50 * 1024)) < 1e-6
    rec = json.load(open(out / "traffic_hiccl_persistent_six_collectives_16r_64MiB.json"))
    assert rec["launches_per_step"] == 6
    md = (out / "hiccl_staged_six_collectives_16r_64MiB.md").read_text()
    mean_us = sum(1000 + i for i in range(L)) / L / 1e3
    assert f"average dispatch duration (trace): {mean_us:.2f} us" in md
    per = (out / "hiccl_staged_per_stage_six_collectives_16r_64MiB.md").read_text()
    assert "| broadcast | 0 |" in per and f"| {RS.bench.SIX[-1]} |" in per
    assert "| 1.0 |" in per          # stage 0's median: 1000 ns


def test_batch_summary_from_synthetic_csv(tmp_path, monkeypatch):
    """The batching-form summary picks the dispatches of hiccl_persistent longer than 6 ms as the three
    merged persistent forms, 4 each (one warm, 3 timed), and reports their median beside bench.py's
    makespan and the executed fraction of peak."""
    import sys
    sys.path.insert(0, ROOT)
    try:
        import rocprof_summary as RS
    except ImportError as e:
        pytest.skip(str(e))
    disp, t = [], 0
    for _ in range(50):                                  # members and the tuning batch: all shorter than 6 ms
        disp.append((PERSIST, t, t + 4_000_000))
        t += 4_000_010
    for base in (9_000_000, 9_100_000, 9_200_000):       # persistent, persistent_sjf, defaults_persistent
        for k in range(4):
            dur = base + (500_000 if k == 0 else 1000 * k)   # the warm run is slower and left out
            disp.append((PERSIST, t, t + dur))
            t += dur + 10
    _trace(str(tmp_path / "batch"), disp)
    line = {"batching": {"sum_exec_bytes": 72 * 10 ** 9,
                         **{k: {"makespan_ms": 9.0, "hbm_frac": 0.8, "latency_us_p50": 1.0, "latency_us_p99": 2.0}
                            for k in ("serial", "persistent", "persistent_sjf", "staged", "defaults_persistent")}}}
    log = tmp_path / "batch.log"
    log.write_text("[bench] progress\n" + json.dumps(line) + "\n")
    out = tmp_path / "profiles"
    out.mkdir()
    monkeypatch.setattr(sys, "argv", ["rocprof_summary.py", "--batch-trace", str(tmp_path / "batch"),
                                      "--batch-log", str(log), "--out", str(out)])
    RS.main()
    md = (out / "hiccl_persistent_batch_512_collectives_8r.md").read_text()
    # persistent: timed runs 9.001, 9.002, 9.003 ms -> median 9.002 ms; 72 GB / 9.002 ms / 8 TB/s = 0.99978
    assert "| persistent | 9.001, 9.002, 9.003 | 9.002 | 9.0 | 1.000 |" in md
    assert "| defaults_persistent | 9.201, 9.202, 9.203 | 9.202 |" in md
    assert "| staged | 9.0 | 0.8 | 1.0 | 2.0 |" in md
