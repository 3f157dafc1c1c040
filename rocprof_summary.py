"""Summaries of the rocprofv3 runs behind bench.py's roofline, written to profiles/.

Reads rocprofv3 CSV output (``--output-format csv``): one kernel-trace run of the headline workload and
four counter runs (FETCH_SIZE, then WRITE_SIZE, for each executor). Writes

  profiles/hiccl_<executor>_six_collectives_16r_64MiB.md        stats, trace-timed dispatches, traffic
  profiles/hiccl_staged_per_stage_six_collectives_16r_64MiB.md  every stage launch of one pass
  profiles/traffic_hiccl_<executor>_six_collectives_16r_64MiB.json  what bench.py reports as `traffic`
  profiles/precision_kernels_allreduce_reducescatter_16r_2e28.md  (with --precision-trace) the kernels of
                                                                  the precision form and its results

Counted bytes: FETCH_SIZE and WRITE_SIZE are read per dispatch in KiB and scaled by what the same counter
reads for a copy of known size in the same process (the 1 GiB device-to-device hipMemcpyAsync that
bench.py times as part of its empirical bound: 1 GiB fetched and 1 GiB written). The algorithmic bytes
come from the planner (the same plans bench.py runs, built here on host buffers).

Usage (from the repository root, after the rocprofv3 runs listed in the written files):

    python rocprof_summary.py --trace DIR --fetch-staged DIR --write-staged DIR \\
        --fetch-persistent DIR --write-persistent DIR [--out profiles]
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402  (workload constants and the plans' shapes)

PEAK = bench.PEAK_HBM
KERNEL = {"staged": "hiccl_staged<256, false>", "persistent": "hiccl_persistent<256, false>"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
WORKLOAD = "six collectives over 16 virtual ranks as {2,4,2}, 64 MiB float32 per rank, stripe 4, pipeline 8"
TRACE_ARGS = "--steps 10 --warmup 2 --no-cpu-baseline --no-batch --no-precision --no-serve"
PMC_ARGS = "--steps 2 --warmup 1 --no-cpu-baseline --no-alt --no-batch --no-precision --no-serve"


def _csv(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def trace_dispatches(d, kernel):
    """(start_ns, end_ns) of every dispatch of `kernel`, in dispatch order."""
    rows = [r for r in _csv(d, "kernel_trace.csv") if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]


def counter_values(d, kernel, counter):
    """Counter value of every dispatch of `kernel`, in dispatch order."""
    rows = [r for r in _csv(d, "counter_collection.csv") if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in rows]


def plans():
    """Per collective: the stages of its plan as (work, tiles, algorithmic bytes), and its executed bytes."""
    import numpy as np

    from paper_2408_05962_amd import collectives as CO
    d = bench.S_BYTES // 4 // bench.P
    out = {}
    for name in bench.SIX:
        snd = [np.zeros(bench.send_len(name, bench.P, d), np.float32) for _ in range(bench.P)]
        rcv = [np.zeros(bench.recv_len(name, bench.P, d), np.float32) for _ in range(bench.P)]
        c = CO.make(name, bench.P, "float32", snd, rcv, d, hierarchy=bench.HIER, stripe=bench.STRIPE,
                    pipeline=bench.PIPE, exec_mode="staged")
        info = c.plan_info()
        te = info["tile_elems"]
        stages = {}
        for t in c.plan_tasks():
            s = stages.setdefault(t["stage"], {"kinds": set(), "tiles": 0, "bytes": 0})
            k = t["nsrc"]
            s["kinds"].add("copy" if t["kind"] == 0 else f"{k}-input reduce")
            s["tiles"] += -(-t["count"] // te)
            s["bytes"] += (k + 1) * t["count"] * 4 if t["kind"] else 2 * t["count"] * 4
        out[name] = {"stages": [stages[i] for i in sorted(stages)], "exec": info["hbm_read"] + info["hbm_written"],
                     "tile_bytes": te * 4}
        c.close()
    return out


def _bench_line(log):
    """bench.py's JSON line in a captured log (None if absent)."""
    if not log or not os.path.exists(log):
        return None
    for line in open(log):
        line = line.strip()
        if line.startswith("{") and '"metric"' in line:
            return json.loads(line)
    return None


def traffic(fetch_dir, write_dir, kernel, launches, warmup, steps):
    """Counted HBM bytes of the last timed step's `launches` dispatches, calibrated on the 1 GiB copy."""
    out = {}
    for label, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        v = counter_values(d, kernel, counter)
        n = launches * (warmup + steps)
        if len(v) < n:
            raise SystemExit(f"{d}: {len(v)} dispatches of {kernel}, expected at least {n}")
        step = v[n - launches:n]
        cal = max(counter_values(d, COPY_KERNEL, counter))
        factor = (1 << 30) / (cal * 1024)
        out[label] = {"kib_step": sum(step), "cal_kib": cal, "factor": factor, "bytes_step": sum(step) * 1024 * factor}
    return out


def _stats_table(trace_dir):
    rows = _csv(trace_dir, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["| kernel | calls | avg ns | total ns | % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        lines.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['TotalDurationNs']} | "
                     f"{float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def _digests():
    import hashlib
    src = hashlib.sha256(open(os.path.join(ROOT, "paper_2408_05962_amd", "csrc", "device.hip"), "rb").read()).hexdigest()
    isa_f = os.path.join(ROOT, "paper_2408_05962_amd", "_build", "device_isa.sha256")
    isa = open(isa_f).read().strip() if os.path.exists(isa_f) else None
    return src, isa


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", help="kernel-trace run of the headline (with the four counter runs below)")
    ap.add_argument("--trace-log", help="captured output of the trace run (bench.py's JSON line)")
    for mode in ("staged", "persistent"):
        ap.add_argument(f"--fetch-{mode}")
        ap.add_argument(f"--write-{mode}")
    ap.add_argument("--precision-trace", help="kernel-trace run of the precision form (optional)")
    ap.add_argument("--precision-log", help="captured output of that run (bench.py's JSON line)")
    ap.add_argument("--batch-trace", help="kernel-trace run of the batching form alone (optional)")
    ap.add_argument("--batch-log", help="captured output of that run (bench.py --only-batch's JSON line)")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    if args.precision_trace:
        _precision(args)
    if args.batch_trace:
        _batch(args)
    if not args.trace:
        print(f"wrote summaries to {args.out}")
        return
    missing = [f"--{k}-{m}" for k in ("fetch", "write") for m in ("staged", "persistent")
               if not getattr(args, f"{k}_{m}")]
    if missing:
        raise SystemExit(f"--trace needs {' '.join(missing)}")
    P = plans()
    src, isa = _digests()
    line = _bench_line(args.trace_log)
    stage_launches = sum(len(P[n]["stages"]) for n in bench.SIX)
    exec_step = sum(P[n]["exec"] for n in bench.SIX)
    for mode in ("staged", "persistent"):
        kern = KERNEL[mode]
        launches = stage_launches if mode == "staged" else len(bench.SIX)
        # trace run: the headline executor is timed with warmup 2 + steps 10, the other with 2 + 5
        w, k = (2, 10) if mode == "staged" else (2, 5)
        disp = trace_dispatches(args.trace, kern)[: launches * (w + k)]
        timed = disp[launches * w:]
        avg_us = statistics.mean(e - s for s, e in timed) / 1e3
        tr = traffic(getattr(args, f"fetch_{mode}"), getattr(args, f"write_{mode}"), kern, launches, 1, 2)
        counted = tr["fetch"]["bytes_step"] + tr["write"]["bytes_step"]
        rec = {"kernel": kern.split("<")[0], "mode": mode, "tile_bytes": "default", "grid": "default",
               "device_source_sha256": src, "device_isa_sha256": isa,
               "traffic_bytes_per_launch": counted / launches, "launches_per_step": launches,
               "algorithmic_bytes_per_step": exec_step}
        base = f"hiccl_{mode}_six_collectives_16r_64MiB"
        with open(os.path.join(args.out, f"traffic_{base.replace('hiccl_', 'hiccl_', 1)}.json"), "w") as f:
            json.dump(rec, f, indent=1)
        ev = ""
        if line and line.get("config", {}).get("executor") == mode:
            ev = (f"- bench.py in the same run (HIP events on the launch stream): {line['roofline']['avg_launch_us']} us "
                  f"per launch, {line['roofline']['bytes_per_launch']} algorithmic bytes per launch\n")
        md = f"""# {kern.split('<')[0]} — {WORKLOAD}

Commands (from the repository root on one MI355X), then this summary:

    rocprofv3 --kernel-trace --stats --output-format csv -d {args.trace} -o kt -- python3 bench.py {TRACE_ARGS}
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d {getattr(args, f'fetch_{mode}')} -o p -- python3 bench.py {PMC_ARGS} --mode {mode}
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d {getattr(args, f'write_{mode}')} -o p -- python3 bench.py {PMC_ARGS} --mode {mode}
    python rocprof_summary.py --trace {args.trace} ... (all five directories)

## Kernel stats (rocprofv3 --stats, trace run)

{_stats_table(args.trace)}

## {kern}: timed dispatches of the trace run

- dispatches per step: {launches}; timed steps: {k}; dispatches averaged: {len(timed)}
- average dispatch duration (trace): {avg_us:.2f} us
{ev}- algorithmic bytes per step (read n + write n per hop, read k*n + write n per k-input node): {exec_step}
- achieved from the trace: {exec_step / launches / (avg_us * 1e3):.1f} GB/s per dispatch on average = {exec_step / launches / (avg_us * 1e3) / PEAK:.4f} of 8 TB/s

## HBM traffic (rocprofv3 --pmc, last timed step, calibrated)

- calibration: the 1 GiB device-to-device hipMemcpyAsync of the same process reads FETCH_SIZE {tr['fetch']['cal_kib']:.0f} KiB and WRITE_SIZE {tr['write']['cal_kib']:.0f} KiB per dispatch: factors {tr['fetch']['factor']:.4f} (fetch), {tr['write']['factor']:.4f} (write)
- one step ({launches} dispatches): fetched {tr['fetch']['bytes_step'] / 1e9:.3f} GB, written {tr['write']['bytes_step'] / 1e9:.3f} GB, total {counted / 1e9:.3f} GB
- counted / algorithmic = {counted / exec_step:.3f}
- traffic per launch: {counted / launches:.0f} bytes; counted bytes over the trace-timed dispatches: {counted / launches / (avg_us * 1e3) / PEAK:.4f} of 8 TB/s

 device.hip sha256 when profiled: {src}
 kernel instructions sha256 (paper_2408_05962_amd/build.py): {isa}
"""
        with open(os.path.join(args.out, f"{base}.md"), "w") as f:
            f.write(md)
        if mode == "staged":
            _per_stage(args, P, disp, launches, w, k, isa)
    print(f"wrote summaries to {args.out}")


PRECISION_ARGS = "--steps 1 --warmup 0 --no-batch --no-alt --no-cpu-baseline --no-serve"
BATCH_ARGS = "--only-batch"
BATCH_FORMS = ("persistent", "persistent_sjf", "defaults_persistent")


def _batch(args):
    """Kernel stats of the batching form run alone, and the merged persistent launches in it.

    The run times its forms in a fixed order (bench.py batch_bench: serial, graph, persistent,
    persistent_sjf, staged, then serial and persistent with the defaults), each as one warm run and 3
    timed runs. A merged persistent launch of the 512-collective batch is the only dispatch of
    hiccl_persistent longer than 6 ms (the 256-collective tuning batch takes about 4 ms, a single member at
    most about 0.5 ms), so those dispatches in order are the three merged persistent forms, 4 each."""
    line = None
    if args.batch_log and os.path.exists(args.batch_log):
        for raw in open(args.batch_log):
            raw = raw.strip()
            if raw.startswith("{") and '"batching"' in raw:
                line = json.loads(raw)["batching"]
    disp = trace_dispatches(args.batch_trace, "hiccl_persistent<256, false>")
    long_ms = [(e - s) / 1e6 for s, e in disp if (e - s) > 6e6]
    rows = []
    if len(long_ms) == 4 * len(BATCH_FORMS):
        for i, form in enumerate(BATCH_FORMS):
            timed = long_ms[4 * i + 1: 4 * i + 4]
            ev = line[form]["makespan_ms"] if line and form in line else "—"
            exec_b = (line or {}).get("sum_exec_bytes")
            frac = f"{exec_b / (statistics.median(timed) * 1e6) / PEAK:.3f}" if exec_b else "—"
            rows.append(f"| {form} | {', '.join(f'{t:.3f}' for t in timed)} | {statistics.median(timed):.3f} | "
                        f"{ev} | {frac} |")
    else:
        rows.append(f"| (found {len(long_ms)} dispatches over 6 ms, expected {4 * len(BATCH_FORMS)}) | | | | |")
    forms = ""
    if line:
        forms = "\n".join(f"| {k} | {line[k]['makespan_ms']} | {line[k]['hbm_frac']} | {line[k]['latency_us_p50']} | "
                          f"{line[k]['latency_us_p99']} |"
                          for k in ("serial", "graph", "persistent", "persistent_sjf", "staged",
                                    "defaults_serial", "defaults_persistent") if k in line)
    _, isa = _digests()
    md = f"""# Batching form: 512 collectives over 8 ranks as {{2,4}}, 4 KiB-64 MiB per rank, float32 / int32

Command (from the repository root on one MI355X), then this summary:

    rocprofv3 --kernel-trace --stats --output-format csv -d {args.batch_trace} -o batch -- python3 bench.py {BATCH_ARGS}
    python rocprof_summary.py --batch-trace {args.batch_trace} --batch-log <captured output>

The merged persistent forms are one `hiccl_persistent<256, false>` dispatch per run (members in groups of about 1 GiB of executed bytes, claimed along group-stage diagonals). Executed bytes per run: {(line or {}).get('sum_exec_bytes', '—')}.

## Kernel stats (rocprofv3 --stats)

{_stats_table(args.batch_trace)}

## Merged persistent launches in the trace (the 3 timed runs of each form, ms)

| form | trace durations | median | bench.py makespan (HIP events) | executed fraction of 8 TB/s (trace) |
|---|---|---|---|---|
{chr(10).join(rows)}

## The same run's bench.py batching results

Under the kernel trace the captured graph replays much more slowly than without it; its figure here is the profiler's, not the form's.

| form | makespan ms | executed fraction of 8 TB/s | latency p50 us | p99 us |
|---|---|---|---|---|
{forms}

 kernel instructions sha256 (paper_2408_05962_amd/build.py): {isa}
"""
    with open(os.path.join(args.out, "hiccl_persistent_batch_512_collectives_8r.md"), "w") as f:
        f.write(md)


def _precision(args):
    """Kernel stats of a run that includes the precision form, and that run's precision results."""
    line = _bench_line(args.precision_log)
    rows = []
    for r in (line or {}).get("precision", {}).get("results", []):
        rows.append(f"| {r['collective']} | {r['payload']} | {r['ms']} | {r['ms_persistent']} | {r['exec_GBps']} | "
                    f"{r['hbm_frac']} | {r['hbm_frac_persistent']} | {r['error_vs_float64']['scaled']:.3e} |")
    _, isa = _digests()
    md = f"""# Precision form kernels: All-Reduce and Reduce-Scatter, 16 ranks as {{2,4,2}}, 2^28 elements per rank, stripe 4, pipeline 8, float32 / bf16 / fp8-e4m3

Command (from the repository root on one MI355X), then this summary:

    rocprofv3 --kernel-trace --stats --output-format csv -d {args.precision_trace} -o prec -- python3 bench.py {PRECISION_ARGS}
    python rocprof_summary.py ... --precision-trace {args.precision_trace} --precision-log <captured output>

`<256, true>` kernels are built with the bf16 / fp8 tile paths; `<256, false>` serve int32 / float32 (here: the float32 payload runs and one headline pass). `k_to_bf16` / `k_to_fp8` convert the float32 inputs to the payload format and `k_from_*` widen results for scoring, outside the timed runs.

## Kernel stats (rocprofv3 --stats)

{_stats_table(args.precision_trace)}

## The same run's bench.py precision results (HIP events, one warm and 3 timed runs per executor)

| collective | payload | staged ms | persistent ms | executed GB/s (staged) | fraction of 8 TB/s (staged) | (persistent) | scaled error vs float64 |
|---|---|---|---|---|---|---|---|
{chr(10).join(rows)}

 kernel instructions sha256 (paper_2408_05962_amd/build.py): {isa}
"""
    with open(os.path.join(args.out, "precision_kernels_allreduce_reducescatter_16r_2e28.md"), "w") as f:
        f.write(md)


def _per_stage(args, P, disp, launches, w, k, isa):
    steps = [disp[launches * (w + i): launches * (w + i + 1)] for i in range(k)]
    rows, total_us, total_b, pos = [], 0.0, 0, 0
    for name in bench.SIX:
        for si, st in enumerate(P[name]["stages"]):
            med = statistics.median((s[pos][1] - s[pos][0]) / 1e3 for s in steps)
            gbs = st["bytes"] / (med * 1e3)
            rows.append(f"| {name} | {si} | {', '.join(sorted(st['kinds']))} | {st['tiles']} | "
                        f"{st['bytes'] / 2**20:.0f} | {med:.1f} | {gbs:.0f} | {gbs / PEAK:.3f} |")
            total_us += med
            total_b += st["bytes"]
            pos += 1
    order = ", ".join(f"{n.replace('_', '-').title()} {len(P[n]['stages'])}" for n in bench.SIX)
    md = f"""# hiccl_staged per dependency stage — {WORKLOAD}

Command (from the repository root on one MI355X; the same trace run as `hiccl_staged_six_collectives_16r_64MiB.md`):

    rocprofv3 --kernel-trace --stats --output-format csv -d {args.trace} -o kt -- python3 bench.py {TRACE_ARGS}

Each step launches {launches} stage kernels in a fixed order: {order}.
The table takes each stage's median dispatch duration (End − Start timestamp) over the {k} timed steps.
Algorithmic bytes per stage are summed over the stage's tasks from the plan (`hiccl_plan_tasks`): read n + write n per copy, read k·n + write n per k-input reduce node. Tiles are {P['broadcast']['tile_bytes'] // 1024} KiB of output.

| collective | stage | work | tiles | algorithmic MiB | median us | GB/s | fraction of 8 TB/s |
|---|---|---|---|---|---|---|---|
{chr(10).join(rows)}

sum of stage medians {total_us:.1f} us for {total_b} bytes: {total_b / (total_us * 1e3):.0f} GB/s = {total_b / (total_us * 1e3) / PEAK:.4f} of 8 TB/s

 kernel instructions sha256 (paper_2408_05962_amd/build.py): {isa}
"""
    with open(os.path.join(args.out, "hiccl_staged_per_stage_six_collectives_16r_64MiB.md"), "w") as f:
        f.write(md)


if __name__ == "__main__":
    main()
