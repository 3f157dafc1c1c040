"""Benchmark of the hierarchical collective executor on one MI355X.

Workload: the six collectives (Broadcast, Reduce, All-Gather,
Reduce-Scatter, All-Reduce, All-to-All) over 16 virtual ranks factorized as
{2 nodes, 4 devices, 2 dies}, 64 MiB of float32 ~ N(0,1) per rank (the
largest per-rank buffer), stripe 4, pipeline depth 8. One step runs all six
collectives once; inputs are resident in device memory before timing.

Prints one JSON line: aggregate algorithm bandwidth (sum of per-rank buffer
sizes over the step time), per-collective detail, the roofline of the
executor kernel (executed device-memory bytes over its event-timed
duration, against 8 TB/s), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SIX = ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_to_all")
P, HIER, STRIPE, PIPE = 16, [2, 4, 2], 4, 8
S_BYTES = 64 * 2 ** 20
PEAK_HBM = 8000.0     # GB/s, MI355X HBM3E
METRIC = "algbw GB/s & %HBM roofline per collective; p50/p99 latency batched vs plain"


def send_len(name, p, d):
    return d if name in ("all_gather", "gather") else d * p


def recv_len(name, p, d):
    return {"broadcast": d * p, "reduce": d * p, "all_gather": d * p, "reduce_scatter": d, "all_reduce": d * p,
            "all_to_all": d * p}[name]


def cpu_baseline(budget_s: float = 20.0) -> dict:
    """The oracle (float64 definitions) timed on host cores over a bounded sample of the same workload."""
    import numpy as np

    import synth
    from oracle import collectives as OC

    # sample: the six collectives at 16 ranks with 4 MiB per rank (1/16 of the workload's buffers)
    n = (4 * 2 ** 20) // 4
    d = n // P
    fns = {
        "broadcast": lambda s: OC.broadcast(s, 0),
        "reduce": lambda s: OC.reduce(s, 0),
        "all_gather": lambda s: OC.all_gather([x[:d] for x in s]),
        "reduce_scatter": lambda s: OC.reduce_scatter(s),
        "all_reduce": lambda s: OC.all_reduce(s),
        "all_to_all": lambda s: OC.all_to_all(s),
    }
    sends = [synth.rank_buffer("float32", 1, 0, r, n) for r in range(P)]
    done_bytes, spent, reps = 0, 0.0, 0
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end:
        for name in SIX:
            t0 = time.perf_counter()
            fns[name](sends)
            spent += time.perf_counter() - t0
            done_bytes += n * 4
        reps += 1
    return {"value": round(done_bytes / spent / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"six collectives x {reps} passes, 16 ranks, 4 MiB float32 per rank (float64 oracle, "
                      f"numpy on one core of {os.cpu_count()})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="persistent", choices=["persistent", "staged"])
    ap.add_argument("--tile", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the virtual ranks of the hierarchy "
                                   "live in one GPU's memory; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_2408_05962_amd import collectives as CO

    torch.cuda.init()
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    S_el = S_BYTES // 4
    d = S_el // P

    comms, bufs, info = {}, {}, {}
    for i, name in enumerate(SIX):
        snd = synth.device_buffers("float32", 100 + i, P, send_len(name, P, d), device="cuda")
        rcv = torch.zeros((P, recv_len(name, P, d)), dtype=torch.float32, device=dev)
        c = CO.make(name, P, "float32", [snd[r] for r in range(P)], [rcv[r] for r in range(P)], d, hierarchy=HIER,
                    stripe=STRIPE, pipeline=PIPE, exec_mode=args.mode, tile_bytes=args.tile)
        comms[name] = c
        bufs[name] = (snd, rcv)
        info[name] = c.plan_info()
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        for name in SIX:
            comms[name].run(st)
    for name in SIX:
        comms[name].wait()
    torch.cuda.synchronize()

    ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)] for name in SIX}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for name in SIX:
            a, b = ev[name][k]
            a.record(st)
            comms[name].run(st)
            b.record(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for name in SIX:
        comms[name].wait()

    step_ms = (t1 - t0) * 1e3 / args.steps
    per, kern_ms, kern_bytes = {}, 0.0, 0
    for name in SIX:
        ms = sum(a.elapsed_time(b) for a, b in ev[name]) / args.steps
        exec_bytes = info[name]["hbm_read"] + info[name]["hbm_written"]
        kern_ms += ms
        kern_bytes += exec_bytes
        per[name] = {"ms": round(ms, 4), "algbw_GBps": round(S_BYTES / ms / 1e6, 1),
                     "exec_bytes": exec_bytes, "exec_GBps": round(exec_bytes / ms / 1e6, 1),
                     "hbm_frac": round(exec_bytes / ms / 1e6 / PEAK_HBM, 4),
                     "tasks": info[name]["ntasks"], "tiles": info[name]["ntiles"], "stages": info[name]["nstages"]}

    # sanity: All-Reduce rows agree and match a host sum at a few sampled elements
    snd, rcv = bufs["all_reduce"]
    idx = torch.tensor([0, 1, S_el // 2, S_el - 1], device=dev)
    got = rcv[:, idx].double().cpu()
    ref = snd[:, idx].double().sum(0).cpu()
    assert torch.all(got == got[0]), "All-Reduce rows differ"
    assert torch.allclose(got[0], ref, rtol=1e-5, atol=1e-4), "All-Reduce disagrees with the sampled sum"

    # empirical copy bound in the same run: a 1 GiB device-to-device copy
    x = torch.empty(2 ** 28, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(st)
    for _ in range(10):
        y.copy_(x)
    c1.record(st)
    torch.cuda.synchronize()
    copy_gbps = 2 * x.numel() * 4 / (c0.elapsed_time(c1) / 10) / 1e6
    del x, y

    achieved = kern_bytes / kern_ms / 1e6
    out = {
        "metric": METRIC,
        "value": round(len(SIX) * S_BYTES / step_ms / 1e6, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "six collectives (broadcast, reduce, all-gather, reduce-scatter, all-reduce, "
                               "all-to-all), 16 virtual ranks as {2,4,2}, 64 MiB float32 N(0,1) per rank, "
                               "stripe 4, pipeline 8",
                   "executor": args.mode, "tile_bytes": args.tile},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM, 4), "traffic": None},
        "per_collective": per,
        "empirical_copy_GBps": round(copy_gbps, 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    for c in comms.values():
        c.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
