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
            "all_to_all": d * p, "scatter": d, "gather": d * p}[name]


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


def _cpu_block_worker(job):
    """One process of the all-cores baseline: the six collectives over 16 ranks on its block of elements
    (n elements per rank), repeated for `budget_s`; returns (bytes done, seconds spent in the oracle)."""
    import synth
    from oracle import collectives as OC
    n, block, budget_s = job
    d = n // P
    fns = {
        "broadcast": lambda s: OC.broadcast(s, 0),
        "reduce": lambda s: OC.reduce(s, 0),
        "all_gather": lambda s: OC.all_gather([x[:d] for x in s]),
        "reduce_scatter": lambda s: OC.reduce_scatter(s),
        "all_reduce": lambda s: OC.all_reduce(s),
        "all_to_all": lambda s: OC.all_to_all(s),
    }
    sends = [synth.rank_buffer("float32", 1, block, r, n) for r in range(P)]
    done, spent = 0, 0.0
    t_end = time.perf_counter() + budget_s
    while time.perf_counter() < t_end:
        for name in SIX:
            t0 = time.perf_counter()
            fns[name](sends)
            spent += time.perf_counter() - t0
            done += n * 4
    return done, spent


def cpu_baseline_all_cores(budget_s: float = 10.0) -> dict:
    """The same oracle and sample split over element blocks, one block per process on the host's cores
    (the machine's CPU share, at most 16): every collective here is elementwise per element block, so the
    blocks are independent. Aggregate rate = sum of the processes' rates (they run concurrently)."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    n = (4 * 2 ** 20) // 4 // workers // (P * 4) * (P * 4)
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_cpu_block_worker, [(n, 1 + w, budget_s) for w in range(workers)])
    rate = sum(b / t for b, t in res if t > 0)
    return {"value": round(rate / 1e9, 3), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"six collectives, 16 ranks, 4 MiB float32 per rank split into {workers} element blocks of "
                      f"{n} elements per rank, one process each, ~{budget_s:.0f} s each (float64 oracle)"}


# ------------------------------------------------------------------ batching form
BATCH_P, BATCH_H = 8, [2, 4]
SIZE_CLASSES = [(4 << 10, 64 << 10), (64 << 10, 1 << 20), (1 << 20, 16 << 20), (16 << 20, 64 << 20)]


def _size_class(nbytes):
    for i, (lo, hi) in enumerate(SIZE_CLASSES):
        if nbytes < hi:
            return i
    return len(SIZE_CLASSES) - 1


def _mk(torch, CO, name, p, h, dtype, per_rank_bytes, seed, s=1, m=1, tile=0, grid=0, ring=1, mode="persistent"):
    """A communicator with its own device buffers for a collective of `per_rank_bytes` (largest buffer)."""
    import synth
    es = 2 if dtype == "bfloat16" else 4
    d = max(1, per_rank_bytes // es // p)
    if dtype == "bfloat16":
        d = max(8, d // 8 * 8)
    kind = "int32" if dtype == "int32" else "float32"
    snd = synth.device_buffers(kind, seed, p, send_len(name, p, d))
    if dtype == "bfloat16":
        snd = snd.to(torch.bfloat16).view(torch.int16)
    rcv = torch.zeros((p, recv_len(name, p, d)), dtype=snd.dtype, device="cuda")
    c = CO.make(name, p, dtype, [snd[r] for r in range(p)], [rcv[r] for r in range(p)], d, hierarchy=h, stripe=s,
                pipeline=m, tile_bytes=tile, grid=grid, ring=ring, exec_mode=mode)
    return c, snd, rcv, d * p * es


def tune_batch_policy(torch, n=256, seed=99):
    """Batched-context tuning: on a batch drawn like the measured one but from another seed, the library's
    batch autotuner (hiccl_autotune_batch) picks (stripe, pipeline, tile) per (collective, size class) by
    coordinate descent on the merged persistent launch, starting from the defaults (s = m = 1, default
    tile). Returns the per-class table, the tuning batch's time under the defaults and tuned, and the time
    spent."""
    import synth
    from paper_2408_05962_amd import Batch, autotune_batch
    from paper_2408_05962_amd import collectives as CO
    rng = synth.choice_stream(seed, 2)
    sizes = synth.log_uniform_sizes(seed, n, 4 << 10, 64 << 20, BATCH_P * 16)
    st = torch.cuda.current_stream()
    comms, keep, classes = [], [], []
    for i in range(n):
        name = SIX[int(rng.integers(0, 6))]
        dtype = "int32" if rng.random() < 0.5 else "float32"
        c, snd, rcv, _ = _mk(torch, CO, name, BATCH_P, BATCH_H, dtype, sizes[i], 9000 + i)
        comms.append(c)
        keep.append((snd, rcv))
        classes.append(SIX.index(name) * len(SIZE_CLASSES) + _size_class(sizes[i]))
    b = Batch(comms, "persistent")
    b.run(st)
    b.wait()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(3):
        b.run(st)
    e1.record(st)
    b.wait()
    torch.cuda.synchronize()
    default_ms = e0.elapsed_time(e1) / 3
    b.close()
    t0 = time.perf_counter()
    res = autotune_batch(comms, classes, [1, 2, 4], [1, 2, 4, 8], [0, 16384, 131072], mode="persistent", reps=3,
                         sweeps=2, stream=st)
    tune_s = time.perf_counter() - t0
    table = {}
    for k, choice in enumerate(res["choice"]):
        table[(SIX[k // len(SIZE_CLASSES)], k % len(SIZE_CLASSES))] = tuple(choice)
    for c in comms:
        c.close()
    del keep
    return table, {"defaults": round(default_ms, 3), "tuned": round(res["ms"], 3)}, tune_s


def batch_bench(torch, n=512, seed=4, reps=3):
    import numpy as np

    import synth
    from paper_2408_05962_amd import Batch
    from paper_2408_05962_amd import collectives as CO
    table, tuning_ms, tune_s = tune_batch_policy(torch)
    _progress(f"batch tuning: {tuning_ms} in {tune_s:.1f} s")
    rng = synth.choice_stream(seed, 2)
    sizes = synth.log_uniform_sizes(seed, n, 4 << 10, 64 << 20, BATCH_P * 16)
    items = []
    t_plan = time.perf_counter()
    for i in range(n):
        name = SIX[int(rng.integers(0, 6))]
        dtype = "int32" if rng.random() < 0.5 else "float32"
        s, m, tile = table[(name, _size_class(sizes[i]))]
        c, snd, rcv, S = _mk(torch, CO, name, BATCH_P, BATCH_H, dtype, sizes[i], 5000 + i, s, m, tile)
        info = c.plan_info()
        items.append((c, snd, rcv, S, info["hbm_read"] + info["hbm_written"], name, dtype))
        if (i + 1) % 128 == 0:
            _progress(f"batch: planned {i + 1} of {n}")
    t_plan = time.perf_counter() - t_plan
    comms = [it[0] for it in items]
    total_S = sum(it[3] for it in items)
    total_exec = sum(it[4] for it in items)
    st = torch.cuda.current_stream()
    out = {"collectives": n, "ranks": BATCH_P, "hierarchy": BATCH_H, "sum_S_bytes": total_S,
           "sum_exec_bytes": total_exec, "tune_s": round(tune_s, 2), "plan_s": round(t_plan, 2),
           "policy": "tuned in the batch (hiccl_autotune_batch, coordinate descent over (collective, size class) "
                     "on a 256-collective tuning batch of another seed)",
           "tuned": {f"{k[0]}/{SIZE_CLASSES[k[1]][0]}": v for k, v in table.items()},
           "tuning_batch_ms": tuning_ms}

    def timed(comms, mode, total_exec):
        b = Batch(comms, mode)
        b.run(st)
        b.wait()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        spans, lat = [], []
        for _ in range(reps):
            e0.record(st)
            b.run(st)
            e1.record(st)
            b.wait()
            torch.cuda.synchronize()
            spans.append(e0.elapsed_time(e1))
            lat.append(np.asarray(b.times_ns(), dtype=np.float64) / 1e3)
        b.close()
        ms = float(np.median(spans))
        L = np.concatenate(lat)
        return {"makespan_ms": round(ms, 3), "algbw_GBps": round(total_S / ms / 1e6, 1),
                "exec_GBps": round(total_exec / ms / 1e6, 1),
                "hbm_frac": round(total_exec / ms / 1e6 / PEAK_HBM, 4),
                "latency_us_p50": round(float(np.percentile(L, 50)), 1),
                "latency_us_p99": round(float(np.percentile(L, 99)), 1)}

    for mode in ("serial", "graph", "persistent", "persistent_sjf", "staged"):
        out[mode] = timed(comms, mode, total_exec)
        _progress(f"batch {mode}: {out[mode]['makespan_ms']:.3f} ms")
    for c in comms:
        c.close()
    # the same collectives on the same buffers with the defaults (s = m = 1, default tile): what tuning is worth
    plain = []
    for i, (c, snd, rcv, S, _, name, dtype) in enumerate(items):
        d = S // (BATCH_P * 4)
        plain.append(CO.make(name, BATCH_P, dtype, [snd[r] for r in range(BATCH_P)], [rcv[r] for r in range(BATCH_P)],
                             d, hierarchy=BATCH_H))
    plain_exec = 0
    for c in plain:
        info = c.plan_info()
        plain_exec += info["hbm_read"] + info["hbm_written"]
    for mode in ("serial", "persistent"):
        out[f"defaults_{mode}"] = timed(plain, mode, plain_exec)
        _progress(f"batch defaults {mode}: {out[f'defaults_{mode}']['makespan_ms']:.3f} ms")
    for c in plain:
        c.close()
    return out


def _time_comm(torch, c, reps=10, warm=2):
    """Mean time (ms) of `reps` back-to-back runs of one communicator, HIP events on the stream."""
    st = torch.cuda.current_stream()
    for _ in range(warm):
        c.run(st)
    c.wait()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        c.run(st)
    e1.record(st)
    c.wait()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sweep_bench(torch):
    """Measurements beside the headline: pipeline depth, ring vs tree, two-step compositions, the
    autotuners, Scatter / Gather and one rank's share."""
    import numpy as np

    import synth
    from paper_2408_05962_amd import collectives as CO
    out = {}
    st = torch.cuda.current_stream()
    d = S_BYTES // 4 // P

    def mk(name, h, s, m, mode, ring=1, seed=1, p=P, dd=d, dtype="float32"):
        kind = "int32" if dtype == "int32" else "float32"
        snd = synth.device_buffers(kind, seed, p, send_len(name, p, dd))
        rcv = torch.zeros((p, recv_len(name, p, dd)), dtype=snd.dtype, device="cuda")
        c = CO.make(name, p, dtype, [snd[r] for r in range(p)], [rcv[r] for r in range(p)], dd, hierarchy=h,
                    stripe=s, pipeline=m, exec_mode=mode, ring=ring)
        return c, snd, rcv

    # pipeline depth (the shape of the paper's pipeline-depth experiment, Sec. 6.4, on HBM)
    rows = []
    for m in (1, 2, 4, 8, 16, 32):
        row = {"pipeline": m}
        for mode in ("staged", "persistent"):
            c, snd, rcv = mk("all_reduce", HIER, STRIPE, m, mode)
            ms = _time_comm(torch, c)
            info = c.plan_info()
            row[mode] = {"ms": round(ms, 4), "exec_GBps": round((info["hbm_read"] + info["hbm_written"]) / ms / 1e6, 1),
                         "stages": info["nstages"], "tasks": info["ntasks"]}
            c.close()
            del snd, rcv
        rows.append(row)
        _progress(f"pipeline sweep m={m}: {row}")
    out["pipeline_depth_all_reduce"] = rows

    # task timeline of the persistent executor (hiccl_set_trace): how much the dependency stages of one
    # All-Reduce overlap in time at pipeline depth 1 and 8 (the picture of Sec. 4.5, from the device clock)
    import numpy as np
    tl = {}
    for m in (1, 8):
        c, snd, rcv = mk("all_reduce", HIER, STRIPE, m, "persistent")
        c.set_trace(True)
        for _ in range(3):
            c.run(st)
            c.wait()
        start, end = c.trace()
        stage = np.array([t["stage"] for t in c.plan_tasks()])
        span = int(end.max())
        windows = [[round(int(start[stage == k].min()) / 1e3, 1), round(int(end[stage == k].max()) / 1e3, 1)]
                   for k in np.unique(stage)]
        busy = sum(w[1] - w[0] for w in windows)
        tl[f"m{m}"] = {"span_us": round(span / 1e3, 1), "stage_windows_us": windows,
                       "stage_busy_over_span": round(busy / (span / 1e3), 3), "tasks": len(start)}
        c.close()
        del snd, rcv
        _progress(f"timeline m={m}: {tl[f'm{m}']}")
    out["task_timeline_all_reduce_persistent"] = tl

    # ring(4) + tree vs tree on 16 ranks as {4,4} (Sec. 4.4)
    ring = {}
    for name in SIX:
        r = {}
        for label, rg in (("tree", 1), ("ring4", 4)):
            for mode in ("staged", "persistent"):
                c, snd, rcv = mk(name, [4, 4], 1, PIPE, mode, ring=rg)
                ms = _time_comm(torch, c)
                info = c.plan_info()
                r[f"{label}_{mode}_ms"] = round(ms, 4)
                r[f"{label}_stages"] = info["nstages"]
                c.close()
                del snd, rcv
        ring[name] = r
        _progress(f"ring {name}: {r}")
    out["ring_vs_tree_16r_4x4_64MiB"] = ring

    # two-step rows of Table 2 (a fence and a scratch buffer of d*p per rank) against the single-step form
    from paper_2408_05962_amd import Comm
    two = {}
    for name in ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast"):
        base = "all_reduce" if name == "all_reduce_bcast" else name
        snd = synth.device_buffers("float32", 7, P, send_len(base, P, d))
        rcv = torch.zeros((P, recv_len(base, P, d)), device="cuda")
        scr = torch.zeros((P, d * P), device="cuda")
        c = Comm(P, "float32")
        CO.compose_multi(c, name, [snd[r] for r in range(P)], [rcv[r] for r in range(P)], [scr[r] for r in range(P)],
                         d, root=0)
        c.set_hierarchy(HIER)
        c.set_stripe(STRIPE)
        c.set_pipeline(PIPE)
        c.set_exec("staged")
        c.init()
        ms2 = _time_comm(torch, c)
        info = c.plan_info()
        c.close()
        c = CO.make(base, P, "float32", [snd[r] for r in range(P)], [rcv[r] for r in range(P)], d, hierarchy=HIER,
                    stripe=STRIPE, pipeline=PIPE, exec_mode="staged")
        ms1 = _time_comm(torch, c)
        c.close()
        two[name] = {"two_step_ms": round(ms2, 4), "single_step_ms": round(ms1, 4),
                     "two_step_exec_GBps": round((info["hbm_read"] + info["hbm_written"]) / ms2 / 1e6, 1)}
        del snd, rcv, scr
    out["two_step_vs_single_step"] = two
    _progress(f"two-step: {two}")

    # the model-guided autotuner against exhaustive search (24 candidates), persistent executor
    from paper_2408_05962_amd import autotune, autotune_model
    tun = {}
    for size in (1 << 20, S_BYTES):
        dd = size // 4 // P
        for name in SIX:
            snd = synth.device_buffers("float32", 11, P, send_len(name, P, dd))
            rcv = torch.zeros((P, recv_len(name, P, dd)), device="cuda")
            res = {}
            for kind in ("exhaustive", "model"):
                c = CO.make(name, P, "float32", [snd[r] for r in range(P)], [rcv[r] for r in range(P)], dd,
                            hierarchy=HIER)
                if kind == "exhaustive":
                    r = autotune(c, [1, 2, 4], [1, 2, 4, 8], [16384, 65536], reps=3, stream=st)
                    r["measured"] = 24
                else:
                    r = autotune_model(c, [1, 2, 4], [1, 2, 4, 8], [16384, 65536], reps=3, anchors=5, top=3, stream=st)
                res[kind] = r
                c.close()
            tun[f"{name}/{size >> 20}MiB"] = {
                "exhaustive_us": round(res["exhaustive"]["us"], 1), "model_us": round(res["model"]["us"], 1),
                "model_over_exhaustive": round(res["model"]["us"] / res["exhaustive"]["us"], 3),
                "model_measured": res["model"]["measured"],
                "exhaustive_pick": [res["exhaustive"][k] for k in ("stripe", "pipeline", "tile_bytes")],
                "model_pick": [res["model"][k] for k in ("stripe", "pipeline", "tile_bytes")]}
            del snd, rcv
    out["autotuner_model_vs_exhaustive"] = tun
    _progress(f"autotuners: {tun}")

    # Scatter / Gather at the headline shape
    sg = {}
    for name in ("scatter", "gather"):
        c, snd, rcv = mk(name, HIER, STRIPE, PIPE, "staged")
        ms = _time_comm(torch, c)
        info = c.plan_info()
        sg[name] = {"ms": round(ms, 4), "algbw_GBps": round(S_BYTES / ms / 1e6, 1),
                    "exec_GBps": round((info["hbm_read"] + info["hbm_written"]) / ms / 1e6, 1)}
        c.close()
        del snd, rcv
    out["scatter_gather"] = sg
    _progress(f"scatter/gather: {sg}")

    # one rank's share at the headline shape: the tasks whose output lies in rank r's memory, i.e. the
    # work one GPU would do if each virtual rank were its own GPU pulling remote operands (Sec. 5.1)
    shares = {}
    for name in SIX:
        c, snd, rcv = mk(name, HIER, STRIPE, PIPE, "staged")
        info = c.plan_info()
        full_ms = _time_comm(torch, c)
        W = torch.empty(max(c.workspace_size(), 256), dtype=torch.uint8, device="cuda")
        c.set_workspace(W, W.numel())
        c.run(st)
        c.wait()
        per = []
        for r in range(P):
            sc = CO.make(name, P, "float32", [snd[q] for q in range(P)], [rcv[q] for q in range(P)], d,
                         hierarchy=HIER, stripe=STRIPE, pipeline=PIPE, exec_mode="staged", share=r)
            sc.set_workspace(W, W.numel())
            si = sc.plan_info()
            per.append((_time_comm(torch, sc), si["hbm_read"] + si["hbm_written"], si["nstages"]))
            sc.close()
        k = max(range(P), key=lambda r: per[r][0])
        shares[name] = {"full_ms": round(full_ms, 4),
                        "full_exec_GB": round((info["hbm_read"] + info["hbm_written"]) / 1e9, 3),
                        "max_share_ms": round(per[k][0], 4), "max_share_rank": k,
                        "max_share_exec_GB": round(per[k][1] / 1e9, 3), "max_share_stages": per[k][2],
                        "max_share_exec_GBps": round(per[k][1] / per[k][0] / 1e6, 1),
                        "mean_share_ms": round(float(np.mean([x[0] for x in per])), 4),
                        "sum_share_ms": round(float(np.sum([x[0] for x in per])), 4),
                        "largest_share_exec_GB": round(max(x[1] for x in per) / 1e9, 3)}
        c.close()
        del snd, rcv, W
        _progress(f"rank shares {name}: {shares[name]}")
    out["one_rank_share_16r_64MiB_staged"] = shares

    return out


def small_all_reduce_bench(torch):
    """The small All-Reduce of the latency-bound configuration: 4 ranks as {2,2}, 65,536 int32 per rank,
    s = m = 1. Device time between events and host time from the call to the result, p50 / p99 over 50
    runs, on each executor and through the device request ring; every form checked against the int32 sum."""
    import numpy as np

    import synth
    from paper_2408_05962_amd import collectives as CO
    st = torch.cuda.current_stream()

    def mk(name, h, s, m, mode, p, dd, dtype):
        snd = synth.device_buffers(dtype, 1, p, send_len(name, p, dd))
        rcv = torch.zeros((p, recv_len(name, p, dd)), dtype=snd.dtype, device="cuda")
        c = CO.make(name, p, dtype, [snd[r] for r in range(p)], [rcv[r] for r in range(p)], dd, hierarchy=h,
                    stripe=s, pipeline=m, exec_mode=mode)
        return c, snd, rcv

    # the small All-Reduce: 4 ranks as {2,2}, 65,536 int32 per rank, s = m = 1 (latency-bound)
    small = {}
    for mode in ("staged", "persistent"):
        c, snd, rcv = mk("all_reduce", [2, 2], 1, 1, mode, 4, 65536 // 4, "int32")
        lat = []
        for _ in range(3):
            c.run(st)
        c.wait()
        host = []
        for _ in range(50):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(st)
            c.run(st)
            e1.record(st)
            c.wait()
            host.append((time.perf_counter() - t0) * 1e6)
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1) * 1e3)
        ok = bool(torch.equal(rcv[0], snd.sum(0, dtype=torch.int32)) and torch.equal(rcv[3], rcv[0]))
        small[mode] = {"latency_us_p50": round(float(np.percentile(lat, 50)), 2),
                       "latency_us_p99": round(float(np.percentile(lat, 99)), 2), "matches_sum": ok,
                       "host_us_p50": round(float(np.percentile(host, 50)), 2),
                       "host_us_p99": round(float(np.percentile(host, 99)), 2)}
        c.close()
        del snd, rcv
    # the same request through the device request ring: host clock from append to the completion word
    from paper_2408_05962_amd import Server
    c, snd, rcv = mk("all_reduce", [2, 2], 1, 1, "persistent", 4, 65536 // 4, "int32")
    srv = Server(1 << 40, 1, ring=True, idle_ms=1000)
    lat = []
    for k in range(53):
        t0 = time.perf_counter()
        tk = srv.admit(1)
        srv.launch(tk, c)
        while not srv.poll(tk)[0]:
            pass
        if k >= 3:
            lat.append((time.perf_counter() - t0) * 1e6)
    srv.close()
    ok = bool(torch.equal(rcv[0], snd.sum(0, dtype=torch.int32)) and torch.equal(rcv[3], rcv[0]))
    small["device_ring"] = {"latency_us_p50": round(float(np.percentile(lat, 50)), 2),
                            "latency_us_p99": round(float(np.percentile(lat, 99)), 2), "matches_sum": ok,
                            "clock": "host, append to completion word"}
    c.close()
    del snd, rcv
    _progress(f"small all-reduce: {small}")
    return small


def _progress(msg):
    """A progress line on stderr (the JSON result stays the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _errors(got, exact, scale):
    """Error of a computed sum against its exact value: largest absolute error; largest error scaled by
    max(|exact|, sum of |inputs|) (what the summation error bound limits); largest plain relative error
    where |exact| >= 1e-3 * sum |inputs|; normwise relative error."""
    import numpy as np
    diff = np.abs(got - exact)
    well = np.abs(exact) >= 1e-3 * scale
    nrm = float(np.linalg.norm(exact))
    return {"max_abs": float(diff.max()),
            "scaled": float((diff / np.where(np.maximum(np.abs(exact), scale) == 0, 1.0,
                                             np.maximum(np.abs(exact), scale))).max()),
            "rel_well_conditioned": float((diff[well] / np.abs(exact[well])).max()) if np.any(well) else 0.0,
            "normwise": float(np.linalg.norm(got - exact) / nrm) if nrm > 0 else float(np.linalg.norm(got - exact))}


# ----------------------------------------------------------------- precision
def precision_bench(torch, reps=3, n=1 << 28):
    """All-Reduce and Reduce-Scatter over 16 ranks as {2,4,2}, 2^28 elements per rank ~ N(0,1) with 1 % of
    entries x 1e3, stripe 4, pipeline 8; payload float32 vs bf16 vs fp8-e4m3 (per-256 power-of-two
    scales), float32 accumulation. Both executors run every result (one warm run, then `reps` timed) and
    must leave the same bytes; the error of that result against the float64 sum of the original float32
    inputs is measured over the whole chunks 0 and p-1 (every stripe, channel and tile boundary of a
    chunk)."""
    import numpy as np

    import synth
    from paper_2408_05962_amd import collectives as CO
    from paper_2408_05962_amd import from_payload, to_payload
    p, h, s, m = 16, [2, 4, 2], 4, 8
    d = n // p
    X = synth.device_buffers("float32_outliers", 301, p, n)
    st = torch.cuda.current_stream()
    chunks = (0, p - 1)
    # the exact sums of the scored chunks, from the original float32 inputs
    exact = {}
    for j in chunks:
        xs = X[:, j * d:(j + 1) * d].cpu().numpy().astype(np.float64)
        exact[j] = (xs.sum(0), np.abs(xs).sum(0))
        del xs
    out = {"ranks": p, "elements_per_rank": n, "stripe": s, "pipeline": m, "timed_reps": reps,
           "scored": f"whole chunks {list(chunks)} ({d} elements each) of every result, against the float64 "
                    "sum of the original float32 inputs", "results": []}
    W = torch.empty(d, dtype=torch.float32, device="cuda")
    for name in ("all_reduce", "reduce_scatter"):
        rl = recv_len(name, p, d)
        for dtype in ("float32", "bfloat16", "fp8_e4m3"):
            es = {"float32": 4, "bfloat16": 2, "fp8_e4m3": 1}[dtype]
            tdt = {"float32": torch.float32, "bfloat16": torch.int16, "fp8_e4m3": torch.uint8}[dtype]
            Y = Sc = None
            if dtype == "float32":
                send = [X[r] for r in range(p)]
            else:
                Y = torch.empty((p, n), dtype=tdt, device="cuda")
                Sc = torch.empty((p, n // 256), dtype=torch.float32, device="cuda") if dtype == "fp8_e4m3" else None
                for r in range(p):
                    to_payload(dtype, X[r], Y[r], Sc[r] if Sc is not None else None, n, st)
                send = [Y[r] for r in range(p)] if Sc is None else [(Y[r], Sc[r]) for r in range(p)]
            times, res, info = {}, {}, None
            for mode in ("staged", "persistent"):
                R = torch.zeros((p, rl), dtype=tdt, device="cuda")
                RS = torch.zeros((p, rl // 256), dtype=torch.float32, device="cuda") if dtype == "fp8_e4m3" else None
                recv = [R[r] for r in range(p)] if RS is None else [(R[r], RS[r]) for r in range(p)]
                c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=s, pipeline=m, exec_mode=mode)
                info = c.plan_info()
                c.run(st)
                c.wait()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                for _ in range(reps):
                    c.run(st)
                e1.record(st)
                c.wait()
                torch.cuda.synchronize()
                times[mode] = e0.elapsed_time(e1) / reps
                c.close()
                res[mode] = (R, RS)
            (R, RS), (R2, RS2) = res["staged"], res["persistent"]
            same = bool(torch.equal(R, R2) and (RS is None or torch.equal(RS, RS2)))
            assert same, f"precision {name} {dtype}: the two executors' results differ"
            del res, R2, RS2
            # error over the scored chunks: the library widens the result to float32 on the device
            errs = []
            for j in chunks:
                col = 0 if name == "reduce_scatter" else j * d
                if dtype == "float32":
                    W.copy_(R[j, col:col + d])
                else:
                    from_payload(dtype, R[j, col:col + d], RS[j, col // 256:(col + d) // 256] if RS is not None else None,
                                 W, d, st)
                torch.cuda.synchronize()
                errs.append(_errors(W.cpu().numpy().astype(np.float64), *exact[j]))
            worst = {k: max(e[k] for e in errs) for k in errs[0]}
            exec_b = info["hbm_read"] + info["hbm_written"]
            ms = times["staged"]
            _progress(f"precision {name} {dtype}: staged {ms:.3f} ms, persistent {times['persistent']:.3f} ms, "
                      f"scaled error {worst['scaled']:.3e}")
            out["results"].append({
                "collective": name, "payload": dtype, "ms": round(ms, 3),
                "ms_persistent": round(times["persistent"], 3),
                "algbw_GBps": round(n * es / ms / 1e6, 1),
                "algbw_float32_equivalent_GBps": round(n * 4 / ms / 1e6, 1),
                "exec_bytes": exec_b, "exec_GBps": round(exec_b / ms / 1e6, 1),
                "hbm_frac": round(exec_b / ms / 1e6 / PEAK_HBM, 4),
                "hbm_frac_persistent": round(exec_b / times["persistent"] / 1e6 / PEAK_HBM, 4),
                "executors_bit_identical": same,
                "error_vs_float64": {k: float(f"{v:.3e}") for k, v in worst.items()}})
            del R, RS, Y, Sc, send
            torch.cuda.empty_cache()
    del X, W
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------- serving form
SERVE_HIERS = [[2, 4], [2, 4, 2], [4, 4]]


def serve_templates(torch, ntemplates=48, seed=8, mode="persistent"):
    """Resident request templates of the serving mix: type uniform over the six, hierarchy from {2x4, 2x4x2,
    4x4}, per-rank size log-uniform in [1 KiB, 256 MiB], dtype from {int32, float32, bf16}. Each is run once
    (buffers and schedule resident from then on)."""
    import numpy as np

    import synth
    from paper_2408_05962_amd import collectives as CO
    rng = synth.choice_stream(seed, 3)
    sizes = synth.log_uniform_sizes(seed, ntemplates, 1 << 10, 256 << 20, 16 * 16)
    temps = []
    for i in range(ntemplates):
        name = SIX[int(rng.integers(0, 6))]
        h = SERVE_HIERS[int(rng.integers(0, 3))]
        p = int(np.prod(h))
        dtype = ["int32", "float32", "bfloat16"][int(rng.integers(0, 3))]
        s = 4 if p == 16 else 2
        m = 8 if sizes[i] >= (1 << 20) else 1
        c, snd, rcv, S = _mk(torch, CO, name, p, h, dtype, sizes[i], 7000 + i, s, m, mode=mode)
        if mode == "persistent":
            c.set_claim(1, 4)    # one tile queue: progress holds however many of its workgroups are resident
        foot = snd.numel() * snd.element_size() + rcv.numel() * rcv.element_size() + c.workspace_size()
        c.run(torch.cuda.current_stream())
        c.wait()
        temps.append({"comm": c, "snd": snd, "rcv": rcv, "S": S, "foot": foot, "name": name, "p": p, "h": h,
                      "dtype": dtype, "stripe": s})
    torch.cuda.synchronize()
    return temps


def serve_bench(torch, ntemplates=48, nreq=2000, fractions=(0.25, 0.5, 0.75, 0.9, 1.2), slots=4,
                budget=200 * 10 ** 9, seed=8, mode="persistent"):
    """Poisson stream of collective requests over resident request templates, served three ways: one
    launch per request on concurrent slots (continuous batching), the device request ring (one resident
    launch serving the requests the host appends), and one request at a time (FIFO).

    Templates are drawn from the serving mix (type uniform over the six, hierarchy from {2x4, 2x4x2, 4x4},
    per-rank size log-uniform in [1 KiB, 256 MiB], dtype from {int32, float32, bf16}); each keeps its
    buffers and schedule resident. A request picks a template; it is admitted when a slot and budget are
    free and its template is idle. Latency = arrival to completion (host clock)."""
    import numpy as np

    import synth
    from paper_2408_05962_amd import Server
    temps = serve_templates(torch, ntemplates, seed, mode)

    def run_stream(arrivals, picks, nslots, ring=False):
        srv = Server(budget, nslots, ring=ring)
        busy = [False] * len(temps)
        queue, inflight, lat = [], {}, []
        t0 = time.perf_counter()
        i = 0
        n = len(arrivals)
        while len(lat) < n:
            now = time.perf_counter() - t0
            while i < n and arrivals[i] <= now:
                queue.append((arrivals[i], picks[i]))
                i += 1
            # admit in arrival order while a slot, budget and the template are free
            k = 0
            while k < len(queue):
                arr, tp = queue[k]
                if busy[tp]:
                    k += 1
                    continue
                tk = srv.admit(temps[tp]["foot"])
                if tk is None:
                    break
                srv.launch(tk, temps[tp]["comm"])
                busy[tp] = True
                inflight[tk] = (arr, tp)
                queue.pop(k)
            srv.progress()
            for tk in list(inflight):
                done, _ = srv.poll(tk)
                if done:
                    arr, tp = inflight.pop(tk)
                    busy[tp] = False
                    lat.append(time.perf_counter() - t0 - arr)
            if not queue and not inflight and i < n:
                time.sleep(max(0.0, min(arrivals[i] - (time.perf_counter() - t0), 0.001)))
        span = time.perf_counter() - t0
        srv.drain()
        srv.close()
        return span, np.asarray(lat)

    g = synth.choice_stream(seed, 4)
    picks = g.integers(0, len(temps), nreq)
    # closed loop: everything arrives at once -> sustained service rate mu
    span, _ = run_stream(np.zeros(nreq), picks, slots)
    mu = nreq / span
    ring_ok = mode == "persistent"          # the device ring serves persistent-executor templates
    mu_ring = nreq / run_stream(np.zeros(nreq), picks, slots, ring=True)[0] if ring_ok else None
    _progress(f"serve closed loop: {mu:.1f} requests/s (device ring: {mu_ring})")
    out = {"executor": mode, "templates": ntemplates, "requests_per_rate": nreq, "slots": slots, "budget_bytes": budget,
           "mu_req_per_s": round(mu, 1), "mu_ring_req_per_s": round(mu_ring, 1) if mu_ring else None, "rates": []}
    for f in fractions:
        lam = f * mu
        arrivals = np.cumsum(g.exponential(1.0 / lam, nreq))
        row = {"fraction_of_mu": f, "lambda_req_per_s": round(lam, 1)}
        forms = (("continuous", slots, False), ("ring", slots, True), ("fifo", 1, False))
        for label, ns, ring in forms:
            if ring and not ring_ok:
                continue
            span, lat = run_stream(arrivals, picks, ns, ring)
            Sb = sum(temps[tp]["S"] for tp in picks)
            row[label] = {"throughput_req_per_s": round(nreq / span, 1), "algbw_GBps": round(Sb / span / 1e9, 2),
                          "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                          "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3)}
        out["rates"].append(row)
        _progress(f"serve rate {f}: {row}")
    for tpl in temps:
        tpl["comm"].close()
    return out


def empirical_bound(torch, nbytes=1 << 30, reps=10):
    """Empirical device-memory bound in the same run (the analog of the paper's empirical bounds): one
    1 GiB copy as the executor's own plan (a one-leaf multicast between two virtual ranks, one copy task
    of 32768 tiles), on each executor, and hipMemcpyAsync device-to-device. Read + write bytes over the
    event-timed duration."""
    import ctypes

    from paper_2408_05962_amd import Comm
    n = nbytes // 4
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    st = torch.cuda.current_stream()
    out = {"bytes_per_copy": nbytes}
    for mode in ("staged", "persistent"):
        c = Comm(2, "float32")
        c.add_multicast([x, x], [y, y], n, 0, [1])
        c.set_hierarchy([2])
        c.set_exec(mode)
        c.init()
        out[f"hiccl_copy_{mode}_GBps"] = round(2 * nbytes / _time_comm(torch, c, reps=reps) / 1e6, 1)
        c.close()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p]
    hip.hipMemcpyAsync.restype = ctypes.c_int
    D2D = 3        # hipMemcpyDeviceToDevice
    for _ in range(3):
        assert hip.hipMemcpyAsync(y.data_ptr(), x.data_ptr(), nbytes, D2D, st.cuda_stream) == 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        assert hip.hipMemcpyAsync(y.data_ptr(), x.data_ptr(), nbytes, D2D, st.cuda_stream) == 0
    e1.record(st)
    torch.cuda.synchronize()
    out["hipMemcpyDtoD_GBps"] = round(2 * nbytes / (e0.elapsed_time(e1) / reps) / 1e6, 1)
    del x, y
    return out


def measured_traffic(mode, tile, grid):
    """HBM bytes per launch of the headline kernel from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when they were taken on other kernel
    code (the digest of the built kernels' instructions differs) or another launch configuration."""
    kname = "hiccl_staged" if mode == "staged" else "hiccl_persistent"
    path = os.path.join(ROOT, "profiles", f"traffic_{kname}_six_collectives_16r_64MiB.json")
    digest = os.path.join(ROOT, "paper_2408_05962_amd", "_build", "device_isa.sha256")
    if tile or grid or not os.path.exists(path) or not os.path.exists(digest):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(digest) as f:
        isa = f.read().strip()
    if rec.get("device_isa_sha256") != isa or rec.get("mode") != mode:
        return None
    return round(rec["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="staged", choices=["persistent", "staged"])
    ap.add_argument("--tile", type=int, default=0, help="tile bytes (0 = the executor's default)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups (0 = the executor's default)")
    ap.add_argument("--no-alt", action="store_true", help="skip timing the other executor")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--batch", action="store_true", help="(default) measure the batching form: 512 collectives, "
                    "batched vs one launch per collective, throughput and p50/p99 latency")
    ap.add_argument("--no-batch", action="store_true", help="skip the batching form")
    ap.add_argument("--only-batch", action="store_true",
                    help="measure only the batching form and print its JSON object (for a kernel trace of it)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving form (Poisson requests)")
    ap.add_argument("--serve-requests", type=int, default=500, help="requests per arrival rate")
    ap.add_argument("--serve-rates", default="0.5,0.9,1.2",
                    help="arrival rates as fractions of the closed-loop service rate")
    ap.add_argument("--serve-exec", default="persistent", choices=["staged", "persistent"],
                    help="executor of the serving templates")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision form (bf16 / fp8)")
    ap.add_argument("--no-small", action="store_true", help="skip the small All-Reduce (4 ranks, 256 KiB per rank)")
    ap.add_argument("--sweep", action="store_true",
                    help="also measure pipeline depth, ring vs tree, two-step compositions, the autotuners, "
                         "Scatter / Gather and one rank's share")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the virtual ranks of the hierarchy "
                                   "live in one GPU's memory; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import synth
    from paper_2408_05962_amd import collectives as CO

    torch.cuda.init()
    if args.only_batch:
        print(json.dumps({"batching": batch_bench(torch)}), flush=True)
        return
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    S_el = S_BYTES // 4
    d = S_el // P

    bufs = {}
    for i, name in enumerate(SIX):
        snd = synth.device_buffers("float32", 100 + i, P, send_len(name, P, d), device="cuda")
        rcv = torch.zeros((P, recv_len(name, P, d)), dtype=torch.float32, device=dev)
        bufs[name] = (snd, rcv)
    torch.cuda.synchronize()

    def measure(mode, tile, grid, steps, warmup):
        """Time `steps` passes of the six collectives with one executor; per-collective HIP events on `st`."""
        comms, info = {}, {}
        for name in SIX:
            snd, rcv = bufs[name]
            c = CO.make(name, P, "float32", [snd[r] for r in range(P)], [rcv[r] for r in range(P)], d,
                        hierarchy=HIER, stripe=STRIPE, pipeline=PIPE, exec_mode=mode, tile_bytes=tile, grid=grid)
            comms[name] = c
            info[name] = c.plan_info()
        for _ in range(warmup):
            for name in SIX:
                comms[name].run(st)
        for name in SIX:
            comms[name].wait()
        torch.cuda.synchronize()
        ev = {name: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                     for _ in range(steps)] for name in SIX}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            for name in SIX:
                a, b = ev[name][k]
                a.record(st)
                comms[name].run(st)
                b.record(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for name in SIX:
            comms[name].wait()
            comms[name].close()
        per, kern_ms, kern_bytes, launches = {}, 0.0, 0, 0
        for name in SIX:
            ms = sum(a.elapsed_time(b) for a, b in ev[name]) / steps
            exec_bytes = info[name]["hbm_read"] + info[name]["hbm_written"]
            nl = info[name]["nstages"] if mode == "staged" else 1
            kern_ms += ms
            kern_bytes += exec_bytes
            launches += nl
            per[name] = {"ms": round(ms, 4), "algbw_GBps": round(S_BYTES / ms / 1e6, 1),
                         "exec_bytes": exec_bytes, "exec_GBps": round(exec_bytes / ms / 1e6, 1),
                         "hbm_frac": round(exec_bytes / ms / 1e6 / PEAK_HBM, 4), "launches": nl,
                         "tasks": info[name]["ntasks"], "tiles": info[name]["ntiles"],
                         "stages": info[name]["nstages"]}
        return {"step_ms": (t1 - t0) * 1e3 / steps, "per": per, "kern_ms": kern_ms, "kern_bytes": kern_bytes,
                "launches": launches, "tile": tile, "grid": grid}

    head = measure(args.mode, args.tile, args.grid, args.steps, args.warmup)
    _progress(f"{args.mode}: {head['step_ms']:.3f} ms per step")
    alt_mode = "persistent" if args.mode == "staged" else "staged"
    alt = None if args.no_alt else measure(alt_mode, 0, 0, max(5, args.steps // 2), 2)
    step_ms, per, kern_ms, kern_bytes = head["step_ms"], head["per"], head["kern_ms"], head["kern_bytes"]

    # sanity: All-Reduce rows agree and match a host sum at a few sampled elements
    snd, rcv = bufs["all_reduce"]
    idx = torch.tensor([0, 1, S_el // 2, S_el - 1], device=dev)
    got = rcv[:, idx].double().cpu()
    ref = snd[:, idx].double().sum(0).cpu()
    assert torch.all(got == got[0]), "All-Reduce rows differ"
    assert torch.allclose(got[0], ref, rtol=1e-5, atol=1e-4), "All-Reduce disagrees with the sampled sum"

    bound = empirical_bound(torch)

    achieved = kern_bytes / kern_ms / 1e6
    kname = "hiccl_staged<256, false>" if args.mode == "staged" else "hiccl_persistent<256, false>"
    traffic = measured_traffic(args.mode, args.tile, args.grid)
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
                   "executor": args.mode, "tile_bytes": head["tile"] or "default", "grid": head["grid"] or "default"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM, 4), "traffic": traffic,
                     # counted HBM bytes (calibrated FETCH_SIZE + WRITE_SIZE per launch) over the launch time
                     "hbm_counted_frac": (round(traffic / (kern_ms * 1e-3 / head["launches"]) / 1e9 / PEAK_HBM, 4)
                                          if traffic else None),
                     "kernel": kname, "launches_per_step": head["launches"],
                     "bytes_per_launch": round(kern_bytes / head["launches"]),
                     "avg_launch_us": round(kern_ms * 1e3 / head["launches"], 2)},
        "per_collective": per,
        "empirical_bound": bound,
    }
    if alt is not None:
        out["other_executor"] = {"executor": alt_mode, "ms_per_step": round(alt["step_ms"], 4),
                                 "value": round(len(SIX) * S_BYTES / alt["step_ms"] / 1e6, 2),
                                 "exec_GBps": round(alt["kern_bytes"] / alt["kern_ms"] / 1e6, 1),
                                 "hbm_frac": round(alt["kern_bytes"] / alt["kern_ms"] / 1e6 / PEAK_HBM, 4),
                                 "per_collective_ms": {n: v["ms"] for n, v in alt["per"].items()},
                                 "per_collective_hbm_frac": {n: v["hbm_frac"] for n, v in alt["per"].items()}}
    del bufs
    torch.cuda.empty_cache()
    if not args.no_precision:
        out["precision"] = precision_bench(torch)
        torch.cuda.empty_cache()
    if not args.no_small:
        out["small_all_reduce_4r_2x2_int32_256KiB"] = small_all_reduce_bench(torch)
    if args.sweep:
        out["sweep"] = sweep_bench(torch)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batching"] = batch_bench(torch)
        torch.cuda.empty_cache()
    if not args.no_serve:
        rates = tuple(float(x) for x in args.serve_rates.split(","))
        out["serving"] = serve_bench(torch, nreq=args.serve_requests, fractions=rates, mode=args.serve_exec)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(args.cpu_budget / 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
