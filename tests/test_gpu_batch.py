"""Batching form on the GPU: many uneven collectives in one persistent launch, a captured hipGraph, or
serial launches. Every result equals the oracle and is bit-identical to the same collective run alone."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2408_05962_amd import hiccl
    hiccl.lib()
    return torch


def _mix(torch, n, seed, p=8, h=(2, 4)):
    """n collectives of mixed type, dtype and size over p ranks; returns (specs, device buffers, host inputs)."""
    import synth
    from paper_2408_05962_amd import collectives as CO
    rng = synth.choice_stream(seed, 1)
    sizes = synth.log_uniform_sizes(seed, n, 4096, 4 << 20, p * 16)      # bytes per rank, multiple of p*16
    items = []
    for i in range(n):
        name = H.SIX[int(rng.integers(0, 6))]
        dtype = "int32" if rng.random() < 0.5 else "float32"
        d = sizes[i] // 4 // p
        if i % 5 == 0:
            d += 3                                   # ragged chunk
        s = [1, 2, 4][int(rng.integers(0, 3))]
        m = [1, 2, 4][int(rng.integers(0, 3))]
        sends = [np.asarray(x) for x in synth.rank_buffers("int32" if dtype == "int32" else "float32", 4, i, p,
                                                           H.send_len(name, p, d))]
        S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
        R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
        c = CO.make(name, p, dtype, [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=list(h),
                    stripe=s, pipeline=m, tile_bytes=16384)
        c.set_spin_limit(1 << 20)
        items.append({"name": name, "dtype": dtype, "d": d, "s": s, "m": m, "comm": c, "S": S, "R": R,
                      "sends": sends})
    return items


def _got(it, p=8):
    out = it["R"].cpu().numpy()
    ranks = [0] if it["name"] in ("reduce", "gather") else range(p)
    return {r: out[r] for r in ranks}


@pytest.mark.parametrize("mode,group_mb", [("persistent", None), ("graph", None), ("serial", None),
                                           ("persistent_sjf", None), ("staged", None),
                                           ("persistent", 1), ("persistent_sjf", 1), ("staged", 1)])
def test_batch_matches_oracle_and_alone(torch_cuda, mode, group_mb, monkeypatch):
    """group_mb = 1: the merged forms split the batch into groups of about 1 MiB of executed bytes (most
    members form a group of their own), so stage launches and claims run group after group (persistent:
    along diagonals of group and stage)."""
    torch = torch_cuda
    from paper_2408_05962_amd import Batch
    if group_mb is not None:
        monkeypatch.setenv("HICCL_BATCH_GROUP_MB", str(group_mb))
    items = _mix(torch, 24, seed=11)
    alone = []
    for it in items:
        it["R"].zero_()
        it["comm"].run(torch.cuda.current_stream())
        it["comm"].wait()
        torch.cuda.synchronize()
        alone.append(it["R"].cpu().numpy().copy())
    b = Batch([it["comm"] for it in items], mode)
    st = torch.cuda.current_stream()
    for rep in range(3):
        for it in items:
            it["R"].zero_()
        b.run(st)
        b.wait()
        torch.cuda.synchronize()
        times = b.times_ns()
        assert all(t > 0 for t in times)
        for k, it in enumerate(items):
            got = it["R"].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), (mode, rep, k, it["name"])
            H.check_result(it["name"], _got(it), it["sends"], it["dtype"], h=[2, 4], s=it["s"])
    b.close()
    for it in items:
        it["comm"].close()


@pytest.mark.parametrize("mode", ["persistent", "graph", "serial", "persistent_sjf", "staged"])
def test_batch_with_empty_members(torch_cuda, mode):
    """Empty collectives (count 0: no task) between real ones: every form runs, the real results equal the
    oracle, the empty members report a completion time of 0 and the others a positive one below a second
    (an empty member must not shift the others' time origin)."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Batch, Comm
    from paper_2408_05962_amd import collectives as CO
    p, h, d = 8, [2, 4], 8192
    comms, real = [], []
    for i in range(5):
        if i % 2 == 0:
            x = torch.zeros(p, device="cuda")
            c = Comm(p, "float32")
            c.add_multicast([x[r] for r in range(p)], [x[r] for r in range(p)], 0, 0, [1, 2, 3])
            c.set_hierarchy(h)
            c.init()
            comms.append(c)
            continue
        sends = [np.asarray(x) for x in synth.rank_buffers("int32", 8, i, p, H.send_len("all_reduce", p, d))]
        S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
        R = torch.zeros((p, H.recv_len("all_reduce", p, d)), dtype=S.dtype, device="cuda")
        c = CO.make("all_reduce", p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h)
        comms.append(c)
        real.append((i, S, R, sends))
    b = Batch(comms, mode)
    st = torch.cuda.current_stream()
    for _ in range(2):
        for _, _, R, _ in real:
            R.zero_()
        b.run(st)
        b.wait()
        torch.cuda.synchronize()
        times = b.times_ns()
        for i, t in enumerate(times):
            if i % 2 == 0:
                assert t == 0, (mode, times)
            else:
                assert 0 < t < 10**9, (mode, times)
        for _, _, R, sends in real:
            out = R.cpu().numpy()
            H.check_result("all_reduce", {r: out[r] for r in range(p)}, sends, "int32", h=h)
    b.close()
    for c in comms:
        c.close()


@pytest.mark.parametrize("mode", ["persistent", "persistent_sjf", "staged"])
def test_grouped_batch_completes_group_by_group(torch_cuda, mode, monkeypatch):
    """With groups of about 1 MiB of executed bytes, the merged forms finish their members in group order:
    batch order for the persistent launch and the stage launches, smallest first for persistent_sjf. The
    members are 32 int32 All-Reduces over 8 ranks whose sizes fall along the batch order, so smallest
    first reverses it. The first eight members to run must finish, in median, before the last eight, and
    every result equals the oracle."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Batch
    from paper_2408_05962_amd import collectives as CO
    monkeypatch.setenv("HICCL_BATCH_GROUP_MB", "1")
    p, h, n = 8, [2, 4], 32
    items = []
    for i in range(n):
        d = 4096 * (n - i)                       # buffers of 4 MiB down to 128 KiB per rank
        sends = [np.asarray(x) for x in synth.rank_buffers("int32", 6, i, p, H.send_len("all_reduce", p, d))]
        S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
        R = torch.zeros((p, H.recv_len("all_reduce", p, d)), dtype=S.dtype, device="cuda")
        c = CO.make("all_reduce", p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h)
        c.set_spin_limit(1 << 20)
        items.append({"comm": c, "S": S, "R": R, "sends": sends})
    b = Batch([it["comm"] for it in items], mode)
    st = torch.cuda.current_stream()
    for rep in range(2):
        for it in items:
            it["R"].zero_()
        b.run(st)
        b.wait()
        torch.cuda.synchronize()
        times = np.array(b.times_ns(), dtype=np.float64)
        run_order = times if mode != "persistent_sjf" else times[::-1]
        assert np.median(run_order[:8]) < np.median(run_order[-8:]), (mode, rep, times.tolist())
    for it in items:
        out = it["R"].cpu().numpy()
        H.check_result("all_reduce", {r: out[r] for r in range(p)}, it["sends"], "int32", h=h)
    b.close()
    for it in items:
        it["comm"].close()


@pytest.mark.parametrize("kind", ["exhaustive", "model"])
def test_autotuners_pick_a_valid_configuration(torch_cuda, kind):
    torch = torch_cuda
    from paper_2408_05962_amd import autotune, autotune_model
    from paper_2408_05962_amd import collectives as CO
    p, h, d = 8, [2, 4], 8192
    sends = [np.random.default_rng(r).integers(-1000, 1001, d * p).astype(np.int32) for r in range(p)]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros_like(S)
    c = CO.make("all_reduce", p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h)
    st = torch.cuda.current_stream()
    if kind == "exhaustive":
        r = autotune(c, [1, 2, 4], [1, 2, 4], [16384, 65536], reps=2, stream=st)
    else:
        r = autotune_model(c, [1, 2, 4], [1, 2, 4], [16384, 65536], reps=2, anchors=4, top=2, stream=st)
        assert r["measured"] <= 6
    assert r["stripe"] in (1, 2, 4) and r["pipeline"] in (1, 2, 4) and r["us"] > 0
    R.zero_()
    c.run(st)
    c.wait()
    torch.cuda.synchronize()
    out = R.cpu().numpy()
    H.check_result("all_reduce", {q: out[q] for q in range(p)}, sends, "int32")
    c.close()


def test_staged_batch_of_program_ordered_plans(torch_cuda):
    """The merged stage-by-stage batch regroups tables by stage even when a plan was ordered otherwise."""
    torch = torch_cuda
    from paper_2408_05962_amd import Batch
    from paper_2408_05962_amd import collectives as CO
    p, h, d = 8, [2, 4], 1000
    outs = []
    for mode in (None, "staged"):
        comms, Rs, sends_all = [], [], []
        for i, name in enumerate(["all_reduce", "broadcast", "all_to_all"]):
            sends = [np.random.default_rng(10 * i + r).standard_normal(H.send_len(name, p, d)).astype(np.float32)
                     for r in range(p)]
            S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
            R = torch.zeros((p, H.recv_len(name, p, d)), dtype=torch.float32, device="cuda")
            c = CO.make(name, p, "float32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h,
                        stripe=2, pipeline=2, tile_bytes=4096, order="program")
            comms.append((c, S))
            Rs.append(R)
            sends_all.append((name, sends))
        st = torch.cuda.current_stream()
        if mode is None:
            for c, _ in comms:
                c.run(st)
                c.wait()
        else:
            b = Batch([c for c, _ in comms], mode)
            b.run(st)
            b.wait()
            b.close()
        torch.cuda.synchronize()
        outs.append([R.cpu().numpy() for R in Rs])
        for (name, sends), R in zip(sends_all, outs[-1]):
            ranks = range(p)
            H.check_result(name, {r: R[r] for r in ranks}, sends, "float32", h=h, s=2)
        for c, _ in comms:
            c.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.timeout(400)
def test_batch_512_full_size(torch_cuda):
    """The measured batch itself: 512 collectives over 8 ranks as {2,4}, 4 KiB-64 MiB per rank, float32 /
    int32, with the bench's seeds and its default policy (s = m = 1, default tile). In one persistent launch
    (batch order and smallest first), in the captured graph and in merged stage launches every result is bit-identical (compared on the device) to the same collective
    run alone; those alone results equal the oracle for every collective up to 4 MiB per rank and for the
    largest collective of each type. The merged forms run the batch in groups of members (1 GiB of executed
    bytes for the persistent launch, 4 GiB for stage launches), so several groups are exercised."""
    torch = torch_cuda
    import bench as B
    import synth
    from paper_2408_05962_amd import Batch
    from paper_2408_05962_amd import collectives as CO
    n, p = 512, B.BATCH_P
    rng = synth.choice_stream(4, 2)
    sizes = synth.log_uniform_sizes(4, n, 4 << 10, 64 << 20, p * 16)
    items = []
    for i in range(n):
        name = B.SIX[int(rng.integers(0, 6))]
        dtype = "int32" if rng.random() < 0.5 else "float32"
        c, snd, rcv, S = B._mk(torch, CO, name, p, B.BATCH_H, dtype, sizes[i], 5000 + i)
        c.set_spin_limit(1 << 20)
        items.append({"name": name, "dtype": dtype, "c": c, "snd": snd, "rcv": rcv, "S": S})
    st = torch.cuda.current_stream()
    alone = []
    for it in items:
        it["rcv"].zero_()
        it["c"].run(st)
        it["c"].wait()
        alone.append(it["rcv"].clone())
    torch.cuda.synchronize()
    largest = {}
    for k, it in enumerate(items):
        if it["S"] > largest.get(it["name"], (-1, 0))[1]:
            largest[it["name"]] = (k, it["S"])
    checked = {k for k, _ in largest.values()} | {k for k, it in enumerate(items) if it["S"] <= 4 << 20}
    for k in sorted(checked):
        it = items[k]
        sends = list(it["snd"].cpu().numpy())
        out = alone[k].cpu().numpy()
        ranks = [0] if it["name"] == "reduce" else range(p)
        # (the float32 tree-order emulation is skipped above 4 MiB per rank to bound the host time)
        H.check_result(it["name"], {r: out[r] for r in ranks}, sends, it["dtype"], h=B.BATCH_H, s=1,
                       order_exact=it["S"] <= 4 << 20)
    for mode in ("persistent", "graph", "staged", "persistent_sjf"):
        for it in items:
            it["rcv"].zero_()
        b = Batch([it["c"] for it in items], mode)
        b.run(st)
        b.wait()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            assert torch.equal(it["rcv"].view(torch.int32), alone[k].view(torch.int32)), (mode, k, it["name"])
        b.close()
    for it in items:
        it["c"].close()


@pytest.mark.parametrize("mode", ["persistent", "graph"])
def test_run_batch_memoized(torch_cuda, mode):
    """hiccl_run_batch: the members run as one memoized batch; waiting on any member waits for all; every
    result is bit-identical to the collective run alone. A member run alone in between leaves the batch,
    and the next call runs it in the batch again."""
    torch = torch_cuda
    from paper_2408_05962_amd import run_batch
    items = _mix(torch, 12, seed=23)
    st = torch.cuda.current_stream()
    alone = []
    for it in items:
        it["R"].zero_()
        it["comm"].run(st)
        it["comm"].wait()
        torch.cuda.synchronize()
        alone.append(it["R"].cpu().numpy().copy())
    comms = [it["comm"] for it in items]
    for rep in range(3):
        for it in items:
            it["R"].zero_()
        run_batch(comms, st, mode)
        comms[(5 * rep) % len(comms)].wait()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            got = it["R"].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), (mode, rep, k, it["name"])
        if rep == 1:
            it = items[3]
            it["R"].zero_()
            it["comm"].run(st)
            it["comm"].wait()
            torch.cuda.synchronize()
            assert np.array_equal(it["R"].cpu().numpy().view(np.uint32), alone[3].view(np.uint32))
    for k, it in enumerate(items):
        H.check_result(it["name"], _got(it), it["sends"], it["dtype"], h=[2, 4], s=it["s"])
        it["comm"].close()


def test_autotune_batch_choices_are_valid_and_results_exact(torch_cuda):
    """hiccl_autotune_batch: per-class choices come from the candidate lists, the members are left planned
    with them, and the batch then gives every collective's oracle result."""
    torch = torch_cuda
    from paper_2408_05962_amd import Batch, autotune_batch
    items = _mix(torch, 12, seed=31)
    for it in items:                       # start every member from the defaults the tuner starts from
        it["comm"].set_stripe(1)
        it["comm"].set_pipeline(1)
        it["comm"].set_exec("persistent", 16384)
        it["comm"].init()
    classes = [H.SIX.index(it["name"]) % 3 for it in items]
    res = autotune_batch([it["comm"] for it in items], classes, [1, 2], [1, 2, 4], [16384, 65536], reps=2,
                         sweeps=1, stream=torch.cuda.current_stream())
    assert len(res["choice"]) == max(classes) + 1 and res["ms"] > 0
    for s, m, t in res["choice"]:
        assert s in (1, 2) and m in (1, 2, 4) and t in (16384, 65536)
    for it, k in zip(items, classes):
        s, m, _ = res["choice"][k]
        it["s"] = s
        it["R"].zero_()
    b = Batch([it["comm"] for it in items], "persistent")
    b.run(torch.cuda.current_stream())
    b.wait()
    torch.cuda.synchronize()
    b.close()
    for it in items:
        H.check_result(it["name"], _got(it), it["sends"], it["dtype"], h=[2, 4], s=it["s"])
        it["comm"].close()
