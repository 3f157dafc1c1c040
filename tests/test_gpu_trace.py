"""The persistent executor's task timeline (hiccl_set_trace / hiccl_trace_tasks) on the GPU: every task is
stamped, and for every dependency edge of the plan the successor started no earlier than its predecessor
finished. That checks the executor's dependency protocol from the device's own clock, on both kernel
instantiations (int32 / float32 tables and bf16 / fp8 tables); the results stay exact."""
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


def _check_timeline(c):
    start, end = c.trace()
    tasks = c.plan_tasks()
    a, b = c.plan_edges()
    assert len(start) == len(tasks) > 0
    assert np.all(end > 0), "a task was never stamped as finished"
    assert start.min() == 0                                   # times count from the earliest start
    assert np.all(start <= end)
    late = [(int(x), int(y)) for x, y in zip(a.tolist(), b.tolist()) if start[y] < end[x]]
    assert not late, f"successors started before their predecessors finished: {late[:5]}"
    return start, end


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_trace_respects_every_dependency(torch_cuda, dtype):
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import collectives as CO
    name, p, h, s, m, d = "all_reduce", 16, [2, 4, 2], 4, 4, 65536
    sends = [np.asarray(x) for x in synth.rank_buffers("float32", 9, 1, p, H.send_len(name, p, d))]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    if dtype == "bfloat16":
        S = S.to(torch.bfloat16).view(torch.int16)
        sends = [x for x in S.view(torch.bfloat16).float().cpu().numpy()]
    R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
    c = CO.make(name, p, dtype, [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=s,
                pipeline=m)
    c.set_trace(True)
    st = torch.cuda.current_stream()
    for _ in range(2):
        R.zero_()
        c.run(st)
        c.wait()
        _check_timeline(c)
    out = R.view(torch.bfloat16).float().cpu().numpy() if dtype == "bfloat16" else R.cpu().numpy()
    if dtype == "float32":
        H.check_result(name, {r: out[r] for r in range(p)}, sends, "float32", h=h, s=s)
    else:
        assert np.all(out == out[0])                          # every rank holds the same bytes
        exact = np.sum(np.asarray(sends, np.float64), axis=0)
        scale = np.sum(np.abs(np.asarray(sends, np.float64)), axis=0)
        assert np.max(np.abs(out[0] - exact) / np.maximum(scale, 1e-30)) < 0.05
    c.set_trace(False)                                        # off again: runs as before, no timeline
    R.zero_()
    c.run(st)
    c.wait()
    from paper_2408_05962_amd.hiccl import ERR_STATE, HicclError
    with pytest.raises(HicclError) as e:
        c.trace()
    assert e.value.code == ERR_STATE
    c.close()


def test_trace_overlaps_channels(torch_cuda):
    """With pipelining (m = 8) the dependency stages of one All-Reduce overlap in time (Sec. 4.5): the
    stages' busy windows add up to more than the run's span. With m = 1 they still overlap less."""
    torch = torch_cuda
    from paper_2408_05962_amd import collectives as CO
    p, h, d = 16, [2, 4, 2], 1 << 20
    S = torch.randn(p, d * p, device="cuda")
    R = torch.zeros_like(S)
    sums = {}
    for m in (1, 8):
        c = CO.make("all_reduce", p, "float32", [S[r] for r in range(p)], [R[r] for r in range(p)], d,
                    hierarchy=h, stripe=4, pipeline=m)
        c.set_trace(True)
        st = torch.cuda.current_stream()
        for _ in range(2):
            c.run(st)
            c.wait()
        start, end = _check_timeline(c)
        stage = np.array([t["stage"] for t in c.plan_tasks()])
        busy = sum(int(end[stage == k].max() - start[stage == k].min()) for k in np.unique(stage))
        sums[m] = busy / int(end.max())
        c.close()
    assert sums[8] > 1.0, sums
    assert sums[8] > sums[1], sums


@pytest.mark.parametrize("name", H.SIX)
def test_trace_dependencies_every_collective(torch_cuda, name):
    """Every one of the six collectives at 16 ranks as {2,4,2}, s = 4, m = 4 (the persistent executor's
    claim orders differ: stage order for the copy-only collectives, diagonal channel groups for the
    reduction ones): no successor starts before its predecessor finished, and the result equals the
    oracle."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import collectives as CO
    p, h, s, m, d = 16, [2, 4, 2], 4, 4, 16384
    sends = [np.asarray(x) for x in synth.rank_buffers("int32", 10, H.SIX.index(name), p, H.send_len(name, p, d))]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
    c = CO.make(name, p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=s,
                pipeline=m)
    c.set_trace(True)
    st = torch.cuda.current_stream()
    c.run(st)
    c.wait()
    _check_timeline(c)
    out = R.cpu().numpy()
    ranks = [0] if name == "reduce" else range(p)
    H.check_result(name, {r: out[r] for r in ranks}, sends, "int32", h=h, s=s)
    c.close()


@pytest.mark.parametrize("name", ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast"])
def test_trace_two_step_fences(torch_cuda, name):
    """The two-step rows of Table 2: a fence between the steps makes a task of the second step wait only
    for the first-step tasks whose ranges overlap its own (Sec. 3.3). On the device clock, every such
    edge is respected, and the result equals the direct definition."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Comm
    from paper_2408_05962_amd import collectives as CO
    p, h, s, m, d = 16, [2, 4, 2], 4, 2, 4096 + 3
    base = "all_reduce" if name == "all_reduce_bcast" else name
    sends = [np.asarray(x) for x in synth.rank_buffers("int32", 11, len(name), p, H.send_len(base, p, d))]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.full((p, H.recv_len(base, p, d)), -7, dtype=torch.int32, device="cuda")
    X = torch.zeros((p, d * p), dtype=torch.int32, device="cuda")
    c = Comm(p, "int32")
    CO.compose_multi(c, name, [S[r] for r in range(p)], [R[r] for r in range(p)], [X[r] for r in range(p)], d,
                     root=p - 1)
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_pipeline(m)
    c.set_trace(True)
    c.init()
    c.run(torch.cuda.current_stream())
    c.wait()
    _check_timeline(c)
    steps = {t["step"] for t in c.plan_tasks()}
    assert len(steps) == 2
    out = R.cpu().numpy()
    ranks = [p - 1] if base in ("reduce", "gather") else range(p)
    H.check_result(base, {r: out[r] for r in ranks}, sends, "int32", root=p - 1)
    c.close()
