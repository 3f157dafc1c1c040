"""Serving form on the GPU: requests admitted under an HBM budget into concurrent slots. Each result is
bit-identical alone and in the mix, and equals the oracle."""
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


def test_results_identical_alone_and_in_the_mix(torch_cuda):
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Server
    from paper_2408_05962_amd import collectives as CO
    rng = synth.choice_stream(3, 9)
    hiers = [[2, 4], [2, 4, 2], [4, 4]]
    temps = []
    for i in range(12):
        name = H.SIX[i % 6]
        h = hiers[int(rng.integers(0, 3))]
        p = int(np.prod(h))
        dtype = "int32" if i % 3 == 0 else "float32"
        d = int(rng.integers(200, 3000))
        sends = synth.rank_buffers(dtype, 21, i, p, H.send_len(name, p, d))
        S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
        R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
        c = CO.make(name, p, dtype, [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h,
                    stripe=2, pipeline=2, tile_bytes=8192, grid=64)
        c.set_spin_limit(1 << 20)
        c.set_claim(1, 4)          # one queue: progress does not depend on how many workgroups are resident
        temps.append({"c": c, "S": S, "R": R, "sends": sends, "name": name, "dtype": dtype, "h": h, "p": p,
                      "foot": (S.numel() + R.numel()) * 4 + c.workspace_size()})
    alone = []
    for tp in temps:
        tp["R"].zero_()
        tp["c"].run(torch.cuda.current_stream())
        tp["c"].wait()
        torch.cuda.synchronize()
        alone.append(tp["R"].cpu().numpy().copy())
        ranks = [0] if tp["name"] == "reduce" else range(tp["p"])
        out = alone[-1]
        H.check_result(tp["name"], {r: out[r] for r in ranks}, tp["sends"], tp["dtype"], h=tp["h"], s=2)
    for tp in temps:
        tp["R"].zero_()
    torch.cuda.synchronize()
    # a budget that fits about three requests: later ones wait until earlier ones finish
    budget = 3 * max(tp["foot"] for tp in temps)
    srv = Server(budget, 4)
    pending = list(range(len(temps)))
    tickets = {}
    refused = 0
    while pending or tickets:
        while pending:
            tk = srv.admit(temps[pending[0]]["foot"])
            if tk is None:
                refused += 1
                break
            srv.launch(tk, temps[pending[0]]["c"])
            tickets[tk] = pending.pop(0)
        srv.progress()
        used, running = srv.usage()
        assert used <= budget and running <= 4
        for tk in list(tickets):
            done, dev_us = srv.poll(tk)
            if done:
                tickets.pop(tk)
    srv.drain()
    srv.close()
    torch.cuda.synchronize()
    assert refused > 0                     # admission really deferred requests
    for k, tp in enumerate(temps):
        got = tp["R"].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), (k, tp["name"])
        tp["c"].close()


def test_admission_errors(torch_cuda):
    from paper_2408_05962_amd import Server
    from paper_2408_05962_amd.hiccl import HicclError
    srv = Server(1000, 2)
    with pytest.raises(HicclError):
        srv.admit(2000)                    # can never fit
    a = srv.admit(600)
    assert a is not None
    assert srv.admit(600) is None          # budget exhausted: deferred
    b = srv.admit(300)
    assert b is not None
    assert srv.admit(10) is None           # both slots taken
    srv.close()


def test_failed_launch_releases_and_timeouts_are_reported(torch_cuda):
    """A launch that fails gives its slot and budget back; a request whose executor gives up a
    dependency wait (forced from the host with a one-poll spin limit) is reported by poll as TIMEOUT,
    and the same template then serves correctly again."""
    torch = torch_cuda
    from paper_2408_05962_amd import Comm, Server
    from paper_2408_05962_amd import collectives as CO
    from paper_2408_05962_amd.hiccl import ERR_STATE, ERR_TIMEOUT, HicclError
    srv = Server(1 << 30, 2)
    bad = Comm(4, "float32")                     # never initialized: hiccl_run refuses it
    tk = srv.admit(1 << 20)
    with pytest.raises(HicclError) as e:
        srv.launch(tk, bad)
    assert e.value.code == ERR_STATE
    assert srv.usage() == (0, 0)                 # the ticket was released
    bad.close()
    p, h, d = 16, [2, 4, 2], 4096
    sends = [np.random.default_rng(r).integers(-1000, 1001, d * p).astype(np.int32) for r in range(p)]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros_like(S)
    c = CO.make("all_reduce", p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h,
                stripe=4, pipeline=2, tile_bytes=1024)
    c.set_claim(1, 4)
    c.set_spin_limit(1)
    timeouts = 0
    for _ in range(3):
        tk = srv.admit(1 << 20)
        srv.launch(tk, c)
        srv.drain()
        try:
            srv.poll(tk)
        except HicclError as err:
            assert err.code == ERR_TIMEOUT
            timeouts += 1
    assert timeouts > 0
    c.set_spin_limit(1 << 20)
    R.zero_()
    tk = srv.admit(1 << 20)
    srv.launch(tk, c)
    srv.drain()
    done, _ = srv.poll(tk)
    assert done
    torch.cuda.synchronize()
    out = R.cpu().numpy()
    H.check_result("all_reduce", {r: out[r] for r in range(p)}, sends, "int32")
    srv.close()
    c.close()


def test_submit_results_identical_alone_and_in_the_mix(torch_cuda):
    """hiccl_server_submit: admission with the footprint the library computes (the caller memory a
    request's primitives touch plus its workspace) and launch in one call. The templates keep the
    default claim setting (8 queues): the server itself makes a launch beside others claim from one
    queue. Every result is bit-identical to the request run alone; the budget and slots are never
    exceeded."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Server
    from paper_2408_05962_amd import collectives as CO
    rng = synth.choice_stream(5, 9)
    hiers = [[2, 4], [2, 4, 2], [4, 4]]
    temps = []
    for i in range(12):
        name = H.SIX[(i + 2) % 6]
        h = hiers[int(rng.integers(0, 3))]
        p = int(np.prod(h))
        dtype = "int32" if i % 2 == 0 else "float32"
        d = int(rng.integers(1000, 20000))
        sends = synth.rank_buffers(dtype, 22, i, p, H.send_len(name, p, d))
        S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
        R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
        c = CO.make(name, p, dtype, [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h,
                    stripe=2, pipeline=2, tile_bytes=8192)
        c.set_spin_limit(1 << 20)
        temps.append({"c": c, "S": S, "R": R, "sends": sends, "name": name, "dtype": dtype, "h": h, "p": p,
                      "foot": (S.numel() + R.numel()) * 4 + c.workspace_size()})
    st = torch.cuda.current_stream()
    alone = []
    for tp in temps:
        tp["R"].zero_()
        tp["c"].run(st)
        tp["c"].wait()
        torch.cuda.synchronize()
        alone.append(tp["R"].cpu().numpy().copy())
        ranks = [0] if tp["name"] == "reduce" else range(tp["p"])
        H.check_result(tp["name"], {r: alone[-1][r] for r in ranks}, tp["sends"], tp["dtype"], h=tp["h"], s=2)
    for tp in temps:
        tp["R"].zero_()
    torch.cuda.synchronize()
    budget = 2 * max(tp["foot"] for tp in temps)
    srv = Server(budget, 4)
    pending = list(range(len(temps)))
    tickets = {}
    while pending or tickets:
        while pending:
            tk = srv.submit(temps[pending[0]]["c"])
            if tk is None:
                break
            tickets[tk] = pending.pop(0)
        srv.progress()
        used, running = srv.usage()
        assert used <= budget and running <= 4
        for tk in list(tickets):
            done, _ = srv.poll(tk)
            if done:
                tickets.pop(tk)
    srv.drain()
    srv.close()
    torch.cuda.synchronize()
    for k, tp in enumerate(temps):
        got = tp["R"].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), (k, tp["name"])
        tp["c"].close()
