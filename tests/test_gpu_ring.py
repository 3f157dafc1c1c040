"""The serving form's device request ring on the GPU: one resident launch serves the requests the host
appends. Each result is bit-identical to the same request run alone (which equals the oracle), an idle
ring exits and the next request starts it again, and a request whose dependency wait expires is reported
as TIMEOUT while the ring keeps serving."""
import time

import numpy as np
import pytest

from tests import harness as H
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2408_05962_amd import hiccl
    hiccl.lib()
    return torch


def _template(torch, name, h, dtype, d, seed, s=2, m=2, tile=8192):
    import synth
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    sends = synth.rank_buffers(dtype, 31, seed, p, H.send_len(name, p, d))
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, H.recv_len(name, p, d)), dtype=S.dtype, device="cuda")
    c = CO.make(name, p, dtype, [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=s,
                pipeline=m, tile_bytes=tile)
    c.set_spin_limit(1 << 20)
    return {"c": c, "S": S, "R": R, "sends": sends, "name": name, "dtype": dtype, "h": h, "p": p, "s": s}


def _serve(torch, srv, temps, order):
    """Admit and launch the templates in `order` as slots free up; wait for all of them."""
    torch.cuda.current_stream().synchronize()      # the buffers' clearing is done before the ring reads them
    pending, tickets = list(order), {}
    t0 = time.time()
    while pending or tickets:
        assert time.time() - t0 < 60, "ring requests did not finish"
        while pending:
            tk = srv.admit(1 << 20)
            if tk is None:
                break
            srv.launch(tk, temps[pending.pop(0)]["c"])
            tickets[tk] = True
        srv.progress()
        for tk in list(tickets):
            done, _ = srv.poll(tk)
            if done:
                tickets.pop(tk)


def test_ring_results_identical_alone_and_in_the_mix(torch_cuda):
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Server
    rng = synth.choice_stream(5, 11)
    hiers = [[2, 4], [2, 4, 2], [4, 4]]
    temps = []
    for i in range(12):
        h = hiers[int(rng.integers(0, 3))]
        temps.append(_template(torch, H.SIX[i % 6], h, "int32" if i % 3 == 0 else "float32",
                               int(rng.integers(200, 3000)), i))
    st = torch.cuda.current_stream()
    alone = []
    for tp in temps:
        tp["R"].zero_()
        tp["c"].run(st)
        tp["c"].wait()
        out = tp["R"].cpu().numpy().copy()
        alone.append(out)
        ranks = [0] if tp["name"] == "reduce" else range(tp["p"])
        H.check_result(tp["name"], {r: out[r] for r in ranks}, tp["sends"], tp["dtype"], h=tp["h"], s=tp["s"])
    srv = Server(1 << 40, 4, ring=True, ring_grid=0, idle_ms=50)
    for rnd in range(3):
        for tp in temps:
            tp["R"].zero_()
        order = list(range(len(temps)))
        if rnd % 2:
            order.reverse()
        _serve(torch, srv, temps, order)
        for k, tp in enumerate(temps):
            got = tp["R"].cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), (rnd, k, tp["name"])
    srv.drain()
    srv.close()
    for tp in temps:
        tp["c"].close()


def test_ring_idle_exit_and_restart(torch_cuda):
    torch = torch_cuda
    from paper_2408_05962_amd import Server
    tp = _template(torch, "all_reduce", [2, 2], "int32", 16384, 3, s=1, m=1)
    srv = Server(1 << 40, 2, ring=True, ring_grid=8, idle_ms=2)
    for _ in range(3):
        tp["R"].zero_()
        _serve(torch, srv, [tp], [0])
        out = tp["R"].cpu().numpy()
        H.check_result("all_reduce", {r: out[r] for r in range(4)}, tp["sends"], "int32")
        time.sleep(0.05)                            # longer than the idle time: the resident launch exits
    srv.close()
    tp["c"].close()


def test_ring_timeout_is_reported_and_ring_recovers(torch_cuda):
    torch = torch_cuda
    from paper_2408_05962_amd import Server
    from paper_2408_05962_amd.hiccl import ERR_TIMEOUT, HicclError
    tp = _template(torch, "all_reduce", [2, 4, 2], "int32", 4096, 4, s=4, m=2, tile=1024)
    srv = Server(1 << 40, 2, ring=True, idle_ms=50)
    tp["c"].set_spin_limit(1)                       # every unmet dependency wait gives up at once
    timeouts = 0
    for _ in range(3):
        tk = srv.admit(1 << 20)
        srv.launch(tk, tp["c"])
        srv.drain()
        try:
            srv.poll(tk)
        except HicclError as err:
            assert err.code == ERR_TIMEOUT
            timeouts += 1
    assert timeouts > 0
    tp["c"].set_spin_limit(1 << 20)
    tp["R"].zero_()
    _serve(torch, srv, [tp], [0])
    out = tp["R"].cpu().numpy()
    H.check_result("all_reduce", {r: out[r] for r in range(16)}, tp["sends"], "int32")
    srv.close()
    tp["c"].close()


def test_ring_argument_errors(torch_cuda):
    torch = torch_cuda
    from paper_2408_05962_amd import Server, lib
    from paper_2408_05962_amd import collectives as CO
    from paper_2408_05962_amd.hiccl import ERR_INVALID_ARG, ERR_STATE, ERR_UNSUPPORTED, HicclError
    srv = Server(1 << 30, 2)
    assert lib().hiccl_server_start_ring(srv.h, 1, 10) == ERR_INVALID_ARG
    assert lib().hiccl_server_start_ring(srv.h, 0, 0) == ERR_INVALID_ARG
    assert lib().hiccl_server_start_ring(srv.h, 4, 10) == 0
    assert lib().hiccl_server_start_ring(srv.h, 4, 10) == ERR_STATE
    S = torch.zeros((4, 64), dtype=torch.int32, device="cuda")
    R = torch.zeros_like(S)
    c = CO.make("all_reduce", 4, "int32", [S[r] for r in range(4)], [R[r] for r in range(4)], 16, hierarchy=[2, 2],
                exec_mode="staged")
    tk = srv.admit(1 << 10)
    with pytest.raises(HicclError) as e:
        srv.launch(tk, c)
    assert e.value.code == ERR_UNSUPPORTED
    assert srv.usage() == (0, 0)                    # the failed launch released its ticket
    srv.close()
    c.close()


@pytest.mark.timeout(400)
def test_serving_mix_full_size_alone_and_in_the_mix(torch_cuda):
    """The measured serving mix itself (the bench's 48 templates, up to 256 MiB per rank, int32 / float32 /
    bf16): a stream of 300 requests served by the device ring, and again by concurrent slots, leaves every
    requested template's result bit-identical to the template run alone. The alone results equal the oracle
    for every template up to 4 MiB per rank (bf16 reductions: the oracle's per-node requantization)."""
    torch = torch_cuda
    import bench as B
    import synth
    from paper_2408_05962_amd import Server
    temps = B.serve_templates(torch, 48, 8, "persistent")
    st = torch.cuda.current_stream()
    alone = []
    for tp in temps:
        tp["rcv"].zero_()
        tp["comm"].run(st)
        tp["comm"].wait()
        alone.append(tp["rcv"].clone())
    torch.cuda.synchronize()
    for k, tp in enumerate(temps):
        if tp["S"] > 4 << 20:
            continue
        if tp["dtype"] == "bfloat16":
            # bf16: copies move the bits unchanged; reductions equal the oracle's per-node widen / sum / narrow
            sends = [x.view(np.uint16) for x in tp["snd"].cpu().numpy()]
            out = alone[k].cpu().numpy().view(np.uint16)
            if tp["name"] in ("reduce", "reduce_scatter", "all_reduce"):
                exp = H.tree_order_payload(tp["name"], sends, tp["h"], tp["stripe"])
            else:
                exp = H.expected(tp["name"], sends)
            for r, e in exp.items():
                assert np.array_equal(out[r], np.asarray(e, np.uint16)), (k, tp["name"], "bf16", r)
            continue
        sends = list(tp["snd"].cpu().numpy())
        out = alone[k].cpu().numpy()
        ranks = [0] if tp["name"] == "reduce" else range(tp["p"])
        H.check_result(tp["name"], {r: out[r] for r in ranks}, sends, tp["dtype"], h=tp["h"], s=tp["stripe"])
    picks = [int(x) for x in synth.choice_stream(8, 4).integers(0, len(temps), 300)]
    for ring in (True, False):
        for tp in temps:
            tp["rcv"].zero_()
        st.synchronize()
        srv = Server(200 * 10 ** 9, 4, ring=ring)
        queue, inflight, busy = list(picks), {}, set()
        t0 = time.time()
        while queue or inflight:
            assert time.time() - t0 < 120, "requests did not finish"
            k = 0
            while k < len(queue):
                tpi = queue[k]
                if tpi in busy:
                    k += 1
                    continue
                tk = srv.admit(temps[tpi]["foot"])
                if tk is None:
                    break
                srv.launch(tk, temps[tpi]["comm"])
                busy.add(tpi)
                inflight[tk] = tpi
                queue.pop(k)
            srv.progress()
            for tk in list(inflight):
                if srv.poll(tk)[0]:
                    busy.discard(inflight.pop(tk))
        srv.drain()
        srv.close()
        for k in sorted(set(picks)):
            assert torch.equal(temps[k]["rcv"], alone[k]), (ring, k, temps[k]["name"], temps[k]["dtype"])
    for tp in temps:
        tp["comm"].close()


@pytest.mark.parametrize("dtype", ["bfloat16", "fp8_e4m3"])
def test_ring_payload_requests_bit_identical(torch_cuda, dtype):
    """bf16 and fp8 requests through the device ring equal the same requests run alone, bit for bit (codes
    and block scales)."""
    torch = torch_cuda
    import synth
    from paper_2408_05962_amd import Server, to_payload
    from paper_2408_05962_amd import collectives as CO
    st = torch.cuda.current_stream()
    temps = []
    for i, (name, h) in enumerate([("all_reduce", [2, 4, 2]), ("reduce_scatter", [4, 4]), ("broadcast", [2, 4]),
                                   ("all_gather", [2, 4, 2])]):
        p = int(np.prod(h))
        d = 256 * 12
        n_s, n_r = H.send_len(name, p, d), H.recv_len(name, p, d)
        X = synth.device_buffers("float32_outliers", 600 + i, p, n_s)
        if dtype == "bfloat16":
            S = torch.empty((p, n_s), dtype=torch.int16, device="cuda")
            for r in range(p):
                to_payload(dtype, X[r], S[r], None, n_s, st)
            R = torch.zeros((p, n_r), dtype=torch.int16, device="cuda")
            send, recv, scales = [S[r] for r in range(p)], [R[r] for r in range(p)], None
            SS = None
        else:
            S = torch.empty((p, n_s), dtype=torch.uint8, device="cuda")
            SS = torch.empty((p, n_s // 256), device="cuda")
            for r in range(p):
                to_payload(dtype, X[r], S[r], SS[r], n_s, st)
            R = torch.zeros((p, n_r), dtype=torch.uint8, device="cuda")
            RS = torch.zeros((p, n_r // 256), device="cuda")
            send, recv, scales = [(S[r], SS[r]) for r in range(p)], [(R[r], RS[r]) for r in range(p)], RS
        c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=2, pipeline=2, tile_bytes=4096)
        c.set_spin_limit(1 << 20)
        c.run(st)
        c.wait()
        alone = (R.clone(), scales.clone() if scales is not None else None)
        # the communicator holds raw addresses: every buffer it names (send scales included) must outlive it
        temps.append({"c": c, "R": R, "scales": scales, "alone": alone, "keep": (X, S, SS)})
    srv = Server(1 << 40, 2, ring=True, idle_ms=50)
    for rnd in range(2):
        for tp in temps:
            tp["R"].zero_()
            if tp["scales"] is not None:
                tp["scales"].zero_()
        _serve(torch, srv, [{"c": tp["c"]} for tp in temps], list(range(len(temps))))
        for k, tp in enumerate(temps):
            assert torch.equal(tp["R"], tp["alone"][0]), (dtype, rnd, k)
            if tp["scales"] is not None:
                assert torch.equal(tp["scales"], tp["alone"][1]), (dtype, rnd, k)
    srv.close()
    for tp in temps:
        tp["c"].close()
