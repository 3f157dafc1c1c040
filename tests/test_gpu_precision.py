"""GPU precision form: bf16 and fp8-e4m3 payloads (per-256 power-of-two scales) through the C ABI.

* the device payload conversion equals the oracle quantizer byte for byte;
* collectives in a payload format equal the oracle's per-node widen / sum / narrow emulation byte for
  byte (the requantization at every reduction node follows the schedule's tree);
* the error against the float64 sum of the original float32 inputs is reported for every result.
"""
import json
import os

import numpy as np
import pytest

from oracle import collectives as OC
from oracle import quant as OQ
from tests.conftest import gpu_available
from tests import harness as H

pytestmark = pytest.mark.gpu

REPORT_DIR = os.environ.get("HICCL_REPORT_DIR")   # where to also write the error reports as JSON


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2408_05962_amd import hiccl
    hiccl.lib()
    return torch


def _payload_tensors(torch, X, dtype):
    """Convert device float32 rows to payload rows on the device (library kernels)."""
    from paper_2408_05962_amd import to_payload
    p, n = X.shape
    if dtype == "bfloat16":
        Y = torch.empty((p, n), dtype=torch.int16, device="cuda")
        for r in range(p):
            to_payload("bfloat16", X[r], Y[r], None, n)
        return Y, None
    Y = torch.empty((p, n), dtype=torch.uint8, device="cuda")
    Sc = torch.empty((p, n // 256), dtype=torch.float32, device="cuda")
    for r in range(p):
        to_payload("fp8_e4m3", X[r], Y[r], Sc[r], n)
    return Y, Sc


def test_payload_conversion_matches_oracle(torch_cuda):
    torch = torch_cuda
    import synth
    n = 1 << 20
    X = synth.device_buffers("float32_outliers", 31, 1, n)
    x = X[0].cpu().numpy()
    Y, _ = _payload_tensors(torch, X, "bfloat16")
    assert np.array_equal(Y[0].cpu().numpy().view(np.uint16), OQ.f32_to_bf16_bits(x))
    Y, Sc = _payload_tensors(torch, X, "fp8_e4m3")
    c, s = OQ.fp8_quantize(x.astype(np.float64))
    assert np.array_equal(Sc[0].cpu().numpy(), s)
    assert np.array_equal(Y[0].cpu().numpy(), c)
    # and back: widening is exact
    from paper_2408_05962_amd import from_payload
    Z = torch.empty(n, dtype=torch.float32, device="cuda")
    from_payload("fp8_e4m3", Y[0], Sc[0], Z, n)
    assert np.array_equal(Z.cpu().numpy().astype(np.float64), OQ.fp8_dequantize(c, s))


EXECS = ("staged", "persistent")


def _run_payload(torch, name, dtype, X, h, s, m, d, ring=1, exec_mode="persistent"):
    from paper_2408_05962_amd import collectives as CO
    p = X.shape[0]
    Y, Sc = _payload_tensors(torch, X, dtype)
    rl = H.recv_len(name, p, d)
    if dtype == "bfloat16":
        R = torch.zeros((p, rl), dtype=torch.int16, device="cuda")
        send = [Y[r] for r in range(p)]
        recv = [R[r] for r in range(p)]
        RS = None
    else:
        R = torch.zeros((p, rl), dtype=torch.uint8, device="cuda")
        RS = torch.zeros((p, rl // 256), dtype=torch.float32, device="cuda")
        send = [(Y[r], Sc[r]) for r in range(p)]
        recv = [(R[r], RS[r]) for r in range(p)]
    c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=s, pipeline=m, ring=ring, exec_mode=exec_mode)
    c.set_spin_limit(1 << 20)
    c.run(torch.cuda.current_stream())
    c.wait()
    torch.cuda.synchronize()
    c.close()
    return Y, Sc, R, RS


def _host_payload(dtype, Yr, Sr):
    if dtype == "bfloat16":
        return Yr.view(np.uint16)
    return H.Fp8Buf(Yr, Sr)


@pytest.mark.parametrize("exec_mode", EXECS)
@pytest.mark.parametrize("dtype", ["bfloat16", "fp8_e4m3"])
@pytest.mark.parametrize("name", ["all_reduce", "reduce_scatter", "reduce"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 2), ([4, 4], 2, 3), ([2, 4], 1, 1), ([8], 1, 2), ([16], 1, 3)])
def test_payload_collectives_bit_exact(torch_cuda, dtype, name, h, s, m, exec_mode):
    """Both executors; the flat hierarchies {8} and {16} make reduction nodes of 8 and 16 operands, which
    take the kernels' general k-operand path (the others have at most 4)."""
    torch = torch_cuda
    import synth
    p = int(np.prod(h))
    d = 256 * s * 4
    X = synth.device_buffers("float32_outliers", 40 + p, p, d * p)
    Y, Sc, R, RS = _run_payload(torch, name, dtype, X, h, s, m, d, exec_mode=exec_mode)
    x = [v for v in X.cpu().numpy()]
    yh, sh = Y.cpu().numpy(), (Sc.cpu().numpy() if Sc is not None else [None] * p)
    pay = [_host_payload(dtype, yh[r], sh[r]) for r in range(p)]
    # the device inputs equal the oracle's own quantization of the float32 inputs
    for r in range(p):
        ref = H.to_payload_host(x[r], dtype)
        if dtype == "bfloat16":
            assert np.array_equal(pay[r], ref)
        else:
            assert np.array_equal(pay[r].codes, ref.codes) and np.array_equal(pay[r].scales, ref.scales)
    exp = H.tree_order_payload(name, pay, h, s)
    rh, rsh = R.cpu().numpy(), (RS.cpu().numpy() if RS is not None else [None] * p)
    exact = H.expected(name, x)
    scale = H.abs_scale(name, x)
    for r, e in exp.items():
        got = _host_payload(dtype, rh[r], rsh[r])
        if dtype == "bfloat16":
            assert np.array_equal(got, e), f"{name} {dtype} rank {r}"
        else:
            assert np.array_equal(got.codes, e.codes) and np.array_equal(got.scales, e.scales), f"{name} {dtype} rank {r}"
        rep = OC.error_report(H.payload_values(got, dtype), exact[r], scale[r])
        assert rep["scaled"] < (0.05 if dtype == "bfloat16" else 0.5)


@pytest.mark.parametrize("dtype", ["float32", "bfloat16", "fp8_e4m3"])
@pytest.mark.parametrize("name", ["all_reduce", "reduce_scatter"])
def test_precision_16_ranks_2e28_elements(torch_cuda, dtype, name):
    """16 ranks as {2,4,2}, 2^28 elements per rank ~ N(0,1) with 1 % of entries x 1e3, stripe 4,
    pipeline 8, on both executors:

    * the staged and the persistent executor give the same bytes on every rank's whole result;
    * All-Reduce leaves the same bytes on every rank;
    * the whole chunks j = 0 and j = p - 1 (every stripe, channel and tile boundary of a chunk) equal the
      oracle's tree-order emulation element by element (float32 sums, or widen / sum / narrow per node);
    * the error against the float64 sum of the original float32 inputs, and against the float64 sum of
      the payload inputs, is computed over those whole chunks and reported."""
    torch = torch_cuda
    import synth
    from concurrent.futures import ThreadPoolExecutor
    from paper_2408_05962_amd import collectives as CO
    p, h, s, m = 16, [2, 4, 2], 4, 8
    n = 1 << 28
    d = n // p
    rl = H.recv_len(name, p, d)
    X = synth.device_buffers("float32_outliers", 77, p, n)
    if dtype == "float32":
        Y = Sc = None
        send = [X[r] for r in range(p)]
    else:
        Y, Sc = _payload_tensors(torch, X, dtype)
        send = [Y[r] for r in range(p)] if Sc is None else [(Y[r], Sc[r]) for r in range(p)]
    tdt = {"float32": torch.float32, "bfloat16": torch.int16, "fp8_e4m3": torch.uint8}[dtype]
    out = {}
    for mode in EXECS:
        print(f"\n[precision 2^28] {name} {dtype} {mode}", flush=True)
        R = torch.zeros((p, rl), dtype=tdt, device="cuda")
        RS = torch.zeros((p, rl // 256), dtype=torch.float32, device="cuda") if dtype == "fp8_e4m3" else None
        recv = [R[r] for r in range(p)] if RS is None else [(R[r], RS[r]) for r in range(p)]
        c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=s, pipeline=m, exec_mode=mode)
        c.set_spin_limit(1 << 20)
        c.run(torch.cuda.current_stream())
        c.wait()
        torch.cuda.synchronize()
        c.close()
        out[mode] = (R, RS)
    (R, RS), (R2, RS2) = out["staged"], out["persistent"]
    assert torch.equal(R, R2), f"{name} {dtype}: staged and persistent results differ"
    assert RS is None or torch.equal(RS, RS2), f"{name} {dtype}: staged and persistent block scales differ"
    del out, R2, RS2
    if name == "all_reduce":
        for r in range(1, p):
            assert torch.equal(R[r], R[0]), f"All-Reduce {dtype}: rank {r} differs from rank 0"
    reports = []
    with ThreadPoolExecutor(8) as pool:
        for j in (0, p - 1):
            xs = X[:, j * d:(j + 1) * d].cpu().numpy()
            exact = OC.combine(list(xs), "sum")
            scale = OC.abs_sum(list(xs))
            col = 0 if name == "reduce_scatter" else j * d
            gy = R[j, col:col + d].cpu().numpy()
            if dtype == "float32":
                want = H.chunk_reduce({r: xs[r] for r in range(p)}, j, d, h, s, "float32", pool)
                assert np.array_equal(gy.view(np.uint32), want.view(np.uint32)), \
                    f"{name} float32 chunk {j}: not the tree-order float32 sums"
                gv = gy.astype(np.float64)
                rep = {"vs_float64_of_inputs": OC.error_report(gv, exact, scale)}
            else:
                ys = Y[:, j * d:(j + 1) * d].cpu().numpy()
                ss = Sc[:, j * d // 256:(j + 1) * d // 256].cpu().numpy() if Sc is not None else [None] * p
                pay = {r: _host_payload(dtype, ys[r], ss[r]) for r in range(p)}
                want = H.chunk_reduce(pay, j, d, h, s, dtype, pool)
                gs = RS[j, col // 256:(col + d) // 256].cpu().numpy() if RS is not None else None
                got = _host_payload(dtype, gy, gs)
                if dtype == "bfloat16":
                    bad = np.nonzero(got != want)[0]
                else:
                    assert np.array_equal(got.scales, want.scales), f"{name} fp8 chunk {j}: block scales differ"
                    bad = np.nonzero(got.codes != want.codes)[0]
                assert bad.size == 0, f"{name} {dtype} chunk {j}: {bad.size} elements differ, first at {bad[:5]}"
                gv = H.payload_values(got, dtype)
                deq = [H.payload_values(pay[r], dtype) for r in range(p)]
                rep = {"vs_float64_of_inputs": OC.error_report(gv, exact, scale),
                       "vs_float64_of_payload_inputs": OC.error_report(gv, OC.combine(deq, "sum"),
                                                                        OC.abs_sum(deq))}
                del ys, pay, deq
            reports.append(rep)
            del xs, exact, scale
    worst = {form: {k: max(r[form][k] for r in reports) for k in reports[0][form]} for form in reports[0]}
    if dtype == "float32":
        assert worst["vs_float64_of_inputs"]["scaled"] <= H.TOL_F32
    if REPORT_DIR:
        os.makedirs(REPORT_DIR, exist_ok=True)
        with open(os.path.join(REPORT_DIR, f"precision_{name}_{dtype}.json"), "w") as f:
            json.dump({"collective": name, "payload": dtype, "ranks": p, "elements_per_rank": n,
                       "chunks_compared_whole": [0, p - 1], "elements_per_chunk": d, "error": worst}, f)
    print(f"{name} {dtype}: error over chunks 0 and {p - 1} (whole): {worst}", flush=True)
    del X, Y, Sc, R, RS
    torch.cuda.empty_cache()


def test_fp8_node_every_code_pair(torch_cuda):
    """One two-operand fp8 reduction node (Reduce over 2 ranks) fed every pair of non-NaN e4m3 codes,
    with per-block scales that vary the operands' relative magnitude: widening, summing, rescaling and
    round-to-nearest-even encoding (ties and subnormals included) equal the oracle's node byte for byte."""
    torch = torch_cuda
    from paper_2408_05962_amd import collectives as CO
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    a = np.repeat(codes, len(codes))
    b = np.tile(codes, len(codes))
    n = (len(a) + 255) // 256 * 256
    n += n % 512                                   # two equal chunks of whole blocks
    A = np.zeros(n, np.uint8)
    B = np.zeros(n, np.uint8)
    A[:len(a)], B[:len(b)] = a, b
    nb = n // 256
    sa = np.ones(nb, np.float32)
    sb = np.exp2(np.arange(nb) % 9 - 4).astype(np.float32)     # 2^-4 .. 2^4
    dev = lambda x: torch.from_numpy(x).to("cuda")  # noqa: E731
    Y = [dev(A), dev(B)]
    S = [dev(sa), dev(sb)]
    R = [torch.zeros(n, dtype=torch.uint8, device="cuda") for _ in range(2)]
    RS = [torch.zeros(nb, dtype=torch.float32, device="cuda") for _ in range(2)]
    c = CO.make("reduce", 2, "fp8_e4m3", [(Y[r], S[r]) for r in range(2)], [(R[r], RS[r]) for r in range(2)], n // 2,
                hierarchy=[2])
    c.set_spin_limit(1 << 20)
    c.run(torch.cuda.current_stream())
    c.wait()
    torch.cuda.synchronize()
    c.close()
    ec, es = OQ.node_fp8([(A, sa), (B, sb)])
    assert np.array_equal(RS[0].cpu().numpy(), es)
    got = R[0].cpu().numpy()
    bad = np.nonzero(got != ec)[0]
    assert bad.size == 0, f"{bad.size} codes differ, first at {bad[:5]}: got {got[bad[:5]]} want {ec[bad[:5]]}"


@pytest.mark.parametrize("exec_mode", EXECS)
@pytest.mark.parametrize("dtype", ["bfloat16", "fp8_e4m3"])
@pytest.mark.parametrize("name", ["all_reduce", "reduce_scatter", "reduce"])
@pytest.mark.parametrize("h,s,m,ring", [([4, 2], 1, 2, 4), ([4, 2], 2, 1, 4), ([2, 4, 2], 2, 2, 2)])
def test_payload_collectives_with_ring_bit_exact(torch_cuda, dtype, name, h, s, m, ring, exec_mode):
    """Payload formats under the hybrid ring+tree factorization (Sec. 4.4): each node of the ring order
    widens, sums and narrows exactly as the oracle's ring reduction emulates it."""
    torch = torch_cuda
    import synth
    p = int(np.prod(h))
    d = 256 * max(s, 1) * 2
    X = synth.device_buffers("float32_outliers", 60 + p + ring, p, d * p)
    Y, Sc, R, RS = _run_payload(torch, name, dtype, X, h, s, m, d, ring=ring, exec_mode=exec_mode)
    yh, sh = Y.cpu().numpy(), (Sc.cpu().numpy() if Sc is not None else [None] * p)
    pay = [_host_payload(dtype, yh[r], sh[r]) for r in range(p)]
    exp = H.tree_order_payload(name, pay, h, s, ring=ring)
    rh, rsh = R.cpu().numpy(), (RS.cpu().numpy() if RS is not None else [None] * p)
    for r, e in exp.items():
        got = _host_payload(dtype, rh[r], rsh[r])
        if dtype == "bfloat16":
            assert np.array_equal(got, e), f"{name} {dtype} rank {r}"
        else:
            assert np.array_equal(got.codes, e.codes) and np.array_equal(got.scales, e.scales), f"{name} {dtype} rank {r}"

