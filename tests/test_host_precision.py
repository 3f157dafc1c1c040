"""Precision form on the host schedule checker: bf16 and fp8 payloads against the oracle's per-node
requantization (bit-exact) and against the float64 sum of the original inputs (error stated)."""
import numpy as np
import pytest

import synth
from oracle import collectives as OC
from tests import harness as H


def _lib():
    from paper_2408_05962_amd import hiccl
    try:
        hiccl.lib()
    except ImportError as e:
        pytest.skip(str(e))


@pytest.mark.parametrize("dtype", ["bfloat16", "fp8_e4m3"])
@pytest.mark.parametrize("name", ["all_reduce", "reduce_scatter", "reduce"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 2), ([4, 4], 2, 1), ([2, 2], 1, 3)])
def test_payload_plans_match_oracle(dtype, name, h, s, m):
    _lib()
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    d = 256 * s * 2
    n = d * p
    x = [synth.rank_buffer("float32_outliers", 3, 0, r, n) for r in range(p)]
    pay = [H.to_payload_host(v, dtype) for v in x]
    rl = H.recv_len(name, p, d)
    if dtype == "bfloat16":
        send = [v.copy() for v in pay]
        recv = [np.zeros(rl, np.uint16) for _ in range(p)]
        sb, rb = send, recv
    else:
        send = [(v.codes.copy(), v.scales.copy()) for v in pay]
        recv = [(np.zeros(rl, np.uint8), np.zeros(rl // 256, np.float32)) for _ in range(p)]
        sb, rb = send, recv
    c = CO.make(name, p, dtype, sb, rb, d, hierarchy=h, stripe=s, pipeline=m)
    c.validate_host(seed=2, norders=3)
    c.close()
    exp = H.tree_order_payload(name, pay, h, s)
    exact = H.expected(name, x)
    scale = H.abs_scale(name, x)
    for r, e in exp.items():
        if dtype == "bfloat16":
            assert np.array_equal(recv[r], e), (r,)
            got = H.payload_values(recv[r], dtype)
        else:
            assert np.array_equal(recv[r][0], e.codes) and np.array_equal(recv[r][1], e.scales), (r,)
            got = H.payload_values(H.Fp8Buf(*recv[r]), dtype)
        rep = OC.error_report(got, exact[r], scale[r])
        # stated, not a pass criterion of the method; a loose sanity bound only
        assert rep["scaled"] < (0.05 if dtype == "bfloat16" else 0.5)


@pytest.mark.parametrize("dtype", ["bfloat16", "fp8_e4m3"])
@pytest.mark.parametrize("name", ["all_reduce", "reduce_scatter", "reduce"])
@pytest.mark.parametrize("h,s,m,ring", [([4, 2], 1, 2, 4), ([4, 2], 2, 1, 4), ([2, 4, 2], 2, 2, 2)])
def test_payload_ring_host_schedule(dtype, name, h, s, m, ring):
    """Payload formats under ring + tree: the library's host schedule checker (random dependency orders)
    equals the oracle's per-node requantization in ring order."""
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    d = 256 * s * 2
    rng = np.random.default_rng(p + ring)
    X = (rng.standard_normal((p, d * p)) * np.where(rng.random((p, d * p)) < 0.01, 1e3, 1.0)).astype(np.float32)
    pay = [H.to_payload_host(X[r], dtype) for r in range(p)]
    rl = H.recv_len(name, p, d)
    if dtype == "bfloat16":
        send = [np.ascontiguousarray(pay[r]) for r in range(p)]
        recv = [np.zeros(rl, np.uint16) for _ in range(p)]
    else:
        send = [(np.ascontiguousarray(pay[r].codes), np.ascontiguousarray(pay[r].scales)) for r in range(p)]
        recv = [(np.zeros(rl, np.uint8), np.zeros(rl // 256, np.float32)) for _ in range(p)]
    c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=s, pipeline=m, ring=ring)
    c.validate_host(seed=1, norders=2)
    c.close()
    for r, e in H.tree_order_payload(name, pay, h, s, ring=ring).items():
        if dtype == "bfloat16":
            assert np.array_equal(recv[r], e), (name, r)
        else:
            assert np.array_equal(recv[r][0], e.codes) and np.array_equal(recv[r][1], e.scales), (name, r)
