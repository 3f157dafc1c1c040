"""Shared helpers of the parity tests: inputs, oracle expectations, comparisons.

Expected values come from ``oracle`` only; inputs from ``synth`` (host) or
torch's seeded device generator (read back to the host before any run).
"""
from __future__ import annotations

import numpy as np

from oracle import collectives as OC
from oracle import quant as OQ
from oracle import tree as OT

SIX = ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_to_all")
EIGHT = SIX + ("scatter", "gather")

NP = {"int32": np.int32, "float32": np.float32}
ALIGN = {"int32": 4, "float32": 4, "bfloat16": 8, "fp8_e4m3": 256}
TOL_F32 = 1e-5      # condition-scaled relative error bound for float32 sums


def send_len(name, p, d):
    return d if name in ("all_gather", "gather") else d * p


def recv_len(name, p, d):
    return {"broadcast": d * p, "reduce": d * p, "all_gather": d * p, "reduce_scatter": d, "all_reduce": d * p,
            "scatter": d, "gather": d * p, "all_to_all": d * p}[name]


def expected(name, sends, root=0, op="sum"):
    """Oracle result per receiving rank (dict rank -> array; float64 for float sums)."""
    p = len(sends)
    if name == "broadcast":
        return dict(enumerate(OC.broadcast(sends, root)))
    if name == "reduce":
        return {root: OC.reduce(sends, root, op)}
    if name == "all_gather":
        return dict(enumerate(OC.all_gather(sends)))
    if name == "reduce_scatter":
        return dict(enumerate(OC.reduce_scatter(sends, op)))
    if name == "all_reduce":
        return dict(enumerate(OC.all_reduce(sends, op)))
    if name == "scatter":
        return dict(enumerate(OC.scatter(sends[root], p)))
    if name == "gather":
        return {root: OC.gather(sends)}
    if name == "all_to_all":
        return dict(enumerate(OC.all_to_all(sends)))
    raise ValueError(name)


def abs_scale(name, sends):
    """Elementwise sum of |inputs| of every sum result (the condition scale), per receiving rank."""
    p = len(sends)
    full = OC.abs_sum(sends)
    if name == "reduce_scatter":
        d = len(sends[0]) // p
        return {r: full[r * d:(r + 1) * d] for r in range(p)}
    return {r: full for r in range(p)}


def is_sum(name, op):
    return op == "sum" and name in ("reduce", "reduce_scatter", "all_reduce")


def _striped_ring(vals, root, n, h, s, ring, align, combine=OT.sum_f32, concat=np.concatenate):
    """R(all, root) under ring(ring) and stripe(s): per stripe, the ring reduction of its owner, each node
    formed by `combine` (default: float32 left-to-right sums)."""
    p = len(vals)
    k = OT.ring_depth(h, ring)
    size = OT.block_sizes(h)[k]
    own = None
    if s > 1:
        B = OT.block_sizes(h)
        for kk in range(len(h), k - 1, -1):
            sz = B[kk]
            if sz >= s and sz % s == 0:
                lo = (root // sz) * sz
                if not all(lo <= x < lo + sz for x in range(p)):
                    own = [lo + ((root - lo) + t * (sz // s)) % sz for t in range(s)]
                break
    if own is None:
        return OT.ring_reduce(vals, range(p), root, h, ring, combine)
    parts = []
    for t, (off, ln) in enumerate(OT.split(n, s, align)):
        if ln == 0:
            continue
        sub = {r: v[off:off + ln] for r, v in vals.items()}
        parts.append(OT.ring_reduce(sub, range(p), own[t], h, ring, combine))
    return concat(parts)


def tree_order_f32(name, sends, h, s, root=0, ring=1):
    """float32 result of the factorized schedule, operands combined in the tree (or ring) order of the oracle."""
    p = len(sends)
    n = len(sends[0])
    vals = dict(enumerate(np.asarray(x, np.float32) for x in sends))

    def red(v, rt, m):
        if ring > 1:
            return _striped_ring(v, rt, m, h, s, ring, 4)
        return OT.striped_reduce(v, range(p), rt, m, h, s, 4, OT.sum_f32)

    if name == "reduce":
        return {root: red(vals, root, n)}
    d = n // p
    out = {}
    for j in range(p):
        chunk = {r: v[j * d:(j + 1) * d] for r, v in vals.items()}
        out[j] = red(chunk, j, d)
    if name == "reduce_scatter":
        return out
    full = np.concatenate([out[j] for j in range(p)])
    return {r: full for r in range(p)}


def check_result(name, got: dict, sends, dtype, op="sum", root=0, h=None, s=1, order_exact=True, ring=1):
    """Compare device results (dict rank -> host array) with the oracle; returns error stats."""
    exp = expected(name, sends, root, op)
    stats = {}
    if dtype == "int32" or not is_sum(name, op):
        for r, y in exp.items():
            g = got[r]
            if not np.array_equal(g.view(np.uint32) if g.dtype == np.float32 else g,
                                  np.asarray(y, g.dtype).view(np.uint32) if g.dtype == np.float32 else np.asarray(y, g.dtype)):
                bad = np.nonzero(np.asarray(g, np.float64) != np.asarray(y, np.float64))[0]
                raise AssertionError(f"{name} {dtype} rank {r}: {len(bad)} mismatches, first at {bad[:5]}")
        stats["exact"] = True
        return stats
    scale = abs_scale(name, sends)
    worst = 0.0
    for r, y in exp.items():
        e = OC.scaled_error(got[r], y, scale[r])
        worst = max(worst, e)
        assert e <= TOL_F32, f"{name} rank {r}: scaled error {e:.3e} > {TOL_F32}"
    stats["scaled_error"] = worst
    if order_exact and h is not None:
        tex = tree_order_f32(name, sends, h, s, root, ring)
        for r, y in tex.items():
            assert np.array_equal(got[r].view(np.uint32), y.view(np.uint32)), \
                f"{name} rank {r}: not bit-identical to the tree-order float32 expectation"
        stats["order_exact"] = True
    return stats


# ---------------------------------------------------------------- precision form
class Fp8Buf:
    """An fp8 operand: e4m3 codes plus one float32 scale per 256 elements (sliceable by elements)."""

    def __init__(self, codes, scales):
        self.codes = np.asarray(codes, np.uint8)
        self.scales = np.asarray(scales, np.float32)

    def __getitem__(self, sl):
        a, b = sl.start or 0, sl.stop if sl.stop is not None else len(self.codes)
        assert a % 256 == 0 and b % 256 == 0
        return Fp8Buf(self.codes[a:b], self.scales[a // 256:b // 256])

    def __len__(self):
        return len(self.codes)


def to_payload_host(x, dtype):
    """Oracle quantization of float32 inputs to the payload format."""
    if dtype == "bfloat16":
        return OQ.f32_to_bf16_bits(x)
    c, s = OQ.fp8_quantize(np.asarray(x, np.float64))
    return Fp8Buf(c, s)


def payload_values(v, dtype):
    """float64 values of a payload operand."""
    if dtype == "bfloat16":
        return OQ.bf16_bits_to_f32(v).astype(np.float64)
    return OQ.fp8_dequantize(v.codes, v.scales)


def _node(dtype):
    if dtype == "bfloat16":
        return OQ.node_bf16
    return lambda ops: Fp8Buf(*OQ.node_fp8([(o.codes, o.scales) for o in ops]))


def _concat(parts, dtype):
    if dtype == "bfloat16":
        return np.concatenate(parts)
    return Fp8Buf(np.concatenate([p.codes for p in parts]), np.concatenate([p.scales for p in parts]))


def tree_order_payload(name, payloads, h, s, ring=1):
    """Result of RS / AR / Reduce in a payload format: every reduction node widens its operands to
    float32, sums them left to right and narrows the result (fresh block scales for fp8), in the tree
    order of the factorization; transfers move payload bytes unchanged."""
    p = len(payloads)
    dtype = "bfloat16" if not isinstance(payloads[0], Fp8Buf) else "fp8_e4m3"
    align = ALIGN[dtype]
    n = len(payloads[0])

    def striped(vals, root, m):
        if ring > 1:
            return _striped_ring(vals, root, m, h, s, ring, align, _node(dtype), lambda parts: _concat(parts, dtype))
        return chunk_reduce(vals, root, m, h, s, dtype)

    vals = dict(enumerate(payloads))
    if name == "reduce":
        return {0: striped(vals, 0, n)}
    d = n // p
    out = {j: striped({r: v[j * d:(j + 1) * d] for r, v in vals.items()}, j, d) for j in range(p)}
    if name == "reduce_scatter":
        return out
    full = _concat([out[j] for j in range(p)], dtype)
    return {r: full for r in range(p)}


def chunk_reduce(vals, root, m, h, s, dtype, pool=None):
    """R(all ranks, root) over m elements in the tree order of the factorization, per stripe when the
    reduction is striped. float32 operands are summed left to right in float32; payload operands go
    through the oracle's widen / sum / narrow node. `pool` (an executor) runs the stripes concurrently."""
    p = len(vals)
    align = ALIGN[dtype]
    node = OT.sum_f32 if dtype == "float32" else _node(dtype)
    own = OT.stripe_owners(root, range(p), h, s)
    if own is None:
        return OT.tree_reduce(vals, range(p), root, h, node)
    jobs = []
    for t, (off, ln) in enumerate(OT.split(m, s, align)):
        jobs.append(({r: v[off:off + ln] for r, v in vals.items()}, own[t]))
    run = (lambda f, xs: list(pool.map(f, xs))) if pool is not None else (lambda f, xs: [f(x) for x in xs])
    parts = run(lambda job: OT.tree_reduce(job[0], range(p), job[1], h, node), jobs)
    if dtype == "float32":
        return np.concatenate(parts)
    return _concat(parts, dtype)
