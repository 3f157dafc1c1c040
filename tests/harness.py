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


def tree_order_f32(name, sends, h, s, root=0):
    """float32 result of the factorized schedule, operands combined in the tree order of the oracle."""
    p = len(sends)
    n = len(sends[0])
    vals = dict(enumerate(np.asarray(x, np.float32) for x in sends))
    if name == "reduce":
        return {root: OT.striped_reduce(vals, range(p), root, n, h, s, 4, OT.sum_f32)}
    d = n // p
    out = {}
    for j in range(p):
        chunk = {r: v[j * d:(j + 1) * d] for r, v in vals.items()}
        out[j] = OT.striped_reduce(chunk, range(p), j, d, h, s, 4, OT.sum_f32)
    if name == "reduce_scatter":
        return out
    full = np.concatenate([out[j] for j in range(p)])
    return {r: full for r in range(p)}


def check_result(name, got: dict, sends, dtype, op="sum", root=0, h=None, s=1, order_exact=True):
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
        tex = tree_order_f32(name, sends, h, s, root)
        for r, y in tex.items():
            assert np.array_equal(got[r].view(np.uint32), y.view(np.uint32)), \
                f"{name} rank {r}: not bit-identical to the tree-order float32 expectation"
        stats["order_exact"] = True
    return stats
