"""Fence-delimited primitive-step interpreter — test oracle.

Executes a composition of the three primitives of Sec. 3.1 on host buffers, with the semantics of Secs. 3.2 and 3.3:

  * multicast M(i, J, n): the root i's ``n`` elements are replicated into
    every leaf j in J;
  * reduction R(I, j, n, op): the ``n``-element operands of the leaves in I
    are combined with ``op`` into the root j (a single leaf is a plain copy,
    the unary operation being omitted);
  * all primitives between two fences run concurrently: each reads the state
    at the start of its step, and the step's writes land after all of them
    have read;
  * a fence orders the steps (the next step sees every write of the last).

Buffers are named numpy arrays held in wide precision (float64 / int64, ints
wrapped modulo 2**32 on every store). Each primitive carries, per rank, a
(buffer name, element offset) pair for its send and receive sides, as the
per-process pointers of the paper's API become per-rank addresses when all
ranks live in one address space.

Parity: pinned by tests/test_oracle_steps.py — every single- and multi-step
row of Table 2, and the
All-Reduce of Listing 2, against the direct definitions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .collectives import wide, wrap_int32


@dataclass
class Prim:
    kind: str                      # "M" (multicast) or "R" (reduction)
    root: int                      # M: sending rank i; R: receiving rank j
    leaves: list[int]              # M: receiving ranks J; R: contributing ranks I
    count: int                     # elements
    send: dict[int, tuple[str, int]] = field(default_factory=dict)   # rank -> (buffer, offset)
    recv: dict[int, tuple[str, int]] = field(default_factory=dict)
    op: str = "sum"


def multicast(root, leaves, count, send, recv) -> Prim:
    return Prim("M", root, list(leaves), count, dict(send), dict(recv))


def reduction(leaves, root, count, send, recv, op="sum") -> Prim:
    return Prim("R", root, list(leaves), count, dict(send), dict(recv), op)


class Memory:
    """Named host buffers in wide precision; ``is_int`` selects the 32-bit wrap on store."""

    def __init__(self, buffers: dict[str, np.ndarray]):
        self.is_int = {k: np.asarray(v).dtype.kind in "iu" for k, v in buffers.items()}
        self.buf = {k: wide(v).copy() for k, v in buffers.items()}

    def read(self, ref, n):
        name, off = ref
        a = self.buf[name]
        if off < 0 or off + n > len(a):
            raise IndexError(f"read {name}[{off}:{off + n}] outside buffer of {len(a)}")
        return a[off:off + n].copy()

    def write(self, ref, values):
        name, off = ref
        a = self.buf[name]
        n = len(values)
        if off < 0 or off + n > len(a):
            raise IndexError(f"write {name}[{off}:{off + n}] outside buffer of {len(a)}")
        if self.is_int[name]:
            values = wrap_int32(values).astype(np.int64)
        a[off:off + n] = values

    def result(self, name, dtype):
        a = self.buf[name]
        if np.dtype(dtype).kind in "iu":
            return wrap_int32(a)
        return a.copy()


def _ranges(prim: Prim):
    """(buffer, lo, hi, is_write) address ranges a primitive touches."""
    out = []
    n = prim.count
    if prim.kind == "M":
        b, o = prim.send[prim.root]
        out.append((b, o, o + n, False))
        for j in prim.leaves:
            b, o = prim.recv[j]
            out.append((b, o, o + n, True))
    else:
        for i in prim.leaves:
            b, o = prim.send[i]
            out.append((b, o, o + n, False))
        b, o = prim.recv[prim.root]
        out.append((b, o, o + n, True))
    return out


def find_races(step: list[Prim]) -> list[tuple[int, int]]:
    """Pairs of primitives of one step that write-write or read-write overlapping elements.

    The paper leaves the result of such a step undefined; a read-read overlap
    is not a race.
    """
    races = []
    rs = [_ranges(p) for p in step]
    for a in range(len(step)):
        for b in range(a + 1, len(step)):
            hit = False
            for (ba, la, ha, wa) in rs[a]:
                for (bb, lb, hb, wb) in rs[b]:
                    if ba == bb and la < hb and lb < ha and (wa or wb) and ha > la and hb > lb:
                        hit = True
            if hit:
                races.append((a, b))
    return races


def run(memory: Memory, steps: list[list[Prim]]) -> Memory:
    """Execute the steps in order; within a step every primitive reads the step's initial state."""
    for step in steps:
        pending = []
        for prim in step:
            n = prim.count
            if n == 0:
                continue
            if prim.kind == "M":
                v = memory.read(prim.send[prim.root], n)
                for j in prim.leaves:
                    pending.append((prim.recv[j], v))
            elif prim.kind == "R":
                vals = [memory.read(prim.send[i], n) for i in sorted(prim.leaves)]
                if not vals:
                    continue
                acc = vals[0].copy()
                for v in vals[1:]:
                    if prim.op == "sum":
                        acc = acc + v
                    elif prim.op == "max":
                        acc = np.maximum(acc, v)
                    elif prim.op == "min":
                        acc = np.minimum(acc, v)
                    else:
                        raise ValueError(prim.op)
                pending.append((prim.recv[prim.root], acc))
            else:
                raise ValueError(prim.kind)
        for ref, v in pending:
            memory.write(ref, v)
    return memory


# ------------------------------------------------ compositions of Table 2
def _all(p):
    return list(range(p))


def compose(name: str, p: int, d: int, op: str = "sum", root: int = 0, form: str = "single"):
    """Steps realising a collective from the composition table.

    Buffers are named ``s{r}`` (send) and ``y{r}`` (receive). Sizes follow the
    paper's convention (largest buffer d*p). ``form`` picks the single-step
    row or one of the multi-step rows (read right to left, the dot being a
    fence). Returns a list of steps.
    """
    U = _all(p)
    S = {r: (f"s{r}", 0) for r in U}
    Y = {r: (f"y{r}", 0) for r in U}

    def s_at(k):   # chunk k of every rank's send buffer
        return {r: (f"s{r}", k * d) for r in U}

    def y_at(k):
        return {r: (f"y{r}", k * d) for r in U}

    if form == "single":
        if name == "broadcast":
            return [[multicast(root, U, d * p, S, Y)]]
        if name == "reduce":
            return [[reduction(U, root, d * p, S, Y, op)]]
        if name == "all_gather":
            return [[multicast(i, U, d, S, y_at(i)) for i in U]]
        if name == "reduce_scatter":
            return [[reduction(U, j, d, s_at(j), Y, op) for j in U]]
        if name == "all_reduce":
            return [[reduction(U, j, d * p, S, Y, op) for j in U]]
        if name == "scatter":
            # a single-leaf reduction is point-to-point (the unary op omitted)
            return [[reduction([root], j, d, s_at(j), Y, op) for j in U]]
        if name == "gather":
            return [[multicast(i, [root], d, S, y_at(i)) for i in U]]
        if name == "all_to_all":
            return [[multicast(i, [j], d, s_at(j), y_at(i)) for i in U for j in U]]
        raise ValueError(name)
    if form == "multi":
        # the intermediate lives in the receive buffers (or a scratch buffer
        # named t{r} where the shapes differ), as in Listing 2
        T = {r: (f"t{r}", 0) for r in U}
        if name == "broadcast":      # All-gather . Scatter
            step1 = [reduction([root], j, d, {root: (f"s{root}", j * d)}, T, op) for j in U]
            step2 = [multicast(i, U, d, T, y_at(i)) for i in U]
            return [step1, step2]
        if name == "reduce":         # Gather . Reduce-scatter
            step1 = [reduction(U, j, d, s_at(j), T, op) for j in U]
            step2 = [multicast(i, [root], d, T, y_at(i)) for i in U]
            return [step1, step2]
        if name == "all_gather":     # Broadcast . Gather
            step1 = [multicast(i, [root], d, S, {root: (f"t{root}", i * d)}) for i in U]
            step2 = [multicast(root, U, d * p, T, Y)]
            return [step1, step2]
        if name == "reduce_scatter":  # Scatter . Reduce
            step1 = [reduction(U, root, d * p, S, T, op)]
            step2 = [reduction([root], j, d, {root: (f"t{root}", j * d)}, Y, op) for j in U]
            return [step1, step2]
        if name == "all_reduce_bcast":  # Broadcast . Reduce
            step1 = [reduction(U, root, d * p, S, T, op)]
            step2 = [multicast(root, U, d * p, T, Y)]
            return [step1, step2]
        if name == "all_reduce":     # All-gather . Reduce-scatter, in place as in the listing
            others = {i: [r for r in U if r != i] for i in U}
            step1 = [reduction(U, j, d, s_at(j), y_at(j), op) for j in U]
            step2 = [multicast(i, others[i], d, y_at(i), y_at(i)) for i in U]
            return [step1, step2]
        raise ValueError(name)
    raise ValueError(form)


def buffers_for(name: str, p: int, d: int, sends: list[np.ndarray], form: str = "single") -> dict:
    """Named buffers for ``compose``: send buffers as given, receive (and scratch) zeroed."""
    dt = np.asarray(sends[0]).dtype
    recv_len = {"broadcast": d * p, "reduce": d * p, "all_gather": d * p, "reduce_scatter": d,
                "all_reduce": d * p, "all_reduce_bcast": d * p, "scatter": d, "gather": d * p,
                "all_to_all": d * p}[name]
    bufs = {}
    for r in range(p):
        bufs[f"s{r}"] = np.asarray(sends[r])
        bufs[f"y{r}"] = np.zeros(recv_len, dtype=dt)
        if form == "multi":
            bufs[f"t{r}"] = np.zeros(d * p, dtype=dt)
    return bufs
