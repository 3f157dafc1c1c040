"""Collectives composed from the three primitives, over the C ABI.

Each helper registers the primitives of one row of Table 2 (single step),
or the Reduce-Scatter / fence / All-Gather All-Reduce of Listing 2, into a
communicator — a loop with one primitive per line, as in Sec. 3.2. The
buffer convention is the paper's: the largest per-rank buffer holds d*p
elements and chunk q is elements [q*d, (q+1)*d).

Buffers are per-rank base addresses (ints, tensors or arrays), or
(data, scales) pairs for the fp8 payload.
"""
from __future__ import annotations

from .hiccl import ELEM_SIZE, FP8_E4M3, Comm, addr

NAMES = ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "scatter", "gather", "all_to_all")


def _at(buf, elems: int, dtype: int):
    """Address of element ``elems`` of a per-rank buffer (and of its fp8 block scale)."""
    es = ELEM_SIZE[dtype]
    if isinstance(buf, tuple):
        data, scales = addr(buf[0]), addr(buf[1])
        if dtype == FP8_E4M3:
            if elems % 256:
                raise ValueError("fp8 chunks must be whole 256-element blocks")
            return (data + elems * es, scales + (elems // 256) * 4)
        return data + elems * es
    return addr(buf) + elems * es


def recv_elems(name: str, p: int, d: int) -> int:
    """Receive-buffer length per rank of a collective (send length is d*p, or d for the gathers)."""
    return {"broadcast": d * p, "reduce": d * p, "all_gather": d * p, "reduce_scatter": d, "all_reduce": d * p,
            "scatter": d, "gather": d * p, "all_to_all": d * p}[name]


def send_elems(name: str, p: int, d: int) -> int:
    return d if name in ("all_gather", "gather") else d * p


def compose(comm: Comm, name: str, send, recv, d: int, root: int = 0, op: str = "sum", form: str = "listing"):
    """Register collective ``name`` over per-rank ``send`` / ``recv`` buffers with chunk ``d``.

    ``form`` matters for All-Reduce only: "listing" is Reduce-Scatter, a
    fence, then an in-place All-Gather to the other ranks (Listing 2);
    "single" is the single-step row of Table 2.
    """
    p, dt = comm.nranks, comm.dtype
    U = list(range(p))
    at = lambda b, e: _at(b, e, dt)  # noqa: E731
    if name == "broadcast":
        comm.add_multicast(send, recv, d * p, root, U)
    elif name == "reduce":
        comm.add_reduction(send, recv, d * p, U, root, op)
    elif name == "all_gather":
        for i in U:
            comm.add_multicast(send, [at(recv[r], i * d) for r in U], d, i, U)
    elif name == "reduce_scatter":
        for j in U:
            comm.add_reduction([at(send[r], j * d) for r in U], recv, d, U, j, op)
    elif name == "all_reduce" and form == "single":
        for j in U:
            comm.add_reduction(send, recv, d * p, U, j, op)
    elif name == "all_reduce":
        for j in U:
            comm.add_reduction([at(send[r], j * d) for r in U], [at(recv[r], j * d) for r in U], d, U, j, op)
        comm.add_fence()
        for i in U:
            chunk = [at(recv[r], i * d) for r in U]
            comm.add_multicast(chunk, chunk, d, i, [r for r in U if r != i])
    elif name == "scatter":
        # a one-leaf primitive is point-to-point
        for j in U:
            comm.add_multicast([at(send[r], j * d) for r in U], recv, d, root, [j])
    elif name == "gather":
        for i in U:
            comm.add_multicast(send, [at(recv[r], i * d) for r in U], d, i, [root])
    elif name == "all_to_all":
        for i in U:
            for j in U:
                comm.add_multicast([at(send[r], j * d) for r in U], [at(recv[r], i * d) for r in U], d, i, [j])
    else:
        raise ValueError(f"unknown collective {name!r}")
    return comm


MULTI = ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast")


def compose_multi(comm: Comm, name: str, send, recv, scratch, d: int, root: int = 0, op: str = "sum"):
    """Register a two-step row of Table 2 (read right to left, the dot being a fence) with a
    per-rank scratch buffer of d*p elements holding the intermediate:

      broadcast        = All-gather . Scatter
      reduce           = Gather . Reduce-scatter
      all_gather       = Broadcast . Gather
      reduce_scatter   = Scatter . Reduce
      all_reduce_bcast = Broadcast . Reduce
    """
    p, dt = comm.nranks, comm.dtype
    U = list(range(p))
    at = lambda b, e: _at(b, e, dt)  # noqa: E731
    if name == "broadcast":
        for j in U:                                   # scatter chunk j of the root's buffer to rank j
            comm.add_multicast([at(send[r], j * d) for r in U], scratch, d, root, [j])
        comm.add_fence()
        for i in U:                                   # all-gather the chunks
            comm.add_multicast(scratch, [at(recv[r], i * d) for r in U], d, i, U)
    elif name == "reduce":
        for j in U:                                   # reduce-scatter into the scratch buffers
            comm.add_reduction([at(send[r], j * d) for r in U], scratch, d, U, j, op)
        comm.add_fence()
        for i in U:                                   # gather at the root
            comm.add_multicast(scratch, [at(recv[r], i * d) for r in U], d, i, [root])
    elif name == "all_gather":
        for i in U:                                   # gather at the root's scratch
            comm.add_multicast(send, [at(scratch[r], i * d) for r in U], d, i, [root])
        comm.add_fence()
        comm.add_multicast(scratch, recv, d * p, root, U)   # broadcast it
    elif name == "reduce_scatter":
        comm.add_reduction(send, scratch, d * p, U, root, op)   # reduce at the root
        comm.add_fence()
        for j in U:                                   # scatter chunk j to rank j
            comm.add_multicast([at(scratch[r], j * d) for r in U], recv, d, root, [j])
    elif name == "all_reduce_bcast":
        comm.add_reduction(send, scratch, d * p, U, root, op)
        comm.add_fence()
        comm.add_multicast(scratch, recv, d * p, root, U)
    else:
        raise ValueError(f"unknown two-step composition {name!r}")
    return comm


def make(name: str, p: int, dtype, send, recv, d: int, hierarchy=None, stripe: int = 1, pipeline: int = 1,
         root: int = 0, op: str = "sum", form: str = "listing", exec_mode: str = "persistent", tile_bytes: int = 0,
         grid: int = 0, order: str = "stage", init: bool = True, ring: int = 1, share: int = -1) -> Comm:
    """Create, compose and (by default) initialize a communicator for one collective."""
    c = Comm(p, dtype)
    compose(c, name, send, recv, d, root=root, op=op, form=form)
    c.set_hierarchy(hierarchy or [p])
    c.set_stripe(stripe)
    c.set_ring(ring)
    c.set_pipeline(pipeline)
    c.set_exec(exec_mode, tile_bytes, grid, order)
    if share >= 0:
        c.set_share(share)
    if init:
        c.init()
    return c
