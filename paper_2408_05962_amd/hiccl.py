"""ctypes binding of the executor's C ABI (include/hiccl.h).

Argument marshalling only: every step of a collective runs inside
libhiccl.so (host planner + HIP kernels). Buffers are passed as integer
addresses; torch tensors and numpy arrays are accepted and converted with
``addr()``. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HICCL_LIB") or os.path.join(HERE, "libhiccl.so")

INT32, FLOAT32, BFLOAT16, FP8_E4M3 = 0, 1, 2, 3
DTYPES = {"int32": INT32, "float32": FLOAT32, "bfloat16": BFLOAT16, "fp8_e4m3": FP8_E4M3}
ELEM_SIZE = {INT32: 4, FLOAT32: 4, BFLOAT16: 2, FP8_E4M3: 1}
OPS = {"sum": 0, "max": 1, "min": 2}
EXEC = {"persistent": 0, "staged": 1}
ORDER = {"stage": 0, "program": 1, "channel": 2, "critical": 3}
BATCH = {"persistent": 0, "graph": 1, "serial": 2, "persistent_sjf": 3, "staged": 4}

SUCCESS, ERR_INVALID_ARG, ERR_STATE, ERR_RACE, ERR_OOM, ERR_HIP, ERR_TIMEOUT, ERR_UNSUPPORTED, ERR_BUSY = \
    0, -1, -2, -3, -4, -5, -6, -7, -8


class HicclError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hiccl error {code}: {msg}")
        self.code = code


class Buf(C.Structure):
    _fields_ = [("data", C.c_void_p), ("scales", C.c_void_p)]


MAX_SRC = 16


class TaskInfo(C.Structure):
    _fields_ = [("kind", C.c_int), ("prim", C.c_int), ("step", C.c_int), ("stripe", C.c_int),
                ("channel", C.c_int), ("stage", C.c_int), ("dst_rank", C.c_int), ("dst_workspace", C.c_int),
                ("nsrc", C.c_int), ("src_rank", C.c_int * MAX_SRC), ("npred", C.c_int), ("ring_step", C.c_int),
                ("count", C.c_uint64), ("offset", C.c_uint64)]


class PlanInfo(C.Structure):
    _fields_ = [("ntasks", C.c_uint64), ("ntiles", C.c_uint64), ("nedges", C.c_uint64), ("nstages", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("hbm_read", C.c_uint64), ("hbm_written", C.c_uint64),
                ("tile_elems", C.c_uint64)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2408_05962_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i, sz, u64 = C.c_void_p, C.c_int, C.c_size_t, C.c_uint64
        pi = C.POINTER(C.c_int)
        sig = {
            "hiccl_comm_create": [i, i, C.POINTER(vp)],
            "hiccl_comm_destroy": [vp],
            "hiccl_add_multicast": [vp, C.POINTER(Buf), C.POINTER(Buf), sz, i, pi, i],
            "hiccl_add_reduction": [vp, C.POINTER(Buf), C.POINTER(Buf), sz, pi, i, i, i],
            "hiccl_add_fence": [vp],
            "hiccl_set_hierarchy": [vp, pi, i],
            "hiccl_set_stripe": [vp, i],
            "hiccl_set_ring": [vp, i],
            "hiccl_set_pipeline": [vp, i],
            "hiccl_set_share": [vp, i],
            "hiccl_set_exec": [vp, i, sz, i, i],
            "hiccl_set_spin_limit": [vp, C.c_uint32],
            "hiccl_set_trace": [vp, i],
            "hiccl_trace_tasks": [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_size_t],
            "hiccl_set_claim": [vp, i, i],
            "hiccl_set_grid": [vp, i],
            "hiccl_init": [vp],
            "hiccl_workspace_size": [vp, C.POINTER(sz)],
            "hiccl_set_workspace": [vp, vp, sz],
            "hiccl_run": [vp, vp],
            "hiccl_run_static": [vp, vp],
            "hiccl_wait": [vp],
            "hiccl_query_bytes": [vp, pi, i, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)],
            "hiccl_plan_info": [vp, C.POINTER(PlanInfo)],
            "hiccl_plan_tasks": [vp, C.POINTER(TaskInfo), sz, C.POINTER(sz)],
            "hiccl_plan_edges": [vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), sz, C.POINTER(sz)],
            "hiccl_validate_host": [vp, u64, i],
            "hiccl_batch_create": [C.POINTER(vp), i, i, C.POINTER(vp)],
            "hiccl_batch_run": [vp, vp],
            "hiccl_batch_wait": [vp],
            "hiccl_batch_times": [vp, C.POINTER(u64), i],
            "hiccl_batch_destroy": [vp],
            "hiccl_run_batch": [C.POINTER(vp), i, vp, i],
            "hiccl_autotune": [vp, pi, i, pi, i, C.POINTER(sz), i, i, vp, pi, pi, C.POINTER(sz),
                               C.POINTER(C.c_double)],
            "hiccl_autotune_model": [vp, pi, i, pi, i, C.POINTER(sz), i, i, i, i, vp, pi, pi, C.POINTER(sz),
                                     C.POINTER(C.c_double), pi],
            "hiccl_autotune_batch": [C.POINTER(vp), i, pi, i, pi, i, pi, i, C.POINTER(sz), i, i, i, i, vp, pi, pi,
                                     C.POINTER(sz), C.POINTER(C.c_double)],
            "hiccl_server_create": [sz, i, C.POINTER(vp)],
            "hiccl_server_admit": [vp, sz, C.POINTER(u64)],
            "hiccl_server_stream": [vp, u64, C.POINTER(vp)],
            "hiccl_server_launch": [vp, u64, vp],
            "hiccl_server_submit": [vp, vp, C.POINTER(u64)],
            "hiccl_server_progress": [vp],
            "hiccl_server_poll": [vp, u64, pi, C.POINTER(C.c_double)],
            "hiccl_server_drain": [vp],
            "hiccl_server_usage": [vp, C.POINTER(sz), pi],
            "hiccl_server_start_ring": [vp, i, i],
            "hiccl_server_destroy": [vp],
            "hiccl_to_payload": [i, vp, vp, vp, sz, vp],
            "hiccl_from_payload": [i, vp, vp, vp, sz, vp],
            "hiccl_version": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.hiccl_last_error.argtypes = []
        L.hiccl_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc != SUCCESS:
        raise HicclError(rc, lib().hiccl_last_error().decode(errors="replace"))
    return rc


def addr(x) -> int:
    """Integer address of a torch tensor, numpy array, ctypes object or int (0 for None)."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if hasattr(x, "ctypes"):
        return int(x.ctypes.data)
    return int(C.addressof(x))


def stream_handle(stream) -> int | None:
    """hipStream_t of a torch stream (or an int / None for the default stream)."""
    if stream is None or isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _bufs(entries, n):
    arr = (Buf * n)()
    for r, e in enumerate(entries):
        if e is None:
            continue
        if isinstance(e, tuple):
            arr[r].data, arr[r].scales = addr(e[0]), addr(e[1]) or None
        else:
            arr[r].data, arr[r].scales = addr(e), None
        if not arr[r].data:
            arr[r].data = None
    return arr


def _ints(xs):
    xs = [int(v) for v in xs]
    return (C.c_int * max(1, len(xs)))(*xs), len(xs)


class Comm:
    """A communicator over ``nranks`` virtual ranks (one GPU's buffers)."""

    def __init__(self, nranks: int, dtype="float32"):
        self.nranks = nranks
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        h = C.c_void_p()
        check(lib().hiccl_comm_create(nranks, self.dtype, C.byref(h)))
        self.h = h
        self._buffers = []   # the buffer objects passed in: the library keeps only their addresses

    # composition (Sec. 3.1) -------------------------------------------------
    def add_multicast(self, send, recv, count, root, leaves):
        """send / recv: per-rank addresses (or (data, scales) pairs); None where unused. Tensors and
        arrays passed here are kept referenced for the communicator's lifetime."""
        lv, n = _ints(leaves)
        check(lib().hiccl_add_multicast(self.h, _bufs(send, self.nranks), _bufs(recv, self.nranks),
                                        int(count), int(root), lv, n))
        self._buffers.append((send, recv))
        return SUCCESS

    def add_reduction(self, send, recv, count, leaves, root, op="sum"):
        lv, n = _ints(leaves)
        check(lib().hiccl_add_reduction(self.h, _bufs(send, self.nranks), _bufs(recv, self.nranks),
                                        int(count), lv, n, int(root), OPS[op] if isinstance(op, str) else op))
        self._buffers.append((send, recv))
        return SUCCESS

    def add_fence(self):
        return check(lib().hiccl_add_fence(self.h))

    # optimization space (Sec. 4.1) --------------------------------------------
    def set_hierarchy(self, factors):
        f, n = _ints(factors)
        return check(lib().hiccl_set_hierarchy(self.h, f, n))

    def set_stripe(self, s):
        return check(lib().hiccl_set_stripe(self.h, int(s)))

    def set_ring(self, n):
        return check(lib().hiccl_set_ring(self.h, int(n)))

    def set_pipeline(self, m):
        return check(lib().hiccl_set_pipeline(self.h, int(m)))

    def set_share(self, rank=-1):
        return check(lib().hiccl_set_share(self.h, int(rank)))

    def set_exec(self, mode="persistent", tile_bytes=0, grid=0, order="stage"):
        return check(lib().hiccl_set_exec(self.h, EXEC.get(mode, mode), int(tile_bytes), int(grid),
                                          ORDER.get(order, order)))

    def set_grid(self, grid=0):
        return check(lib().hiccl_set_grid(self.h, int(grid)))

    def set_claim(self, queues=0, batch=0):
        return check(lib().hiccl_set_claim(self.h, int(queues), int(batch)))

    def set_spin_limit(self, polls):
        return check(lib().hiccl_set_spin_limit(self.h, int(polls)))

    def set_trace(self, on=True):
        return check(lib().hiccl_set_trace(self.h, 1 if on else 0))

    def trace(self):
        """(start_ns, end_ns) of every plan task in the last traced run (numpy uint64 arrays)."""
        import numpy as np
        n = self.plan_info()["ntasks"]
        start = np.zeros(max(1, n), np.uint64)
        end = np.zeros(max(1, n), np.uint64)
        p = C.POINTER(C.c_uint64)
        check(lib().hiccl_trace_tasks(self.h, start.ctypes.data_as(p), end.ctypes.data_as(p), n))
        return start[:n], end[:n]

    def init(self):
        return check(lib().hiccl_init(self.h))

    def workspace_size(self) -> int:
        v = C.c_size_t()
        check(lib().hiccl_workspace_size(self.h, C.byref(v)))
        return v.value

    def set_workspace(self, buf, nbytes):
        check(lib().hiccl_set_workspace(self.h, addr(buf), int(nbytes)))
        self._buffers.append(buf)
        return SUCCESS

    # execution ------------------------------------------------------------------
    def run(self, stream=None):
        return check(lib().hiccl_run(self.h, stream_handle(stream)))

    def run_static(self, stream=None):
        """hiccl_run without any device allocation: tables, counters and workspace in the library's static
        device scratch (calls that overlap on one GPU race)."""
        return check(lib().hiccl_run_static(self.h, stream_handle(stream)))

    def wait(self):
        return check(lib().hiccl_wait(self.h))

    # inspection -----------------------------------------------------------------
    def query_bytes(self, acct=None):
        if acct:
            a, n = _ints(acct)
        else:
            a, n = None, 0
        nl = (len(acct) if acct else 16) + 1
        lb = (C.c_uint64 * nl)()
        rd, wr = C.c_uint64(), C.c_uint64()
        check(lib().hiccl_query_bytes(self.h, a, n, lb, C.byref(rd), C.byref(wr)))
        return list(lb), rd.value, wr.value

    def plan_info(self) -> dict:
        pi = PlanInfo()
        check(lib().hiccl_plan_info(self.h, C.byref(pi)))
        return {k: getattr(pi, k) for k, _ in PlanInfo._fields_}

    def plan_tasks(self) -> list[dict]:
        n = C.c_size_t()
        check(lib().hiccl_plan_tasks(self.h, None, 0, C.byref(n)))
        arr = (TaskInfo * max(1, n.value))()
        check(lib().hiccl_plan_tasks(self.h, arr, n.value, C.byref(n)))
        out = []
        for t in arr[:n.value]:
            d = {k: getattr(t, k) for k, _ in TaskInfo._fields_ if k != "src_rank"}
            d["src_rank"] = list(t.src_rank[:min(t.nsrc, MAX_SRC)])
            out.append(d)
        return out

    def plan_edges(self):
        """Dependency edges (from, to) of the plan, as two numpy uint32 arrays of task indices."""
        import numpy as np
        n = C.c_size_t()
        check(lib().hiccl_plan_edges(self.h, None, None, 0, C.byref(n)))
        a = np.zeros(max(1, n.value), np.uint32)
        b = np.zeros(max(1, n.value), np.uint32)
        p = C.POINTER(C.c_uint32)
        check(lib().hiccl_plan_edges(self.h, a.ctypes.data_as(p), b.ctypes.data_as(p), n.value, C.byref(n)))
        return a[:n.value], b[:n.value]

    def validate_host(self, seed=0, norders=3):
        return check(lib().hiccl_validate_host(self.h, int(seed), int(norders)))

    def close(self):
        if getattr(self, "h", None):
            lib().hiccl_comm_destroy(self.h)
            self.h = None
            self._buffers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several initialized communicators executed together."""

    def __init__(self, comms, mode="persistent"):
        self.comms = list(comms)
        arr = (C.c_void_p * len(self.comms))(*[c.h for c in self.comms])
        h = C.c_void_p()
        check(lib().hiccl_batch_create(arr, len(self.comms), BATCH.get(mode, mode), C.byref(h)))
        self.h = h

    def run(self, stream=None):
        return check(lib().hiccl_batch_run(self.h, stream_handle(stream)))

    def wait(self):
        return check(lib().hiccl_batch_wait(self.h))

    def times_ns(self) -> list[int]:
        n = len(self.comms)
        arr = (C.c_uint64 * n)()
        check(lib().hiccl_batch_times(self.h, arr, n))
        return list(arr)

    def close(self):
        if getattr(self, "h", None):
            lib().hiccl_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(comms, stream=None, mode="persistent"):
    """Run initialized communicators as one memoized batch (hiccl_run_batch); ``comm.wait()`` on any member
    waits for the whole batch."""
    comms = list(comms)
    arr = (C.c_void_p * len(comms))(*[c.h for c in comms])
    return check(lib().hiccl_run_batch(arr, len(comms), stream_handle(stream), BATCH.get(mode, mode)))


def autotune(comm: Comm, stripes, pipes, tiles, reps=3, stream=None):
    s, ns = _ints(stripes)
    p, np_ = _ints(pipes)
    t = (C.c_size_t * len(tiles))(*[int(v) for v in tiles])
    bs, bp, bt, us = C.c_int(), C.c_int(), C.c_size_t(), C.c_double()
    check(lib().hiccl_autotune(comm.h, s, ns, p, np_, t, len(tiles), int(reps), stream_handle(stream),
                               C.byref(bs), C.byref(bp), C.byref(bt), C.byref(us)))
    return {"stripe": bs.value, "pipeline": bp.value, "tile_bytes": bt.value, "us": us.value}


def autotune_model(comm: Comm, stripes, pipes, tiles, reps=3, anchors=4, top=2, stream=None):
    """Model-guided autotune: fit a bytes / tiles / stages cost model to a few timed anchors, time the best
    predicted candidates, keep the fastest measured."""
    s, ns = _ints(stripes)
    p, np_ = _ints(pipes)
    t = (C.c_size_t * len(tiles))(*[int(v) for v in tiles])
    bs, bp, bt, us, nm = C.c_int(), C.c_int(), C.c_size_t(), C.c_double(), C.c_int()
    check(lib().hiccl_autotune_model(comm.h, s, ns, p, np_, t, len(tiles), int(reps), int(anchors), int(top),
                                     stream_handle(stream), C.byref(bs), C.byref(bp), C.byref(bt), C.byref(us),
                                     C.byref(nm)))
    return {"stripe": bs.value, "pipeline": bp.value, "tile_bytes": bt.value, "us": us.value, "measured": nm.value}


_live_servers: "weakref.WeakSet[Server]" = weakref.WeakSet()


def autotune_batch(comms, classes, stripes, pipes, tiles, mode="persistent", reps=5, sweeps=2, stream=None):
    """Per-class (stripe, pipeline, tile) by coordinate descent on the merged launch of the whole batch
    (hiccl_autotune_batch); the members are left planned with the choice. Returns {"choice": [(s, m, tile)
    per class], "ms": the batch's median time}."""
    comms = list(comms)
    ncls = max(classes) + 1
    arr = (C.c_void_p * len(comms))(*[c.h for c in comms])
    cl, _ = _ints(classes)
    s, ns = _ints(stripes)
    p, np_ = _ints(pipes)
    t = (C.c_size_t * len(tiles))(*[int(v) for v in tiles])
    bs, bp, bt = (C.c_int * ncls)(), (C.c_int * ncls)(), (C.c_size_t * ncls)()
    ms = C.c_double()
    check(lib().hiccl_autotune_batch(arr, len(comms), cl, ncls, s, ns, p, np_, t, len(tiles), BATCH.get(mode, mode),
                                     int(reps), int(sweeps), stream_handle(stream), bs, bp, bt, C.byref(ms)))
    return {"choice": [(bs[k], bp[k], bt[k]) for k in range(ncls)], "ms": ms.value}


@atexit.register
def _close_servers():
    # a server's device ring keeps a resident launch: stop it before the process ends
    for s in list(_live_servers):
        s.close()


class Server:
    """Admission under a device-memory budget with concurrent slots; with ``ring=True`` the
    requests are served by a resident launch from a device request ring."""

    def __init__(self, hbm_budget: int, slots: int, ring: bool = False, ring_grid: int = 0, idle_ms: int = 200):
        h = C.c_void_p()
        check(lib().hiccl_server_create(int(hbm_budget), int(slots), C.byref(h)))
        self.h = h
        _live_servers.add(self)
        if ring:
            check(lib().hiccl_server_start_ring(self.h, int(ring_grid), int(idle_ms)))

    def admit(self, footprint: int):
        """A ticket, or None when the request must wait (no slot or budget free now)."""
        t = C.c_uint64()
        rc = lib().hiccl_server_admit(self.h, int(footprint), C.byref(t))
        if rc == ERR_BUSY:
            return None
        check(rc)
        return t.value

    def submit(self, comm: Comm):
        """Admit (footprint computed by the library) and launch in one call; None when the request must wait."""
        t = C.c_uint64()
        rc = lib().hiccl_server_submit(self.h, comm.h, C.byref(t))
        if rc == ERR_BUSY:
            return None
        check(rc)
        return t.value

    def stream(self, ticket) -> int:
        s = C.c_void_p()
        check(lib().hiccl_server_stream(self.h, int(ticket), C.byref(s)))
        return s.value or 0

    def launch(self, ticket, comm: Comm):
        return check(lib().hiccl_server_launch(self.h, int(ticket), comm.h))

    def progress(self):
        return check(lib().hiccl_server_progress(self.h))

    def poll(self, ticket):
        d, us = C.c_int(), C.c_double()
        check(lib().hiccl_server_poll(self.h, int(ticket), C.byref(d), C.byref(us)))
        return bool(d.value), us.value

    def drain(self):
        return check(lib().hiccl_server_drain(self.h))

    def usage(self):
        u, r = C.c_size_t(), C.c_int()
        check(lib().hiccl_server_usage(self.h, C.byref(u), C.byref(r)))
        return u.value, r.value

    def close(self):
        if getattr(self, "h", None):
            check(lib().hiccl_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_payload(dtype, src, out, scales, n, stream=None):
    d = DTYPES[dtype] if isinstance(dtype, str) else dtype
    return check(lib().hiccl_to_payload(d, addr(src), addr(out), addr(scales) or None, int(n), stream_handle(stream)))


def from_payload(dtype, src, scales, out, n, stream=None):
    d = DTYPES[dtype] if isinstance(dtype, str) else dtype
    return check(lib().hiccl_from_payload(d, addr(src), addr(scales) or None, addr(out), int(n),
                                          stream_handle(stream)))
