"""The C-ABI library on the CPU: exports, argument and state errors, and the
factorizer's plans against the paper's worked examples and the oracle's
per-level byte counts. No kernel is launched here."""
import json
import os
import re

import numpy as np
import pytest

from oracle import tree as OT
from tests import harness as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def hc():
    from paper_2408_05962_amd import hiccl
    try:
        hiccl.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return hiccl


def test_every_declared_symbol_is_exported(hc):
    with open(os.path.join(ROOT, "include", "hiccl.h")) as f:
        text = f.read()
    names = set(re.findall(r"^\s*(?:int|const char\*)\s+(hiccl_[a-z_0-9]+)\s*\(", text, re.M))
    assert len(names) >= 35
    lib = hc.lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert lib.hiccl_version() >= 10000


def _bufs(p, n, dtype=np.float32):
    return [np.zeros(n, dtype) for _ in range(p)]


def _code(fn, *a):
    from paper_2408_05962_amd.hiccl import HicclError
    try:
        fn(*a)
    except HicclError as e:
        return e.code
    return 0


def test_argument_and_state_errors(hc):
    import ctypes as C
    lib = hc.lib()
    h = C.c_void_p()
    assert lib.hiccl_comm_create(0, 1, C.byref(h)) == hc.ERR_INVALID_ARG
    assert lib.hiccl_comm_create(4, 9, C.byref(h)) == hc.ERR_INVALID_ARG
    assert lib.hiccl_init(None) == hc.ERR_INVALID_ARG
    c = hc.Comm(4, "float32")
    s, r = _bufs(4, 8), _bufs(4, 8)
    assert _code(c.set_hierarchy, [2, 3]) == hc.ERR_INVALID_ARG          # product != nranks
    assert _code(c.add_multicast, s, r, 8, 0, [1, 1]) == hc.ERR_INVALID_ARG   # duplicate leaf
    assert _code(c.add_multicast, s, r, 8, 4, [1]) == hc.ERR_INVALID_ARG      # root out of range
    assert _code(c.add_multicast, s, r, 8, 0, [7]) == hc.ERR_INVALID_ARG      # leaf out of range
    assert _code(c.run) == hc.ERR_STATE                                       # not initialized
    c.add_multicast(s, r, 8, 0, [1, 2])
    # a second primitive writing rank 2's receive buffer in the same step is a race ...
    assert _code(c.add_multicast, s, r, 8, 3, [2]) == hc.ERR_RACE
    # ... and reading a buffer the step writes is a race too
    assert _code(c.add_multicast, r, s, 8, 1, [3]) == hc.ERR_RACE
    c.add_fence()
    c.add_multicast(s, r, 8, 3, [2])                                         # fine after a fence
    c.set_hierarchy([2, 2])
    c.set_stripe(3)
    assert _code(c.init) == hc.ERR_INVALID_ARG                               # 3 divides no group of {2,2}
    c.set_stripe(2)
    c.init()
    assert _code(c.add_fence) == hc.ERR_STATE
    assert _code(c.add_multicast, s, r, 8, 0, [1]) == hc.ERR_STATE
    assert _code(c.init) == hc.ERR_STATE
    c.set_pipeline(2)                                                        # re-plans
    c.init()
    assert c.plan_info()["ntasks"] > 0
    c.close()


def test_payload_type_errors(hc):
    c = hc.Comm(2, "fp8_e4m3")
    d = [np.zeros(512, np.uint8) for _ in range(2)]
    sc = [np.ones(2, np.float32) for _ in range(2)]
    bufs = list(zip(d, sc))
    assert _code(c.add_multicast, bufs, bufs[::-1], 100, 0, [1]) == hc.ERR_INVALID_ARG   # not whole blocks
    assert _code(c.add_multicast, d, d[::-1], 256, 0, [1]) == hc.ERR_INVALID_ARG         # scales missing
    assert _code(c.add_reduction, bufs, [bufs[1], bufs[0]], 256, [0, 1], 0, "max") == hc.ERR_UNSUPPORTED
    c.add_reduction([bufs[0], bufs[1]], [(np.zeros(256, np.uint8), np.ones(1, np.float32))] * 2, 256, [0, 1], 0)
    c.close()
    b = hc.Comm(2, "bfloat16")
    x = [np.zeros(8, np.uint16) for _ in range(4)]
    assert _code(b.add_reduction, x[:2], x[2:], 8, [0, 1], 0, "min") == hc.ERR_UNSUPPORTED
    b.close()


def test_ring_length_is_validated(hc):
    c = hc.Comm(4, "float32")
    s, r = _bufs(4, 4), _bufs(4, 4)
    c.add_multicast(s, r, 4, 0, [1, 2, 3])
    c.set_hierarchy([2, 2])
    c.set_ring(3)
    assert _code(c.init) in (hc.ERR_INVALID_ARG, hc.ERR_UNSUPPORTED)
    c.close()


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _bcast_plan(hc, h, s=1, m=1, root=0, n=96):
    p = int(np.prod(h))
    send, recv = _bufs(p, n), _bufs(p, n)
    c = hc.Comm(p, "float32")
    c.add_multicast(send, recv, n, root, list(range(p)))
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_pipeline(m)
    c.init()
    return c


def test_library_reproduces_worked_broadcast(hc):
    g = _gold("broadcast_2x2x3_tree.json")
    c = _bcast_plan(hc, g["hierarchy"])
    hops = {}
    for t in c.plan_tasks():
        a, b = t["src_rank"][0], t["dst_rank"]
        if a != b:
            hops.setdefault(str(OT.depth(a, b, g["hierarchy"])), []).append([a, b])
    for k, v in g["hops_by_depth"].items():
        assert sorted(hops[k]) == sorted(v)
    # the local root copy has no predecessor; the leaf hops wait for their staging rank (3 stages)
    assert c.plan_info()["nstages"] == g["stages_unstriped"]
    c.close()


def test_library_reproduces_striped_broadcast(hc):
    g = _gold("broadcast_2x2x3_striped.json")
    c = _bcast_plan(hc, g["hierarchy"], s=g["stripes"], n=96)
    tasks = c.plan_tasks()
    # the scatter hops carry stripes 1 and 2 from the root to their owners (stripe 0 stays at the root)
    scat = sorted([t["src_rank"][0], t["dst_rank"]] for t in tasks if t["stage"] == 0 and t["src_rank"][0] == 0
                  and t["stripe"] > 0 and t["dst_rank"] == g["owners"][t["stripe"]])
    assert scat == g["scatter_hops"]
    assert c.plan_info()["nstages"] == g["stages_striped"]
    c.close()
    # with at least as many channels as stages every channel can be in flight at once
    c = _bcast_plan(hc, g["hierarchy"], s=g["stripes"], m=g["min_channels_full_overlap"], n=96 * 4)
    chans = {t["channel"] for t in c.plan_tasks() if t["stage"] == 0}
    assert chans == set(range(g["min_channels_full_overlap"]))
    c.close()


def test_direct_vs_hierarchical_cross_node_copies(hc):
    g = _gold("broadcast_direct_vs_hierarchical_2x3.json")
    for key, hier in (("cross_node_copies_direct", g["direct_hierarchy"]),
                      ("cross_node_copies_hierarchical", g["hierarchical_hierarchy"])):
        c = _bcast_plan(hc, hier, n=64)
        lb, _, _ = c.query_bytes(g["accounting_hierarchy"])
        assert lb[1] == g[key] * 64 * 4
        c.close()


def test_listing_allreduce_fine_grain_dependencies(hc):
    """Three ranks: each in-place multicast M_i waits for its reduction R_i only, not for a barrier."""
    g = _gold("allreduce_listing_3ranks.json")
    from paper_2408_05962_amd import collectives as CO
    p, d = g["p"], 8
    send, recv = _bufs(p, d * p), _bufs(p, d * p)
    c = CO.make("all_reduce", p, "float32", send, recv, d, hierarchy=[p])
    tasks = c.plan_tasks()
    red = [t for t in tasks if t["step"] == 0]
    mc = [t for t in tasks if t["step"] == 1]
    assert [t["kind"] for t in red] == [1] * p and len(mc) == p * (p - 1)
    assert all(t["npred"] == 1 for t in mc)            # exactly the reduction of the same chunk
    for t in mc:
        assert t["src_rank"][0] == red[t["prim"] - p]["dst_rank"]
    c.close()


COLL = ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_to_all", "scatter", "gather"]


@pytest.mark.parametrize("h,s", [([2, 4, 2], 1), ([2, 4, 2], 4), ([2, 2, 3], 3), ([4, 4], 2), ([2, 4], 1)])
@pytest.mark.parametrize("name", COLL)
def test_level_bytes_match_oracle(hc, name, h, s):
    """Per-level logical bytes of the library's factorization equal the oracle's, and the top level
    carries exactly the minimum implied by Table 3."""
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    d = 16 * s
    send = _bufs(p, H.send_len(name, p, d))
    recv = _bufs(p, H.recv_len(name, p, d))
    c = CO.make(name, p, "float32", send, recv, d, hierarchy=h, stripe=s, pipeline=3)
    lb, rd, wr = c.query_bytes()
    c.close()
    ref = OT.collective_level_bytes(name, h, d, s=s, esize=4, align=4)
    assert lb[1:len(h) + 1] == ref[1:], (lb, ref)
    assert lb[1] == OT.min_top_bytes(name, p, p // h[0], d) * 4


@pytest.mark.parametrize("name,coef", [("broadcast", 32), ("reduce", 38.5), ("all_gather", 32),
                                       ("reduce_scatter", 38.5), ("all_reduce", 68.5), ("all_to_all", 44)])
def test_executed_bytes_16_ranks_2x4x2_shape(hc, name, coef):
    """Executed device-memory bytes of the {2,4,2}, s = 4 schedules as multiples of the per-rank buffer S."""
    from paper_2408_05962_amd import collectives as CO
    p, h, s, m = 16, [2, 4, 2], 4, 8
    d = 4096
    S = d * p * 4
    send = _bufs(p, H.send_len(name, p, d))
    recv = _bufs(p, H.recv_len(name, p, d))
    c = CO.make(name, p, "float32", send, recv, d, hierarchy=h, stripe=s, pipeline=m)
    _, rd, wr = c.query_bytes()
    c.close()
    assert (rd + wr) == coef * S


def test_tree_reduction_traffic(hc):
    """A full-leaf reduction on {2,4,2} reads 26 n and writes 11 n (8 + 2 + 1 fused nodes)."""
    p, n = 16, 64
    send, recv = _bufs(p, n), _bufs(p, n)
    c = hc.Comm(p, "float32")
    c.add_reduction(send, recv, n, list(range(p)), 0)
    c.set_hierarchy([2, 4, 2])
    c.init()
    _, rd, wr = c.query_bytes()
    ks = sorted(t["nsrc"] for t in c.plan_tasks())
    c.close()
    assert rd == 26 * n * 4 and wr == 11 * n * 4
    assert ks == [2] * 9 + [4] * 2


def test_workspace_and_plan_info(hc):
    from paper_2408_05962_amd import collectives as CO
    p, d = 16, 1024
    send, recv = _bufs(p, d * p), _bufs(p, d)
    c = CO.make("reduce_scatter", p, "float32", send, recv, d, hierarchy=[2, 4, 2], stripe=4, pipeline=8,
                tile_bytes=4096)
    info = c.plan_info()
    assert c.workspace_size() == info["workspace_bytes"] > 0
    assert info["tile_elems"] == 1024
    assert info["ntiles"] >= info["ntasks"]
    tasks = c.plan_tasks()
    assert all(t["stage"] == 0 or t["npred"] > 0 for t in tasks)
    assert [t["stage"] for t in tasks] == sorted(t["stage"] for t in tasks)   # claim order is stage order
    c.close()


@pytest.mark.parametrize("order", ["stage", "program", "channel", "critical"])
def test_claim_orders_are_topological(hc, order):
    from paper_2408_05962_amd import collectives as CO
    p, d = 16, 2048
    for name in ("all_reduce", "broadcast", "all_to_all"):
        send = _bufs(p, H.send_len(name, p, d))
        recv = _bufs(p, H.recv_len(name, p, d))
        c = CO.make(name, p, "float32", send, recv, d, hierarchy=[2, 4, 2], stripe=4, pipeline=8, order=order)
        tasks = c.plan_tasks()
        c.close()
        # every task's stage is 1 + the largest stage of its predecessors, so a topological order
        # never places a task before a task of a lower stage it could depend on; check the weaker
        # invariant that stage 0 tasks with no predecessors exist and channels are grouped when asked
        assert tasks and all((t["stage"] == 0) == (t["npred"] == 0) for t in tasks)
        if order == "channel":
            ch = [t["channel"] for t in tasks]
            assert ch == sorted(ch)
        if order in ("stage", "critical"):
            # a predecessor always has a lower stage, so stage-sorted tables are topological
            st = [t["stage"] for t in tasks]
            assert st == sorted(st)


def test_tile_limits(hc):
    """Device tile offsets are 32-bit and tile indices 31-bit: out-of-range tiles are argument errors."""
    c = hc.Comm(2, "float32")
    assert _code(c.set_exec, "persistent", 128) == hc.ERR_INVALID_ARG
    assert _code(c.set_exec, "persistent", (1 << 30) + 16) == hc.ERR_INVALID_ARG
    c.set_exec("staged", 1 << 30)
    # 2^32 elements per rank in 256-byte tiles would need 2^26 tiles per hop: fine; 2^39 bytes would not be
    c.add_multicast([1 << 40, 1 << 41], [1 << 42, 1 << 43], 1 << 37, 0, [1])
    c.set_exec("persistent", 256)
    assert _code(c.init) == hc.ERR_INVALID_ARG
    c.set_exec("persistent", 1 << 20)
    c.init()
    assert c.plan_info()["ntiles"] == (1 << 39) // (1 << 20)
    c.close()


@pytest.mark.parametrize("name", H.EIGHT)
def test_rank_shares_partition_the_plan(hc, name):
    """One rank's share keeps exactly the full plan's tasks whose output lies in that rank's memory, in
    the same claim order and with stages renumbered densely; the shares of all ranks partition the
    plan, its executed bytes and its edges' endpoints."""
    from paper_2408_05962_amd import collectives as CO
    p, d, h = 16, 256, [2, 4, 2]
    send, recv = _bufs(p, H.send_len(name, p, d)), _bufs(p, H.recv_len(name, p, d))
    kw = dict(hierarchy=h, stripe=4, pipeline=2, root=5, tile_bytes=1024)
    full = CO.make(name, p, "float32", send, recv, d, **kw)
    ft, fi = full.plan_tasks(), full.plan_info()
    full.close()

    def key(t):
        return (t["kind"], t["prim"], t["step"], t["stripe"], t["channel"], t["dst_rank"], t["dst_workspace"],
                tuple(t["src_rank"]), t["count"], t["offset"], t["ring_step"])

    ntasks = rd = wr = 0
    for r in range(p):
        c = CO.make(name, p, "float32", send, recv, d, share=r, **kw)
        st, si = c.plan_tasks(), c.plan_info()
        mine = [t for t in ft if t["dst_rank"] == r]
        assert [key(t) for t in st] == [key(t) for t in mine]
        # dense stages, a monotone renumbering of the full plan's, and edges only among kept tasks
        assert sorted({t["stage"] for t in st}) == list(range(si["nstages"]))
        remap = {s: i for i, s in enumerate(sorted({t["stage"] for t in mine}))}
        assert [t["stage"] for t in st] == [remap[t["stage"]] for t in mine]
        assert all(a["npred"] <= b["npred"] for a, b in zip(st, mine))
        assert si["workspace_bytes"] == fi["workspace_bytes"]
        assert _code(c.validate_host) == hc.ERR_STATE
        ntasks += si["ntasks"]
        rd += si["hbm_read"]
        wr += si["hbm_written"]
        c.close()
    assert (ntasks, rd, wr) == (fi["ntasks"], fi["hbm_read"], fi["hbm_written"])


def test_share_rank_is_validated(hc):
    c = hc.Comm(4, "int32")
    assert _code(c.set_share, -2) == hc.ERR_INVALID_ARG
    assert _code(c.set_share, 4) == hc.ERR_INVALID_ARG
    c.set_share(3)
    c.set_share(-1)
    c.close()


def _copy_comm(hc, src, dst, n=64):
    """A one-hop communicator: rank 0's `src` to rank 1's `dst` (host addresses; nothing is launched)."""
    c = hc.Comm(2, "float32")
    c.add_multicast([src, None], [None, dst], n, 0, [1])
    c.init()
    return c


def test_batch_members_must_be_disjoint(hc):
    """Batch members run unordered: a communicator twice, or one member writing memory another reads or
    writes, is rejected before anything touches the device. Read-read sharing passes the check."""
    import ctypes as C
    lib = hc.lib()
    a, b, c_, d = (np.zeros(64, np.float32) for _ in range(4))
    x = _copy_comm(hc, a, b)
    y_rw = _copy_comm(hc, b, c_)          # reads what x writes
    y_ww = _copy_comm(hc, d, b)           # writes what x writes
    y_rr = _copy_comm(hc, a, c_)          # reads what x reads: allowed
    y_half = hc.Comm(2, "float32")        # writes only the second half of b: still overlaps
    y_half.add_multicast([d, None], [None, b[32:]], 32, 0, [1])
    y_half.init()
    y_next = hc.Comm(2, "float32")        # writes right after b's range ends: no overlap
    e = np.zeros(128, np.float32)
    x2 = _copy_comm(hc, a, e[:64])
    y_next.add_multicast([d, None], [None, e[64:]], 64, 0, [1])
    y_next.init()

    def create(*cs):
        arr = (C.c_void_p * len(cs))(*[q.h for q in cs])
        h = C.c_void_p()
        rc = lib.hiccl_batch_create(arr, len(cs), 0, C.byref(h))
        if rc == 0:
            lib.hiccl_batch_destroy(h)
        return rc

    assert create(x, x) == hc.ERR_INVALID_ARG
    assert create(x, y_rw) == hc.ERR_INVALID_ARG
    assert create(y_rw, x) == hc.ERR_INVALID_ARG
    assert create(x, y_ww) == hc.ERR_INVALID_ARG
    assert create(x, y_half) == hc.ERR_INVALID_ARG
    assert create(y_rr, y_half, x) == hc.ERR_INVALID_ARG
    # disjoint members get past the check (on a host without a GPU the device upload then fails)
    assert create(x, y_rr) != hc.ERR_INVALID_ARG
    assert create(x2, y_next) != hc.ERR_INVALID_ARG
    # the memoized form applies the same rule
    arr = (C.c_void_p * 2)(x.h, y_ww.h)
    assert lib.hiccl_run_batch(arr, 2, None, 0) == hc.ERR_INVALID_ARG
    for q in (x, y_rw, y_ww, y_rr, y_half, y_next, x2):
        q.close()


def test_batch_caller_workspaces_must_not_overlap(hc):
    """A caller-provided workspace is memory its member writes."""
    import ctypes as C
    lib = hc.lib()
    p, n = 4, 256
    sends = [np.zeros(n, np.float32) for _ in range(2 * p)]
    recvs = [np.zeros(n, np.float32) for _ in range(2 * p)]
    cs = []
    for k in range(2):
        c = hc.Comm(p, "float32")
        c.add_reduction(sends[k * p:(k + 1) * p], recvs[k * p:(k + 1) * p], n, list(range(p)), 0)
        c.set_hierarchy([2, 2])
        c.init()
        cs.append(c)
    ws = np.zeros(4 * cs[0].workspace_size() // 4 + 1024, np.float32)
    base = (ws.ctypes.data + 255) // 256 * 256
    cs[0].set_workspace(base, cs[0].workspace_size())
    cs[1].set_workspace(base, cs[1].workspace_size())        # the same memory
    arr = (C.c_void_p * 2)(cs[0].h, cs[1].h)
    h = C.c_void_p()
    assert lib.hiccl_batch_create(arr, 2, 0, C.byref(h)) == hc.ERR_INVALID_ARG
    for c in cs:
        c.close()


def test_run_batch_and_submit_argument_errors(hc):
    import ctypes as C
    lib = hc.lib()
    assert lib.hiccl_run_batch(None, 1, None, 0) == hc.ERR_INVALID_ARG
    arr = (C.c_void_p * 1)(None)
    assert lib.hiccl_run_batch(arr, 0, None, 0) == hc.ERR_INVALID_ARG
    assert lib.hiccl_run_batch(arr, 1, None, 0) == hc.ERR_INVALID_ARG          # NULL member
    c = hc.Comm(2, "float32")
    a, b = np.zeros(8, np.float32), np.zeros(8, np.float32)
    c.add_multicast([a, None], [None, b], 8, 0, [1])
    arr = (C.c_void_p * 1)(c.h)
    assert lib.hiccl_run_batch(arr, 1, None, 0) == hc.ERR_STATE                # not initialized
    t = C.c_uint64()
    assert lib.hiccl_server_submit(None, c.h, C.byref(t)) == hc.ERR_INVALID_ARG
    c.close()


def test_run_static_checks_before_any_device_call(hc):
    """hiccl_run_static (the allocation-free entry point): NULL and uninitialized communicators are
    refused, and a plan whose workspace and tables exceed the static scratch is refused with
    INVALID_ARG before anything touches a device (this runs on a host without one)."""
    import ctypes as C
    lib = hc.lib()
    assert lib.hiccl_run_static(None, None) == hc.ERR_INVALID_ARG
    p, d = 16, 1 << 20
    s, r = _bufs(p, d * p), _bufs(p, d * p)
    c = hc.Comm(p, "float32")
    from paper_2408_05962_amd import collectives as CO
    CO.compose(c, "all_reduce", s, r, d)
    c.set_hierarchy([2, 4, 2])
    c.set_stripe(4)
    assert lib.hiccl_run_static(c.h, None) == hc.ERR_STATE
    c.init()
    assert c.workspace_size() > (64 << 20)        # 16 ranks x 4 MiB chunks: workspace alone exceeds 64 MiB
    assert lib.hiccl_run_static(c.h, None) == hc.ERR_INVALID_ARG
    assert b"static scratch" in lib.hiccl_last_error()
    c.close()


def test_autotune_batch_argument_errors(hc):
    """hiccl_autotune_batch refuses empty candidate lists and out-of-range classes before any device call."""
    import ctypes as C
    lib = hc.lib()
    c = hc.Comm(4, "float32")
    s, r = _bufs(4, 64), _bufs(4, 64)
    from paper_2408_05962_amd import collectives as CO
    CO.compose(c, "all_reduce", s, r, 16)
    c.init()
    arr = (C.c_void_p * 1)(c.h)
    one = (C.c_int * 1)(1)
    bad = (C.c_int * 1)(3)
    tiles = (C.c_size_t * 1)(0)
    out_i, out_p, out_t, ms = (C.c_int * 4)(), (C.c_int * 4)(), (C.c_size_t * 4)(), C.c_double()
    args = lambda cls, ncls, ns: (arr, 1, cls, ncls, one, ns, one, 1, tiles, 1, 0, 1, 1, None, out_i, out_p, out_t,  # noqa: E731
                                  C.byref(ms))
    assert lib.hiccl_autotune_batch(*args(bad, 2, 1)) == hc.ERR_INVALID_ARG        # class 3 of 2
    assert lib.hiccl_autotune_batch(*args(one, 2, 0)) == hc.ERR_INVALID_ARG        # no stripe candidate
    assert lib.hiccl_autotune_batch(None, 0, one, 1, one, 1, one, 1, tiles, 1, 0, 1, 1, None, out_i, out_p, out_t,
                                    C.byref(ms)) == hc.ERR_INVALID_ARG
    c.close()


def test_trace_argument_and_state_errors(hc):
    """hiccl_set_trace takes 0 or 1; hiccl_trace_tasks wants the plan's task count and a traced persistent
    run of the communicator itself, and says STATE (before any device call) when there is none."""
    import ctypes as C
    lib = hc.lib()
    assert lib.hiccl_set_trace(None, 1) == hc.ERR_INVALID_ARG
    c = hc.Comm(4, "float32")
    s, r = _bufs(4, 64), _bufs(4, 64)
    from paper_2408_05962_amd import collectives as CO
    CO.compose(c, "all_reduce", s, r, 16)
    c.set_hierarchy([2, 2])
    assert lib.hiccl_set_trace(c.h, 2) == hc.ERR_INVALID_ARG
    buf = (C.c_uint64 * 64)()
    assert lib.hiccl_trace_tasks(c.h, buf, buf, 0) == hc.ERR_STATE              # not initialized
    c.init()
    nt = c.plan_info()["ntasks"]
    assert lib.hiccl_trace_tasks(c.h, buf, buf, nt) == hc.ERR_STATE             # trace off
    c.set_trace(True)
    assert lib.hiccl_trace_tasks(c.h, buf, buf, nt + 1) == hc.ERR_INVALID_ARG   # wrong count
    assert lib.hiccl_trace_tasks(c.h, None, buf, nt) == hc.ERR_INVALID_ARG
    assert lib.hiccl_trace_tasks(c.h, buf, buf, nt) == hc.ERR_STATE             # no run yet
    c.set_exec("staged", 0, 0, "stage")                                        # discards the plan
    c.init()
    assert lib.hiccl_trace_tasks(c.h, buf, buf, c.plan_info()["ntasks"]) == hc.ERR_STATE   # staged executor
    c.close()


def test_plan_edges_match_the_plan(hc):
    """hiccl_plan_edges: as many edges as hiccl_plan_info counts, each task's in-degree equals its npred,
    every edge runs from a lower stage to a higher one, and inside one primitive's tree the edges stay
    within a channel (Sec. 4.5: channel c of a node depends on channel c of its predecessors)."""
    import numpy as np
    from paper_2408_05962_amd import collectives as CO
    p, d = 16, 4096
    s, r = _bufs(p, d * p), _bufs(p, d * p)
    c = hc.Comm(p, "float32")
    CO.compose(c, "all_reduce", s, r, d)
    c.set_hierarchy([2, 4, 2])
    c.set_stripe(4)
    c.set_pipeline(4)
    c.init()
    info = c.plan_info()
    tasks = c.plan_tasks()
    a, b = c.plan_edges()
    assert len(a) == info["nedges"] > 0
    indeg = np.bincount(b, minlength=len(tasks))
    assert [int(x) for x in indeg] == [t["npred"] for t in tasks]
    for x, y in zip(a.tolist(), b.tolist()):
        assert tasks[x]["stage"] < tasks[y]["stage"]
        if tasks[x]["prim"] == tasks[y]["prim"]:
            assert tasks[x]["channel"] == tasks[y]["channel"]
    c.close()
