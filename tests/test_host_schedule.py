"""The library's plans executed on host memory by its schedule checker, against the oracle.

The checker runs each plan in several random dependency-respecting orders
with poisoned workspace, so a missing dependency edge fails here on the CPU.
"""
import zlib

import numpy as np
import pytest

from tests import harness as H

pytest.importorskip("ctypes")


def _lib():
    from paper_2408_05962_amd import hiccl
    try:
        hiccl.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return hiccl


def _inputs(name, p, d, dtype, seed):
    rng = np.random.default_rng(seed)
    n = H.send_len(name, p, d)
    if dtype == "int32":
        return [rng.integers(-1000, 1001, n).astype(np.int32) for _ in range(p)]
    return [rng.standard_normal(n).astype(np.float32) for _ in range(p)]


def host_run(name, p, h, dtype, d, s=1, m=1, root=0, op="sum", seed=0, norders=3, tile=0, form="listing", ring=1):
    _lib()
    from paper_2408_05962_amd import collectives as CO
    sends = _inputs(name, p, d, dtype, seed)
    recvs = [np.full(H.recv_len(name, p, d), -7, H.NP[dtype]) for _ in range(p)]
    c = CO.make(name, p, dtype, sends, recvs, d, hierarchy=h, stripe=s, pipeline=m, root=root, op=op, tile_bytes=tile,
                form=form, init=False)
    c.set_ring(ring)
    c.init()
    c.validate_host(seed=seed, norders=norders)
    info = c.plan_info()
    c.close()
    exp_ranks = [root] if name in ("reduce", "gather") else range(p)
    return sends, {r: recvs[r] for r in exp_ranks}, info


@pytest.mark.parametrize("name", H.EIGHT)
@pytest.mark.parametrize("dtype", ["int32", "float32"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 8), ([2, 3], 3, 2), ([4, 4], 2, 3), ([16], 1, 1),
                                   ([2, 2, 2, 2], 2, 1), ([2, 2], 1, 1)])
def test_plans_match_oracle(name, dtype, h, s, m):
    p = int(np.prod(h))
    d = 37 if name not in ("all_gather", "gather") else 61
    seed = zlib.crc32(f"{name}{dtype}{h}".encode()) % 1000
    sends, got, _ = host_run(name, p, h, dtype, d, s=s, m=m, seed=seed)
    H.check_result(name, got, sends, dtype, h=h, s=s)


@pytest.mark.parametrize("op", ["max", "min"])
def test_max_min_plans(op):
    for name in ("all_reduce", "reduce_scatter", "reduce"):
        for dtype in ("int32", "float32"):
            sends, got, _ = host_run(name, 8, [2, 4], dtype, 33, s=2, m=2, op=op, seed=4)
            H.check_result(name, got, sends, dtype, op=op)


def test_roots_and_sparse_hierarchy():
    for name in ("broadcast", "reduce", "scatter", "gather"):
        for root in (5, 11):
            sends, got, _ = host_run(name, 12, [2, 2, 3], "int32", 29, s=3, m=2, root=root, seed=root)
            H.check_result(name, got, sends, "int32", root=root)


def test_single_step_allreduce_form():
    sends, got, _ = host_run("all_reduce", 8, [2, 4], "float32", 16, s=2, m=2, form="single")
    H.check_result("all_reduce", got, sends, "float32", order_exact=False)


def test_allreduce_4_ranks_2x2_schedule_shape():
    """All-Reduce of 4 ranks as {2,2}, 65,536 int32 per rank: 4 stages (RS node, RS top, AG top, AG leaf)."""
    import synth
    _lib()
    from paper_2408_05962_amd import collectives as CO
    p, n = 4, 65536
    sends = [synth.rank_buffer("int32", 0, 0, r, n) for r in range(p)]
    recvs = [np.zeros(n, np.int32) for _ in range(p)]
    c = CO.make("all_reduce", p, "int32", sends, recvs, n // p, hierarchy=[2, 2])
    c.validate_host(seed=9, norders=3)
    info = c.plan_info()
    lb, rd, wr = c.query_bytes()
    c.close()
    H.check_result("all_reduce", dict(enumerate(recvs)), sends, "int32")
    assert info["nstages"] == 4
    assert lb[1] == 512 * 1024 and lb[2] == 1024 * 1024      # top 512 KiB, intra-node 1 MiB
    assert rd + wr == 15 * n * 4                              # 15 S executed bytes


@pytest.mark.parametrize("name", H.EIGHT)
@pytest.mark.parametrize("dtype", ["int32", "float32"])
@pytest.mark.parametrize("h,ring,s,m", [([4, 3], 4, 3, 5), ([4, 4, 2], 4, 2, 2), ([2, 4, 2], 2, 4, 3), ([4, 2], 4, 1, 1),
                                        ([8, 2], 8, 2, 4)])
def test_ring_plans_match_oracle(name, dtype, h, ring, s, m):
    p = int(np.prod(h))
    d = 24 * s if name not in ("all_gather", "gather") else 40 * s
    seed = zlib.crc32(f"ring{name}{dtype}{h}".encode()) % 1000
    sends, got, info = host_run(name, p, h, dtype, d, s=s, m=m, seed=seed, ring=ring)
    H.check_result(name, got, sends, dtype, h=h, s=s, ring=ring)


def test_ring_broadcast_stages_and_rails():
    """ring(4), stripe(3) on 4 nodes x 3 GPUs: five stages (Fig. 6(b)) and the same hops as the oracle."""
    from oracle import tree as OT
    _lib()
    from paper_2408_05962_amd import Comm
    p, n = 12, 96
    send = [np.zeros(n, np.float32) for _ in range(p)]
    recv = [np.zeros(n, np.float32) for _ in range(p)]
    c = Comm(p, "float32")
    c.add_multicast(send, recv, n, 0, list(range(p)))
    c.set_hierarchy([4, 3])
    c.set_stripe(3)
    c.set_ring(4)
    c.init()
    assert c.plan_info()["nstages"] == 5
    lib_hops = sorted((t["src_rank"][0], t["dst_rank"]) for t in c.plan_tasks() if t["src_rank"][0] != t["dst_rank"])
    hops, nst = OT.ring_multicast_hops(0, range(p), [4, 3], 4, s=3)
    assert nst == 5
    assert lib_hops == sorted((hp.src, hp.dst) for hp in hops)
    ring_steps = {t["ring_step"] for t in c.plan_tasks()}
    assert ring_steps == {0, 1, 2, 3}
    c.close()


def test_ring_one_equals_tree_plan():
    _lib()
    from paper_2408_05962_amd import collectives as CO
    p, d = 16, 64
    sends = [np.zeros(d * p, np.float32) for _ in range(p)]
    recvs = [np.zeros(d * p, np.float32) for _ in range(p)]
    a = CO.make("all_reduce", p, "float32", sends, recvs, d, hierarchy=[2, 4, 2], stripe=4, pipeline=2)
    b = CO.make("all_reduce", p, "float32", sends, recvs, d, hierarchy=[2, 4, 2], stripe=4, pipeline=2, init=False)
    b.set_ring(1)
    b.init()
    ta, tb = a.plan_tasks(), b.plan_tasks()
    assert [(t["kind"], t["src_rank"], t["dst_rank"], t["count"]) for t in ta] == \
        [(t["kind"], t["src_rank"], t["dst_rank"], t["count"]) for t in tb]


@pytest.mark.parametrize("name", ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast"])
@pytest.mark.parametrize("dtype", ["int32", "float32"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 2), ([2, 3], 3, 1), ([4, 4], 1, 3)])
def test_two_step_compositions(name, dtype, h, s, m):
    """The multi-step rows of Table 2 through the library equal the direct definitions (and, for
    sums, the oracle's own step interpreter running the same composition)."""
    _lib()
    from oracle import steps as OS
    from paper_2408_05962_amd import Comm
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    d = 24
    seed = zlib.crc32(f"multi{name}{dtype}{h}".encode()) % 1000
    base = "all_reduce" if name == "all_reduce_bcast" else name
    sends = _inputs(base, p, d, dtype, seed)
    recvs = [np.full(H.recv_len(base, p, d), -7, H.NP[dtype]) for _ in range(p)]
    scratch = [np.zeros(d * p, H.NP[dtype]) for _ in range(p)]
    c = Comm(p, dtype)
    CO.compose_multi(c, name, sends, recvs, scratch, d, root=p - 1)
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_pipeline(m)
    c.init()
    c.validate_host(seed=seed, norders=3)
    c.close()
    root = p - 1
    ranks = [root] if base in ("reduce",) else range(p)
    exp = H.expected(base, sends, root)
    mem = OS.run(OS.Memory(OS.buffers_for(base, p, d, sends, "multi")), OS.compose(base if name != "all_reduce_bcast" else name, p, d, root=root, form="multi"))
    for r in ranks:
        y = exp[r]
        if dtype == "int32":
            assert np.array_equal(recvs[r], y), (name, r)
        else:
            assert np.max(np.abs(recvs[r] - y) / np.maximum(1, np.abs(y))) < 1e-5, (name, r)
        assert np.allclose(mem.result(f"y{r}", np.float64 if dtype == "float32" else np.int32), y)


@pytest.mark.parametrize("p,h,s,m,ring,seed", [(12, [2, 2, 3], 3, 2, 1, 1), (12, [2, 2, 3], 2, 3, 1, 2),
                                              (8, [2, 4], 2, 2, 2, 3), (16, [4, 4], 4, 1, 4, 4),
                                              (8, [8], 1, 4, 1, 5)])
def test_random_sparse_leaf_programs_host(p, h, s, m, ring, seed):
    """The GPU parity programs of random sparse-leaf primitives, run by the host schedule checker in
    random dependency orders, against the oracle's step interpreter."""
    from oracle import steps as OS
    from paper_2408_05962_amd import Comm
    from tests.test_gpu_parity import _random_program
    rng = np.random.default_rng(seed)
    L, slot = 4096, 512
    steps = _random_program(rng, p, L, 3, slot)
    A0 = rng.integers(-1000, 1001, (p, L)).astype(np.int32)
    B0 = rng.integers(-1000, 1001, (p, L)).astype(np.int32)
    A, B = A0.copy(), B0.copy()
    base = {"a": A, "b": B}

    def addr(ref):
        name, off = ref
        return base[name[0]][int(name[1:])].ctypes.data + off * 4

    c = Comm(p, "int32")
    for k, step in enumerate(steps):
        if k:
            c.add_fence()
        for pr in step:
            send = [addr(pr.send[r]) for r in range(p)]
            recv = [addr(pr.recv[r]) for r in range(p)]
            if pr.kind == "M":
                c.add_multicast(send, recv, pr.count, pr.root, pr.leaves)
            else:
                c.add_reduction(send, recv, pr.count, pr.leaves, pr.root, "sum")
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_ring(ring)
    c.set_pipeline(m)
    c.set_exec("persistent", 1024)
    c.init()
    c.validate_host(seed=seed, norders=3)
    c.close()
    mem = OS.Memory({**{f"a{r}": A0[r] for r in range(p)}, **{f"b{r}": B0[r] for r in range(p)}})
    OS.run(mem, steps)
    for r in range(p):
        assert np.array_equal(A[r], mem.result(f"a{r}", np.int32)), f"rank {r} buffer a"
        assert np.array_equal(B[r], mem.result(f"b{r}", np.int32)), f"rank {r} buffer b"
