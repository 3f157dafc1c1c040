"""GPU parity: the HIP executor against the CPU oracle, through the C ABI."""
import zlib

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2408_05962_amd import hiccl
    hiccl.lib()          # must load: a GPU run without the native library is a failure, not a skip
    return torch


def _host_inputs(name, p, d, dtype, seed):
    rng = np.random.default_rng(seed)
    n = H.send_len(name, p, d)
    if dtype == "int32":
        return [rng.integers(-1000, 1001, n).astype(np.int32) for _ in range(p)]
    return [rng.standard_normal(n).astype(np.float32) for _ in range(p)]


def _run(torch, name, p, h, dtype, d, s=1, m=1, mode="persistent", sends=None, seed=0, reps=1, tile=0, root=0,
         op="sum", order="stage", ring=1, grid=0, claim=None):
    from paper_2408_05962_amd import collectives as CO
    if sends is None:
        sends = _host_inputs(name, p, d, dtype, seed)
    tdt = torch.int32 if dtype == "int32" else torch.float32
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.full((p, H.recv_len(name, p, d)), -7, dtype=tdt, device="cuda")
    send = [S[r] for r in range(p)]
    recv = [R[r] for r in range(p)]
    c = CO.make(name, p, dtype, send, recv, d, hierarchy=h, stripe=s, pipeline=m, exec_mode=mode, tile_bytes=tile,
                root=root, op=op, order=order, ring=ring, grid=grid)
    if claim:
        c.set_claim(*claim)
    c.set_spin_limit(1 << 20)    # a stalled dependency fails the test within seconds
    st = torch.cuda.current_stream()
    outs = []
    for _ in range(reps):
        R.fill_(-7)
        c.run(st)
        c.wait()
        torch.cuda.synchronize()
        outs.append(R.cpu().numpy().copy())
    c.close()
    return sends, outs


def _got(name, out, p, root):
    exp_ranks = [root] if name in ("reduce", "gather") else range(p)
    return {r: out[r] for r in exp_ranks}


def test_allreduce_4_ranks_2x2_int32_bit_exact(torch_cuda):
    """All-Reduce over 4 ranks as {2,2}, 65,536 int32 per rank in [-1000, 1000], s = m = 1."""
    import synth
    p, n = 4, 65536
    sends = [synth.rank_buffer("int32", 0, 0, r, n) for r in range(p)]
    for mode in ("persistent", "staged"):
        _, outs = _run(torch_cuda, "all_reduce", p, [2, 2], "int32", n // p, sends=sends, reps=3, mode=mode)
        for out in outs:
            H.check_result("all_reduce", _got("all_reduce", out, p, 0), sends, "int32")


@pytest.mark.parametrize("name", H.EIGHT)
@pytest.mark.parametrize("dtype", ["int32", "float32"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 8), ([2, 3], 3, 2), ([4, 4], 2, 3), ([16], 1, 1), ([2, 2, 2, 2], 2, 1)])
def test_collectives_small(torch_cuda, name, dtype, h, s, m):
    p = int(np.prod(h))
    d = 1003 if name not in ("all_gather", "gather") else 2051   # ragged: not a multiple of the vector width
    sends, outs = _run(torch_cuda, name, p, h, dtype, d, s=s, m=m, seed=zlib.crc32(f"{name}{dtype}{h}".encode()) % 1000,
                       reps=2, tile=4096)
    for out in outs:
        H.check_result(name, _got(name, out, p, 0), sends, dtype, h=h, s=s)
    assert np.array_equal(outs[0], outs[1])   # re-runs reset their counters and reproduce bit for bit


@pytest.mark.parametrize("name", H.SIX)
def test_staged_matches_persistent(torch_cuda, name):
    h, s, m = [2, 4, 2], 4, 4
    p = 16
    sends, a = _run(torch_cuda, name, p, h, "float32", 4096, s=s, m=m, seed=5, mode="persistent", tile=8192)
    _, b = _run(torch_cuda, name, p, h, "float32", 4096, s=s, m=m, sends=sends, mode="staged", tile=8192)
    _, c = _run(torch_cuda, name, p, h, "float32", 4096, s=s, m=m, sends=sends, mode="persistent", tile=8192,
                order="program")
    _, e = _run(torch_cuda, name, p, h, "float32", 4096, s=s, m=m, sends=sends, mode="persistent", tile=8192,
                order="channel")
    _, f = _run(torch_cuda, name, p, h, "float32", 4096, s=s, m=m, sends=sends, mode="persistent", tile=8192,
                order="critical")
    assert np.array_equal(a[0].view(np.uint32), f[0].view(np.uint32))
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
    assert np.array_equal(a[0].view(np.uint32), c[0].view(np.uint32))
    assert np.array_equal(a[0].view(np.uint32), e[0].view(np.uint32))


@pytest.mark.parametrize("name", ["all_reduce", "broadcast", "all_gather"])
@pytest.mark.parametrize("mode", ["persistent", "staged"])
@pytest.mark.parametrize("grid,claim", [(1, None), (7, (8, 1)), (300, (3, 5)), (1000, (8, 16))])
def test_launch_shapes_do_not_change_results(torch_cuda, name, mode, grid, claim):
    """Grid, queue count and claim batch decide only who runs which tile (and on which XCD), never the
    arithmetic; Broadcast and All-Gather exercise the grouping of same-source tiles."""
    h, s, m, p = [2, 4, 2], 4, 2, 16
    sends, ref = _run(torch_cuda, name, p, h, "float32", 2048 + 5, s=s, m=m, seed=21, tile=4096)
    _, got = _run(torch_cuda, name, p, h, "float32", 2048 + 5, s=s, m=m, sends=sends, tile=4096, mode=mode,
                  grid=grid, claim=claim, reps=2)
    for out in got:
        assert np.array_equal(out.view(np.uint32), ref[0].view(np.uint32))
    H.check_result(name, _got(name, ref[0], p, 0), sends, "float32", h=h, s=s)


@pytest.mark.parametrize("op", ["max", "min"])
@pytest.mark.parametrize("dtype", ["int32", "float32"])
def test_max_min(torch_cuda, op, dtype):
    for name in ("all_reduce", "reduce_scatter", "reduce"):
        sends, outs = _run(torch_cuda, name, 8, [2, 4], dtype, 777, s=2, m=2, op=op, seed=3)
        H.check_result(name, _got(name, outs[0], 8, 0), sends, dtype, op=op)


def test_root_and_odd_hierarchies(torch_cuda):
    for name in ("broadcast", "reduce", "scatter", "gather"):
        for root in (5, 11):
            sends, outs = _run(torch_cuda, name, 12, [2, 2, 3], "int32", 513, s=3, m=2, root=root, seed=root)
            H.check_result(name, _got(name, outs[0], 12, root), sends, "int32", root=root)


def test_empty_and_tiny(torch_cuda):
    for name in ("all_reduce", "all_to_all", "broadcast"):
        sends, outs = _run(torch_cuda, name, 4, [2, 2], "float32", 1, s=2, m=4, seed=1)
        H.check_result(name, _got(name, outs[0], 4, 0), sends, "float32", h=[2, 2], s=2)
    from paper_2408_05962_amd import Comm
    import torch
    x = torch.zeros(4, device="cuda")
    c = Comm(4, "float32")
    c.add_multicast([x] * 4, [x] * 4, 0, 0, [1, 2, 3])   # count 0: a no-op
    c.set_hierarchy([2, 2])
    c.init()
    c.run()
    c.wait()
    assert c.plan_info()["ntasks"] == 0


def test_many_reruns_stress(torch_cuda):
    """Many small tasks, many repeats: device counters reset themselves and ordering holds."""
    import torch
    from paper_2408_05962_amd import collectives as CO
    p, d = 16, 2048
    sends = _host_inputs("all_reduce", p, d, "int32", 11)
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, d * p), dtype=torch.int32, device="cuda")
    c = CO.make("all_reduce", p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=[2, 4, 2],
                stripe=4, pipeline=8, tile_bytes=1024)
    exp = H.expected("all_reduce", sends)[0]
    st = torch.cuda.current_stream()
    for it in range(50):
        R.zero_()
        c.run(st)
    c.wait()
    got = R.cpu().numpy()
    for r in range(p):
        assert np.array_equal(got[r], exp)
    c.close()


@pytest.mark.parametrize("name", H.SIX)
@pytest.mark.parametrize("mode", ["staged", "persistent"])
def test_six_collectives_16_ranks_64MiB_full_size(torch_cuda, name, mode):
    """Six collectives, 16 ranks as {2,4,2}, 64 MiB float32 per rank ~ N(0,1), stripe 4, pipeline 8, default tile
    and grid: the bench's launch configuration (staged) and its other executor (persistent)."""
    import torch
    import synth
    from paper_2408_05962_amd import collectives as CO
    p, h, s, m = 16, [2, 4, 2], 4, 8
    S_el = 64 * 2 ** 20 // 4
    d = S_el // p
    sl, rl = H.send_len(name, p, d), H.recv_len(name, p, d)
    Sd = synth.device_buffers("float32", 2000 + H.SIX.index(name), p, sl)
    R = torch.full((p, rl), float("nan"), device="cuda")
    c = CO.make(name, p, "float32", [Sd[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=s,
                pipeline=m, exec_mode=mode)
    sends = [x for x in Sd.cpu().numpy()]
    c.run(torch.cuda.current_stream())
    c.wait()
    torch.cuda.synchronize()
    got = R.cpu().numpy()
    c.close()
    H.check_result(name, _got(name, got, p, 0), sends, "float32", h=h, s=s, order_exact=True)


@pytest.mark.parametrize("name", H.EIGHT)
@pytest.mark.parametrize("h,ring,s,m", [([4, 4, 2], 4, 2, 4), ([4, 3], 4, 3, 5), ([8, 2], 8, 1, 8)])
def test_ring_collectives(torch_cuda, name, h, ring, s, m):
    """Hybrid ring + tree (Sec. 4.4) on the device: bit-exact data movement and tree/ring-order float32 sums."""
    p = int(np.prod(h))
    d = 1536 + 5 if name not in ("all_gather", "gather") else 4099
    for dtype in ("int32", "float32"):
        sends, outs = _run(torch_cuda, name, p, h, dtype, d, s=s, m=m, ring=ring, tile=8192, reps=2,
                           seed=zlib.crc32(f"ring{name}{h}{dtype}".encode()) % 1000)
        for out in outs:
            H.check_result(name, _got(name, out, p, 0), sends, dtype, h=h, s=s, ring=ring)


def _random_program(rng, p, L, nsteps, slot):
    """Steps of random multicasts / reductions over sparse leaf sets. Step k reads buffer X_k and writes
    Y_k (alternating "a" / "b"), each primitive into its own slot of Y, so no step has a race."""
    from oracle import steps as OS
    steps = []
    for k in range(nsteps):
        X, Y = ("a", "b") if k % 2 == 0 else ("b", "a")
        prims = []
        for q in range(L // slot):
            n = int(rng.integers(1, slot + 1))                      # ragged counts
            so = int(rng.integers(0, L - n + 1))                    # any read offset
            wo = q * slot + int(rng.integers(0, slot - n + 1))      # inside this primitive's slot
            k_leaves = int(rng.integers(1, p + 1))
            leaves = sorted(int(x) for x in rng.choice(p, k_leaves, replace=False))
            root = int(rng.integers(0, p))
            send = {r: (f"{X}{r}", so) for r in range(p)}
            recv = {r: (f"{Y}{r}", wo) for r in range(p)}
            if rng.random() < 0.5:
                prims.append(OS.multicast(root, leaves, n, send, recv))
            else:
                prims.append(OS.reduction(leaves, root, n, send, recv))
        steps.append(prims)
    return steps


@pytest.mark.parametrize("p,h,s,m,ring,seed", [(12, [2, 2, 3], 3, 2, 1, 1), (12, [2, 2, 3], 2, 3, 1, 2),
                                              (8, [2, 4], 2, 2, 2, 3), (16, [4, 4], 4, 1, 4, 4),
                                              (8, [8], 1, 4, 1, 5)])
@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_random_sparse_leaf_programs(torch_cuda, p, h, s, m, ring, seed, mode):
    """Custom collectives: multicasts and reductions over random leaf subsets and roots, ragged counts,
    several fenced steps, against the oracle's step interpreter (int32, bit-exact)."""
    torch = torch_cuda
    from oracle import steps as OS
    from paper_2408_05962_amd import Comm
    rng = np.random.default_rng(seed)
    L, slot = 4096, 512
    steps = _random_program(rng, p, L, 3, slot)
    A0 = rng.integers(-1000, 1001, (p, L)).astype(np.int32)
    B0 = rng.integers(-1000, 1001, (p, L)).astype(np.int32)
    A, B = torch.from_numpy(A0).to("cuda"), torch.from_numpy(B0).to("cuda")
    base = {"a": A, "b": B}

    def addr(ref):
        name, off = ref
        return base[name[0]][int(name[1:])].data_ptr() + off * 4

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
    c.set_exec(mode, 1024)
    c.set_spin_limit(1 << 20)
    c.init()
    c.run(torch.cuda.current_stream())
    c.wait()
    torch.cuda.synchronize()
    c.close()
    mem = OS.Memory({**{f"a{r}": A0[r] for r in range(p)}, **{f"b{r}": B0[r] for r in range(p)}})
    OS.run(mem, steps)
    gotA, gotB = A.cpu().numpy(), B.cpu().numpy()
    for r in range(p):
        assert np.array_equal(gotA[r], mem.result(f"a{r}", np.int32)), f"rank {r} buffer a"
        assert np.array_equal(gotB[r], mem.result(f"b{r}", np.int32)), f"rank {r} buffer b"


def test_spin_limit_abort_is_clean_and_recoverable(torch_cuda):
    """A spin limit of one poll makes the persistent executor give up its first unmet dependency wait:
    the run ends (every workgroup exits), hiccl_wait reports TIMEOUT, and the same communicator then
    runs correctly with the normal limit (the last workgroup out reset every counter)."""
    torch = torch_cuda
    from paper_2408_05962_amd import collectives as CO
    from paper_2408_05962_amd.hiccl import ERR_TIMEOUT, HicclError
    name, p, h, d = "all_reduce", 16, [2, 4, 2], 4096
    sends = _host_inputs(name, p, d, "int32", 77)
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, H.recv_len(name, p, d)), dtype=torch.int32, device="cuda")
    c = CO.make(name, p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=4,
                pipeline=2, tile_bytes=1024)
    st = torch.cuda.current_stream()
    c.set_spin_limit(1)
    timeouts = 0
    for _ in range(3):
        c.run(st)
        try:
            c.wait()
        except HicclError as e:
            assert e.code == ERR_TIMEOUT
            timeouts += 1
        torch.cuda.synchronize()
    assert timeouts > 0
    c.set_spin_limit(1 << 20)
    for _ in range(2):
        R.zero_()
        c.run(st)
        c.wait()
        torch.cuda.synchronize()
        out = R.cpu().numpy()
        H.check_result(name, {r: out[r] for r in range(p)}, sends, "int32")
    c.close()


@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_debug_counter_check_after_runs(torch_cuda, mode, monkeypatch):
    """HICCL_DEBUG=1 makes every wait read back the task table's counters: after normal runs, after runs
    that gave up a dependency wait (TIMEOUT, counters still reset by the last workgroup) and after a batch
    run, every counter is where the next run expects it, so no wait reports STATE, and results stay exact."""
    torch = torch_cuda
    from paper_2408_05962_amd import Batch
    from paper_2408_05962_amd import collectives as CO
    from paper_2408_05962_amd.hiccl import ERR_TIMEOUT, HicclError
    monkeypatch.setenv("HICCL_DEBUG", "1")
    name, p, h, d = "all_reduce", 16, [2, 4, 2], 4096
    sends = _host_inputs(name, p, d, "int32", 78)
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, H.recv_len(name, p, d)), dtype=torch.int32, device="cuda")
    c = CO.make(name, p, "int32", [S[r] for r in range(p)], [R[r] for r in range(p)], d, hierarchy=h, stripe=4,
                pipeline=2, tile_bytes=1024, exec_mode=mode)
    st = torch.cuda.current_stream()
    for _ in range(3):
        R.zero_()
        c.run(st)
        c.wait()
        out = R.cpu().numpy()
        H.check_result(name, {r: out[r] for r in range(p)}, sends, "int32")
    if mode == "persistent":
        c.set_spin_limit(1)
        for _ in range(3):
            c.run(st)
            try:
                c.wait()
            except HicclError as e:
                assert e.code == ERR_TIMEOUT
        c.set_spin_limit(1 << 20)
    R.zero_()
    b = Batch([c], "persistent" if mode == "persistent" else "staged")
    b.run(st)
    b.wait()
    out = R.cpu().numpy()
    H.check_result(name, {r: out[r] for r in range(p)}, sends, "int32")
    b.close()
    c.close()


@pytest.mark.parametrize("name,p,h", [("all_reduce", 1, [1]), ("broadcast", 1, [1]), ("all_reduce", 2, [1, 2]),
                                      ("all_reduce", 4, [4, 1]), ("all_to_all", 3, [3]), ("reduce_scatter", 6, [3, 1, 2])])
@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_degenerate_hierarchies(torch_cuda, name, p, h, mode):
    """One rank, unit factors and odd factors: the factorization degenerates to copies or flat levels."""
    sends, outs = _run(torch_cuda, name, p, h, "int32", 37, seed=3, reps=2, mode=mode, tile=1024)
    for out in outs:
        H.check_result(name, _got(name, out, p, 0), sends, "int32", h=h)


@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_unaligned_operands(torch_cuda, mode):
    """Buffers that start one element past a 16-byte boundary take the 4-byte (and byte) paths."""
    torch = torch_cuda
    from paper_2408_05962_amd import collectives as CO
    name, p, h, d = "all_reduce", 8, [2, 4], 1000
    sends = _host_inputs(name, p, d, "float32", 9)
    n = H.send_len(name, p, d)
    S = torch.zeros((p, n + 1), dtype=torch.float32, device="cuda")
    S[:, 1:] = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.zeros((p, n + 1), dtype=torch.float32, device="cuda")
    c = CO.make(name, p, "float32", [S[r, 1:] for r in range(p)], [R[r, 1:] for r in range(p)], d, hierarchy=h,
                stripe=2, pipeline=3, exec_mode=mode, tile_bytes=2048)
    c.set_spin_limit(1 << 20)
    c.run(torch.cuda.current_stream())
    c.wait()
    torch.cuda.synchronize()
    c.close()
    out = R[:, 1:].cpu().numpy()
    assert np.all(R[:, 0].cpu().numpy() == 0)           # nothing written before the buffers
    H.check_result(name, {r: out[r] for r in range(p)}, sends, "float32", h=h, s=2)


@pytest.mark.parametrize("name", ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast"])
@pytest.mark.parametrize("h,s,m", [([2, 4, 2], 4, 2), ([2, 3], 3, 1)])
@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_two_step_compositions(torch_cuda, name, h, s, m, mode):
    """The two-step rows of Table 2 (a fence between the steps, an intermediate scratch buffer) on the
    GPU, int32: equal to the direct definitions bit for bit."""
    torch = torch_cuda
    from paper_2408_05962_amd import Comm
    from paper_2408_05962_amd import collectives as CO
    p = int(np.prod(h))
    d = 1000 + 3
    base = "all_reduce" if name == "all_reduce_bcast" else name
    sends = _host_inputs(base, p, d, "int32", zlib.crc32(f"two{name}{h}".encode()) % 1000)
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.full((p, H.recv_len(base, p, d)), -7, dtype=torch.int32, device="cuda")
    X = torch.zeros((p, d * p), dtype=torch.int32, device="cuda")
    c = Comm(p, "int32")
    CO.compose_multi(c, name, [S[r] for r in range(p)], [R[r] for r in range(p)], [X[r] for r in range(p)], d,
                     root=p - 1)
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_pipeline(m)
    c.set_exec(mode, 4096)
    c.set_spin_limit(1 << 20)
    c.init()
    for _ in range(2):
        R.fill_(-7)
        c.run(torch.cuda.current_stream())
        c.wait()
        torch.cuda.synchronize()
        out = R.cpu().numpy()
        H.check_result(base, _got(base, out, p, p - 1), sends, "int32", root=p - 1)
    c.close()


def _two_step_f32_expected(name, sends, h, s, root):
    """Tree-order float32 result of a two-step row of Table 2: the reduction step is summed in the
    oracle's tree order (per stripe), and the copy step moves its bits unchanged."""
    p = len(sends)
    if name in ("broadcast", "all_gather"):
        return None                                             # pure data movement: checked exactly
    if name == "reduce":                                        # Gather . Reduce-scatter
        return {root: H.tree_order_f32("all_reduce", sends, h, s)[0]}
    full = H.tree_order_f32("reduce", sends, h, s, root=root)[root]     # Reduce at the root first
    if name == "reduce_scatter":                                # Scatter . Reduce
        d = len(full) // p
        return {j: full[j * d:(j + 1) * d] for j in range(p)}
    return {r: full for r in range(p)}                          # all_reduce_bcast = Broadcast . Reduce


@pytest.mark.parametrize("name", ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce_bcast"])
@pytest.mark.parametrize("mode", ["persistent", "staged"])
def test_two_step_compositions_float32(torch_cuda, name, mode):
    """The two-step rows of Table 2 in float32 at {2,4,2}, stripe 4, pipeline 2, with a ragged chunk:
    within the condition-scaled 1e-5 of the float64 definitions, and bit-identical to the oracle's
    tree-order sums carried through the scratch buffer."""
    torch = torch_cuda
    from paper_2408_05962_amd import Comm
    from paper_2408_05962_amd import collectives as CO
    h, s, m = [2, 4, 2], 4, 2
    p, root = 16, 15
    d = 4096 + 3
    base = "all_reduce" if name == "all_reduce_bcast" else name
    sends = _host_inputs(base, p, d, "float32", zlib.crc32(f"two-f32{name}".encode()) % 1000)
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.full((p, H.recv_len(base, p, d)), -7, dtype=torch.float32, device="cuda")
    X = torch.zeros((p, d * p), dtype=torch.float32, device="cuda")
    c = Comm(p, "float32")
    CO.compose_multi(c, name, [S[r] for r in range(p)], [R[r] for r in range(p)], [X[r] for r in range(p)], d,
                     root=root)
    c.set_hierarchy(h)
    c.set_stripe(s)
    c.set_pipeline(m)
    c.set_exec(mode)
    c.set_spin_limit(1 << 20)
    c.init()
    exp = _two_step_f32_expected(name, sends, h, s, root)
    for _ in range(2):
        R.fill_(-7)
        c.run(torch.cuda.current_stream())
        c.wait()
        torch.cuda.synchronize()
        out = R.cpu().numpy()
        got = _got(base, out, p, root)
        H.check_result(base, got, sends, "float32", root=root)
        if exp is not None:
            for r, y in exp.items():
                assert np.array_equal(got[r].view(np.uint32), y.view(np.uint32)), \
                    f"{name} {mode} rank {r}: not the tree-order float32 sums"
    c.close()
