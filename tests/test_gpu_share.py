"""One rank's share of a plan on the GPU (the tasks whose output lies in that rank's memory, as one GPU
would run them if every virtual rank were its own GPU). Run after the full plan on the same workspace,
a share rebuilds exactly its rank's receive buffer and writes no other rank's."""
import zlib

import numpy as np
import pytest

from tests import harness as H
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2408_05962_amd import hiccl
    hiccl.lib()
    return torch


@pytest.mark.parametrize("name", H.EIGHT)
@pytest.mark.parametrize("mode", ["staged", "persistent"])
@pytest.mark.parametrize("h,s,ring", [([2, 4, 2], 4, 1), ([4, 4], 2, 4)])
def test_share_rebuilds_its_rank_only(torch_cuda, name, mode, h, s, ring):
    torch = torch_cuda
    from paper_2408_05962_amd import collectives as CO
    p, root = int(np.prod(h)), 5
    d = 24 * s * 7 + 8
    rng = np.random.default_rng(zlib.crc32(f"share{name}{h}".encode()) % 1000)
    sends = [rng.integers(-1000, 1001, H.send_len(name, p, d)).astype(np.int32) for _ in range(p)]
    S = torch.stack([torch.from_numpy(x) for x in sends]).to("cuda")
    R = torch.full((p, H.recv_len(name, p, d)), -7, dtype=torch.int32, device="cuda")
    send, recv = [S[r] for r in range(p)], [R[r] for r in range(p)]
    kw = dict(hierarchy=h, stripe=s, pipeline=2, exec_mode=mode, root=root, tile_bytes=1024, ring=ring)
    full = CO.make(name, p, "int32", send, recv, d, **kw)
    W = torch.zeros(max(full.workspace_size(), 256), dtype=torch.uint8, device="cuda")
    full.set_workspace(W, W.numel())
    full.set_spin_limit(1 << 20)
    st = torch.cuda.current_stream()
    for r in (0, root, p - 1):
        # the full plan leaves every receive buffer and workspace region at its final value
        R.fill_(-7)
        full.run(st)
        full.wait()
        torch.cuda.synchronize()
        ref = R.cpu().numpy().copy()
        H.check_result(name, {q: ref[q] for q in ([root] if name in ("reduce", "gather") else range(p))},
                       sends, "int32", root=root)
        c = CO.make(name, p, "int32", send, recv, d, share=r, **kw)
        c.set_workspace(W, W.numel())
        c.set_spin_limit(1 << 20)
        R[r].fill_(-7)
        c.run(st)
        c.wait()
        torch.cuda.synchronize()
        assert np.array_equal(R.cpu().numpy(), ref), f"rank {r}'s share did not rebuild its buffer"
        others = [q for q in range(p) if q != r]
        R[others] = -9
        c.run(st)
        c.wait()
        torch.cuda.synchronize()
        assert (R.cpu().numpy()[others] == -9).all(), f"rank {r}'s share wrote another rank's buffer"
        c.close()
    full.close()
