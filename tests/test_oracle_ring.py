"""Pins of the ring + tree reading (Sec. 4.4, Fig. 6(b), Eq. (1))."""
import numpy as np
import pytest

from oracle import collectives as OC
from oracle import tree as T


def test_ring_four_nodes_three_gpus_five_stages():
    """ring(4), stripe(3) on 4 nodes x 3 GPUs: scatter, three ring hops, intra-node assembly: stages 0..4."""
    hops, nst = T.ring_multicast_hops(0, range(12), [4, 3], 4, s=3)
    assert nst == 5
    ring = sorted((hp.src, hp.dst) for hp in hops if hp.depth == 1)
    # three rails g_t -> g_{t+3} -> g_{t+6} -> g_{t+9}
    want = sorted([(t + 3 * c, t + 3 * (c + 1)) for t in range(3) for c in range(3)])
    assert ring == want
    # every GPU but the root receives every stripe exactly once
    got = {}
    for hp in hops:
        got.setdefault(hp.stripe, []).append(hp.dst)
    for t in range(3):
        assert sorted(got[t]) == sorted(set(range(1, 12)))


def test_ring_one_is_the_tree():
    hops, nst = T.ring_multicast_hops(0, range(12), [2, 2, 3], 1)
    tree = T.multicast_hops(0, range(12), [2, 2, 3])
    assert sorted((h.src, h.dst) for h in hops) == sorted((h.src, h.dst) for h in tree)
    assert nst == 1 + max(h.stage for h in tree)


@pytest.mark.parametrize("n,m", [(4, 1), (4, 5), (4, 32), (8, 3)])
def test_pipelined_ring_steps_eq1(n, m):
    """Eq. (1): a pipelined ring over n nodes with m channels takes n + m - 2 link steps."""
    hops, _ = T.ring_multicast_hops(0, range(n * 2), [n, 2], n)
    ring = [hp for hp in hops if hp.depth == 1]
    assert len(ring) == n - 1                 # one chain of n - 1 hops per channel
    # list schedule: channel c may cross link l once it crossed link l-1 and link l carried channel c-1
    done = {}
    for c in range(m):
        for l in range(len(ring)):
            done[(c, l)] = max(done.get((c, l - 1), 0), done.get((c - 1, l), 0)) + 1
    assert max(done.values()) == n + m - 2


def test_ring_top_level_volume_is_minimal():
    for h, n in (([4, 3], 4), ([4, 4, 2], 4), ([2, 4, 2], 2)):
        p = int(np.prod(h))
        hops, _ = T.ring_multicast_hops(0, range(p), h, n)
        assert sum(1 for hp in hops if hp.depth == 1) == h[0] - 1


@pytest.mark.parametrize("h,n", [([4, 3], 4), ([4, 4, 2], 4), ([2, 4, 2], 2), ([2, 2], 2)])
def test_ring_reduce_is_the_sum(h, n):
    p = int(np.prod(h))
    rng = np.random.default_rng(p)
    vals = {r: rng.integers(-1000, 1001, 33).astype(np.int64) for r in range(p)}
    for root in (0, p - 1):
        got = T.ring_reduce(vals, range(p), root, h, n, lambda ops: sum(ops[1:], ops[0]))
        assert np.array_equal(got, OC.combine([vals[r] for r in range(p)], "sum"))
    # operand order: the farthest node's partial arrives last at each hop
    seen = []
    T.ring_reduce({r: r for r in range(p)}, range(p), 0, h, n, lambda ops: seen.append(list(ops)) or ops[0])
    assert seen[-1][-1] != 0 or n == 1


def test_ring_requires_a_group_boundary():
    with pytest.raises(ValueError):
        T.ring_depth([2, 3], 3)
    assert T.ring_depth([4, 3], 4) == 1
