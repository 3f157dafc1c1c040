"""Pins of the factorization oracle against the paper's worked examples and closed forms."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import tree as T

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_worked_broadcast_2x2x3():
    g = _gold("broadcast_2x2x3_tree.json")
    h = g["hierarchy"]
    hops = T.multicast_hops(g["root"], range(12), h)
    by_depth = {}
    for hp in hops:
        by_depth.setdefault(str(hp.depth), []).append([hp.src, hp.dst])
    for k, v in g["hops_by_depth"].items():
        assert sorted(by_depth[k]) == sorted(v)
    assert 1 + max(hp.stage for hp in hops) == g["stages_unstriped"]


def test_striped_broadcast_2x2x3():
    g = _gold("broadcast_2x2x3_striped.json")
    h, s, root = g["hierarchy"], g["stripes"], g["root"]
    own = T.stripe_owners(root, range(12), h, s)
    assert own == g["owners"]
    scat = [[root, o] for o in own if o != root]
    assert scat == g["scatter_hops"]
    # stages: scatter (0), then each owner's tree starts after its stripe arrived
    stages = 0
    for o in own:
        start = 1 if o != root else 0
        hops = T.multicast_hops(o, set(range(12)) - {o, root}, h, stage0=start)
        stages = max(stages, 1 + max(hp.stage for hp in hops))
    assert stages == g["stages_striped"] == g["min_channels_full_overlap"]


def test_direct_vs_hierarchical_cross_node_copies():
    g = _gold("broadcast_direct_vs_hierarchical_2x3.json")
    acct = g["accounting_hierarchy"]
    d = 1
    for key, hier in (("cross_node_copies_direct", g["direct_hierarchy"]),
                      ("cross_node_copies_hierarchical", g["hierarchical_hierarchy"])):
        tr = T.prim_transfers("M", g["root"], range(6), d, hier)
        lb = T.level_bytes(tr, acct, 1)
        assert lb[1] == g[key]


@pytest.mark.parametrize("h", [[2, 4, 2], [2, 2, 3], [4, 4], [2, 3, 2, 2], [3, 5], [6]])
def test_full_leaf_multicast_hop_counts_closed_form(h):
    p = int(np.prod(h))
    for root in {0, p - 1, p // 3}:
        hops = T.multicast_hops(root, range(p), h)
        assert len(hops) == p - 1
        assert sorted(hp.dst for hp in hops) == sorted(set(range(p)) - {root})
        for k in range(1, len(h) + 1):
            want = int(np.prod(h[:k])) - int(np.prod(h[:k - 1]))
            assert sum(1 for hp in hops if hp.depth == k) == want


@pytest.mark.parametrize("h", [[2, 4, 2], [2, 2], [2, 4], [4, 4], [2, 2, 3]])
def test_full_leaf_reduction_node_counts(h):
    """Per level k: prod(f_1..f_{k-1}) nodes each combining f_k operands."""
    p = int(np.prod(h))
    tree = T.reduction_tree(range(p), 0, h)
    nodes = T.reduction_nodes(tree)
    for k in range(1, len(h) + 1):
        at = [nd for nd in nodes if nd.depth == k]
        assert len(at) == int(np.prod(h[:k - 1]))
        assert all(len(nd.children) == h[k - 1] for nd in at)
    reads = sum(len(nd.children) for nd in nodes)
    writes = len(nodes)
    assert reads == sum(int(np.prod(h[:k])) for k in range(1, len(h) + 1))
    assert writes == sum(int(np.prod(h[:k - 1])) for k in range(1, len(h) + 1))
    assert T.tree_depth_stages(tree) == len(h)


def test_reduction_2x4x2_traffic_coefficients():
    # reads 26 n, writes 11 n for a full-leaf reduction on {2,4,2}
    nodes = T.reduction_nodes(T.reduction_tree(range(16), 5, [2, 4, 2]))
    assert sum(len(nd.children) for nd in nodes) == 26
    assert len(nodes) == 11
    assert nodes[-1].host == 5


COLL = ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_to_all", "scatter", "gather"]


@pytest.mark.parametrize("h", [[2, 2], [2, 4, 2], [4, 4], [2, 4], [2, 2, 3], [3, 2]])
@pytest.mark.parametrize("name", COLL)
def test_top_level_bytes_equal_minimum(h, name):
    """The factorized schedule moves exactly the least volume across the top level (s = 1)."""
    p = int(np.prod(h))
    g = p // h[0]
    d = 4
    lb = T.collective_level_bytes(name, h, d)
    assert lb[1] == T.min_top_bytes(name, p, g, d)


@pytest.mark.parametrize("h", [[2, 4, 2], [2, 2, 3]])
@pytest.mark.parametrize("name", COLL)
def test_every_depth_meets_its_minimum(h, name):
    """Bytes crossing depth-k boundaries equal the same minimum with B_k as the group size."""
    p = int(np.prod(h))
    d = 4
    lb = T.collective_level_bytes(name, h, d)
    B = T.block_sizes(h)
    for k in range(1, len(h) + 1):
        crossing = sum(lb[1:k + 1])
        assert crossing == T.min_top_bytes(name, p, B[k], d), (k, lb)


def test_minimum_is_a_true_lower_bound_brute_force():
    """For a broadcast on 2x2, no set of copies that reaches every rank crosses the top level less."""
    h = [2, 2]
    ranks = range(4)
    best = None
    # every spanning arborescence rooted at 0 over 4 ranks: parent choice per non-root rank
    for parents in itertools.product(ranks, repeat=3):
        par = dict(zip([1, 2, 3], parents))
        ok = True
        for v in (1, 2, 3):
            seen, x = set(), v
            while x != 0:
                if x in seen or par[x] == x:
                    ok = False
                    break
                seen.add(x)
                x = par[x]
            if not ok:
                break
        if not ok:
            continue
        top = sum(1 for v, u in par.items() if T.depth(u, v, h) == 1)
        best = top if best is None else min(best, top)
    assert best == T.min_top_bytes("broadcast", 4, 2, 1) // 4


@pytest.mark.parametrize("h,s", [([2, 4, 2], 4), ([2, 2, 3], 3), ([4, 4], 2), ([2, 4], 4)])
def test_striping_keeps_top_level_volume(h, s):
    """Striping reroutes inside the stripe group; the top level still carries the minimum."""
    p = int(np.prod(h))
    g = p // h[0]
    d = 8 * s
    for name in ("broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_to_all"):
        lb = T.collective_level_bytes(name, h, d, s=s)
        assert lb[1] == T.min_top_bytes(name, p, g, d), name


def test_stripe_owners_reading():
    # {2,4,2}, s = 4: one owner per device of the root's node, starting at the root
    assert T.stripe_owners(0, range(16), [2, 4, 2], 4) == [0, 2, 4, 6]
    assert T.stripe_owners(3, range(16), [2, 4, 2], 4) == [3, 5, 7, 1]
    # all leaves inside the stripe group: not striped
    assert T.stripe_owners(0, [1, 2, 3], [2, 4, 2], 4) is None
    assert T.stripe_owners(0, range(16), [2, 4, 2], 1) is None


def test_split_pieces():
    assert T.split(10, 3, 1) == [(0, 4), (4, 3), (7, 3)]
    assert T.split(18, 2, 4) == [(0, 8), (8, 10)]
    assert T.split(3, 4, 4) == [(0, 0), (0, 0), (0, 0), (0, 3)]
    for n, parts, al in [(1000, 7, 4), (4096, 8, 256), (5, 2, 1)]:
        pcs = T.split(n, parts, al)
        assert sum(ln for _, ln in pcs) == n
        assert all(off % al == 0 for off, _ in pcs)


def test_sparse_reduction_and_single_leaf():
    h = [2, 4, 2]
    # one leaf: a plain point-to-point value, no node
    assert T.reduction_tree([13], 0, h) == 13
    # two leaves in different nodes meet at the root's node
    tr = T.reduction_tree([3, 12], 0, h)
    assert isinstance(tr, T.Node) and tr.host == 0 and tr.children == [3, 12]
    # pruning: no hop enters a group without leaves
    hops = T.multicast_hops(0, [5, 14], h)
    # staging falls back to the lowest leaf when the same-offset rank is not a leaf
    assert {(hp.src, hp.dst, hp.depth) for hp in hops} == {(0, 14, 1), (0, 5, 2)}
    touched = {hp.dst for hp in hops}
    for grp in range(8):          # device groups of two
        members = {2 * grp, 2 * grp + 1}
        if not members & {5, 14}:
            assert not (touched & members)


def test_sum_f32_is_left_to_right():
    a = np.array([1e8], np.float32)
    b = np.array([1.0], np.float32)
    c = np.array([-1e8], np.float32)
    assert T.sum_f32([a, b, c])[0] == np.float32(0.0)      # (1e8 + 1) rounds back to 1e8
    assert T.sum_f32([a, c, b])[0] == np.float32(1.0)


@pytest.mark.parametrize("h", [[2, 2, 3], [2, 4, 2], [4, 4], [3, 2, 2]])
def test_reduction_is_the_mirror_of_the_multicast(h):
    """A full-leaf reduction moves data along exactly the reversed hops of the multicast from the same
    root (Sec. 4.2 describes one tree; the worked {2,2,3} broadcast of Sec. 4.3 fixes its hops)."""
    p = int(np.prod(h))
    for root in (0, p - 1, p // 2 + 1):
        mc = {(hp.dst, hp.src) for hp in T.multicast_hops(root, range(p), h)}
        red = set()
        for nd in T.reduction_nodes(T.reduction_tree(range(p), root, h)):
            for ch in nd.children:
                if T.host(ch) != nd.host:
                    red.add((T.host(ch), nd.host))
        assert red == mc, (h, root)
