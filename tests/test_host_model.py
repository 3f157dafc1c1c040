"""The planner's pipelined schedules against the communication model of Sec. 4.6 (host only).

Each sending rank has one link that carries one chunk (one channel of one hop) at a time, and a hop
can start once its sender holds that channel. A list schedule over the planner's own task table (its
claim order) then gives the model's step counts: n + m - 2 chunk steps for a pipelined ring over n
nodes (Eq. ring) and m * log2(n) for the tree over {2, ..., 2} (Eq. tree with no latency term), so a
ring on four nodes approaches half the tree's time as the pipeline deepens.
"""
import math

import pytest

from paper_2408_05962_amd import collectives as CO


def _plan(p, h, m, ring=1):
    send = [0x10000000000 + r * (1 << 32) for r in range(p)]
    recv = [0x20000000000 + r * (1 << 32) for r in range(p)]
    c = CO.make("broadcast", p, "float32", send, recv, 4096, hierarchy=h, pipeline=m, ring=ring, init=False,
                order="critical")
    c.init()
    tasks = c.plan_tasks()
    c.close()
    return tasks


def _makespan(tasks, root=0):
    """Link-serialized list schedule in table order; returns the finish time in chunk steps."""
    have = {}                              # (rank, channel) -> time the rank holds that channel
    free = {}                              # rank -> time its link is free
    end = 0
    hops = [t for t in tasks if t["kind"] == 0 and t["src_rank"][0] != t["dst_rank"]]
    for t in sorted(hops, key=lambda t: t["stage"]):     # stable: table order within a stage
        src, dst, ch = t["src_rank"][0], t["dst_rank"], t["channel"]
        ready = 0 if src == root else have[(src, ch)]
        start = max(ready, free.get(src, 0))
        free[src] = start + 1
        have[(dst, ch)] = start + 1
        end = max(end, start + 1)
    return end


@pytest.mark.parametrize("n", [2, 3, 4, 8])
@pytest.mark.parametrize("m", [1, 2, 5, 16])
def test_ring_takes_n_plus_m_minus_2_steps(n, m):
    assert _makespan(_plan(n, [n], m, ring=n)) == n + m - 2


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("m", [1, 2, 5, 16])
def test_tree_takes_m_log_n_steps(levels, m):
    n = 2 ** levels
    assert _makespan(_plan(n, [2] * levels, m)) == m * int(math.log2(n))


def test_ring_is_twice_as_fast_as_tree_on_four_nodes():
    ratios = [_makespan(_plan(4, [2, 2], m)) / _makespan(_plan(4, [4], m, ring=4)) for m in (1, 8, 64, 256)]
    assert ratios == sorted(ratios) and abs(ratios[-1] - 2.0) < 0.02


def test_stage_order_keeps_hops_of_one_source_together():
    """The default stage order lists a sender's hops of one stage together (cache reuse of the source on
    one GPU); the critical-path order interleaves them by the length of their downstream chains."""
    send = [0x10000000000 + r * (1 << 32) for r in range(8)]
    recv = [0x20000000000 + r * (1 << 32) for r in range(8)]
    srcs = {}
    for order in ("stage", "critical"):
        c = CO.make("broadcast", 8, "float32", send, recv, 4096, hierarchy=[2, 2, 2], order=order)
        srcs[order] = [(t["stage"], t["src_rank"][0], t["dst_rank"]) for t in c.plan_tasks() if t["kind"] == 0]
        c.close()
    first = [x for x in srcs["critical"] if x[0] == 0 and x[1] != x[2]]
    assert [x[2] for x in first] == [4, 2, 1]          # farthest subtree first
    assert sorted(srcs["stage"]) == sorted(srcs["critical"])

