"""Pins of the primitive-step interpreter: every composition row equals the direct definition."""
import numpy as np
import pytest

from oracle import collectives as C
from oracle import steps as S

SINGLE = ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "scatter", "gather",
          "all_to_all"]
MULTI = ["broadcast", "reduce", "all_gather", "reduce_scatter", "all_reduce", "all_reduce_bcast"]


def _sends(name, p, d, seed, dtype=np.int32):
    rng = np.random.default_rng(seed)
    n = d if name == "all_gather" or name == "gather" else d * p
    if dtype == np.int32:
        return [rng.integers(-1000, 1001, n).astype(np.int32) for _ in range(p)]
    return [rng.standard_normal(n).astype(np.float32) for _ in range(p)]


def _expected(name, sends, p, root):
    if name == "broadcast":
        return {r: y for r, y in enumerate(C.broadcast(sends, root))}
    if name == "reduce":
        return {root: C.reduce(sends, root)}
    if name == "all_gather":
        return dict(enumerate(C.all_gather(sends)))
    if name == "reduce_scatter":
        return dict(enumerate(C.reduce_scatter(sends)))
    if name in ("all_reduce", "all_reduce_bcast"):
        return dict(enumerate(C.all_reduce(sends)))
    if name == "scatter":
        return dict(enumerate(C.scatter(sends[root], p)))
    if name == "gather":
        return {root: C.gather(sends)}
    if name == "all_to_all":
        return dict(enumerate(C.all_to_all(sends)))
    raise ValueError(name)


@pytest.mark.parametrize("form,names", [("single", SINGLE), ("multi", MULTI)])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("d", [1, 3])
def test_composition_rows_equal_definitions(form, names, p, d):
    for k, name in enumerate(names):
        root = (p - 1) if p > 1 else 0
        sends = _sends(name, p, d, seed=1000 * p + 10 * d + k)
        steps = S.compose(name, p, d, root=root, form=form)
        mem = S.run(S.Memory(S.buffers_for(name, p, d, sends, form)), steps)
        exp = _expected(name, sends, p, root)
        for r, y in exp.items():
            got = mem.result(f"y{r}", np.int32)
            assert np.array_equal(got, y), (form, name, p, d, r)


def test_listing_allreduce_three_ranks_float():
    """Reduce-scatter, fence, in-place All-gather to `others` on three ranks (Fig. 4)."""
    p, d = 3, 4
    sends = _sends("all_reduce", p, d, 7, np.float32)
    steps = S.compose("all_reduce", p, d, form="multi")
    assert [len(st) for st in steps] == [3, 3]
    assert all(pr.kind == "R" for pr in steps[0]) and all(pr.kind == "M" for pr in steps[1])
    mem = S.run(S.Memory(S.buffers_for("all_reduce", p, d, sends, "multi")), steps)
    exp = C.all_reduce(sends)[0]
    for r in range(p):
        assert np.array_equal(mem.result(f"y{r}", np.float32), exp)


def test_step_reads_snapshot():
    """Two primitives of one step: the second must not see the first one's write."""
    bufs = {"a": np.array([1, 2], np.int32), "b": np.array([0, 0], np.int32), "c": np.array([0, 0], np.int32)}
    m1 = S.multicast(0, [1], 2, {0: ("a", 0)}, {1: ("b", 0)})
    m2 = S.multicast(1, [2], 2, {1: ("b", 0)}, {2: ("c", 0)})
    # in one step m2 reads b before m1's write lands (and this is a race the checker reports)
    assert S.find_races([m1, m2]) == [(0, 1)]
    mem = S.run(S.Memory(bufs), [[m1, m2]])
    assert list(mem.result("c", np.int32)) == [0, 0]
    # with a fence between them, the dependency is honoured
    mem = S.run(S.Memory(bufs), [[m1], [m2]])
    assert list(mem.result("c", np.int32)) == [1, 2]


def test_race_finder_read_read_is_not_a_race():
    bufs = {"a": 4}
    del bufs
    m1 = S.multicast(0, [1], 4, {0: ("a", 0)}, {1: ("b", 0)})
    m2 = S.multicast(0, [2], 4, {0: ("a", 0)}, {2: ("c", 0)})
    assert S.find_races([m1, m2]) == []
    m3 = S.multicast(0, [2], 4, {0: ("a", 2)}, {2: ("b", 2)})   # overlaps m1's write
    assert S.find_races([m1, m3]) == [(0, 1)]


def test_single_leaf_reduction_is_copy():
    bufs = {"a": np.array([5, 6, 7], np.int32), "b": np.zeros(3, np.int32)}
    r = S.reduction([0], 1, 3, {0: ("a", 0)}, {1: ("b", 0)}, "sum")
    mem = S.run(S.Memory(bufs), [[r]])
    assert list(mem.result("b", np.int32)) == [5, 6, 7]


def test_max_min_reductions_hand_values():
    """max and min reductions of the interpreter on hand-checked values, with negatives (int32 and
    float32), a fenced second step that reads the first step's results, and a one-leaf max (a copy)."""
    s = {"s0": np.array([3, -7, 0, 1000], np.int32), "s1": np.array([-1, 5, 2, -1000], np.int32),
         "s2": np.array([2, 2, -9, 999], np.int32)}
    bufs = dict(s, ya=np.zeros(4, np.int32), yb=np.zeros(4, np.int32), yc=np.zeros(4, np.int32),
                yd=np.zeros(4, np.int32))
    send = {0: ("s0", 0), 1: ("s1", 0), 2: ("s2", 0)}
    r_max = S.reduction([0, 1, 2], 0, 4, send, {0: ("ya", 0)}, "max")
    r_min = S.reduction([2, 1, 0], 1, 4, send, {1: ("yb", 0)}, "min")
    # second step: max over the two results of the first step (rank 0 holds ya, rank 1 holds yb)
    r_mix = S.reduction([0, 1], 2, 4, {0: ("ya", 0), 1: ("yb", 0)}, {2: ("yc", 0)}, "max")
    r_one = S.reduction([1], 0, 4, {1: ("s1", 0)}, {0: ("yd", 0)}, "min")
    mem = S.run(S.Memory(bufs), [[r_max, r_min, r_one], [r_mix]])
    assert list(mem.result("ya", np.int32)) == [3, 5, 2, 1000]
    assert list(mem.result("yb", np.int32)) == [-1, -7, -9, -1000]
    assert list(mem.result("yc", np.int32)) == [3, 5, 2, 1000]
    assert list(mem.result("yd", np.int32)) == [-1, 5, 2, -1000]
    f = {"a": np.array([-0.5, 2.25, -3.0], np.float32), "b": np.array([-0.25, -2.5, 1.5], np.float32),
         "m": np.zeros(3, np.float32), "n": np.zeros(3, np.float32)}
    fs = {0: ("a", 0), 1: ("b", 0)}
    mem = S.run(S.Memory(f), [[S.reduction([0, 1], 0, 3, fs, {0: ("m", 0)}, "max"),
                               S.reduction([0, 1], 1, 3, fs, {1: ("n", 0)}, "min")]])
    assert list(mem.result("m", np.float32)) == [-0.25, 2.25, 1.5]
    assert list(mem.result("n", np.float32)) == [-0.5, -2.5, -3.0]


@pytest.mark.parametrize("name", ["reduce", "reduce_scatter", "all_reduce"])
@pytest.mark.parametrize("op", ["max", "min"])
@pytest.mark.parametrize("form", ["single", "multi"])
def test_max_min_compositions_brute_force(name, op, form):
    """Composition rows with max / min against a brute-force loop over every element and rank."""
    p, d = 3, 2
    rng = np.random.default_rng(11)
    sends = [rng.integers(-50, 51, d * p).astype(np.int32) for _ in range(p)]
    steps = S.compose(name, p, d, op=op, form=form)
    mem = S.run(S.Memory(S.buffers_for(name, p, d, sends, form)), steps)
    pick = max if op == "max" else min
    full = [pick(int(sends[r][e]) for r in range(p)) for e in range(d * p)]
    if name == "reduce":
        assert list(mem.result("y0", np.int32)) == full
    elif name == "reduce_scatter":
        for r in range(p):
            assert list(mem.result(f"y{r}", np.int32)) == full[r * d:(r + 1) * d]
    else:
        for r in range(p):
            assert list(mem.result(f"y{r}", np.int32)) == full
