"""Pins of the oracle's order-exact reduction evaluators (the source of the bit-exact float32 and
payload expectations) and of its integer helpers.

* with an exact node operation (int64 sums) a factorized tree, striped or not, equals the plain sum
  over the leaves: every leaf contributes exactly once, whatever the hierarchy, root or leaf set;
* a recording node operation shows the nesting and the ascending child-group operand order of the
  reduction tree (Sec. 4.2, mirrored), including pruned groups that form no node;
* the int32 wrap equals numpy's own int32 overflow arithmetic.
"""
import numpy as np
import pytest

from oracle import collectives as OC
from oracle import tree as OT

HIERS = [[2, 2], [2, 2, 3], [2, 4, 2], [4, 4], [3, 2], [8]]


def _rec(ops):
    return ("n",) + tuple(ops)


@pytest.mark.parametrize("h", HIERS)
def test_tree_reduce_of_exact_integers_is_the_sum(h):
    p = int(np.prod(h))
    rng = np.random.default_rng(p)
    for root in sorted({0, p - 1, p // 2}):
        for leaves in (list(range(p)), sorted(int(x) for x in rng.choice(p, max(1, p // 2), replace=False)),
                       [p - 1]):
            vals = {r: rng.integers(-10 ** 6, 10 ** 6, 7).astype(np.int64) for r in range(p)}
            got = OT.tree_reduce(vals, leaves, root, h, lambda ops: np.sum(ops, axis=0))
            assert np.array_equal(got, np.sum([vals[r] for r in leaves], axis=0)), (h, root, leaves)


@pytest.mark.parametrize("h", HIERS)
@pytest.mark.parametrize("s", [1, 2, 4])
def test_striped_reduce_of_exact_integers_is_the_sum(h, s):
    p = int(np.prod(h))
    n = 4 * 37 + 3                                   # ragged: not a multiple of the stripe alignment
    rng = np.random.default_rng(s * 100 + p)
    vals = {r: rng.integers(-10 ** 6, 10 ** 6, n).astype(np.int64) for r in range(p)}
    want = np.sum([vals[r] for r in range(p)], axis=0)
    for root in (0, p - 1):
        if not any(B % s == 0 and B >= s for B in OT.block_sizes(h)):
            continue
        try:
            got = OT.striped_reduce(vals, range(p), root, n, h, s, 4, lambda ops: np.sum(ops, axis=0))
        except ValueError:
            continue                                  # s divides no group enclosing the root
        assert len(got) == n and np.array_equal(got, want)


def test_tree_reduce_nesting_2x2():
    got = OT.tree_reduce({r: r for r in range(4)}, range(4), 0, [2, 2], _rec)
    assert got == ("n", ("n", 0, 1), ("n", 2, 3))
    # the root's position changes the hosts, never the operand order (ascending child groups)
    assert OT.tree_reduce({r: r for r in range(4)}, range(4), 3, [2, 2], _rec) == got


def test_tree_reduce_nesting_2x2x3_full_and_pruned():
    vals = {r: r for r in range(12)}
    full = OT.tree_reduce(vals, range(12), 0, [2, 2, 3], _rec)
    assert full == ("n", ("n", ("n", 0, 1, 2), ("n", 3, 4, 5)), ("n", ("n", 6, 7, 8), ("n", 9, 10, 11)))
    # leaves {1, 5, 6}, root 0 (not a leaf): subgroups with one contributor form no node
    assert OT.tree_reduce(vals, [1, 5, 6], 0, [2, 2, 3], _rec) == ("n", ("n", 1, 5), 6)
    # a single leaf is its own result
    assert OT.tree_reduce(vals, [7], 0, [2, 2, 3], _rec) == 7


def test_wrap_int32_matches_numpy_int32_overflow():
    rng = np.random.default_rng(3)
    a = rng.integers(-2 ** 31, 2 ** 31, 10000, dtype=np.int64).astype(np.int32)
    b = rng.integers(-2 ** 31, 2 ** 31, 10000, dtype=np.int64).astype(np.int32)
    with np.errstate(over="ignore"):
        want = a + b                                  # numpy int32 arithmetic wraps modulo 2^32
    assert np.array_equal(OC.wrap_int32(a.astype(np.int64) + b.astype(np.int64)), want)
    edge = np.array([2 ** 31, -2 ** 31 - 1, 2 ** 32, -1, 0], dtype=np.int64)
    assert OC.wrap_int32(edge).tolist() == [-2 ** 31, 2 ** 31 - 1, 0, -1, 0]
    assert OC.finish(np.array([2 ** 31], np.int64), np.int32).tolist() == [-2 ** 31]
    assert OC.finish(np.array([0.5]), np.float32).tolist() == [0.5]


def test_abs_sum_is_the_condition_scale():
    x = np.array([1.5, -2.0, 0.0])
    y = np.array([-1.0, 4.0, -3.0])
    assert OC.abs_sum([x, -x, y]).tolist() == [4.0, 8.0, 3.0]
