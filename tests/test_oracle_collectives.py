"""Pins of the direct-definition oracle: hand-computed values, brute force, invariants."""
import numpy as np
import pytest

from oracle import collectives as C


def test_hand_values_p2():
    s = [np.array([1, 2], np.int32), np.array([3, 4], np.int32)]
    assert [list(y) for y in C.all_reduce(s)] == [[4, 6], [4, 6]]
    assert [list(y) for y in C.reduce_scatter(s)] == [[4], [6]]
    assert [list(y) for y in C.all_to_all(s)] == [[1, 3], [2, 4]]
    assert [list(y) for y in C.broadcast(s, 1)] == [[3, 4], [3, 4]]
    assert list(C.reduce(s, 0, "max")) == [3, 4]
    assert list(C.reduce(s, 0, "min")) == [1, 2]
    assert [list(y) for y in C.scatter(np.array([7, 8], np.int32), 2)] == [[7], [8]]
    assert list(C.gather([np.array([5], np.int32), np.array([6], np.int32)])) == [5, 6]
    assert [list(y) for y in C.all_gather([np.array([5], np.int32), np.array([6], np.int32)])] == [[5, 6], [5, 6]]


def test_hand_values_p3_all_to_all():
    # rank i holds [10i+0, 10i+1, 10i+2]; chunk i of rank j's output = chunk j of rank i's input
    s = [np.array([10 * i + q for q in range(3)], np.int32) for i in range(3)]
    y = C.all_to_all(s)
    assert [list(v) for v in y] == [[0, 10, 20], [1, 11, 21], [2, 12, 22]]


def test_int32_sum_wraps_twos_complement():
    big = np.iinfo(np.int32).max
    s = [np.array([big, -big - 1], np.int32), np.array([1, -1], np.int32)]
    y = C.all_reduce(s)[0]
    assert y.dtype == np.int32
    assert list(y) == [-(2 ** 31), 2 ** 31 - 1]


def test_float_sum_is_float64_exact_for_small_ints():
    rng = np.random.default_rng(1)
    s = [rng.integers(-50, 50, 64).astype(np.float32) for _ in range(5)]
    y = C.all_reduce(s)[0]
    assert y.dtype == np.float64
    assert np.array_equal(y, np.sum(np.stack(s).astype(np.float64), axis=0))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("d", [0, 1, 3, 7, 16])
def test_brute_force_elementwise(p, d):
    """Element by element, straight from the definitions, with Python integers."""
    rng = np.random.default_rng(100 * p + d)
    s = [rng.integers(-1000, 1001, d * p).astype(np.int32) for _ in range(p)]
    ar = C.all_reduce(s)
    rs = C.reduce_scatter(s)
    a2a = C.all_to_all(s)
    for r in range(p):
        for e in range(d * p):
            assert ar[r][e] == sum(int(s[q][e]) for q in range(p))
        for e in range(d):
            assert rs[r][e] == sum(int(s[q][r * d + e]) for q in range(p))
        for i in range(p):
            for e in range(d):
                assert a2a[r][i * d + e] == s[i][r * d + e]
    ag_in = [x[:d] for x in s]
    ag = C.all_gather(ag_in)
    for r in range(p):
        for q in range(p):
            assert np.array_equal(ag[r][q * d:(q + 1) * d], ag_in[q])


@pytest.mark.parametrize("p", [2, 3, 4, 8, 16])
def test_invariants(p):
    rng = np.random.default_rng(p)
    d = 5
    s = [rng.integers(-1000, 1001, d * p).astype(np.int32) for _ in range(p)]
    ar = C.all_reduce(s)
    # All-Gather after Reduce-Scatter is All-Reduce (exact for integers)
    ag_rs = C.all_gather(C.reduce_scatter(s))
    for r in range(p):
        assert np.array_equal(ag_rs[r], ar[r])
        assert np.array_equal(ar[r], ar[0])
    # All-to-All twice is the identity
    back = C.all_to_all(C.all_to_all(s))
    for r in range(p):
        assert np.array_equal(back[r], s[r])
    # Gather of a Scatter returns the root's buffer
    assert np.array_equal(C.gather(C.scatter(s[0], p)), s[0])
    # max / min are the elementwise extremes
    st = np.stack(s)
    assert np.array_equal(C.reduce(s, 0, "max"), st.max(axis=0))
    assert np.array_equal(C.reduce(s, 0, "min"), st.min(axis=0))


def test_reduce_matches_library_sum_for_floats():
    rng = np.random.default_rng(3)
    s = [rng.standard_normal(1000).astype(np.float32) for _ in range(16)]
    y = C.reduce(s, 0)
    ref = np.stack(s).astype(np.float64).sum(axis=0)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_inputs_untouched():
    s = [np.arange(6, dtype=np.int32) for _ in range(3)]
    keep = [x.copy() for x in s]
    C.all_reduce(s)
    C.all_to_all(s)
    C.reduce_scatter(s)
    for a, b in zip(s, keep):
        assert np.array_equal(a, b)


def test_scaled_error_metric():
    exact = np.array([1.0, -2.0, 0.0])
    scale = np.array([1.0, 2.0, 4.0])
    got = np.array([1.0 + 1e-6, -2.0, 4e-6])
    assert C.scaled_error(got, exact, scale) == pytest.approx(1e-6)
    rep = C.error_report(got, exact, scale)
    assert rep["max_abs"] == pytest.approx(4e-6)


def test_error_report_hand_values():
    """Every field of the error report against values worked out by hand.

    exact = (1, -2, 0, 1e-4), scale = (1, 2, 4, 1), errors (1e-6, -4e-6, 4e-6, 1e-6):
      * well conditioned where |exact| >= 1e-3 * scale: elements 0 and 1 only, so the plain relative
        error is max(1e-6 / 1, 4e-6 / 2) = 2e-6 (element 3 would give 1e-2, element 2 a division by 0);
      * normwise = ||err||_2 / ||exact||_2 = sqrt(34e-12) / sqrt(5 + 1e-8);
      * scaled = max |err| / max(|exact|, scale) = max(1e-6, 2e-6, 1e-6, 1e-6) = 2e-6.
    An infinity-norm or 1-norm in place of the 2-norm gives 2e-6 or 3.3e-6, not 2.61e-6."""
    exact = np.array([1.0, -2.0, 0.0, 1e-4])
    scale = np.array([1.0, 2.0, 4.0, 1.0])
    err = np.array([1e-6, -4e-6, 4e-6, 1e-6])
    rep = C.error_report(exact + err, exact, scale)
    assert rep["max_abs"] == pytest.approx(4e-6, rel=1e-9)
    assert rep["scaled"] == pytest.approx(2e-6, rel=1e-9)
    assert rep["rel_well_conditioned"] == pytest.approx(2e-6, rel=1e-9)
    assert rep["normwise"] == pytest.approx(np.sqrt(34e-12 / (5 + 1e-8)), rel=1e-9)
    assert rep["normwise"] == pytest.approx(2.6076809e-6, rel=1e-6)


def test_error_report_special_cases():
    # an exact result of all zeros: the normwise error falls back to the absolute 2-norm (3-4-5)
    rep = C.error_report(np.array([3e-6, -4e-6]), np.zeros(2), np.ones(2))
    assert rep["normwise"] == pytest.approx(5e-6, rel=1e-9)
    assert rep["rel_well_conditioned"] == 0.0           # nothing is well conditioned
    assert rep["scaled"] == pytest.approx(4e-6, rel=1e-9)
    # the whole array is one vector: a (2, 2) block reports what its flattening reports, whatever axis
    ex = np.array([[1.0, 2.0], [3.0, 4.0]])
    got = ex + np.array([[1e-3, 0.0], [0.0, -2e-3]])
    sc = np.abs(ex)
    r2 = C.error_report(got, ex, sc)
    r1 = C.error_report(got.ravel(), ex.ravel(), sc.ravel())
    assert r2 == r1
    assert r2["normwise"] == pytest.approx(np.sqrt(5e-6 / 30.0), rel=1e-9)
    assert r2["rel_well_conditioned"] == pytest.approx(1e-3, rel=1e-9)
    # exact agreement reports zero everywhere
    assert all(v == 0.0 for v in C.error_report(ex, ex, sc).values())
    # empty input
    assert all(v == 0.0 for v in C.error_report(np.zeros(0), np.zeros(0), np.zeros(0)).values())
