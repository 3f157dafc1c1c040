"""Plant plausible mistakes in the oracle (on the CPU) and check that its pins catch each one.

Every mutation is a monkeypatched copy of an oracle function with one typical error: a dropped
operand, a transposed index, a wrong staging rank, a wrong host, truncation instead of rounding,
an off-by-one exponent, a missing factor. The pin tests, run against the mutated oracle, must fail.
"""
import numpy as np
import pytest

from oracle import collectives as OC
from oracle import quant as OQ
from oracle import tree as OT
from tests import test_oracle_collectives as PC
from tests import test_oracle_quant as PQ
from tests import test_oracle_tree as PT


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_operand_is_caught(monkeypatch):
    real = OC.combine
    monkeypatch.setattr(OC, "combine", lambda arrays, op: real(arrays[:-1] if len(arrays) > 1 else arrays, op))
    _fails(PC.test_brute_force_elementwise, 3, 3)


def test_transposed_all_to_all_is_caught(monkeypatch):
    def wrong(sends):
        p, d = len(sends), len(sends[0]) // len(sends)
        return [np.concatenate([sends[j][i * d:(i + 1) * d] for i in range(p)]) for j in range(p)]
    monkeypatch.setattr(OC, "all_to_all", wrong)
    _fails(PC.test_hand_values_p3_all_to_all)


def test_wrong_staging_rank_is_caught(monkeypatch):
    real = OT.multicast_hops

    def highest_leaf(root, leaves, h, stage0=0, stripe=0):
        hops = real(root, leaves, h, stage0, stripe)
        # a plausible slip: stage through the highest leaf of each group instead of the same offset
        B = OT.block_sizes(h)
        out = []
        for hp in hops:
            if hp.depth < len(h):
                lo = hp.dst // B[hp.depth] * B[hp.depth]
                hp = OT.Hop(hp.src, lo + B[hp.depth] - 1, hp.depth, hp.stage, hp.stripe)
            out.append(hp)
        return out
    monkeypatch.setattr(OT, "multicast_hops", highest_leaf)
    _fails(PT.test_worked_broadcast_2x2x3)


def test_wrong_reduction_host_is_caught(monkeypatch):
    real = OT.reduction_tree

    def lowest_host(leaves, root, h):
        t = real(leaves, root, h)

        def fix(n):
            if isinstance(n, OT.Node):
                n.host = min(x if isinstance(x, int) else x.host for x in n.children)
                for c in n.children:
                    fix(c)
        fix(t)
        return t
    monkeypatch.setattr(OT, "reduction_tree", lowest_host)
    _fails(PT.test_reduction_is_the_mirror_of_the_multicast, [2, 4, 2])


def test_truncating_encoder_is_caught(monkeypatch):
    def trunc(x):
        x = np.asarray(x, dtype=np.float64)
        a = np.abs(x)
        sign = np.where(np.signbit(x), 0x80, 0)
        out = np.zeros(a.shape, np.int64)
        sub = a < 2.0 ** -6
        out[sub] = np.floor(a[sub] / 2.0 ** -9)
        nrm = ~sub
        _, ex = np.frexp(a[nrm])
        e = ex - 1
        q = np.floor(a[nrm] / np.exp2(e - 3.0)).astype(np.int64)
        code = np.minimum(((e + 7) << 3) | (q - 8), 0x7E)
        out[nrm] = code
        return (out | sign).astype(np.uint8)
    monkeypatch.setattr(OQ, "e4m3_encode", trunc)
    _fails(PQ.test_e4m3_round_half_even_and_saturation)


def test_scale_off_by_one_is_caught(monkeypatch):
    real = OQ.block_scales
    monkeypatch.setattr(OQ, "block_scales", lambda x, block=256: real(x, block) * np.float32(2.0))
    _fails(PQ.test_block_scales_power_of_two_and_tight)


def test_missing_all_reduce_factor_is_caught(monkeypatch):
    real = OT.min_top_bytes
    monkeypatch.setattr(OT, "min_top_bytes",
                        lambda name, p, g, d: real("all_gather", p, g, d) if name == "all_reduce" else real(name, p, g, d))
    _fails(PT.test_top_level_bytes_equal_minimum, [2, 4, 2], "all_reduce")


def test_wrong_bf16_rounding_is_caught(monkeypatch):
    def trunc(x):
        return (np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32) >> 16).astype(np.uint16)
    monkeypatch.setattr(OQ, "f32_to_bf16_bits", trunc)
    _fails(PQ.test_bf16_hand_values)


def test_reversed_operand_order_is_caught(monkeypatch):
    real = OT.reduction_tree

    def reversed_children(leaves, root, h):
        t = real(leaves, root, h)

        def flip(n):
            if isinstance(n, OT.Node):
                n.children = list(reversed(n.children))
                for ch in n.children:
                    flip(ch)
        flip(t)
        return t
    monkeypatch.setattr(OT, "reduction_tree", reversed_children)
    from tests import test_oracle_reduce as PR
    _fails(PR.test_tree_reduce_nesting_2x2)


def test_dropped_leaf_in_tree_reduce_is_caught(monkeypatch):
    real = OT.tree_reduce
    monkeypatch.setattr(OT, "tree_reduce", lambda values, leaves, root, h, combine:
                        real(values, list(leaves)[:-1] or list(leaves), root, h, combine))
    from tests import test_oracle_reduce as PR
    _fails(PR.test_tree_reduce_of_exact_integers_is_the_sum, [2, 2, 3])
