"""Pins of the bf16 / e4m3 oracle quantizers against the format definitions and torch's CPU casts."""
import numpy as np
import pytest
import torch

from oracle import quant as Q


def test_bf16_hand_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.0, 0.0, 1.0 + 2 ** -7], np.float32)
    # 1 + 2^-8 is a tie and goes to the even neighbour 1.0; 1 + 3*2^-8 goes up to 1 + 2^-6
    assert [hex(v) for v in Q.f32_to_bf16_bits(x)] == ["0x3f80", "0x3f80", "0x3f82", "0xc000", "0x0", "0x3f81"]
    assert np.array_equal(Q.bf16_bits_to_f32(Q.f32_to_bf16_bits(x)).astype(np.float64),
                          [1.0, 1.0, 1.0 + 2 ** -6, -2.0, 0.0, 1.0 + 2 ** -7])


def test_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    ours = Q.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_hand_codes():
    vals = [0.0, 1.0, -2.0, 448.0, 2.0 ** -9, 2.0 ** -6, 0.875 * 2 ** -6, 240.0, 1.125, -448.0]
    want = [0x00, 0x38, 0xC0, 0x7E, 0x01, 0x08, 0x07, 0x77, 0x39, 0xFE]
    assert list(Q.e4m3_encode(np.array(vals))) == want


def test_e4m3_round_half_even_and_saturation():
    # between 1.0 (0x38) and 1.125 (0x39): 1.0625 is a tie -> even mantissa 0x38
    assert Q.e4m3_encode(np.array([1.0625]))[0] == 0x38
    # between 1.125 and 1.25: 1.1875 is a tie -> 1.25 (0x3A, even)
    assert Q.e4m3_encode(np.array([1.1875]))[0] == 0x3A
    # subnormal tie: 1.5 * 2^-9 -> 2 * 2^-9 (even), 0.5 * 2^-9 -> 0
    assert list(Q.e4m3_encode(np.array([1.5 * 2 ** -9, 0.5 * 2 ** -9]))) == [0x02, 0x00]
    # above the largest finite value: saturate, never NaN
    assert list(Q.e4m3_encode(np.array([460.0, 1e6, -1e6]))) == [0x7E, 0x7E, 0xFE]


def test_e4m3_all_codes_round_trip():
    codes = np.arange(256, dtype=np.uint8)
    finite = ~np.isin(codes, [0x7F, 0xFF])
    vals = Q.e4m3_decode(codes[finite])
    back = Q.e4m3_encode(vals)
    # +0 and -0 both decode to zero; -0 encodes back with its sign bit
    assert np.array_equal(back, codes[finite])
    assert np.isnan(Q.e4m3_decode(np.array([0x7F, 0xFF], np.uint8))).all()
    assert np.nanmax(np.abs(vals)) == 448.0


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = (rng.uniform(-448, 448, 200000) * np.exp2(rng.integers(-14, 1, 200000))).astype(np.float32)
    ours = Q.e4m3_encode(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_relative_error_bound():
    rng = np.random.default_rng(2)
    x = rng.uniform(2 ** -6, 448, 100000)
    y = Q.e4m3_decode(Q.e4m3_encode(x))
    assert np.max(np.abs(y - x) / x) <= 2 ** -4


def test_block_scales_power_of_two_and_tight():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(256 * 64) * np.repeat(np.exp2(rng.integers(-30, 30, 64)), 256)
    x[:256] = 0.0
    sc = Q.block_scales(x).astype(np.float64)
    assert sc[0] == 1.0
    m, e = np.frexp(sc)
    assert np.all(m == 0.5)                                  # powers of two
    amax = np.abs(x.reshape(-1, 256)).max(axis=1)
    nz = amax > 0
    assert np.all(amax[nz] <= 448 * sc[nz])                  # fits
    assert np.all(amax[nz] > 448 * sc[nz] / 2)               # and is the least such power
    # boundary: amax exactly 448 * 2^k gives scale 2^k
    b = np.zeros(256)
    b[7] = 448 * 2.0 ** 5
    assert Q.block_scales(b)[0] == 32.0
    b[7] = np.nextafter(448 * 2.0 ** 5, np.inf)
    assert Q.block_scales(b)[0] == 64.0


def test_fp8_quantize_dequantize_error():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(256 * 100).astype(np.float32)
    c, s = Q.fp8_quantize(x)
    y = Q.fp8_dequantize(c, s)
    amax = np.repeat(np.abs(x.reshape(-1, 256)).max(axis=1), 256)
    # normal-range values: relative 2^-4; anything: below half a subnormal step of the block
    err = np.abs(y - x)
    assert np.all(err <= np.maximum(np.abs(x) * 2 ** -4, 2.0 ** -10 * amax / 448 * 2))


def test_node_ops_in_payload_format():
    a = Q.f32_to_bf16_bits(np.array([1.0, 2.0], np.float32))
    b = Q.f32_to_bf16_bits(np.array([2 ** -8, 3.0], np.float32))
    out = Q.node_bf16([a, b])
    assert list(Q.bf16_bits_to_f32(out)) == [1.0, 5.0]          # 1 + 2^-8 ties to 1.0
    x = np.linspace(-3, 3, 512)
    c1, s1 = Q.fp8_quantize(x)
    c2, s2 = Q.fp8_quantize(-x)
    c, s = Q.node_fp8([(c1, s1), (c2, s2)])
    assert np.all(Q.fp8_dequantize(c, s) == 0.0)
    assert np.all(s == 1.0)
