"""bf16 and OCP fp8-e4m3 payload formats — test oracle.

Written from the format definitions, in float64 arithmetic (exact for
every step used here):

  bf16      the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent, 7
            fraction bits); conversion from binary32 rounds to nearest,
            ties to even.
  e4m3      OCP 8-bit float "E4M3": 1 sign, 4 exponent bits (bias 7), 3
            fraction bits; exponent field 0 holds subnormals m * 2**-9; no
            infinities; S.1111.111 is NaN, so the largest finite magnitude
            is 1.75 * 2**8 = 448. Conversion rounds to nearest, ties to even,
            and saturates to +-448.
  scales    one binary32 scale per block of 256 consecutive elements: the
            smallest power of two 2**e with amax <= 448 * 2**e (e clamped to
            the binary32 normal range), 1 for an all-zero block. A power of
            two makes the scaling exact, so a quantizer that follows these
            rules reproduces any other's bytes bit for bit.

These carry the precision form of the executor: payloads move in the
narrow format, every reduction node widens its operands to float32, sums
them, and narrows the result again with fresh block scales.

Parity: pinned by tests/test_oracle_quant.py (hand-checked codes, all 256
codes round-tripped, torch's CPU float8_e4m3fn / bfloat16 conversions on
in-range values, the relative error bound 2**-4 of a normal e4m3 value).
"""
from __future__ import annotations

import numpy as np

FP8_MAX = 448.0
FP8_BLOCK = 256


# ------------------------------------------------------------------ bf16
def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """binary32 -> bf16 bit patterns (uint16), round to nearest even. Inputs must be finite."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if not np.all(np.isfinite(x)):
        raise ValueError("bf16 conversion of a non-finite value")
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f32(u: np.ndarray) -> np.ndarray:
    """bf16 bit patterns -> binary32 values (exact)."""
    u = np.asarray(u, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


# ------------------------------------------------------------------ e4m3
def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    """e4m3 codes (uint8) -> float64 values (NaN for the two NaN codes)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    mag = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((e == 15) & (m == 7), np.nan, mag)
    return s * mag


def e4m3_encode(x: np.ndarray) -> np.ndarray:
    """float values -> e4m3 codes (uint8), round to nearest even, saturating to +-448."""
    x = np.asarray(x, dtype=np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("e4m3 conversion of a non-finite value")
    sign = np.where(np.signbit(x), 0x80, 0).astype(np.int64)
    a = np.abs(x)
    out = np.zeros(a.shape, dtype=np.int64)
    # subnormal range: a < 2**-6, step 2**-9; a rounded count of 8 is the least normal (code 8)
    sub = a < 2.0 ** -6
    out[sub] = np.rint(a[sub] / 2.0 ** -9).astype(np.int64)
    nrm = ~sub
    if np.any(nrm):
        an = a[nrm]
        _, ex = np.frexp(an)            # an = f * 2**ex, f in [0.5, 1)
        e = ex - 1                      # an in [2**e, 2**(e+1))
        q = np.rint(an / np.exp2(e - 3.0)).astype(np.int64)   # in [8, 16]
        carry = q == 16
        e = np.where(carry, e + 1, e)
        q = np.where(carry, 8, q)
        code = ((e + 7) << 3) | (q - 8)
        code = np.where((e > 8) | (code > 0x7E), 0x7E, code)   # saturate at 448
        out[nrm] = code
    return (out | sign).astype(np.uint8)


def block_scales(x: np.ndarray, block: int = FP8_BLOCK) -> np.ndarray:
    """Power-of-two binary32 scale of every ``block``-element block of x (len(x) % block == 0)."""
    x = np.asarray(x, dtype=np.float64)
    if len(x) % block:
        raise ValueError("length must be a multiple of the scale block")
    amax = np.abs(x.reshape(-1, block)).max(axis=1) if len(x) else np.zeros(0)
    f, ex = np.frexp(amax)              # amax = f * 2**ex
    e = np.where(f <= 0.875, ex - 9, ex - 8)   # least e with amax <= 0.875 * 2**(9 + e) = 448 * 2**e
    e = np.clip(e, -126, 127)
    sc = np.exp2(e.astype(np.float64))
    sc = np.where(amax == 0, 1.0, sc)
    return sc.astype(np.float32)


def fp8_quantize(x: np.ndarray, block: int = FP8_BLOCK):
    """float values -> (e4m3 codes, per-block binary32 scales)."""
    x = np.asarray(x, dtype=np.float64)
    sc = block_scales(x, block)
    q = x / np.repeat(sc.astype(np.float64), block)
    return e4m3_encode(q), sc


def fp8_dequantize(codes: np.ndarray, scales: np.ndarray, block: int = FP8_BLOCK) -> np.ndarray:
    """(codes, scales) -> float64 values (each exactly representable in binary32)."""
    return e4m3_decode(codes) * np.repeat(np.asarray(scales, dtype=np.float64), block)


# ------------------------------------------ one reduction node in each payload format
def node_bf16(ops: list[np.ndarray]) -> np.ndarray:
    """bf16 operands (uint16 bits) -> widen to binary32, sum left to right, narrow (RNE)."""
    acc = bf16_bits_to_f32(ops[0]).copy()
    for v in ops[1:]:
        acc = (acc + bf16_bits_to_f32(v)).astype(np.float32)
    return f32_to_bf16_bits(acc)


def node_fp8(ops: list[tuple[np.ndarray, np.ndarray]]):
    """fp8 operands (codes, scales) -> widen to binary32, sum left to right, requantize."""
    acc = fp8_dequantize(*ops[0]).astype(np.float32)
    for c, s in ops[1:]:
        acc = (acc + fp8_dequantize(c, s).astype(np.float32)).astype(np.float32)
    return fp8_quantize(acc)
