"""Reduced-precision table formats (an extension beyond the paper: the paper
states no storage precision for its renderer).

BF16: the upper 16 bits of the float32 pattern after round-to-nearest-even
(NaN -> 0x7FC0).  Decoding shifts the 16 bits back up (exact).

FP8: OCP E4M3FN -- 1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits, no
infinities, NaN = S.1111.111, largest finite 448, subnormals m * 2^-9.
Scaling: one float32 scale per (level, channel), s = fl32(amax / 448) with
amax the largest |x| of that level and channel (s = 1 when amax = 0);
code q = nearest E4M3FN value to fl32(x / s), ties to the even code,
saturating at +-448, sign bit copied from the input (so -0 -> 0x80).  A stored value reads back as decode(q) * s.

Encoding here is defined by search over the explicit table of all 256 code
values, independent of any bit trick.
"""
from __future__ import annotations

import numpy as np

from .exact32 import F32


def bf16_encode(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=F32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)
    return np.where(np.isnan(x), np.uint16(0x7FC0), rounded).astype(np.uint16)


def bf16_decode(q: np.ndarray) -> np.ndarray:
    return (np.asarray(q, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(F32)


def fp8_e4m3_value(code: int) -> float:
    """Value of one E4M3FN code, from the format's definition."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


FP8_TABLE = np.array([fp8_e4m3_value(c) for c in range(256)], dtype=np.float64)


def fp8_decode(q: np.ndarray) -> np.ndarray:
    return FP8_TABLE[np.asarray(q, dtype=np.uint8)].astype(F32)


_POS_CODES = np.arange(0, 0x7F)          # 0x00 .. 0x7E: all finite non-negative codes
_POS_VALS = FP8_TABLE[_POS_CODES]        # strictly increasing


def fp8_encode(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even, saturating E4M3FN encoding of float32 values."""
    x = np.asarray(x, dtype=F32).astype(np.float64)
    a = np.minimum(np.abs(x), 448.0)
    hi = np.searchsorted(_POS_VALS, a, side="left")       # first value >= a
    hi = np.clip(hi, 0, len(_POS_VALS) - 1)
    lo = np.clip(hi - 1, 0, len(_POS_VALS) - 1)
    d_hi = _POS_VALS[hi] - a
    d_lo = a - _POS_VALS[lo]
    pick_lo = (d_lo < d_hi) | ((d_lo == d_hi) & (_POS_CODES[lo] % 2 == 0))
    code = np.where(pick_lo, _POS_CODES[lo], _POS_CODES[hi]).astype(np.uint8)
    code = np.where(a == _POS_VALS[hi], _POS_CODES[hi], code).astype(np.uint8)
    sign = np.signbit(x).astype(np.uint8) << np.uint8(7)
    code = code | sign
    return np.where(np.isnan(x), np.uint8(0x7F), code).astype(np.uint8)


def fp8_scales(tables: np.ndarray) -> np.ndarray:
    """Per (level, channel) float32 scales of a [L, T, C] float32 table."""
    amax = np.max(np.abs(tables.astype(F32)), axis=1)          # [L, C], exact
    s = amax / F32(448.0)
    return np.where(amax == 0, F32(1.0), s).astype(F32)


def quantize_tables_fp8(tables: np.ndarray):
    """Codes uint8 [L, T, C] and scales float32 [L, C]."""
    t = tables.astype(F32)
    s = fp8_scales(t)
    q = fp8_encode(t / s[:, None, :])
    return q, s


def quantize_tables_bf16(tables: np.ndarray) -> np.ndarray:
    return bf16_encode(tables.astype(F32))
