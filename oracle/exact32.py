"""Float32 arithmetic of the decision chain, written op by op in numpy.

Every operation on float32 arrays below is a single IEEE-754 binary32
operation with round-to-nearest-even (numpy never fuses a multiply and an
add).  The chain that decides integers -- lattice positions, voxel and corner
indices, trilinear weights, the interpolated density and logits, the
softmax across levels, the density activation and the transmittance -- is
defined in terms of these operations only, plus a project-defined
exponential (below), so that a CPU and a GPU evaluating it produce the same
bits.

exp32 (project definition, Cody-Waite argument reduction + Taylor series):
    x NaN          -> NaN
    x > 88         -> +inf
    x < -86        -> 0
    k  = floor(x * LOG2E + 0.5)            (float32 ops)
    r  = (x - k * LN2_HI) - k * LN2_LO
    p  = Horner(r; 1/7!, 1/6!, ..., 1/1!, 1/0!)   (p = p * r + c, unfused)
    result = p * 2^k   (2^k built from its exponent bits, exact)
with LOG2E = fl32(log2 e) = 0x3FB8AA3B, LN2_HI = 0.693359375 (0x3F318000),
LN2_LO = fl32(ln 2 - LN2_HI) = 0xB95E8083, and c_j = fl32(1/j!).
Its error against the true exponential is a few ulp (pinned in the tests).

Sums over hash levels are taken in level order, l = 0, 1, ..., L - 1.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def _bits_to_f32(u: int) -> np.float32:
    return np.array([u], dtype=np.uint32).view(np.float32)[0]


LOG2E = _bits_to_f32(0x3FB8AA3B)
LN2_HI = _bits_to_f32(0x3F318000)
LN2_LO = _bits_to_f32(0xB95E8083)
TAYLOR = [_bits_to_f32(b) for b in (0x3F800000, 0x3F800000, 0x3F000000, 0x3E2AAAAB,
                                     0x3D2AAAAB, 0x3C088889, 0x3AB60B61, 0x39500D01)]


def exp32(x) -> np.ndarray:
    """Project-defined float32 exponential (see module docstring)."""
    x = np.asarray(x, dtype=F32)
    scalar = x.ndim == 0
    x = np.atleast_1d(x)
    out = np.empty_like(x)
    hi = x > F32(88.0)
    lo = x < F32(-86.0)
    nan = np.isnan(x)
    mid = ~(hi | lo | nan)
    xm = x[mid]
    k = np.floor(xm * LOG2E + F32(0.5))
    r = (xm - k * LN2_HI) - k * LN2_LO
    p = np.full_like(r, TAYLOR[7])
    for j in range(6, -1, -1):
        p = p * r + TAYLOR[j]
    n = k.astype(np.int32)
    two_n = ((n + 127).astype(np.uint32) << np.uint32(23)).view(F32)
    out[mid] = p * two_n
    out[hi] = np.inf
    out[lo] = F32(0.0)
    out[nan] = np.nan
    return out[0] if scalar else out


def sqrt32(x) -> np.ndarray:
    """Correctly rounded float32 square root."""
    return np.sqrt(np.asarray(x, dtype=F32))
