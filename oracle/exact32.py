"""Float32 arithmetic of the decision chain, written op by op in numpy.

Every operation on float32 arrays below is a single IEEE-754 binary32
operation with round-to-nearest-even (numpy never fuses a multiply and an
add); a fused multiply-add, where the chain takes one, is fma32 (one
rounding, emulated exactly).  The chain that decides integers -- lattice positions, voxel and corner
indices, trilinear weights, the interpolated density and logits, the
softmax across levels, the density activation and the transmittance -- is
defined in terms of these operations only, plus a project-defined
exponential (below), so that a CPU and a GPU evaluating it produce the same
bits.

exp32 (project definition, Cody-Waite argument reduction + Taylor series;
fma(a, b, c) = a * b + c rounded once):
    x NaN          -> NaN
    x > 88         -> +inf
    x < -86        -> 0
    k  = floor(fma(x, LOG2E, 0.5))
    r  = fma(-k, LN2_LO, fma(-k, LN2_HI, x))
    p  = Horner(r; 1/7!, 1/6!, ..., 1/1!, 1/0!)   (p = fma(p, r, c))
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
    k = np.floor(fma32(xm, LOG2E, F32(0.5)))
    r = fma32(-k, LN2_LO, fma32(-k, LN2_HI, xm))
    p = np.full_like(r, TAYLOR[7])
    for j in range(6, -1, -1):
        p = fma32(p, r, TAYLOR[j])
    n = k.astype(np.int32)
    two_n = ((n + 127).astype(np.uint32) << np.uint32(23)).view(F32)
    out[mid] = p * two_n
    out[hi] = np.inf
    out[lo] = F32(0.0)
    out[nan] = np.nan
    return out[0] if scalar else out


def fma32(a, b, c) -> np.ndarray:
    """fl32(a * b + c) rounded once (to nearest, ties to even), for float32
    arrays: what a fused multiply-add computes.  The product of two float32
    values is exact in float64 (48 significant bits); the float64 sum is
    rounded to odd (the exact error of the sum, by TwoSum, is nonzero and the
    rounded sum has an even last bit: step one ulp toward the error), and a
    rounding to odd at 53 bits followed by a rounding to nearest at 24 bits
    equals the single rounding to nearest, since 53 >= 2 * 24 + 2 (Boldo and
    Melquiond, "Emulation of FMA and correctly rounded sums: proved
    algorithms using rounding to odd", IEEE TC 2008).  Finite inputs."""
    a64 = np.asarray(a, dtype=F32).astype(np.float64)
    b64 = np.asarray(b, dtype=F32).astype(np.float64)
    c64 = np.asarray(c, dtype=F32).astype(np.float64)
    p = a64 * b64
    s = p + c64
    # TwoSum: s + e == p + c exactly
    bb = s - p
    e = (p - (s - bb)) + (c64 - bb)
    even = (np.asarray(s).view(np.int64) & 1) == 0
    toward = np.where(e > 0, np.inf, -np.inf)
    s_odd = np.where((e != 0) & even, np.nextafter(s, toward), s)
    return np.asarray(s_odd).astype(F32)


def sqrt32(x) -> np.ndarray:
    """Correctly rounded float32 square root."""
    return np.sqrt(np.asarray(x, dtype=F32))
