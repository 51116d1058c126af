"""Multi-level spatial hash tables: corner indexing and trilinear lookup.

Follows the multi-resolution hash encoding the method builds on (Sec. 3,
Eq. 3; Sec. 4.1 "fine-grained" hash levels holding explicit 8-D deferred
features, supplement "Multi-level Hash Features"):

* grid coordinate u = (x - lo) * inv_extent in [0, 1]^3;
* level l of resolution N_l: p = u * N_l, i0 = clamp(floor(p), 0, N_l - 1)
  (p rounded to float32: the cell is decided in float32 arithmetic),
  f = u * N_l - i0, corners i0 + b for b in {0,1}^3 (bit 0 -> x, 1 -> y, 2 -> z);
* spatial hash h = (cx * 1) xor (cy * 2654435761) xor (cz * 805459861),
  each product taken modulo 2^32, then h mod T (T a power of two);
* trilinear weight of corner b: prod over axes of (f if b else 1 - f).

Each level is hashed, coarse levels included.
"""
from __future__ import annotations

import numpy as np

from .exact32 import F32

PRIMES = (1, 2654435761, 805459861)
MASK32 = np.uint64(0xFFFFFFFF)


def spatial_hash(cx, cy, cz, table_size: int) -> np.ndarray:
    """Hash of integer corner coordinates (numpy, uint32 wrap-around)."""
    cx = np.asarray(cx, dtype=np.uint64)
    cy = np.asarray(cy, dtype=np.uint64)
    cz = np.asarray(cz, dtype=np.uint64)
    h = ((cx * np.uint64(PRIMES[0])) & MASK32) ^ ((cy * np.uint64(PRIMES[1])) & MASK32) \
        ^ ((cz * np.uint64(PRIMES[2])) & MASK32)
    return (h & np.uint64(table_size - 1)).astype(np.int64)


def spatial_hash_py(cx: int, cy: int, cz: int, table_size: int) -> int:
    """The same hash with Python integers (used to pin the numpy version)."""
    h = ((cx * PRIMES[0]) % 2 ** 32) ^ ((cy * PRIMES[1]) % 2 ** 32) ^ ((cz * PRIMES[2]) % 2 ** 32)
    return h % table_size


def cell32(u: np.ndarray, N: int) -> np.ndarray:
    """Cell index per axis as the float32 decision chain takes it:
    i0 = clamp(floor(fl32(u N)), 0, N - 1), u rounded to float32 first.

    The cell is an integer decided in floating point, so the float64 values
    use the same one.  Where u N lies within half an ulp below an integer
    the float32 product rounds up to it: i0 is then the cell above and the
    fraction u N - i0 is slightly negative (by at most half an ulp of u N),
    which the trilinear formula takes as it is."""
    p = np.asarray(u, dtype=F32) * F32(N)
    return np.clip(np.floor(p), 0, N - 1).astype(np.int64)


def corners32(u: np.ndarray, N: int, table_size: int):
    """Corner indices [m, 8] and float32 trilinear weights [m, 8] of one level.

    u is float32 [m, 3].  p = fl32(u N) picks the cell; the fraction
    f = fl32(u N - i0) is rounded once (a fused multiply-add), so it is
    accurate to half an ulp of f even where u N is large; the weights follow
    the float32 op order w = (wx * wy) * wz.
    """
    u = np.asarray(u, dtype=F32)
    i0 = cell32(u, N)
    # f = u*N - i0 rounded once (a fused multiply-add): the product of a
    # float32 and an integer below 2^20 and the difference are exact in float64
    f = (u.astype(np.float64) * N - i0).astype(F32)
    g = F32(1.0) - f
    idx = np.empty((u.shape[0], 8), dtype=np.int64)
    w = np.empty((u.shape[0], 8), dtype=F32)
    for c in range(8):
        b = ((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1)
        wa = [f[:, a] if b[a] else g[:, a] for a in range(3)]
        w[:, c] = (wa[0] * wa[1]) * wa[2]
        idx[:, c] = spatial_hash(i0[:, 0] + b[0], i0[:, 1] + b[1], i0[:, 2] + b[2], table_size)
    return idx, w


def corners64(u: np.ndarray, N: int, table_size: int):
    """Same as corners32 in float64 (for values): the cell decided in
    float32 (cell32; u holds float32 values), the fraction u N - i0 and the
    weights in float64."""
    u = np.asarray(u, dtype=np.float64)
    i0 = cell32(u, N)
    f = u * N - i0
    idx = np.empty((u.shape[0], 8), dtype=np.int64)
    w = np.empty((u.shape[0], 8), dtype=np.float64)
    for c in range(8):
        b = ((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1)
        wa = [f[:, a] if b[a] else 1.0 - f[:, a] for a in range(3)]
        w[:, c] = wa[0] * wa[1] * wa[2]
        idx[:, c] = spatial_hash(i0[:, 0] + b[0], i0[:, 1] + b[1], i0[:, 2] + b[2], table_size)
    return idx, w


def interp32(table_ch: np.ndarray, idx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Float32 interpolation of one channel: acc = 0; acc = acc + w_c * v_c, c = 0..7."""
    acc = np.zeros(idx.shape[0], dtype=F32)
    for c in range(8):
        acc = acc + w[:, c] * table_ch[idx[:, c]].astype(F32)
    return acc
