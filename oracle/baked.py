"""Oracle of the paper's own feature construction (test infrastructure).

Sec. 4.1, Eq. 6: the deferred feature at x is f = f~ + f^, where
f~ = Interp(F~, x) and a = Interp(A, x) come from a coarse grid of
resolution L_C (here one block-sparse vertex grid holds both: 8 feature
channels [sigma~, c_d~ (3), v_s~ (4)] and the 2L attention parameters
[omega_1, beta_1, ..., omega_L, beta_L]), and f^ = Att(f^_1..f^_L; a) fuses
the L fine hash levels.  Sec. 4.2, Eq. 7-8: separate attention,
f^ = [sum_l omega_l sigma^_l, sum_l beta_l c^_l, sum_l beta_l v^_l]; the
supplement ("Activation Layers" 2) normalises each per-point, per-level
attention parameter to [0, 1] with a sigmoid.

Coarse grid storage: vertex (vx, vy, vz), 0 <= v <= L_C, lives in block
(vx >> 3, vy >> 3, vz >> 3) at local (vx & 7, vy & 7, vz & 7);
block_index[bz, by, bx] is its atlas row or -1 (empty block: every vertex
takes the default vector); atlas[bid, lz, ly, lx, :] the C values.
Interpolation uses the hash levels' cell convention: p = u L_C,
i0 = clamp(floor(p), 0, L_C - 1), corners i0 + {0, 1}^3, f = u L_C - i0
rounded once.

Aggregation variants (Sec. 5.2, Table 3): Separate-Att (V) is the design
above; Shared-Att (V) stores one a_l per vertex and gates density and
colour with g(a_l); the (Inv) variants take omega_l, beta_l (or a_l) as
scene constants instead of interpolated values; SUM drops the gates
(f^ = sum_l f^_l).  The coarse grid then holds 8 + L or 8 channels.

Float32 decision chain (bit-exact with the GPU): coarse channels
acc = acc + w_c v_c (c = 0..7, plain float32 operations); fine level l as
the hash levels (density channel acc = acc + w_c v_c; FP8 then times the
scale); g = 1 / (1 + exp32(-a)) for each attention parameter;
f_0 = sigma~, then for l = 1..L in order f_0 = f_0 + g_omega_l * sigma^_l.
Reported values are float64.
"""
from __future__ import annotations

import numpy as np

from .exact32 import F32, exp32, fma32
from .hashgrid import cell32, corners32, corners64

BLOCK = 8


def _vertex_values(inp, vx, vy, vz) -> np.ndarray:
    """Stored coarse values [m, C] (float32) of integer vertices."""
    bx, by, bz = vx >> 3, vy >> 3, vz >> 3
    bid = inp.block_index[bz, by, bx]
    if inp.atlas.shape[0] == 0:                          # no stored block at all
        return np.broadcast_to(inp.coarse_default, (len(vx), len(inp.coarse_default))).astype(F32)
    rows = inp.atlas[np.maximum(bid, 0), vz & 7, vy & 7, vx & 7]
    return np.where((bid >= 0)[:, None], rows, inp.coarse_default[None, :]).astype(F32)


def coarse_corners32(u: np.ndarray, Lc: int):
    """Integer corner vertices [m, 8, 3] (x, y, z) and float32 weights [m, 8]."""
    u = np.asarray(u, dtype=F32)
    i0 = cell32(u, Lc)
    f = (u.astype(np.float64) * Lc - i0).astype(F32)     # rounded once
    g = F32(1.0) - f
    v = np.empty((u.shape[0], 8, 3), dtype=np.int64)
    w = np.empty((u.shape[0], 8), dtype=F32)
    for c in range(8):
        b = ((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1)
        wa = [f[:, a] if b[a] else g[:, a] for a in range(3)]
        w[:, c] = (wa[0] * wa[1]) * wa[2]
        for a in range(3):
            v[:, c, a] = i0[:, a] + b[a]
    return v, w


def coarse32(inp, u: np.ndarray) -> np.ndarray:
    """Float32 interpolation of all C coarse channels, corners in order."""
    v, w = coarse_corners32(u, inp.coarse_res)
    acc = np.zeros((u.shape[0], inp.coarse_channels), dtype=F32)
    for c in range(8):
        vals = _vertex_values(inp, v[:, c, 0], v[:, c, 1], v[:, c, 2])
        acc = fma32(w[:, c:c + 1], vals, acc)
    return acc


def coarse64(inp, u: np.ndarray) -> np.ndarray:
    """Float64 trilinear interpolation of the coarse channels."""
    u = np.asarray(u, dtype=np.float64)
    Lc = inp.coarse_res
    i0 = cell32(u, Lc)               # the cell decided in float32
    f = u * Lc - i0
    acc = np.zeros((u.shape[0], inp.coarse_channels))
    for c in range(8):
        b = ((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1)
        wc = np.ones(u.shape[0])
        for a in range(3):
            wc = wc * (f[:, a] if b[a] else 1.0 - f[:, a])
        vals = _vertex_values(inp, i0[:, 0] + b[0], i0[:, 1] + b[1], i0[:, 2] + b[2])
        acc += wc[:, None] * vals.astype(np.float64)
    return acc


def sigmoid32(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=F32)
    return (F32(1.0) / (F32(1.0) + exp32(-a))).astype(F32)


SEPARATE_V, SHARED_V, SEPARATE_INV, SHARED_INV, SUM = 0, 1, 2, 3, 4


def gate_params(inp, co: np.ndarray, l: int):
    """Attention parameters (omega_l, beta_l) of fine level l per point, before
    the sigmoid, under the scene's aggregation; None for SUM (gates 1)."""
    agg = getattr(inp, "aggregation", SEPARATE_V)
    m = co.shape[0]
    if agg == SEPARATE_V:
        return co[:, 8 + 2 * l], co[:, 9 + 2 * l]
    if agg == SHARED_V:
        return co[:, 8 + l], co[:, 8 + l]
    p = np.asarray(inp.gate_params, dtype=co.dtype)
    if agg == SEPARATE_INV:
        return np.full(m, p[2 * l], co.dtype), np.full(m, p[2 * l + 1], co.dtype)
    if agg == SHARED_INV:
        return np.full(m, p[l], co.dtype), np.full(m, p[l], co.dtype)
    if agg == SUM:
        return None
    raise ValueError("unknown aggregation")


def fused32(inp, u: np.ndarray):
    """Float32 decision chain: fused channels [m, 8] (channel 0 bit-exact,
    colour channels to rounding), density gates g_omega [m, L], fine corner
    indices [m, L, 8]."""
    m = u.shape[0]
    co = coarse32(inp, u)
    fused = co[:, :8].copy()
    gws, idxs = [], []
    for l, N in enumerate(inp.resolutions):
        idx, w = corners32(u, N, inp.T)
        idxs.append(idx)
        g = inp.deq32[l][idx]                            # [m, 8 corners, 9]
        acc = np.zeros((m, 8), dtype=F32)
        for c in range(8):
            acc = fma32(w[:, c:c + 1], g[:, c, :8], acc)
        if inp.scales is not None:
            acc = inp.scales[l][None, :8] * acc
        a = gate_params(inp, co, l)
        if a is None:
            gw = gb = np.ones(m, dtype=F32)
        else:
            gw, gb = sigmoid32(a[0]), sigmoid32(a[1])
        fused[:, 0] = fma32(gw, acc[:, 0], fused[:, 0])
        fused[:, 1:] = fma32(gb[:, None], acc[:, 1:], fused[:, 1:])
        gws.append(gw)
    return fused.astype(F32), np.stack(gws, axis=1).astype(F32), np.stack(idxs, axis=1)


def fused64(inp, u: np.ndarray):
    """Float64 feature construction; returns fused [m, 8] and g_omega [m, L]."""
    u = np.asarray(u, dtype=np.float64)
    m = u.shape[0]
    co = coarse64(inp, u)
    fused = co[:, :8].copy()
    gws = []
    for l, N in enumerate(inp.resolutions):
        idx, w = corners64(u, N, inp.T)
        v = np.zeros((m, 8))
        for c in range(8):
            v += w[:, c:c + 1] * inp.val64[l][idx[:, c], :8]
        a = gate_params(inp, co, l)
        if a is None:
            gw = gb = np.ones(m)
        else:
            gw, gb = 1.0 / (1.0 + np.exp(-a[0])), 1.0 / (1.0 + np.exp(-a[1]))
        fused[:, 0] += gw * v[:, 0]
        fused[:, 1:] += gb[:, None] * v[:, 1:]
        gws.append(gw)
    return fused, np.stack(gws, axis=1)


# --------------------------------------------------------------------------
# float64 forward intermediates and the adjoint of the feature construction
# (for the training extension; the sample list is frozen)


def forward64_parts(atlas64, default, block_index, Lc, fine64, resolutions, u):
    """fused [m, 8] and the intermediates the adjoint needs, at float64 grid
    coordinates u (fine64: [L, T, >=8] float64 fine tables)."""
    u = np.asarray(u, dtype=np.float64)
    m = u.shape[0]
    T = fine64.shape[1]
    i0 = cell32(u, Lc)               # the cell decided in float32
    f = u * Lc - i0
    C = atlas64.shape[-1]
    co = np.zeros((m, C))
    cv, cw, cb = [], [], []
    for c in range(8):
        b = ((c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1)
        wc = np.ones(m)
        for a in range(3):
            wc = wc * (f[:, a] if b[a] else 1.0 - f[:, a])
        vx, vy, vz = i0[:, 0] + b[0], i0[:, 1] + b[1], i0[:, 2] + b[2]
        bid = block_index[vz >> 3, vy >> 3, vx >> 3]
        if atlas64.shape[0]:
            rows = atlas64[np.maximum(bid, 0), vz & 7, vy & 7, vx & 7]
            vals = np.where((bid >= 0)[:, None], rows, np.asarray(default, np.float64)[None, :])
        else:
            vals = np.broadcast_to(np.asarray(default, np.float64), (m, C))
        co += wc[:, None] * vals
        cv.append(np.stack([vx, vy, vz], axis=1))
        cw.append(wc)
        cb.append(bid)
    fused = co[:, :8].copy()
    fidx, fw, fval, gws, gbs = [], [], [], [], []
    for l, N in enumerate(resolutions):
        idx, w = corners64(u, N, T)
        v = np.einsum("mc,mcd->md", w, fine64[l][idx][:, :, :8])
        gw = 1.0 / (1.0 + np.exp(-co[:, 8 + 2 * l]))
        gb = 1.0 / (1.0 + np.exp(-co[:, 9 + 2 * l]))
        fused[:, 0] += gw * v[:, 0]
        fused[:, 1:] += gb[:, None] * v[:, 1:]
        fidx.append(idx); fw.append(w); fval.append(v); gws.append(gw); gbs.append(gb)
    return fused, dict(co=co, cv=np.stack(cv, 1), cw=np.stack(cw, 1), cb=np.stack(cb, 1),
                       fidx=fidx, fw=fw, fval=fval, gw=gws, gb=gbs)


def scatter64(parts, g_fused, n_blocks, C, fine_shape):
    """Adjoint of the feature construction: dL/d(atlas) [n_blocks, 8, 8, 8, C]
    and dL/d(fine tables) [L, T, 9] (channel 8 zero) from dL/dfused [m, 8].
    f_0 = co_0 + sum_l g(omega_l) s_l, f_j = co_j + sum_l g(beta_l) v_lj:
    dco_j = df_j (j < 8); dco_omega_l = df_0 s_l g'(omega_l);
    dco_beta_l = sum_{j>=1} df_j v_lj g'(beta_l); dv_l0 = df_0 g(omega_l);
    dv_lj = df_j g(beta_l).  Empty-block vertices (the default vector) take
    no gradient."""
    m = g_fused.shape[0]
    g_co = np.zeros((m, C))
    g_co[:, :8] = g_fused
    g_fine = np.zeros(fine_shape)
    for l in range(len(parts["fidx"])):
        gw, gb, v = parts["gw"][l], parts["gb"][l], parts["fval"][l]
        g_co[:, 8 + 2 * l] = g_fused[:, 0] * v[:, 0] * gw * (1.0 - gw)
        g_co[:, 9 + 2 * l] = (g_fused[:, 1:] * v[:, 1:]).sum(axis=1) * gb * (1.0 - gb)
        gv = np.concatenate([(g_fused[:, 0] * gw)[:, None], g_fused[:, 1:] * gb[:, None]], axis=1)
        for c in range(8):
            np.add.at(g_fine[l][:, :8], parts["fidx"][l][:, c], parts["fw"][l][:, c][:, None] * gv)
    g_atlas = np.zeros((n_blocks, 8, 8, 8, C))
    for c in range(8):
        bid = parts["cb"][:, c]
        ok = bid >= 0
        vx, vy, vz = parts["cv"][ok, c, 0], parts["cv"][ok, c, 1], parts["cv"][ok, c, 2]
        np.add.at(g_atlas, (bid[ok], vz & 7, vy & 7, vx & 7), parts["cw"][ok, c][:, None] * g_co[ok])
    return g_atlas, g_fine
