"""Oracle renderer: march, lookup, attention, compositing, deferred MLP.

What one ray computes (paper sections in brackets):

1. Ray setup (a ray with a non-finite component or a zero direction has no
   samples).  Box scenes: the ray enters and leaves the cube ROI at
   [t0, t1) by the slab test; lattice t_k = t0 + k * step.  Contracted scenes:
   the scene lives in the image of x -> x (|x| <= 1), (2 - 1/|x|) x/|x|
   (|x| > 1); the ray starts at t = 0 and advances by equal contracted arc
   length, t_{k+1} = t_k + step / |J(x_k) d|, ending once it moves outward
   with 1/|x| < step (or |x|^2 overflows).  Every sample carries delta = step (the lattice
   interval it opens) [Eq. 2].
2. Occupancy test at each lattice point; occupied points are sampled.  The
   skip march reads the distance grid G (Eq. 9): after reading G = g > 0 at a
   lattice point, points within g voxels of it (less a margin) are known to be
   empty and are not read.  Box scenes turn that into a jump of
   floor(g * (voxel / step) / |d|) lattice points (at most 2^16, the
   lattice bound); contracted scenes keep a
   ball of radius g * voxel - voxel/1024 around the read point.  The naive
   march reads every lattice point; both must yield the same samples
   (the paper's Table 4: the occupied-point count is unchanged by G).
3. At a sample: trilinear lookup in every hash level [Sec. 3 Eq. 3,
   Sec. 4.1 Eq. 6] of 8 feature channels and 1 attention logit.
4. Attention across levels [Sec. 4.2 Eq. 7-8, softmax reading]: weights
   w_l = softmax_l(logit_l), fused channel = sum_l w_l v_l; density and
   colour share the weights.
5. Activation and compositing [Eq. 2, Eq. 5; supplement "Activation
   Layers"]: sigma = exp(fused_0); alpha = 1 - exp(-sigma * delta);
   C_d += T alpha c_d, F += T alpha v_s, T *= 1 - alpha; the ray stops once
   T < threshold (after compositing that sample) [supplement "Real-time
   Rendering" item 2] or after max_samples samples.
6. Deferred MLP once per ray [Eq. 5]: C = sigmoid(C_d + MLP(C_d, F)), MLP
   7 -> 16 -> 16 -> 3 with ReLU hidden layers and a linear output.

Decisions (steps 1-2 and the termination test) are taken in the float32
mirror of exact32; all reported values are recomputed in float64 on the
decided sample list, at the float32 grid coordinates u = fl32((x - lo) *
inv_extent) of the decided lattice points (a sample's position is part of
what the float32 lattice defines, like its index).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .exact32 import F32, exp32, fma32, sqrt32
from .hashgrid import corners32, corners64
from . import baked, pyramid, quant, sh

BOX = 0
CONTRACT = 1
DT_F32, DT_BF16, DT_FP8 = 0, 1, 2
MAX_LATTICE = 1 << 16


@dataclass
class OracleInputs:
    tables: np.ndarray            # float32 [L, T, 9]
    occ: np.ndarray               # uint8 [R, R, R]
    dist: np.ndarray              # uint8 [R, R, R]
    mlp: np.ndarray               # float32 [451]
    resolutions: List[int]
    domain: int
    roi_half: float
    step: float
    max_samples: int
    t_threshold: float
    dtype: int = DT_F32
    mlp_dims: tuple = (7, 16, 16, 3)
    # baked feature model (coarse grid + sigmoid-gated fine levels); 0 = hash model
    coarse_res: int = 0
    block_index: Optional[np.ndarray] = None   # int32 [nb, nb, nb]
    atlas: Optional[np.ndarray] = None         # float32 [n_blocks, 8, 8, 8, C]
    coarse_default: Optional[np.ndarray] = None  # float32 [C]
    # fusion of the fine levels (Table 3's variants; 0 = Separate-Att (V))
    aggregation: int = 0
    gate_params: tuple = ()                      # constant gates of the Inv variants
    # multi-level occupancy (Eq. 9's s_O branch): uint8 grids [O_0 (finest), O_1, ...];
    # occ / dist are then the pyramid level of the distance grid's resolution and its G
    pyramid: Optional[list] = None
    use_dist: bool = True
    # derived
    stored: Optional[np.ndarray] = None     # stored codes / values [L, T, 9]
    scales: Optional[np.ndarray] = None     # float32 [L, 9] (FP8 only)
    deq32: Optional[np.ndarray] = None      # float32 decoded code values (before scale)
    val64: Optional[np.ndarray] = None      # float64 dequantised values [L, T, 9]

    def __post_init__(self):
        t = np.asarray(self.tables, dtype=F32)
        if self.dtype == DT_F32:
            self.stored = t
            self.deq32 = t
            self.scales = None
            self.val64 = t.astype(np.float64)
        elif self.dtype == DT_BF16:
            self.stored = quant.quantize_tables_bf16(t)
            self.deq32 = quant.bf16_decode(self.stored)
            self.scales = None
            self.val64 = self.deq32.astype(np.float64)
        elif self.dtype == DT_FP8:
            self.stored, self.scales = quant.quantize_tables_fp8(t)
            self.deq32 = quant.fp8_decode(self.stored)
            self.val64 = self.deq32.astype(np.float64) * self.scales.astype(np.float64)[:, None, :]
        else:
            raise ValueError("unknown table dtype")
        self.occ_flat = np.ascontiguousarray(self.occ, dtype=np.uint8).ravel()
        self.dist_flat = np.ascontiguousarray(self.dist, dtype=np.uint8).ravel()

    @property
    def L(self):
        return len(self.resolutions)

    @property
    def T(self):
        return self.tables.shape[1]

    @property
    def R(self):
        return self.occ.shape[0]

    @property
    def coarse_channels(self):
        return 8 + {0: 2 * self.L, 1: self.L}.get(self.aggregation, 0)


# --------------------------------------------------------------------------
# per-sample lookup + attention


def fused32(inp: OracleInputs, u: np.ndarray):
    """Float32 mirror of the lookup + attention chain at grid coordinates u.

    Softmax across levels (Eq. 8, softmax reading) in one pass over the
    levels with a running maximum (the online softmax of Milakov and
    Gimelshein, 2018), so no level's term underflows unless it is negligible
    against the sample's own largest logit.  Per level, in order, with a_l
    the interpolated logit and m the running maximum (m = -inf before level
    0):
        d = a_l - m;  x = exp32(-|d|)
        d > 0:  the new maximum is a_l; the sums so far scale by x, e_l = 1
        else:   the sums keep their scale, e_l = x
        S = fma(S, scale, e_l);   N_j = fma(e_l, v_l[j], N_j * scale)
    fused_j = N_j / S; attention weights w_l = exp32(a_l - m) / S with m the
    final maximum.  S >= 1 always (the level holding the maximum adds 1).

    Returns fused channels [m, 8], attention weights [m, L], corner indices
    [m, L, 8].  (Baked model: see oracle.baked.fused32.)"""
    if inp.coarse_res:
        return baked.fused32(inp, u)
    m = u.shape[0]
    run_max = np.full(m, -np.inf, dtype=F32)
    esum = np.zeros(m, dtype=F32)
    num = np.zeros((m, 8), dtype=F32)
    logits, idxs = [], []
    for l, N in enumerate(inp.resolutions):
        idx, w = corners32(u, N, inp.T)
        idxs.append(idx)
        g = inp.deq32[l][idx]                        # [m, 8 corners, 9 channels]
        acc = np.zeros((m, 9), dtype=F32)
        for c in range(8):                           # acc = fma(w_c, v_c, acc), c = 0..7
            acc = fma32(w[:, c:c + 1], g[:, c, :], acc)
        if inp.scales is not None:
            acc = inp.scales[l][None, :] * acc
        a = acc[:, 8]
        with np.errstate(invalid="ignore"):
            dlt = a - run_max
        x = exp32(-np.abs(dlt))
        up = dlt > F32(0.0)
        scale = np.where(up, x, F32(1.0)).astype(F32)
        e = np.where(up, F32(1.0), x).astype(F32)
        run_max = np.where(up, a, run_max).astype(F32)
        esum = fma32(esum, scale, e)
        num = fma32(e[:, None], acc[:, :8], num * scale[:, None])
        logits.append(a)
    fused = (num / esum[:, None]).astype(F32)
    wl = np.stack([exp32(a - run_max) / esum for a in logits], axis=1).astype(F32)
    return fused, wl, np.stack(idxs, axis=1)


def fused64(inp: OracleInputs, u: np.ndarray):
    """Float64 lookup + attention; returns fused [m, 8], weights [m, L]."""
    if inp.coarse_res:
        return baked.fused64(inp, u)
    u = np.asarray(u, dtype=np.float64)
    m = u.shape[0]
    logits, vals = [], []
    for l, N in enumerate(inp.resolutions):
        idx, w = corners64(u, N, inp.T)
        v = np.zeros((m, 9))
        for c in range(8):
            v += w[:, c:c + 1] * inp.val64[l][idx[:, c]]
        logits.append(v[:, 8])
        vals.append(v[:, :8])
    a = np.stack(logits, axis=1)
    a = a - a.max(axis=1, keepdims=True)
    e = np.exp(a)
    wl = e / e.sum(axis=1, keepdims=True)
    fused = np.einsum("ml,mlc->mc", wl, np.stack(vals, axis=1))
    return fused, wl


def grid_coords32(inp: OracleInputs, pos: np.ndarray) -> np.ndarray:
    """u = (x - lo) * inv_extent, float32."""
    lo = F32(-inp.roi_half)
    inv = F32(1.0) / (F32(inp.roi_half) - lo)
    return (np.asarray(pos, dtype=F32) - lo) * inv


def grid_coords64(inp: OracleInputs, pos: np.ndarray) -> np.ndarray:
    lo = -float(inp.roi_half)
    return (np.asarray(pos, dtype=np.float64) - lo) / (2.0 * inp.roi_half)


def sample_coords64(inp: OracleInputs, o: np.ndarray, d: np.ndarray, s_ray: np.ndarray,
                    s_t: np.ndarray) -> np.ndarray:
    """Grid coordinates of decided samples recomputed in float64 from the ray
    and the sample's lattice parameter t [Sec. 3: x = o + t d; contracted
    scenes map |x| > 1 to (2 - 1/|x|) x / |x|].  The float32 path takes u
    from the float32 position instead; the two differ by the rounding of the
    position (about 1e-7 in u), which this lets one measure."""
    o64 = np.asarray(o, dtype=np.float64)[s_ray]
    d64 = np.asarray(d, dtype=np.float64)[s_ray]
    x = o64 + np.asarray(s_t, dtype=np.float64)[:, None] * d64
    if inp.domain == CONTRACT:
        r = np.sqrt(np.sum(x * x, axis=1))
        outer = r > 1.0
        x[outer] = ((2.0 - 1.0 / r[outer]) / r[outer])[:, None] * x[outer]
    return grid_coords64(inp, x)


# --------------------------------------------------------------------------
# ray setup


def ray_box32(o: np.ndarray, d: np.ndarray, half: float):
    """Slab test in float32: entry t0 (clamped at 0), exit t1, validity."""
    lo, hi = F32(-half), F32(half)
    n = o.shape[0]
    t0 = np.zeros(n, dtype=F32)
    t1 = np.full(n, np.inf, dtype=F32)
    valid = np.isfinite(o).all(axis=1) & np.isfinite(d).all(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            da, oa = d[:, a], o[:, a]
            nz = da != 0
            ta = (lo - oa) / da
            tb = (hi - oa) / da
            t0 = np.where(nz, np.maximum(t0, np.minimum(ta, tb)), t0)
            t1 = np.where(nz, np.minimum(t1, np.maximum(ta, tb)), t1)
            valid &= nz | ((oa >= lo) & (oa <= hi))
    valid &= t0 < t1
    return t0, t1, valid


@dataclass
class RenderResult:
    n_samples: np.ndarray         # int32 [n]
    n_reads: np.ndarray           # int32 [n]
    t_final32: np.ndarray         # float32 [n] (decision mirror)
    t_final: np.ndarray           # float64 [n]
    c_d: np.ndarray               # float64 [n, 3]
    feat: np.ndarray              # float64 [n, 4]
    depth: np.ndarray             # float64 [n]
    rgb: np.ndarray               # float64 [n, 3]
    s_ray: np.ndarray             # int64 [S] samples sorted by (ray, k)
    s_k: np.ndarray               # int64 [S] lattice index of each sample
    s_t: np.ndarray               # float32 [S]
    s_pos: np.ndarray             # float32 [S, 3] grid-domain position
    extra: dict = field(default_factory=dict)


def march(inp: OracleInputs, o: np.ndarray, d: np.ndarray, naive: bool = False,
          terminate: bool = True, intervals=None, hi_guard: float = 0.0):
    """March all rays in lock-step over the lattice index k.

    intervals: optional float32 [n, 2] (t_lo, t_hi) restricting a ray to the
    lattice points with t in [t_lo, t_hi] (NaN rows: no restriction).  Box
    scenes start at lattice index max(0, floor((t_lo - t0) / step)); in the
    contracted domain points with t < t_lo are visited without a read.
    hi_guard > 0: a ray that reaches t > t_hi holding samples whose float32
    transmittance is not below hi_guard drops its t_hi and marches on.

    Returns per-ray sample lists and counts; transmittance decisions in the
    float32 mirror."""
    o = np.asarray(o, dtype=F32)
    d = np.asarray(d, dtype=F32)
    n = o.shape[0]
    R = inp.R
    RF = F32(R)
    step = F32(inp.step)
    thr = F32(inp.t_threshold) if terminate else F32(0.0)
    vox = (F32(inp.roi_half) - F32(-inp.roi_half)) / RF
    T = np.ones(n, dtype=F32)
    nsamp = np.zeros(n, dtype=np.int64)
    nreads = np.zeros(n, dtype=np.int64)
    nmem = np.zeros(n, dtype=np.int64)          # pyramid: grid words read
    dn2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    dn = sqrt32(dn2)
    if inp.domain == BOX:
        t0, t1, alive = ray_box32(o, d, inp.roi_half)
        alive &= dn2 > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            rho = (vox / step) / dn
        next_read = np.zeros(n, dtype=np.int64)
    else:
        alive = np.isfinite(o).all(axis=1) & np.isfinite(d).all(axis=1) & (dn2 > 0)
        t = np.zeros(n, dtype=F32)
        has_ball = np.zeros(n, dtype=bool)
        ball_c = np.zeros((n, 3), dtype=F32)
        ball_r2 = np.zeros(n, dtype=F32)
        margin = vox * F32(1.0 / 1024.0)
    t_lo = np.full(n, -np.inf, dtype=F32)
    t_hi = np.full(n, np.inf, dtype=F32)
    stopped_hi = np.zeros(n, dtype=bool)
    if intervals is not None:
        iv = np.asarray(intervals, dtype=F32)
        use = ~np.isnan(iv[:, 0])
        t_lo[use] = iv[use, 0]
        t_hi[use] = iv[use, 1]
        if inp.domain == BOX:
            with np.errstate(invalid="ignore"):
                kf = np.floor((t_lo - t0) / step)
            kstart = np.where(kf > 0, np.where(kf < F32(MAX_LATTICE), kf, F32(MAX_LATTICE)), 0)
            next_read = np.where(use, kstart, 0).astype(np.int64)
    rec_ray, rec_k, rec_t, rec_pos, rec_T = [], [], [], [], []
    k = 0
    while alive.any() and k < MAX_LATTICE:
        ids = np.nonzero(alive)[0]
        if inp.domain == BOX:
            tk = t0[ids] + F32(k) * step
            if hi_guard > 0:
                go_on = (tk > t_hi[ids]) & (nsamp[ids] > 0) & ~(T[ids] < F32(hi_guard))
                t_hi[ids[go_on]] = np.inf
            at_hi = (tk < t1[ids]) & (tk > t_hi[ids])
            stopped_hi[ids[at_hi]] = True
            inside = (tk < t1[ids]) & ~(tk > t_hi[ids])
            alive[ids[~inside]] = False
            ids, tk = ids[inside], tk[inside]
            pos = o[ids] + tk[:, None] * d[ids]
            if naive:
                need = np.ones(len(ids), dtype=bool)
                if intervals is not None:
                    need = k >= next_read[ids]
            else:
                need = k >= next_read[ids]
        else:
            tk = t[ids]
            if hi_guard > 0:
                go_on = (tk > t_hi[ids]) & (nsamp[ids] > 0) & ~(T[ids] < F32(hi_guard))
                t_hi[ids[go_on]] = np.inf
            at_hi = tk > t_hi[ids]               # checked before the exit test
            stopped_hi[ids[at_hi]] = True
            alive[ids[at_hi]] = False
            ids, tk = ids[~at_hi], tk[~at_hi]
            x = o[ids] + tk[:, None] * d[ids]
            r2 = (x[:, 0] * x[:, 0] + x[:, 1] * x[:, 1]) + x[:, 2] * x[:, 2]
            outer = r2 > F32(1.0)
            pos = x.copy()
            jn = dn[ids].copy()
            with np.errstate(divide="ignore", invalid="ignore"):
                r = sqrt32(r2)
                inv_r = F32(1.0) / r
                s = (F32(2.0) - inv_r) * inv_r
                xd = ((x[:, 0] * d[ids, 0] + x[:, 1] * d[ids, 1]) + x[:, 2] * d[ids, 2]) * inv_r
                perp2 = np.maximum(dn2[ids] - xd * xd, F32(0.0))
                rad = xd * (inv_r * inv_r)
                jn_o = sqrt32((s * s) * perp2 + rad * rad)
            pos[outer] = s[outer, None] * x[outer]
            jn[outer] = jn_o[outer]
            gone = (outer & (inv_r < step) & (xd >= F32(0.0))) | ~np.isfinite(r2)
            alive[ids[gone]] = False
            keep = ~gone
            ids, tk, pos, jn = ids[keep], tk[keep], pos[keep], jn[keep]
            if naive:
                need = np.ones(len(ids), dtype=bool)
            else:
                dv = pos - ball_c[ids]
                dd = (dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1]) + dv[:, 2] * dv[:, 2]
                need = ~(has_ball[ids] & (dd < ball_r2[ids]))
            need &= ~(tk < t_lo[ids])
        # occupancy / distance read
        u = grid_coords32(inp, pos)
        q = np.clip(np.floor(u * RF), 0, R - 1).astype(np.int64)
        vflat = q[:, 0] + R * (q[:, 1] + R * q[:, 2])
        rd = ids[need]
        if inp.pyramid is not None:
            occv = _pyramid_read(inp, rd, u[need], pos[need], tk[need], o, d, vflat[need], naive,
                                 nreads, nmem, k, next_read if inp.domain == BOX else None,
                                 rho if inp.domain == BOX else None,
                                 None if inp.domain == BOX else (has_ball, ball_c, ball_r2, margin),
                                 step, vox)
        else:
            nreads[rd] += 1
            occv = inp.occ_flat[vflat[need]] != 0
            g = inp.dist_flat[vflat[need]].astype(np.int64)
        if not naive and inp.pyramid is None:
            if inp.domain == BOX:
                jf = np.floor(g.astype(F32) * rho[rd])
                jump = np.where(jf < F32(MAX_LATTICE), jf, F32(MAX_LATTICE)).astype(np.int64)
                upd = (~occv) & (g > 0)
                next_read[rd[upd]] = k + np.maximum(jump[upd], 1)
            else:
                upd = (~occv) & (g > 0)
                has_ball[rd] = upd
                rb = g.astype(F32) * vox - margin
                ball_r2[rd[upd]] = (rb * rb)[upd]
                ball_c[rd[upd]] = pos[need][upd]
        # samples
        smp = rd[occv]
        if len(smp):
            spos = pos[need][occv]
            su = u[need][occv]
            fz, _, _ = fused32(inp, su)
            sigma = exp32(fz[:, 0])
            e = exp32(-(sigma * step))
            T[smp] = T[smp] * e
            nsamp[smp] += 1
            rec_ray.append(smp)
            rec_k.append(np.full(len(smp), k, dtype=np.int64))
            rec_t.append(tk[need][occv])
            rec_pos.append(spos)
            rec_T.append(T[smp].copy())
            stop = (T[smp] < thr) | (nsamp[smp] >= inp.max_samples)
            alive[smp[stop]] = False
        if inp.domain == CONTRACT:
            with np.errstate(divide="ignore"):
                t[ids] = tk + step / jn
        k += 1
    if rec_ray:
        s_ray = np.concatenate(rec_ray)
        s_k = np.concatenate(rec_k)
        s_t = np.concatenate(rec_t).astype(F32)
        s_pos = np.concatenate(rec_pos).astype(F32)
        s_T = np.concatenate(rec_T).astype(F32)
        order = np.lexsort((s_k, s_ray))
        s_ray, s_k, s_t, s_pos, s_T = s_ray[order], s_k[order], s_t[order], s_pos[order], s_T[order]
    else:
        s_ray = np.zeros(0, np.int64)
        s_k = np.zeros(0, np.int64)
        s_t = np.zeros(0, F32)
        s_pos = np.zeros((0, 3), F32)
        s_T = np.zeros(0, F32)
    return dict(n_samples=nsamp.astype(np.int32), n_reads=nreads.astype(np.int32),
                t_final32=T, s_ray=s_ray, s_k=s_k, s_t=s_t, s_pos=s_pos, s_T=s_T,
                stopped_hi=stopped_hi, n_mem=nmem)


def _pyramid_read(inp, rd, u, pos, tk, o, d, vflat, naive, nreads, nmem, k, next_read, rho, ball,
                  step, vox):
    """Reads and skip decisions of the multi-level occupancy march at the
    lattice points of rays rd (see oracle.pyramid); returns the sampled mask."""
    pyr = inp.pyramid
    R0 = pyr[0].shape[0]
    nreads[rd] += 1                               # one marching point each
    if naive:
        q0 = np.clip(np.floor(u * F32(R0)), 0, R0 - 1).astype(np.int64)
        nmem[rd] += 1
        return pyr[0][q0[:, 2], q0[:, 1], q0[:, 0]] != 0
    lev, reads, qx = pyramid.exit_level(pyr, u)
    empty = lev >= 0
    r_lev = np.where(empty, R0 >> np.maximum(lev, 0), R0)
    use_g = inp.use_dist & empty & (r_lev < inp.R)
    g = np.where(use_g, inp.dist_flat[vflat].astype(np.int64), 0)
    nmem[rd] += reads + use_g                     # grid words read
    h = F32(inp.roi_half)
    vj = ((h - (-h)) / r_lev.astype(F32)).astype(F32)
    if ball is None:                              # box domain: lattice jumps
        with np.errstate(invalid="ignore"):
            t_exit = pyramid.voxel_exit_t(o[rd], d[rd], qx, -h, vj)
            jo = np.floor((t_exit - tk) / step)
            jo = np.where(np.isnan(jo), F32(1.0), jo)
            jo = np.clip(jo, 1, MAX_LATTICE).astype(np.int64)
            jg = np.floor(g.astype(F32) * rho[rd])
            jg = np.where(jg < F32(MAX_LATTICE), jg, F32(MAX_LATTICE)).astype(np.int64)
        jg = np.where(use_g & (g > 0), jg, 0)
        jump = np.maximum(jo, jg)
        next_read[rd[empty]] = k + jump[empty]
    else:                                         # contracted domain: known-empty balls
        has_ball, ball_c, ball_r2, margin = ball
        r_o = pyramid.inscribed_radius(pos, qx, -h, vj) - margin
        r_g = np.where(use_g & (g > 0), g.astype(F32) * vox - margin, F32(-np.inf)).astype(F32)
        rb = np.maximum(r_o, r_g).astype(F32)
        upd = empty & (rb > 0)
        has_ball[rd] = upd
        ball_r2[rd[upd]] = (rb * rb)[upd]
        ball_c[rd[upd]] = pos[upd]
    return ~empty


def mlp64(params: np.ndarray, x: np.ndarray, dims=(7, 16, 16, 3)) -> np.ndarray:
    """Deferred MLP: W2 relu(W1 relu(W0 x + b0) + b1) + b2 (float64)."""
    p = np.asarray(params, dtype=np.float64)
    i, h1, h2, o = dims
    off = 0
    W0 = p[off:off + h1 * i].reshape(h1, i); off += h1 * i
    b0 = p[off:off + h1]; off += h1
    W1 = p[off:off + h2 * h1].reshape(h2, h1); off += h2 * h1
    b1 = p[off:off + h2]; off += h2
    W2 = p[off:off + o * h2].reshape(o, h2); off += o * h2
    b2 = p[off:off + o]
    a1 = np.maximum(x @ W0.T + b0, 0.0)
    a2 = np.maximum(a1 @ W1.T + b1, 0.0)
    return a2 @ W2.T + b2


def deferred_mlp(inp: OracleInputs, c_d, feat, d):
    """MLP(C_d, F) or, with a 64-unit hidden layer, the view-dependent
    MLP_psi(C_d, F, SH(d)) (Eq. 5)."""
    if tuple(inp.mlp_dims) == sh.DIMS_VIEW:
        return sh.mlp_view64(inp.mlp, c_d, feat, np.asarray(d, np.float64))
    return mlp64(inp.mlp, np.concatenate([c_d, feat], axis=1), inp.mlp_dims)


def composite64(inp: OracleInputs, n: int, s_ray, s_t, fused):
    """Front-to-back compositing of decided samples (float64)."""
    sigma = np.exp(fused[:, 0])
    alpha = 1.0 - np.exp(-sigma * float(F32(inp.step)))
    c_d = np.zeros((n, 3))
    feat = np.zeros((n, 4))
    depth = np.zeros(n)
    T = np.ones(n)
    # samples are sorted by (ray, k): walk them by their rank within the ray
    if len(s_ray):
        starts = np.r_[0, np.nonzero(np.diff(s_ray))[0] + 1]
        rank = np.arange(len(s_ray)) - np.repeat(starts, np.diff(np.r_[starts, len(s_ray)]))
        for r in range(int(rank.max()) + 1):
            sel = rank == r
            rays = s_ray[sel]
            w = T[rays] * alpha[sel]
            c_d[rays] += w[:, None] * fused[sel, 1:4]
            feat[rays] += w[:, None] * fused[sel, 4:8]
            depth[rays] += w * s_t[sel].astype(np.float64)
            T[rays] = T[rays] * (1.0 - alpha[sel])
    return c_d, feat, depth, T


def render(inp: OracleInputs, o: np.ndarray, d: np.ndarray, naive: bool = False,
           terminate: bool = True, coords: str = "f32") -> RenderResult:
    """coords: "f32" evaluates the decided samples at their float32 grid
    coordinates (the lattice's own positions); "f64" recomputes each
    position in float64 from (o, d, t) (sample_coords64)."""
    o = np.asarray(o, dtype=F32)
    n = o.shape[0]
    m = march(inp, o, d, naive=naive, terminate=terminate)
    if len(m["s_ray"]):
        if coords == "f64":
            u = sample_coords64(inp, o, np.asarray(d, dtype=F32), m["s_ray"], m["s_t"])
        else:
            u = grid_coords32(inp, m["s_pos"]).astype(np.float64)
        fz, _ = fused64(inp, u)
    else:
        fz = np.zeros((0, 8))
    c_d, feat, depth, T = composite64(inp, n, m["s_ray"], m["s_t"], fz)
    rgb = 1.0 / (1.0 + np.exp(-(c_d + deferred_mlp(inp, c_d, feat, d))))
    return RenderResult(n_samples=m["n_samples"], n_reads=m["n_reads"],
                        t_final32=m["t_final32"], t_final=T, c_d=c_d, feat=feat,
                        depth=depth, rgb=rgb, s_ray=m["s_ray"], s_k=m["s_k"],
                        s_t=m["s_t"], s_pos=m["s_pos"], extra={"s_T": m["s_T"], "n_mem": m["n_mem"]})


def scene_occupancy(scene) -> np.ndarray:
    """The occupancy grid behind the distance grid (Sec. 4.3): the scene's
    single grid, or, for an occupancy pyramid, its level of resolution
    occ_res, OR-pooled here from the finest level."""
    if getattr(scene, "occ_fine", None) is not None:
        for level in pyramid.build_pyramid(scene.occ_fine, scene.cfg.occ_levels):
            if level.shape[0] == scene.cfg.occ_res:
                return level
        raise ValueError("occ_res is not a resolution of the occupancy pyramid")
    return scene.occ


def inputs_from_scene(scene, dist: np.ndarray, dtype: int = DT_F32) -> OracleInputs:
    cfg = scene.cfg
    extra = {}
    if getattr(scene, "occ_fine", None) is not None:
        extra.update(pyramid=pyramid.build_pyramid(scene.occ_fine, cfg.occ_levels))
    if getattr(scene, "block_index", None) is not None:
        extra.update(coarse_res=cfg.coarse_res, block_index=scene.block_index, atlas=scene.atlas,
                     coarse_default=scene.default, aggregation=getattr(cfg, "aggregation", 0),
                     gate_params=tuple(np.asarray(getattr(cfg, "gate_params", ()), F32)))
    return OracleInputs(tables=scene.tables, occ=scene_occupancy(scene), dist=dist, mlp=scene.mlp,
                        resolutions=list(cfg.resolutions), domain=cfg.domain,
                        roi_half=cfg.roi_half, step=cfg.step, max_samples=cfg.max_samples,
                        t_threshold=cfg.t_threshold, dtype=dtype, mlp_dims=cfg.mlp_dims, **extra)


def valid_rays(inp: OracleInputs, o, d):
    """Rays the march accepts: finite, nonzero direction, and (box) hitting the ROI."""
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    dn2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    if inp.domain == BOX:
        return ray_box32(o, d, inp.roi_half)[2] & (dn2 > 0)
    return np.isfinite(o).all(axis=1) & np.isfinite(d).all(axis=1) & (dn2 > 0)


def render_proposal(inp: OracleInputs, o, d, proposal, conf_threshold=0.9, margin=0.0, use_near=True,
                    far_guard=0.0):
    """Render with a per-ray proposal [t_near, t_far, t_term, conf] (an
    extension).  A ray with conf >= conf_threshold marches only the lattice
    points with t in [t_near - margin, t_far + margin] (use_near false: from
    its start); with far_guard > 0 the far end stops a ray only once its
    transmittance is below far_guard, else the ray marches on.  If the padded
    interval holds no occupied lattice point the ray marches again from its
    start as the plain march (its samples are then the plain march's, its
    read count the sum of both marches).  Other rays march plainly.  Returns
    the result and the fallback mask."""
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    n = len(o)
    prop = np.asarray(proposal, F32)
    conf = prop[:, 3] >= F32(conf_threshold)
    iv = np.full((n, 2), np.nan, F32)
    iv[conf, 0] = prop[conf, 0] - F32(margin) if use_near else -np.inf
    iv[conf, 1] = prop[conf, 1] + F32(margin)
    m = march(inp, o, d, intervals=iv, hi_guard=far_guard)
    plain = march(inp, o, d)
    fb = conf & (m["n_samples"] == 0)
    if fb.any():
        idx = np.nonzero(fb)[0]
        keep = ~np.isin(m["s_ray"], idx)
        take = np.isin(plain["s_ray"], idx)
        for key in ("s_ray", "s_k", "s_t", "s_pos", "s_T"):
            m[key] = np.concatenate([m[key][keep], plain[key][take]])
        order = np.lexsort((m["s_k"], m["s_ray"]))
        for key in ("s_ray", "s_k", "s_t", "s_pos", "s_T"):
            m[key] = m[key][order]
        m["n_reads"][idx] = m["n_reads"][idx] + plain["n_reads"][idx]
        for key in ("n_samples", "t_final32"):
            m[key][idx] = plain[key][idx]
    if len(m["s_ray"]):
        fz, _ = fused64(inp, grid_coords32(inp, m["s_pos"]).astype(np.float64))
    else:
        fz = np.zeros((0, 8))
    c_d, feat, depth, T = composite64(inp, n, m["s_ray"], m["s_t"], fz)
    rgb = 1.0 / (1.0 + np.exp(-(c_d + deferred_mlp(inp, c_d, feat, d))))
    res = RenderResult(n_samples=m["n_samples"], n_reads=m["n_reads"], t_final32=m["t_final32"],
                       t_final=T, c_d=c_d, feat=feat, depth=depth, rgb=rgb, s_ray=m["s_ray"],
                       s_k=m["s_k"], s_t=m["s_t"], s_pos=m["s_pos"], extra={"s_T": m["s_T"]})
    return res, fb
