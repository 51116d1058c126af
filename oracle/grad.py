"""Analytic float64 gradients of the render path (an extension beyond the
paper, which trains but states no gradient code), and the finite-difference
loss they are checked against.

Per ray, with the sample list frozen (decided by the forward march):
  f_i = Att(Interp(levels, x_i))            fused channels [sigma_raw, c(3), v(4)]
  sigma_i = exp(f_i0), e_i = exp(-sigma_i delta), T_i = prod_{j<i} e_j,
  w_i = T_i (1 - e_i)                        (Eq. 2)
  C_d = sum w_i c_i, F = sum w_i v_i         (Eq. 5)
  C = sigmoid(C_d + MLP(C_d, F))             (Eq. 5 + supplement activations)
Loss (reading of the training objective used here): mean over rays and
colour channels of (C - C*)^2.

Backward, per ray:
  g_z = dL/dC * C (1 - C); MLP backprop gives dL/dW, dL/db and g_x = dL/d[C_d; F];
  g_Cd = g_z + g_x[:3], g_F = g_x[3:];
  s_i = g_Cd . c_i + g_F . v_i, S = sum_i w_i s_i = g_Cd . C_d + g_F . F,
  P_i = sum_{j<=i} w_j s_j;
  dL/dc_i = w_i g_Cd, dL/dv_i = w_i g_F,
  dL/dsigma_i = delta (T_{i+1} s_i - (S - P_i)),  dL/df_i0 = sigma_i dL/dsigma_i;
  attention (softmax over levels of the interpolated logits a_l):
  dL/dv_l = w_l dL/df, dL/dw_l = dL/df . v_l, dL/da_l = w_l (dL/dw_l - sum_k w_k dL/dw_k);
  trilinear: every corner entry receives its trilinear weight times the
  level's gradient (all 9 channels).
"""
from __future__ import annotations

import numpy as np

from . import baked, distortion
from .hashgrid import corners64
from .render import OracleInputs, grid_coords64, march, mlp64

MLP_DIMS = (7, 16, 16, 3)


def _split_mlp(p):
    p = np.asarray(p, dtype=np.float64)
    W0 = p[0:112].reshape(16, 7); b0 = p[112:128]
    W1 = p[128:384].reshape(16, 16); b1 = p[384:400]
    W2 = p[400:448].reshape(3, 16); b2 = p[448:451]
    return W0, b0, W1, b1, W2, b2


def frozen_samples(inp: OracleInputs, o, d, with_k: bool = False):
    """Sample lists decided by the forward march (no termination changes
    under the perturbations of a finite-difference check)."""
    m = march(inp, o, d)
    if with_k:
        return m["s_ray"], m["s_pos"], m["s_t"], m["s_k"]
    return m["s_ray"], m["s_pos"], m["s_t"]


def ray_distortion(n_rays, s_ray, s_k, w, step):
    """Per-ray distortion regulariser (supplement Eq. S2) on the lattice
    intervals [k step, (k + 1) step] and dL_dist/dw per sample."""
    step = float(np.float32(step))
    loss = np.zeros(n_rays)
    gw = np.zeros(len(s_ray))
    if len(s_ray):
        starts = np.r_[0, np.nonzero(np.diff(s_ray))[0] + 1]
        ends = np.r_[starts[1:], len(s_ray)]
        for a, b in zip(starts, ends):
            t = np.asarray(s_k[a:b], np.float64) * step
            l, g = distortion.dist_loss_and_grad(w[a:b], t, np.full(b - a, step))
            loss[s_ray[a]] = l
            gw[a:b] = g
    return loss, gw


def grid_u(s_pos, roi_half):
    """Float32 grid coordinates of sample positions, as float64."""
    lo = np.float32(-roi_half)
    inv = np.float32(1.0) / (np.float32(roi_half) - lo)
    return ((np.asarray(s_pos, np.float32) - lo) * inv).astype(np.float64)


def _levels64(tables64, resolutions, T, u):
    """Per-level interpolated values [m, L, 9], corner indices and weights."""
    vals, idxs, ws = [], [], []
    for l, N in enumerate(resolutions):
        idx, w = corners64(u, N, T)
        vals.append(np.einsum("mc,mcd->md", w, tables64[l][idx]))
        idxs.append(idx)
        ws.append(w)
    return np.stack(vals, axis=1), np.stack(idxs, axis=1), np.stack(ws, axis=1)


def forward64(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, roi_half=1.0, coarse=None):
    """Float64 forward on a frozen sample list; returns rgb and intermediates.
    coarse: None (hash model: tables64 are the hash levels, fused by softmax)
    or dict(atlas=, default=, block_index=, res=) for the baked model
    (tables64 are then the fine levels; see oracle.baked)."""
    T = tables64.shape[1]
    u = grid_u(s_pos, roi_half)
    if coarse is not None:
        fused, parts = baked.forward64_parts(coarse["atlas"], coarse["default"], coarse["block_index"],
                                             coarse["res"], tables64, resolutions, u)
        lv = idx = wc = wl = None
    else:
        parts = None
        lv, idx, wc = _levels64(tables64, resolutions, T, u)
        a = lv[:, :, 8]
        a = a - a.max(axis=1, keepdims=True)
        e = np.exp(a)
        wl = e / e.sum(axis=1, keepdims=True)
        fused = np.einsum("ml,mlc->mc", wl, lv[:, :, :8])
    sigma = np.exp(fused[:, 0])
    delta = float(np.float32(step))
    ee = np.exp(-sigma * delta)
    # per-ray transmittance before each sample (samples sorted by ray, k)
    Tb = np.ones(len(s_ray))
    if len(s_ray):
        logs = -sigma * delta
        cs = np.cumsum(logs)
        starts = np.r_[0, np.nonzero(np.diff(s_ray))[0] + 1]
        first = np.repeat(starts, np.diff(np.r_[starts, len(s_ray)]))
        before = cs - logs - np.where(first > 0, cs[first - 1], 0.0)
        Tb = np.exp(before)
    w = Tb * (1.0 - ee)
    c_d = np.zeros((n_rays, 3))
    feat = np.zeros((n_rays, 4))
    np.add.at(c_d, s_ray, w[:, None] * fused[:, 1:4])
    np.add.at(feat, s_ray, w[:, None] * fused[:, 4:8])
    x = np.concatenate([c_d, feat], axis=1)
    z1 = h1 = z2 = h2 = rgb = None
    if mlp is not None:                      # None: the caller handles the MLP (view-dependent)
        W0, b0, W1, b1, W2, b2 = _split_mlp(mlp)
        z1 = x @ W0.T + b0
        h1 = np.maximum(z1, 0)
        z2 = h1 @ W1.T + b1
        h2 = np.maximum(z2, 0)
        o = h2 @ W2.T + b2
        rgb = 1.0 / (1.0 + np.exp(-(c_d + o)))
    return dict(rgb=rgb, c_d=c_d, feat=feat, x=x, z1=z1, h1=h1, z2=z2, h2=h2, fused=fused,
                sigma=sigma, ee=ee, Tb=Tb, w=w, wl=wl, lv=lv, idx=idx, wc=wc, delta=delta,
                parts=parts)


def loss64(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, target, roi_half=1.0):
    f = forward64(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, roi_half)
    return float(np.mean((f["rgb"] - target) ** 2))


def backward64(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, grad_rgb, roi_half=1.0,
               grad_dist=None, s_k=None, coarse=None, upstream=None):
    """dL/dtables [L, T, 9] and dL/dmlp [451] for an upstream dL/drgb [n, 3]
    and, optionally, dL/d(distortion regulariser) per ray [n] (s_k: the
    samples' lattice indices).  The regulariser enters as dL/dw_i, which
    adds g_r dL_dist/dw_i to s_i and g_r sum_i w_i dL_dist/dw_i = 2 g_r L_dist
    to S.  With `coarse` (the baked model) the first result is the pair
    (dL/datlas [n_blocks, 8, 8, 8, C], dL/dfine tables [L, T, 9]).  With
    `upstream` = (dL/dC_d [n, 3], dL/dF [n, 4]) the MLP is skipped (grad_rgb
    unused, dL/dmlp None): the view-dependent MLP's adjoint supplies them."""
    f = forward64(tables64, None if upstream is not None else mlp, resolutions, step, n_rays, s_ray,
                  s_pos, roi_half, coarse)
    if upstream is not None:
        # dL/dC_d [n, 3] and dL/dF [n, 4] given (the view-dependent MLP's adjoint)
        g_cd, g_f = (np.asarray(a, np.float64) for a in upstream)
        gmlp = None
    else:
        W0, b0, W1, b1, W2, b2 = _split_mlp(mlp)
        rgb = f["rgb"]
        gz = grad_rgb * rgb * (1.0 - rgb)
        g_o = gz
        gW2 = g_o.T @ f["h2"]
        gb2 = g_o.sum(axis=0)
        gz2 = (g_o @ W2) * (f["z2"] > 0)
        gW1 = gz2.T @ f["h1"]
        gb1 = gz2.sum(axis=0)
        gz1 = (gz2 @ W1) * (f["z1"] > 0)
        gW0 = gz1.T @ f["x"]
        gb0 = gz1.sum(axis=0)
        gx = gz1 @ W0
        g_cd = gz + gx[:, :3]
        g_f = gx[:, 3:]
        gmlp = np.concatenate([gW0.ravel(), gb0, gW1.ravel(), gb1, gW2.ravel(), gb2])

    fused, w, Tb, ee, sigma = f["fused"], f["w"], f["Tb"], f["ee"], f["sigma"]
    s = (g_cd[s_ray] * fused[:, 1:4]).sum(axis=1) + (g_f[s_ray] * fused[:, 4:8]).sum(axis=1)
    S = (g_cd * f["c_d"]).sum(axis=1) + (g_f * f["feat"]).sum(axis=1)
    if grad_dist is not None:
        dl, gw = ray_distortion(n_rays, s_ray, s_k, w, step)
        gd = np.asarray(grad_dist, np.float64)
        s = s + gd[s_ray] * gw
        S = S + gd * 2.0 * dl
    ws = w * s
    P = np.zeros(len(s_ray))
    if len(s_ray):
        cs = np.cumsum(ws)
        starts = np.r_[0, np.nonzero(np.diff(s_ray))[0] + 1]
        first = np.repeat(starts, np.diff(np.r_[starts, len(s_ray)]))
        P = cs - np.where(first > 0, cs[first - 1], 0.0)
    T_after = Tb * ee
    g_sigma = f["delta"] * (T_after * s - (S[s_ray] - P))
    g_fused = np.zeros_like(fused)
    g_fused[:, 0] = g_sigma * sigma
    g_fused[:, 1:4] = w[:, None] * g_cd[s_ray]
    g_fused[:, 4:8] = w[:, None] * g_f[s_ray]
    if coarse is not None:
        atlas = coarse["atlas"]
        g_atlas, g_fine = baked.scatter64(f["parts"], g_fused, atlas.shape[0], atlas.shape[-1],
                                          tables64.shape)
        return (g_atlas, g_fine), gmlp, f
    wl, lv = f["wl"], f["lv"]
    g_v = wl[:, :, None] * g_fused[:, None, :]                   # [m, L, 8]
    g_w = np.einsum("mc,mlc->ml", g_fused, lv[:, :, :8])
    g_a = wl * (g_w - (wl * g_w).sum(axis=1, keepdims=True))
    g_lv = np.concatenate([g_v, g_a[:, :, None]], axis=2)      # [m, L, 9]
    gtab = np.zeros_like(tables64)
    idx, wc = f["idx"], f["wc"]
    for l in range(len(resolutions)):
        for c in range(8):
            np.add.at(gtab[l], idx[:, l, c], wc[:, l, c][:, None] * g_lv[:, l, :])
    return gtab, gmlp, f


def mse_grad(rgb, target):
    return 2.0 * (rgb - target) / rgb.size


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.99, eps=1e-8):
    """Adam (the paper's optimiser hyper-parameters: beta1 0.9, beta2 0.99,
    eps 1e-8; supplement "Optimization"), float64, bias-corrected."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def fd_table_grad(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, target, entries,
                  h=1e-3, roi_half=1.0):
    """Central finite differences of the loss w.r.t. table entries (l, t, ch).

    Only rays with a sample touching the entry change, so the loss
    difference is summed over those rays alone (same value, less work)."""
    T = tables64.shape[1]
    u = grid_u(s_pos, roi_half)
    idx = np.stack([corners64(u, N, T)[0] for N in resolutions], axis=1)   # [m, L, 8]
    out = []
    for (l, t, ch) in entries:
        hit = np.any(idx[:, l, :] == t, axis=1)
        rays = np.unique(s_ray[hit])
        if len(rays) == 0:
            out.append(0.0)
            continue
        keep = np.isin(s_ray, rays)
        sub_ray = np.searchsorted(rays, s_ray[keep])
        sub_pos = s_pos[keep]
        tgt = target[rays]
        orig = tables64[l, t, ch]
        vals = []
        for sgn in (1.0, -1.0):
            tables64[l, t, ch] = orig + sgn * h
            f = forward64(tables64, mlp, resolutions, step, len(rays), sub_ray, sub_pos, roi_half)
            vals.append(np.sum((f["rgb"] - tgt) ** 2))
        tables64[l, t, ch] = orig
        out.append((vals[0] - vals[1]) / (2 * h) / (3.0 * n_rays))
    return np.array(out)


def fd_mlp_grad(tables64, mlp, resolutions, step, n_rays, s_ray, s_pos, target, params, h=1e-3,
                roi_half=1.0):
    p = np.asarray(mlp, dtype=np.float64).copy()
    out = []
    for j in params:
        orig = p[j]
        vals = []
        for sgn in (1.0, -1.0):
            p[j] = orig + sgn * h
            vals.append(loss64(tables64, p, resolutions, step, n_rays, s_ray, s_pos, target, roi_half))
        p[j] = orig
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


def pick_entries(gtab, n_touched, n_untouched, rng):
    """Random (l, t, ch) entries: n_touched with a nonzero analytic gradient
    row, n_untouched from rows no sample reached."""
    L, T, C = gtab.shape
    touched = np.argwhere(np.any(gtab != 0, axis=2))
    untouched = np.argwhere(~np.any(gtab != 0, axis=2))
    a = touched[rng.choice(len(touched), size=min(n_touched, len(touched)), replace=False)]
    b = untouched[rng.choice(len(untouched), size=min(n_untouched, len(untouched)), replace=False)]
    ch_a = rng.integers(0, C, size=len(a))
    ch_b = rng.integers(0, C, size=len(b))
    return [(int(l), int(t), int(c)) for (l, t), c in zip(a, ch_a)], \
        [(int(l), int(t), int(c)) for (l, t), c in zip(b, ch_b)]
