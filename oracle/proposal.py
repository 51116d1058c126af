"""Learned per-ray sample-interval proposal (an extension: the paper only
mentions adaptive sampling as orthogonal related work, Sec. 2).

Network: r = [o; d] (6-D) -> Fourier features sin/cos(2^k pi r_j), k = 0..3
(48-D, feature 8j + 2k = sin, 8j + 2k + 1 = cos) -> 64 -> 64 -> 4, ReLU
hidden layers, outputs [t_near, t_far, t_term, conf logit].  Parameters,
flattened: W1[64][48], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
(7556 values).

Labels come from the plain renderer's decided samples: t_near = t of the
first evaluated sample; t_far = t of the sample after which the
transmittance first drops below 1e-3 (the last sample's t if it never does;
the paper's own renderer stops at 2e-3, supplement "Real-time Rendering"
item 2, and the workload at 1e-4: beyond 1e-3 a ray's remaining colour weight
is below 0.1 %); t_term = t of the sample after which the transmittance first
drops below 0.5 (the last sample's t if never); rays without samples are
marked invalid.

Loss per batch of n rays (sums divided by n), over valid rays:
  t_near  pinball loss at quantile 0.05 (the prediction learns to sit low),
  t_far   pinball loss at quantile 0.95 (learns to sit high),
  t_term  squared error;
  pinball_q(r) = q r for r = y - pred >= 0, else (q - 1) r.
Second phase adds the binary cross-entropy of sigmoid(out_3) against
target = valid and [out_0 - m, out_1 + m] contains [y_0, y_1].

The GPU trains with bfloat16 GEMM operands and float32 accumulation; the
oracle reproduces the operand rounding (bf16_operands=True) and computes in
float64, so the two agree up to accumulation order.
"""
from __future__ import annotations

import numpy as np

from . import quant

N_FREQ = 4
N_IN, N_H, N_OUT = 48, 64, 4
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_OUT * N_H + N_OUT   # 7556


def fourier(o: np.ndarray, d: np.ndarray) -> np.ndarray:
    r = np.concatenate([np.asarray(o, np.float64), np.asarray(d, np.float64)], axis=1)
    enc = np.empty((r.shape[0], N_IN))
    for j in range(6):
        for k in range(N_FREQ):
            a = (2.0 ** k) * np.pi * r[:, j]
            enc[:, 8 * j + 2 * k] = np.sin(a)
            enc[:, 8 * j + 2 * k + 1] = np.cos(a)
    return enc


def split(p):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    W3 = p[o:o + N_OUT * N_H].reshape(N_OUT, N_H); o += N_OUT * N_H
    b3 = p[o:o + N_OUT]
    return W1, b1, W2, b2, W3, b3


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fin, fout in ((N_IN, N_H), (N_H, N_H), (N_H, N_OUT)):
        a = np.sqrt(6.0 / fin)
        parts.append(rng.uniform(-a, a, size=(fout, fin)).ravel())
        parts.append(np.zeros(fout))
    return np.concatenate(parts).astype(np.float32)


def _q(x, on):
    """Round to bfloat16 through float32 (as the GPU casts float32 values)."""
    if not on:
        return np.asarray(x, np.float64)
    return quant.bf16_decode(quant.bf16_encode(np.asarray(x, np.float32))).astype(np.float64)


def forward(p, enc, bf16_operands=True):
    W1, b1, W2, b2, W3, b3 = split(p)
    q = lambda x: _q(x, bf16_operands)
    z1 = q(enc) @ q(W1).T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = q(h1) @ q(W2).T + b2
    h2 = np.maximum(z2, 0.0)
    out = q(h2) @ q(W3).T + b3
    return dict(enc=enc, z1=z1, h1=h1, z2=z2, h2=h2, out=out)


def conf_target(out, labels, valid, margin):
    return (valid & (out[:, 0] - margin <= labels[:, 0]) & (out[:, 1] + margin >= labels[:, 1])).astype(np.float64)


Q_NEAR, Q_FAR = 0.05, 0.95


def _pinball(pred, y, q):
    r = y - pred
    loss = np.where(r >= 0, q * r, (q - 1.0) * r)
    grad = np.where(pred > y, 1.0 - q, -q)
    return loss, grad


def loss_and_grad_out(out, labels, valid, phase, margin):
    """Loss and dL/dout for one batch."""
    n = out.shape[0]
    v = valid.astype(np.float64)
    l0, g0 = _pinball(out[:, 0], labels[:, 0], Q_NEAR)
    l1, g1 = _pinball(out[:, 1], labels[:, 1], Q_FAR)
    df = out[:, 2] - labels[:, 2]
    loss = float(np.sum(v * (l0 + l1 + df * df))) / n
    g = np.zeros_like(out)
    g[:, 0] = v * g0 / n
    g[:, 1] = v * g1 / n
    g[:, 2] = v * 2.0 * df / n
    if phase >= 2:
        tgt = conf_target(out, labels, valid, margin)
        s = 1.0 / (1.0 + np.exp(-out[:, 3]))
        eps = 1e-12
        loss += float(-np.sum(tgt * np.log(s + eps) + (1 - tgt) * np.log(1 - s + eps))) / n
        g[:, 3] = (s - tgt) / n
    return loss, g


def backward(p, fwd, g_out, bf16_operands=True):
    W1, b1, W2, b2, W3, b3 = split(p)
    q = lambda x: _q(x, bf16_operands)
    go = q(g_out)
    gW3 = go.T @ q(fwd["h2"])
    gb3 = g_out.sum(axis=0)
    gz2 = (go @ q(W3)) * (fwd["z2"] > 0)
    gW2 = q(gz2).T @ q(fwd["h1"])
    gb2 = gz2.sum(axis=0)
    gz1 = (q(gz2) @ q(W2)) * (fwd["z1"] > 0)
    gW1 = q(gz1).T @ q(fwd["enc"])
    gb1 = gz1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


T_FAR = np.float32(1e-3)
T_TERM = np.float32(0.5)


def labels_from_march(n_rays, s_ray, s_t, s_T):
    """(t_near, t_far, t_term, valid) per ray from decided samples sorted by
    (ray, k) with the float32 transmittance after each sample."""
    lab = np.zeros((n_rays, 4), np.float32)
    valid = np.zeros(n_rays, bool)
    if len(s_ray) == 0:
        return lab, valid
    starts = np.r_[0, np.nonzero(np.diff(s_ray))[0] + 1]
    ends = np.r_[starts[1:], len(s_ray)]
    rays = s_ray[starts]
    valid[rays] = True
    lab[rays, 0] = s_t[starts]
    for a, b, r in zip(starts, ends, rays):
        for col, thr in ((1, T_FAR), (2, T_TERM)):
            below = np.nonzero(s_T[a:b] < thr)[0]
            lab[r, col] = s_t[a + below[0]] if len(below) else s_t[b - 1]
    lab[:, 3] = valid
    return lab, valid
