"""Real spherical harmonics up to degree 3 (16 functions) of a unit
direction, and the view-dependent deferred MLP (test infrastructure).

The paper's MLP_psi (Eq. 5; supplement "Network Design") takes the
composited diffuse colour C_d, the specular feature F and a 16-dimensional
embedding of the view direction by spherical harmonics ("4-degree", i.e.
degrees l = 0..3), through two hidden layers of 64 ReLU units to 3 outputs;
C = sigmoid(C_d + MLP_psi(C_d, F, SH(d))).

Basis (orthonormal on the unit sphere, no Condon-Shortley phase), for
d = (x, y, z) with |d| = 1, in the order l = 0..3, m = -l..l:
  l=0: 1/2 sqrt(1/pi)
  l=1: sqrt(3/(4 pi)) * (y, z, x)
  l=2: 1/2 sqrt(15/pi) xy, 1/2 sqrt(15/pi) yz, 1/4 sqrt(5/pi) (3z^2 - 1),
       1/2 sqrt(15/pi) xz, 1/4 sqrt(15/pi) (x^2 - y^2)
  l=3: 1/4 sqrt(35/(2 pi)) y (3x^2 - y^2), 1/2 sqrt(105/pi) xyz,
       1/4 sqrt(21/(2 pi)) y (5z^2 - 1), 1/4 sqrt(7/pi) (5z^3 - 3z),
       1/4 sqrt(21/(2 pi)) x (5z^2 - 1), 1/4 sqrt(105/pi) z (x^2 - y^2),
       1/4 sqrt(35/(2 pi)) x (x^2 - 3y^2)
The direction is normalised first (d / |d|); a zero or non-finite direction
gives SH = 0.

MLP_psi parameters, flattened row-major (out x in): W0[64][23], b0[64],
W1[64][64], b1[64], W2[3][64], b2[3] (5891 values); input order
[C_d (3), F (4), SH (16)].
"""
from __future__ import annotations

import math

import numpy as np

N_SH = 16
DIMS_VIEW = (23, 64, 64, 3)
N_PARAMS_VIEW = 64 * 23 + 64 + 64 * 64 + 64 + 3 * 64 + 3      # 5891


def sh16(d: np.ndarray) -> np.ndarray:
    """[m, 16] float64 real SH of the directions d [m, 3]."""
    d = np.asarray(d, dtype=np.float64)
    n = np.linalg.norm(d, axis=1, keepdims=True)
    ok = np.isfinite(d).all(axis=1) & (n[:, 0] > 0)
    u = np.where(ok[:, None], d / np.where(n > 0, n, 1.0), 0.0)
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    pi = math.pi
    c0 = 0.5 * math.sqrt(1.0 / pi)
    c1 = math.sqrt(3.0 / (4.0 * pi))
    c2a = 0.5 * math.sqrt(15.0 / pi)
    c2b = 0.25 * math.sqrt(5.0 / pi)
    c2c = 0.25 * math.sqrt(15.0 / pi)
    c3a = 0.25 * math.sqrt(35.0 / (2.0 * pi))
    c3b = 0.5 * math.sqrt(105.0 / pi)
    c3c = 0.25 * math.sqrt(21.0 / (2.0 * pi))
    c3d = 0.25 * math.sqrt(7.0 / pi)
    c3e = 0.25 * math.sqrt(105.0 / pi)
    out = np.stack([
        np.full_like(x, c0),
        c1 * y, c1 * z, c1 * x,
        c2a * x * y, c2a * y * z, c2b * (3 * z * z - 1), c2a * x * z, c2c * (x * x - y * y),
        c3a * y * (3 * x * x - y * y), c3b * x * y * z, c3c * y * (5 * z * z - 1),
        c3d * (5 * z ** 3 - 3 * z), c3c * x * (5 * z * z - 1), c3e * z * (x * x - y * y),
        c3a * x * (x * x - 3 * y * y),
    ], axis=1)
    return np.where(ok[:, None], out, 0.0)


def mlp_view64(params: np.ndarray, c_d: np.ndarray, feat: np.ndarray, d: np.ndarray) -> np.ndarray:
    """MLP_psi(C_d, F, SH(d)) in float64 -> [m, 3]."""
    p = np.asarray(params, dtype=np.float64)
    i, h1, h2, o = DIMS_VIEW
    off = 0
    W0 = p[off:off + h1 * i].reshape(h1, i); off += h1 * i
    b0 = p[off:off + h1]; off += h1
    W1 = p[off:off + h2 * h1].reshape(h2, h1); off += h2 * h1
    b1 = p[off:off + h2]; off += h2
    W2 = p[off:off + o * h2].reshape(o, h2); off += o * h2
    b2 = p[off:off + o]
    x = np.concatenate([c_d, feat, sh16(d)], axis=1)
    a1 = np.maximum(x @ W0.T + b0, 0.0)
    a2 = np.maximum(a1 @ W1.T + b1, 0.0)
    return a2 @ W2.T + b2


def _split_view(params):
    p = np.asarray(params, dtype=np.float64)
    i, h1, h2, o = DIMS_VIEW
    sizes = [h1 * i, h1, h2 * h1, h2, o * h2, o]
    parts, off = [], 0
    for s in sizes:
        parts.append(p[off:off + s])
        off += s
    W0, b0, W1, b1, W2, b2 = parts
    return W0.reshape(h1, i), b0, W1.reshape(h2, h1), b1, W2.reshape(o, h2), b2


def mlp_view_backward64(params, c_d, feat, d, grad_rgb):
    """Adjoint of rgb = sigmoid(C_d + MLP_psi(C_d, F, SH(d))) in float64 for an
    upstream dL/drgb [m, 3]: dL/dC_d [m, 3], dL/dF [m, 4] and dL/dpsi [5891]
    (same flattened order as the parameters).  SH(d) is a constant input."""
    W0, b0, W1, b1, W2, b2 = _split_view(params)
    x = np.concatenate([np.asarray(c_d, np.float64), np.asarray(feat, np.float64), sh16(d)], axis=1)
    z1 = x @ W0.T + b0
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W1.T + b1
    a2 = np.maximum(z2, 0.0)
    out = a2 @ W2.T + b2
    rgb = 1.0 / (1.0 + np.exp(-(x[:, :3] + out)))
    gz = np.asarray(grad_rgb, np.float64) * rgb * (1.0 - rgb)       # dL/d(C_d + out)
    g2 = (gz @ W2) * (z2 > 0)
    g1 = (g2 @ W1) * (z1 > 0)
    gx = g1 @ W0
    g_params = np.concatenate([(g1.T @ x).ravel(), g1.sum(0), (g2.T @ a1).ravel(), g2.sum(0),
                               (gz.T @ a2).ravel(), gz.sum(0)])
    return gz + gx[:, :3], gx[:, 3:7], g_params
