"""Distortion regulariser and marching-step auto-tuning of the paper's
training (supplement "Loss Functions", Eq. S2, and "Auto-tuning of Marching
Step Size", Eq. S3); test infrastructure.

Distortion loss of one ray with rendering weights w_i on intervals
[t_i, t_i + delta_i] (the mip-NeRF 360 regulariser the paper adopts):
    L_dist = sum_{i,j} w_i w_j |m_i - m_j| + 1/3 sum_i w_i^2 delta_i,
    m_i = t_i + delta_i / 2.
Its derivative with respect to w_i:
    dL_dist/dw_i = 2 sum_j w_j |m_i - m_j| + 2/3 w_i delta_i.
With the samples in increasing t, sum_j w_j |m_i - m_j| =
m_i W_<i - S_<i + (S_>i - m_i W_>i), with W and S the sums of w_j and
w_j m_j over j < i or j > i, so both take one pass.

Step auto-tuning (Eq. S3): s = gamma s_0 with, after each batch,
gamma <- min(1, (1 + kappa) gamma) if the batch's mean sample count
reaches N_min, else max(gamma_min, (1 - kappa) gamma); the paper uses
N_min = 3, kappa = 0.001, gamma_min = 0.2217 and gamma = 1 at the start.
"""
from __future__ import annotations

import numpy as np

N_MIN, KAPPA, GAMMA_MIN = 3.0, 0.001, 0.2217


def dist_loss_bruteforce(w, t, delta):
    """L_dist of one ray by the double sum (float64)."""
    w = np.asarray(w, np.float64)
    m = np.asarray(t, np.float64) + 0.5 * np.asarray(delta, np.float64)
    return float((w[:, None] * w[None, :] * np.abs(m[:, None] - m[None, :])).sum()
                 + (w * w * np.asarray(delta, np.float64)).sum() / 3.0)


def dist_loss_and_grad(w, t, delta):
    """L_dist and dL_dist/dw of one ray by prefix sums (samples in
    increasing t; float64)."""
    w = np.asarray(w, np.float64)
    dl = np.asarray(delta, np.float64)
    m = np.asarray(t, np.float64) + 0.5 * dl
    W_lt = np.concatenate([[0.0], np.cumsum(w)[:-1]])
    S_lt = np.concatenate([[0.0], np.cumsum(w * m)[:-1]])
    W_gt = w.sum() - W_lt - w
    S_gt = (w * m).sum() - S_lt - w * m
    pair = m * W_lt - S_lt + (S_gt - m * W_gt)          # sum_j w_j |m_i - m_j|
    loss = float((w * pair).sum() + (w * w * dl).sum() / 3.0)
    grad = 2.0 * pair + (2.0 / 3.0) * w * dl
    return loss, grad


def autotune_gamma(gamma: float, mean_samples: float, n_min=N_MIN, kappa=KAPPA,
                   gamma_min=GAMMA_MIN) -> float:
    """One update of the step scaler gamma (Eq. S3)."""
    if mean_samples >= n_min:
        return min(1.0, (1.0 + kappa) * gamma)
    return max(gamma_min, (1.0 - kappa) * gamma)
