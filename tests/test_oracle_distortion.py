"""Pins of the distortion regulariser and the step auto-tuning rule
(supplement Eq. S2, S3): the prefix-sum form against the double sum, closed
forms for one and two samples, the gradient against central differences,
and the gamma recurrence's fixed points and bounds."""
import numpy as np
import pytest

from oracle import distortion as D


def test_prefix_form_equals_double_sum():
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 40):
        w = rng.random(n)
        t = np.sort(rng.random(n)) * 3
        dl = np.full(n, 0.01)
        loss, _ = D.dist_loss_and_grad(w, t, dl)
        assert abs(loss - D.dist_loss_bruteforce(w, t, dl)) < 1e-12


def test_closed_forms():
    loss, g = D.dist_loss_and_grad([0.7], [1.0], [0.2])
    assert abs(loss - 0.7 ** 2 * 0.2 / 3) < 1e-15
    assert abs(g[0] - 2 / 3 * 0.7 * 0.2) < 1e-15
    w, t, dl = [0.3, 0.5], [1.0, 2.0], [0.1, 0.1]
    want = 2 * 0.3 * 0.5 * 1.0 + (0.09 + 0.25) * 0.1 / 3
    loss, g = D.dist_loss_and_grad(w, t, dl)
    assert abs(loss - want) < 1e-15
    assert abs(g[0] - (2 * 0.5 * 1.0 + 2 / 3 * 0.3 * 0.1)) < 1e-15


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    w = rng.random(12)
    t = np.sort(rng.random(12)) * 2
    dl = rng.random(12) * 0.05
    _, g = D.dist_loss_and_grad(w, t, dl)
    h = 1e-6
    for i in range(12):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (D.dist_loss_bruteforce(wp, t, dl) - D.dist_loss_bruteforce(wm, t, dl)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7


def test_autotune_gamma_recurrence():
    g = 1.0
    for _ in range(10):
        g = D.autotune_gamma(g, 5.0)                    # enough samples: stays at 1
    assert g == 1.0
    g = D.autotune_gamma(1.0, 2.0)
    assert abs(g - 0.999) < 1e-15
    for _ in range(5000):
        g = D.autotune_gamma(g, 0.5)                    # collapses to the floor
    assert g == D.GAMMA_MIN
    g2 = D.autotune_gamma(g, 3.0)                       # N_min reached: grows by (1 + kappa)
    assert abs(g2 - D.GAMMA_MIN * 1.001) < 1e-15
