"""Pins of the oracle's analytic gradients: central finite differences in
float64 (h = 1e-3), untouched entries exactly zero, softmax shift
invariance, and the Adam update against its closed form."""
import numpy as np
import pytest

import synth
from oracle.distgrid import distance_grid_edt
from oracle.grad import (adam_step, backward64, fd_mlp_grad, fd_table_grad, forward64,
                         frozen_samples, loss64, mse_grad, pick_entries)
from oracle.render import inputs_from_scene, render, scene_occupancy


def _setup(n_rays_stride=8):
    cfg = synth.tiny()
    sc = synth.make_scene(cfg)
    teacher = synth.make_scene(cfg, seed=1)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::n_rays_stride], d[::n_rays_stride]
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    tab = sc.tables.astype(np.float64)
    target = forward64(teacher.tables.astype(np.float64), teacher.mlp, cfg.resolutions, cfg.step,
                       len(o), s_ray, s_pos)["rgb"]
    return cfg, sc, inp, o, d, s_ray, s_pos, tab, target


def test_forward64_matches_render_values():
    cfg, sc, inp, o, d, s_ray, s_pos, tab, target = _setup(16)
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos)
    r = render(inp, o, d)
    assert np.allclose(f["rgb"], r.rgb, atol=1e-12)
    assert np.allclose(f["c_d"], r.c_d, atol=1e-12)


@pytest.mark.parametrize("n_touched,n_untouched", [(90, 10)])
def test_table_gradient_matches_finite_differences(n_touched, n_untouched):
    cfg, sc, inp, o, d, s_ray, s_pos, tab, target = _setup(8)
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos)
    g = mse_grad(f["rgb"], target)
    gtab, gmlp, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, g)
    rng = np.random.default_rng(0)
    tch, unt = pick_entries(gtab, n_touched, n_untouched, rng)
    fd = fd_table_grad(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target, tch + unt)
    an = np.array([gtab[e] for e in tch + unt])
    scale = np.abs(an).max()
    assert np.all(np.abs(an - fd) <= 1e-4 * scale + 1e-5 * np.abs(fd))
    assert np.all(an[len(tch):] == 0.0) and np.all(fd[len(tch):] == 0.0)


def test_mlp_gradient_matches_finite_differences():
    cfg, sc, inp, o, d, s_ray, s_pos, tab, target = _setup(8)
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos)
    gtab, gmlp, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos,
                               mse_grad(f["rgb"], target))
    params = list(range(0, 451, 11)) + [111, 127, 383, 399, 447, 450]
    # h = 1e-5: a +-1e-3 step on a first-layer weight or bias moves some rays
    # across a ReLU kink, where the loss is not differentiable
    fd = fd_mlp_grad(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target, params,
                     h=1e-5)
    assert np.allclose(gmlp[params], fd, rtol=1e-6, atol=1e-8 * np.abs(gmlp).max())


def test_logit_gradient_sums_to_zero():
    # adding one constant to every logit leaves the softmax unchanged, and the
    # trilinear weights of each level sum to one: the logit channel's gradient
    # summed over all entries of all levels is zero
    cfg, sc, inp, o, d, s_ray, s_pos, tab, target = _setup(8)
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos)
    gtab, _, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos,
                            mse_grad(f["rgb"], target))
    assert abs(gtab[:, :, 8].sum()) < 1e-12 * np.abs(gtab[:, :, 8]).sum()
    # and a finite difference of that uniform shift is zero
    base = loss64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target)
    t2 = tab.copy()
    t2[:, :, 8] += 0.37
    assert abs(loss64(t2, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target) - base) < 1e-14


def test_adam_closed_form_first_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    p1, m, v = adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # first bias-corrected step: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))


def test_distortion_gradient_matches_finite_differences():
    """The regulariser's gradient through the rendering weights (supplement
    Eq. S2): a loss sum_r g_r L_dist(r) differentiated analytically against
    central differences of the table entries."""
    from oracle.grad import ray_distortion
    cfg, sc, inp, o, d, s_ray, s_pos, tab, target = _setup(8)
    s_ray, s_pos, _, s_k = frozen_samples(inp, o, d, with_k=True)
    n = len(o)
    gd = np.random.default_rng(3).uniform(0.5, 1.5, size=n)
    gtab, _, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, n, s_ray, s_pos, np.zeros((n, 3)),
                            grad_dist=gd, s_k=s_k)
    rng = np.random.default_rng(4)
    tch, unt = pick_entries(gtab, 40, 5, rng)

    def loss(t64):
        f = forward64(t64, sc.mlp, cfg.resolutions, cfg.step, n, s_ray, s_pos)
        return float((gd * ray_distortion(n, s_ray, s_k, f["w"], cfg.step)[0]).sum())
    h = 1e-4
    an, fd = [], []
    for (l, t, ch) in tch + unt:
        orig = tab[l, t, ch]
        tab[l, t, ch] = orig + h
        lp = loss(tab)
        tab[l, t, ch] = orig - h
        lm = loss(tab)
        tab[l, t, ch] = orig
        fd.append((lp - lm) / (2 * h))
        an.append(gtab[l, t, ch])
    an, fd = np.array(an), np.array(fd)
    scale = np.abs(an).max()
    assert scale > 0
    assert np.all(np.abs(an - fd) <= 1e-4 * scale + 1e-4 * np.abs(fd)), np.abs(an - fd).max() / scale
    assert np.all(an[len(tch):] == 0.0)


def test_ray_distortion_matches_double_sum():
    from oracle import distortion
    from oracle.grad import ray_distortion
    s_ray = np.array([0, 0, 0, 2, 2])
    s_k = np.array([3, 4, 9, 0, 7])
    w = np.array([0.2, 0.3, 0.4, 0.6, 0.1])
    step = 0.01
    loss, _ = ray_distortion(3, s_ray, s_k, w, step)
    st = float(np.float32(step))
    assert abs(loss[0] - distortion.dist_loss_bruteforce(w[:3], s_k[:3] * st, [st] * 3)) < 1e-15
    assert loss[1] == 0.0
    assert abs(loss[2] - distortion.dist_loss_bruteforce(w[3:], s_k[3:] * st, [st] * 2)) < 1e-15
