"""GPU backward (hand-written kernels through the C ABI) against the oracle's
float64 analytic gradients and central finite differences, plus the Adam
kernel and the autograd wrapper."""
import numpy as np
import pytest

import synth
from oracle.distgrid import distance_grid_edt
from oracle.grad import (adam_step as adam64, backward64, fd_table_grad, forward64, frozen_samples,
                         mse_grad, pick_entries)
from oracle.render import inputs_from_scene, render

from helpers import gpu_renderer, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _problem(stride=8):
    sc, dist = scene_and_dist("tiny")
    cfg = sc.cfg
    teacher = synth.make_scene(cfg, seed=1)
    inp = inputs_from_scene(sc, dist)
    tinp = inputs_from_scene(teacher, dist)
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::stride], d[::stride]
    target = render(tinp, o, d).rgb
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    tab = sc.tables.astype(np.float64)
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos)
    g_rgb = mse_grad(f["rgb"], target)
    return cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb


def _gpu_grads(o, d, g_rgb):
    import torch
    r = gpu_renderer("tiny")
    go, gd, gg = to_gpu(o, d, g_rgb.astype(np.float32))
    gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
    gm = torch.zeros((451,), dtype=torch.float32, device="cuda")
    r.backward(go, gd, gg, gt, gm)
    torch.cuda.synchronize()
    return _np(gt), _np(gm)


def test_backward_matches_oracle_analytic():
    print("[backward vs oracle]", flush=True)
    cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb = _problem()
    gtab64, gmlp64, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, g_rgb)
    gt, gm = _gpu_grads(o, d, g_rgb)
    scale = np.abs(gtab64).max()
    err = np.abs(gt - gtab64)
    assert np.all(err <= 1e-4 * scale + 1e-3 * np.abs(gtab64)), err.max() / scale
    assert np.array_equal(gt == 0, gtab64 == 0)
    assert np.allclose(gm, gmlp64, rtol=1e-3, atol=1e-5 * np.abs(gmlp64).max())


def test_backward_matches_finite_differences_1000_entries():
    print("[backward vs FD]", flush=True)
    cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb = _problem()
    gt, _ = _gpu_grads(o, d, g_rgb)
    rng = np.random.default_rng(7)
    touched, untouched = pick_entries(gt.astype(np.float64), 900, 100, rng)
    fd = fd_table_grad(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target,
                       touched + untouched, h=1e-3)
    an = np.array([gt[e] for e in touched + untouched], dtype=np.float64)
    scale = np.abs(an).max()
    assert np.all(np.abs(an - fd) <= 2e-4 * scale + 2e-3 * np.abs(fd)), np.abs(an - fd).max() / scale
    assert np.all(an[len(touched):] == 0) and np.all(fd[len(touched):] == 0)


def test_backward_run_to_run_spread():
    cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb = _problem(16)
    a, am = _gpu_grads(o, d, g_rgb)
    b, bm = _gpu_grads(o, d, g_rgb)
    assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()
    assert np.array_equal(am, bm)          # the MLP partials are reduced in a fixed order


def test_adam_kernel_matches_oracle():
    import torch
    from paper_2407_10482_amd.renderer import adam_step
    rng = np.random.default_rng(0)
    n = 100_003
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    gp, gm_, gv = to_gpu(p, m, v)
    p64, m64, v64 = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        (gg,) = to_gpu(g)
        adam_step(gp, gg, gm_, gv, step, 0.01)
        p64, m64, v64 = adam64(p64, g.astype(np.float64), m64, v64, step, 0.01)
    torch.cuda.synchronize()
    assert np.abs(_np(gp) - p64).max() < 1e-5


def test_autograd_function_and_training_reduces_loss():
    import torch
    from paper_2407_10482_amd.renderer import adam_step, render_differentiable
    print("[training steps]", flush=True)
    cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb = _problem(4)
    r = gpu_renderer("tiny")
    go, gd, gtarget = to_gpu(o, d, target.astype(np.float32))
    tables = torch.from_numpy(sc.tables).cuda().requires_grad_(True)
    mlp = torch.from_numpy(sc.mlp).cuda().requires_grad_(True)
    rgb = render_differentiable(r, tables, mlp, go, gd)
    loss = torch.mean((rgb - gtarget) ** 2)
    loss.backward()
    # the autograd path returns exactly what the direct call accumulates
    gt, gm = _gpu_grads(o, d, mse_grad(rgb.detach().cpu().numpy().astype(np.float64), target))
    assert np.abs(_np(tables.grad) - gt).max() <= 1e-6 * np.abs(gt).max()
    mt, vt = torch.zeros_like(tables), torch.zeros_like(tables)
    mm, vm = torch.zeros_like(mlp), torch.zeros_like(mlp)
    losses = []
    with torch.no_grad():
        tabs, mlps = tables.detach().clone(), mlp.detach().clone()
    for step in range(1, 21):
        tabs.requires_grad_(True)
        mlps.requires_grad_(True)
        rgb = render_differentiable(r, tabs, mlps, go, gd)
        loss = torch.mean((rgb - gtarget) ** 2)
        loss.backward()
        losses.append(loss.item())
        with torch.no_grad():
            adam_step(tabs, tabs.grad, mt, vt, step, 0.01)
            adam_step(mlps, mlps.grad, mm, vm, step, 0.01)
        tabs.grad = None
        mlps.grad = None
        tabs, mlps = tabs.detach(), mlps.detach()
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_autograd_refuses_a_scene_changed_after_the_forward():
    """The backward recomputes the forward from the renderer's loaded scene:
    a load (here another model's tables) between forward and backward is
    refused instead of giving the other model's gradients."""
    import torch
    from paper_2407_10482_amd.renderer import render_differentiable
    print("[autograd: scene changed]", flush=True)
    cfg, sc, o, d, target, s_ray, s_pos, tab, g_rgb = _problem(16)
    r = gpu_renderer("tiny")
    go, gd = to_gpu(o, d)
    tables = torch.from_numpy(sc.tables).cuda().requires_grad_(True)
    mlp = torch.from_numpy(sc.mlp).cuda().requires_grad_(True)
    rgb = render_differentiable(r, tables, mlp, go, gd)
    other = synth.make_scene(cfg, seed=1)
    r.load_tables(torch.from_numpy(other.tables).cuda())
    with pytest.raises(RuntimeError, match="changed between"):
        rgb.sum().backward()
    # a fresh forward on the current scene differentiates as usual
    rgb2 = render_differentiable(r, tables, mlp, go, gd)
    rgb2.sum().backward()
    torch.cuda.synchronize()
    assert tables.grad is not None and torch.isfinite(tables.grad).all()
