"""Gradient parity at the shapes that are timed or shipped: the 16-level
backward instantiation (the 16 x 2^19 training measurement), the contracted
domain (the hd scene's geometry and tables), and the baked backward with
three and four fine levels.  Each is compared with the oracle's float64
analytic gradient and, for a few hundred entries, with central finite
differences of the float64 loss."""
import numpy as np
import pytest

import synth
from oracle.grad import backward64, fd_table_grad, forward64, frozen_samples, mse_grad, pick_entries
from oracle.render import inputs_from_scene

from helpers import gpu_renderer, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rays(name, n, seed):
    sc, dist = scene_and_dist(name)
    cfg = sc.cfg
    if cfg.domain == synth.DOMAIN_CONTRACT:
        cams = synth.camera_positions(cfg)[:2]
        o, d, _ = synth.scene_rays(cfg, cams=cams, width=256, height=128)
    else:
        o, d, _ = synth.scene_rays(cfg)
    sel = np.sort(np.random.default_rng(seed).choice(len(o), size=n, replace=False))
    return sc, dist, cfg, o[sel], d[sel]


def _hash_problem(name, n, seed=0):
    sc, dist, cfg, o, d = _rays(name, n, seed)
    inp = inputs_from_scene(sc, dist)
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    tab = sc.tables.astype(np.float64)
    target = np.random.default_rng(seed + 1).random((len(o), 3))
    f = forward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, roi_half=cfg.roi_half)
    return cfg, sc, o, d, s_ray, s_pos, tab, target, mse_grad(f["rgb"], target)


def _gpu_hash(name, o, d, g_rgb):
    import torch
    r = gpu_renderer(name)
    go, gd, gg = to_gpu(o, d, g_rgb.astype(np.float32))
    gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
    gm = torch.zeros((451,), dtype=torch.float32, device="cuda")
    r.backward(go, gd, gg, gt, gm)
    torch.cuda.synchronize()
    return _np(gt), _np(gm)


def _close(got, want, what):
    scale = np.abs(want).max()
    assert scale > 0, what
    err = np.abs(got - want)
    assert np.all(err <= 1e-4 * scale + 1e-3 * np.abs(want)), (what, err.max() / scale)
    assert np.all((got != 0) <= (want != 0)), what
    assert np.all(got[np.abs(want) > 1e-6 * scale] != 0), what


@pytest.mark.parametrize("name,n", [("train_large", 1024), ("hd", 384)])
def test_hash_backward_at_timed_shapes(name, n):
    """16 levels (16..4096, 2^19 entries): the box-domain training tables
    and the contracted hd scene."""
    print(f"[backward {name} {n} rays]", flush=True)
    cfg, sc, o, d, s_ray, s_pos, tab, target, g_rgb = _hash_problem(name, n)
    assert len(cfg.resolutions) == 16 and len(s_ray) > 0
    gtab64, gmlp64, _ = backward64(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, g_rgb,
                                   roi_half=cfg.roi_half)
    gt, gm = _gpu_hash(name, o, d, g_rgb)
    _close(gt, gtab64, "tables")
    assert np.allclose(gm, gmlp64, rtol=1e-3, atol=1e-5 * np.abs(gmlp64).max())
    rng = np.random.default_rng(5)
    touched, untouched = pick_entries(gtab64, 250, 50, rng)
    fd = fd_table_grad(tab, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, target,
                       touched + untouched, h=1e-3, roi_half=cfg.roi_half)
    an = np.array([gt[e] for e in touched + untouched], dtype=np.float64)
    scale = np.abs(an).max()
    assert np.all(np.abs(an - fd) <= 2e-4 * scale + 2e-3 * np.abs(fd)), np.abs(an - fd).max() / scale
    assert np.all(an[len(touched):] == 0) and np.all(fd[len(touched):] == 0)


@pytest.mark.parametrize("name", ["baked_tiny_l3", "baked_tiny_l4"])
def test_baked_backward_three_and_four_fine_levels(name):
    import torch
    print(f"[baked backward {name}]", flush=True)
    sc, dist = scene_and_dist(name)
    cfg = sc.cfg
    inp = inputs_from_scene(sc, dist)
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::8], d[::8]
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    coarse = dict(atlas=sc.atlas.astype(np.float64), default=sc.default.astype(np.float64),
                  block_index=sc.block_index, res=cfg.coarse_res)
    fine = sc.tables.astype(np.float64)
    target = np.random.default_rng(3).random((len(o), 3))
    f = forward64(fine, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, coarse=coarse)
    g_rgb = mse_grad(f["rgb"], target)
    (ga64, gf64), gm64, _ = backward64(fine, sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray, s_pos, g_rgb,
                                       coarse=coarse)
    r = gpu_renderer(name)
    arrs = to_gpu(o, d, g_rgb.astype(np.float32))
    gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
    ga = torch.zeros(sc.atlas.shape, dtype=torch.float32, device="cuda")
    gm = torch.zeros((451,), dtype=torch.float32, device="cuda")
    r.backward_baked(*arrs, gt, ga, gm)
    torch.cuda.synchronize()
    _close(_np(gt), gf64, "fine tables")
    _close(_np(ga), ga64, "atlas")
    assert np.allclose(_np(gm), gm64, rtol=1e-3, atol=1e-5 * np.abs(gm64).max())


@pytest.mark.parametrize("name", ["tiny", "train_large", "hd", "baked_tiny"])
def test_backward_from_forward_outputs_matches(name):
    """ngprt_render_backward_fwd (the forward's C_d and F given, first
    re-march skipped) against the backward that re-marches for them: MLP
    gradient bit for bit (fixed-order sums), table and atlas gradients to
    the rounding of the atomic adds' order."""
    import torch
    print(f"[backward from forward outputs {name}]", flush=True)
    sc, dist, cfg, o, d = _rays(name, 2048, 7)
    r = gpu_renderer(name)
    go, gd = to_gpu(o, d)
    n = len(o)
    out = {"rgb": torch.empty((n, 3), dtype=torch.float32, device="cuda"),
           "c_d": torch.empty((n, 3), dtype=torch.float32, device="cuda"),
           "feat": torch.empty((n, 4), dtype=torch.float32, device="cuda")}
    r.render(go, gd, out=out)
    g_rgb = torch.from_numpy(np.random.default_rng(2).standard_normal((n, 3)).astype(np.float32)).cuda()
    baked = sc.cfg.model == synth.MODEL_BAKED
    grads = []
    for use_fwd in (False, True):
        gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
        gm = torch.zeros((451,), dtype=torch.float32, device="cuda")
        ga = torch.zeros(sc.atlas.shape, dtype=torch.float32, device="cuda") if baked else None
        if use_fwd:
            r.backward_fwd(go, gd, out["c_d"], out["feat"], g_rgb, gt, gm, ga)
        elif baked:
            r.backward_baked(go, gd, g_rgb, gt, ga, gm)
        else:
            r.backward(go, gd, g_rgb, gt, gm)
        torch.cuda.synchronize()
        grads.append((_np(gt), _np(gm), None if ga is None else _np(ga)))
    (t0, m0, a0), (t1, m1, a1) = grads
    assert np.array_equal(m0.view(np.uint32), m1.view(np.uint32))
    assert np.abs(t0).max() > 0
    assert np.allclose(t1, t0, rtol=1e-5, atol=1e-6 * np.abs(t0).max())
    assert np.array_equal(t0 != 0, t1 != 0)
    if baked:
        assert np.allclose(a1, a0, rtol=1e-5, atol=1e-6 * np.abs(a0).max())
