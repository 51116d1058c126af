"""GPU backward with the view-dependent MLP (Eq. 5; MLP_psi of C_d, F and
SH(d)) through the C ABI: the MLP's adjoint (dL/dC_d, dL/dF, dL/dpsi)
against the oracle's float64 adjoint, the render adjoint driven by given
dL/dC_d and dL/dF (hash and baked models) against the oracle's, and
training through the autograd wrapper."""
import numpy as np
import pytest

import synth
from oracle import sh
from oracle.grad import backward64, frozen_samples
from oracle.render import inputs_from_scene

from helpers import gpu_renderer, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def test_view_mlp_backward_matches_oracle():
    import torch
    print("[view mlp backward]", flush=True)
    sc, _ = scene_and_dist("tiny_view")
    o, d, _ = synth.scene_rays(sc.cfg)
    n = 3001                                         # ragged: 46 full waves + 57 rays
    go, gd = to_gpu(o[:n], d[:n])
    r = gpu_renderer("tiny_view")
    out = r.render(go, gd)
    c_d, feat = out["c_d"], out["feat"]
    g = np.random.default_rng(5).normal(size=(n, 3))
    gm = torch.zeros((r.n_mlp,), device="cuda")
    (gg,) = to_gpu(g.astype(np.float32))
    gcf = _np(r.view_mlp_backward(gd, c_d, feat, gg, gm))
    w_cd, w_f, w_p = sh.mlp_view_backward64(sc.mlp, _np(c_d).astype(np.float64), _np(feat).astype(np.float64),
                                            d[:n], g)
    want = np.concatenate([w_cd, w_f], axis=1)
    assert np.abs(gcf - want).max() <= 1e-4 * np.abs(want).max()
    gp = _np(gm)
    assert np.abs(gp - w_p).max() <= 1e-4 * np.abs(w_p).max()


@pytest.mark.parametrize("name", ["tiny_view", "paper_tiny"])
def test_render_backward_from_features_matches_oracle(name):
    import torch
    print(f"[render backward from features] {name}", flush=True)
    sc, dist = scene_and_dist(name)
    cfg = sc.cfg
    inp = inputs_from_scene(sc, dist)
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::8], d[::8]
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    rng = np.random.default_rng(6)
    g_cd, g_f = rng.normal(size=(len(o), 3)), rng.normal(size=(len(o), 4))
    baked = cfg.model == synth.MODEL_BAKED
    coarse = None
    if baked:
        coarse = dict(atlas=sc.atlas.astype(np.float64), default=sc.default.astype(np.float64),
                      block_index=sc.block_index, res=cfg.coarse_res)
    want, gm, _ = backward64(sc.tables.astype(np.float64), sc.mlp, cfg.resolutions, cfg.step, len(o), s_ray,
                             s_pos, None, coarse=coarse, upstream=(g_cd, g_f))
    assert gm is None
    r = gpu_renderer(name)
    go, gd, gcf = to_gpu(o, d, np.concatenate([g_cd, g_f], axis=1).astype(np.float32))
    gt = torch.zeros((r.L, r.T, 9), device="cuda")
    ga = torch.zeros(sc.atlas.shape, device="cuda") if baked else None
    r.backward_features(go, gd, gcf, gt, ga)
    torch.cuda.synchronize()
    pairs = [(_np(gt), want[1] if baked else want)]
    if baked:
        pairs.append((_np(ga), want[0]))
    for got, ref in pairs:
        scale = np.abs(ref).max()
        assert scale > 0
        assert np.all(np.abs(got - ref) <= 1e-4 * scale + 1e-3 * np.abs(ref)), np.abs(got - ref).max() / scale


def test_training_with_the_view_mlp_reduces_loss():
    """The paper's representation (baked model, pyramid march, MLP_psi)
    trained through the autograd wrapper against a seed-1 teacher."""
    import torch
    from paper_2407_10482_amd.renderer import adam_step, render_differentiable_view
    from synth.baked import make_baked_scene
    print("[view mlp training]", flush=True)
    sc, _ = scene_and_dist("paper_tiny")
    cfg = sc.cfg
    teacher = make_baked_scene(cfg, seed=1)
    r = gpu_renderer("paper_tiny")
    o, d, _ = synth.scene_rays(cfg)
    go, gd = to_gpu(o[::2], d[::2])
    r.load_tables(torch.from_numpy(teacher.tables).cuda())
    r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(teacher.atlas).cuda(),
                  teacher.default)
    target = r.render(go, gd)["rgb"].clone()
    params = [torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.atlas).cuda(),
              torch.from_numpy(sc.mlp).cuda()]
    moments = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    losses = []
    for step in range(1, 21):
        for p in params:
            p.requires_grad_(True)
        rgb = render_differentiable_view(r, params[0], params[2], go, gd, atlas=params[1])
        loss = torch.mean((rgb - target) ** 2)
        loss.backward()
        losses.append(loss.item())
        with torch.no_grad():
            for p, (m, v) in zip(params, moments):
                adam_step(p, p.grad, m, v, step, 0.01)
        params = [p.detach() for p in params]
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_render_backward_from_features_with_regulariser_matches_oracle():
    """The distortion regulariser (supplement Eq. S2) through the
    feature-driven render backward, baked model on the pyramid."""
    import torch
    print("[render backward from features + dist] paper_tiny", flush=True)
    sc, dist = scene_and_dist("paper_tiny")
    cfg = sc.cfg
    inp = inputs_from_scene(sc, dist)
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::8], d[::8]
    s_ray, s_pos, _, s_k = frozen_samples(inp, o, d, with_k=True)
    rng = np.random.default_rng(9)
    g_cd, g_f = rng.normal(size=(len(o), 3)), rng.normal(size=(len(o), 4))
    g_dist = np.full(len(o), 0.05)
    coarse = dict(atlas=sc.atlas.astype(np.float64), default=sc.default.astype(np.float64),
                  block_index=sc.block_index, res=cfg.coarse_res)
    (ga64, gf64), _, _ = backward64(sc.tables.astype(np.float64), sc.mlp, cfg.resolutions, cfg.step, len(o),
                                    s_ray, s_pos, None, grad_dist=g_dist, s_k=s_k, coarse=coarse,
                                    upstream=(g_cd, g_f))
    r = gpu_renderer("paper_tiny")
    go, gd, gcf, gdd = to_gpu(o, d, np.concatenate([g_cd, g_f], axis=1).astype(np.float32),
                             g_dist.astype(np.float32))
    gt = torch.zeros((r.L, r.T, 9), device="cuda")
    ga = torch.zeros(sc.atlas.shape, device="cuda")
    r.backward_features(go, gd, gcf, gt, ga, gdd)
    torch.cuda.synchronize()
    for got, ref in ((_np(gt), gf64), (_np(ga), ga64)):
        scale = np.abs(ref).max()
        assert scale > 0
        assert np.all(np.abs(got - ref) <= 1e-4 * scale + 1e-3 * np.abs(ref)), np.abs(got - ref).max() / scale


def test_feature_backward_and_view_backward_reject_unsupported_contexts():
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[feature backward errors]", flush=True)
    o = torch.zeros((8, 3), device="cuda")
    gcf = torch.zeros((8, 7), device="cuda")
    bf = gpu_renderer("tiny_view", 1)                   # bf16 tables: no backward
    with pytest.raises(NgprtError):
        bf.backward_features(o, o, gcf, torch.zeros((bf.L, bf.T, 9), device="cuda"))
    sm = gpu_renderer("baked_tiny_sum")                 # SUM aggregation: no backward
    with pytest.raises(NgprtError):
        sm.backward_features(o, o, gcf, torch.zeros((sm.L, sm.T, 9), device="cuda"),
                             torch.zeros((sm.n_blocks, 8, 8, 8, 12), device="cuda"))
    pl = gpu_renderer("tiny")                           # plain MLP: no MLP_psi backward
    with pytest.raises(NgprtError):
        pl.view_mlp_backward(o, o, torch.zeros((8, 4), device="cuda"), o, torch.zeros((451,), device="cuda"))
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["tiny_view", "paper_tiny"])
def test_backward_features_from_forward_outputs(name):
    """The features backward given the forward's C_d and F (first re-march
    skipped) equals the one that re-marches for them, up to the order of
    the atomic adds; one of the two alone, or with the regulariser, is an
    error."""
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    from paper_2407_10482_amd import renderer as rmod
    print(f"[backward features from forward outputs] {name}", flush=True)
    sc, _ = scene_and_dist(name)
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer(name)
    go, gd = to_gpu(o, d)
    n = len(o)
    out = {"rgb": torch.empty((n, 3), device="cuda"), "c_d": torch.empty((n, 3), device="cuda"),
           "feat": torch.empty((n, 4), device="cuda")}
    r.render(go, gd, out=out)
    gcf = torch.from_numpy(np.random.default_rng(4).standard_normal((n, 7)).astype(np.float32)).cuda()
    baked = sc.cfg.model == synth.MODEL_BAKED
    res = []
    for fwd in (False, True):
        gt = torch.zeros((r.L, r.T, 9), device="cuda")
        ga = torch.zeros(sc.atlas.shape, device="cuda") if baked else None
        if fwd:
            r.backward_features(go, gd, gcf, gt, ga, None, out["c_d"], out["feat"])
        else:
            r.backward_features(go, gd, gcf, gt, ga)
        torch.cuda.synchronize()
        res.append((_np(gt), None if ga is None else _np(ga)))
    (t0, a0), (t1, a1) = res
    assert np.abs(t0).max() > 0
    assert np.allclose(t1, t0, rtol=1e-5, atol=1e-6 * np.abs(t0).max())
    if baked:
        assert np.allclose(a1, a0, rtol=1e-5, atol=1e-6 * np.abs(a0).max())
    gt = torch.zeros((r.L, r.T, 9), device="cuda")
    ga = torch.zeros(sc.atlas.shape, device="cuda") if baked else None
    with pytest.raises(NgprtError):
        rmod.check(r.lib.ngprt_render_backward_features(r.ctx, n, rmod._ptr(go), rmod._ptr(gd), rmod._ptr(gcf),
                                                        None, rmod._ptr(gt), rmod._ptr(ga), rmod._ptr(out["c_d"]),
                                                        None, rmod._stream()), r.ctx)
    gdd = torch.ones((n,), device="cuda")
    with pytest.raises(NgprtError):
        r.backward_features(go, gd, gcf, gt, ga, gdd, out["c_d"], out["feat"])
