"""GPU parity of the view-dependent deferred MLP (Eq. 5; MLP_psi
23 -> 64 -> 64 -> 3 of C_d, F and the spherical harmonics of the view
direction) against the float64 oracle, through the C ABI."""
import numpy as np
import pytest

import synth
from oracle.exact32 import F32
from oracle.render import render, scene_occupancy

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu
COLOUR_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


def test_view_mlp_render_parity_and_ragged_batches():
    print("[view mlp render]", flush=True)
    inp = oracle_inputs("tiny_view")
    sc, _ = scene_and_dist("tiny_view")
    o, d, _ = synth.scene_rays(sc.cfg)
    extra_o = np.array([[0.1, 0.1, 0.1], [np.nan, 0, 0], [0.2, 0.1, -3.0]], F32)
    extra_d = np.array([[0, 0, 0], [0, 0, 1], [0, 0, 1]], F32)      # zero direction: SH = 0
    rng = np.random.default_rng(4)
    r = gpu_renderer("tiny_view")
    for n in (1, 63, 65, 257, len(o)):
        sel = rng.choice(len(o), size=n, replace=False) if n < len(o) else np.arange(len(o))
        oo = np.concatenate([extra_o, o[sel]])
        dd = np.concatenate([extra_d, d[sel]])
        go, gd = to_gpu(oo, dd)
        out = r.render(go, gd)
        ref = render(inp, oo, dd)
        assert np.array_equal(_np(out["n_samples"]), ref.n_samples)
        for k, v in (("rgb", ref.rgb), ("c_d", ref.c_d), ("feat", ref.feat)):
            err = np.abs(_np(out[k]).astype(np.float64) - v).max()
            assert err < COLOUR_TOL, (n, k, err)


def test_view_mlp_needs_cd_and_feat_outputs_and_rejects_the_fused_backward():
    import ctypes
    import torch
    from paper_2407_10482_amd._lib import NgprtError, NgprtOutputs, check
    print("[view mlp errors]", flush=True)
    sc, _ = scene_and_dist("tiny_view")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("tiny_view")
    go, gd = to_gpu(o[:64], d[:64])
    rgb = torch.empty((64, 3), device="cuda")
    outs = NgprtOutputs()
    outs.rgb = rgb.data_ptr()
    with pytest.raises(NgprtError):
        check(r.lib.ngprt_render(r.ctx, 64, go.data_ptr(), gd.data_ptr(), ctypes.byref(outs), None), r.ctx)
    with pytest.raises(NgprtError):
        r.backward(go, gd, torch.zeros((64, 3), device="cuda"), torch.zeros((r.L, r.T, 9), device="cuda"),
                   torch.zeros((r.n_mlp,), device="cuda"))
    torch.cuda.synchronize()


def test_view_mlp_hd_full_frame_sampled():
    """The 8-view 1080p workload with MLP_psi, in the benchmark's launch
    configuration: sampled rays against the oracle."""
    import torch
    from oracle.distgrid import distance_grid_edt
    from oracle.render import inputs_from_scene
    from paper_2407_10482_amd.renderer import Renderer
    print("[view mlp hd]", flush=True)
    cfg = synth.hd()
    cfg.mlp_dims = (23, 64, 64, 3)
    sc = synth.make_scene(cfg)
    o, d, _ = synth.scene_rays(cfg)
    r = Renderer.from_config(cfg)
    r.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                 torch.from_numpy(sc.mlp).cuda())
    go, gd = to_gpu(o, d)
    out = {"rgb": torch.empty((len(o), 3), device="cuda")}
    r.render(go, gd, out=out)
    torch.cuda.synchronize()
    sel = np.sort(np.random.default_rng(0).choice(len(o), size=1000, replace=False))
    ref = render(inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc))), o[sel], d[sel])
    assert np.abs(_np(out["rgb"])[sel].astype(np.float64) - ref.rgb).max() < COLOUR_TOL
