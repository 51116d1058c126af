"""GPU parity of the baked feature model (coarse block-sparse grid +
sigmoid-gated separate attention over fine hash levels) against the oracle,
through the C ABI.  Integer outputs and the float32 decision chain
bit-exact; colours within 1e-5 of the float64 oracle."""
import numpy as np
import pytest

import synth
from oracle.exact32 import F32
from oracle.render import fused32, fused64, grid_coords32, render, scene_occupancy

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu
COLOUR_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_baked_eval_points_parity(dtype):
    print(f"[baked eval points dtype {dtype}]", flush=True)
    inp = oracle_inputs("baked_tiny", dtype)
    r = gpu_renderer("baked_tiny", dtype)
    rng = np.random.default_rng(10 + dtype)
    n = 3000
    pos = rng.uniform(-1.0, 1.0, size=(n, 3)).astype(F32)
    pos[:8] = np.array([[-1, -1, -1], [1, 1, 1], [1, -1, 0.5], [0, 0, 0],
                        [0.75, 0.75, 0.75], [-0.75, 0.0, 1.0], [0.5, 0.5, -0.5], [1, 1, -1]], F32)
    (p,) = to_gpu(pos)
    idx, fused, gw = (_np(x) for x in r.eval_points(p))
    u = grid_coords32(inp, pos)
    f32, g32, idx32 = fused32(inp, u)
    assert np.array_equal(idx, idx32.astype(np.int32))
    assert np.array_equal(gw.view(np.uint32), g32.view(np.uint32))
    assert np.array_equal(fused[:, 0].view(np.uint32), f32[:, 0].view(np.uint32))
    f64, g64 = fused64(inp, u.astype(np.float64))
    assert np.abs(fused - f64).max() < COLOUR_TOL
    assert np.abs(gw - g64).max() < 1e-6


def _check_render(out, ref, tol=COLOUR_TOL):
    assert np.array_equal(_np(out["n_samples"]), ref.n_samples)
    assert np.array_equal(_np(out["n_reads"]), ref.n_reads)
    assert np.array_equal(_np(out["t_final"]).view(np.uint32), ref.t_final32.view(np.uint32))
    for k, v in (("rgb", ref.rgb), ("c_d", ref.c_d), ("feat", ref.feat)):
        err = np.abs(_np(out[k]).astype(np.float64) - v).max()
        assert err < tol, (k, err)


@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_baked_render_parity_tiny(dtype):
    print(f"[baked render tiny dtype {dtype}]", flush=True)
    inp = oracle_inputs("baked_tiny", dtype)
    sc, _ = scene_and_dist("baked_tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("baked_tiny", dtype)
    go, gd = to_gpu(o, d)
    out = r.render(go, gd)
    ref = render(inp, o, d)
    assert ref.n_samples.mean() > 5
    _check_render(out, ref)


def test_baked_march_bit_exact():
    print("[baked march]", flush=True)
    inp = oracle_inputs("baked_tiny")
    sc, _ = scene_and_dist("baked_tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("baked_tiny")
    go, gd = to_gpu(o, d)
    cap = 128
    sk, ns, nr = (_np(x) for x in r.march(go, gd, cap=cap))
    ref = render(inp, o, d)
    assert np.array_equal(ns, ref.n_samples) and np.array_equal(nr, ref.n_reads)
    assert ref.n_samples.max() <= cap
    starts = np.r_[0, np.cumsum(ref.n_samples)[:-1]]
    for i in range(0, len(o), 7):
        assert np.array_equal(sk[i, :ref.n_samples[i]], ref.s_k[starts[i]:starts[i] + ref.n_samples[i]])


def test_baked_empty_atlas_and_errors():
    """No stored block (every vertex takes the default), index entries out of
    range, a hash-model context, and unsupported backward."""
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[baked empty atlas + errors]", flush=True)
    sc, dist = scene_and_dist("baked_tiny")
    cfg = sc.cfg
    nb = sc.block_index.shape[0]
    r = gpu_renderer("baked_tiny")
    empty_idx = torch.full((nb, nb, nb), -1, dtype=torch.int32, device="cuda")
    empty_atlas = torch.empty((0, 8, 8, 8, cfg.coarse_channels), dtype=torch.float32, device="cuda")
    default = sc.default.copy()
    default[0] = 3.0
    r.load_coarse(empty_idx, empty_atlas, default)
    inp = oracle_inputs("baked_tiny")
    inp.block_index = np.full((nb, nb, nb), -1, np.int32)
    inp.atlas = np.zeros((0, 8, 8, 8, cfg.coarse_channels), F32)
    inp.coarse_default = default
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::11], d[::11]
    go, gd = to_gpu(o, d)
    _check_render(r.render(go, gd), render(inp, o, d))
    bad = torch.from_numpy(sc.block_index.copy()).cuda()
    bad[0, 0, 0] = sc.atlas.shape[0]          # one past the last atlas row
    with pytest.raises(NgprtError):
        r.load_coarse(bad, torch.from_numpy(sc.atlas).cuda(), sc.default)
    with pytest.raises(NgprtError):                # backward: hash model only
        r.backward(go, gd, torch.zeros((len(o), 3), device="cuda"),
                   torch.zeros((r.L, r.T, 9), device="cuda"), torch.zeros((451,), device="cuda"))
    import ctypes
    from paper_2407_10482_amd._lib import check
    h = gpu_renderer("tiny")                       # a hash-model context
    dflt = (ctypes.c_float * len(default))(*[float(x) for x in default])
    with pytest.raises(NgprtError):
        check(h.lib.ngprt_load_coarse(h.ctx, 0, empty_idx.data_ptr(), None, dflt, None), h.ctx)
    torch.cuda.synchronize()


def test_baked_hd_full_frame_sampled():
    """The 8-view 1080p baked workload in the benchmark's launch
    configuration: sampled rays against the oracle one by one."""
    print("[baked hd full frame]", flush=True)
    import torch
    from synth.baked import make_baked_scene
    from oracle.distgrid import distance_grid_edt
    from oracle.render import inputs_from_scene
    from paper_2407_10482_amd.renderer import Renderer
    cfg = synth.baked_hd(n_fine=2)
    sc = make_baked_scene(cfg)
    dist = distance_grid_edt(scene_occupancy(sc))
    o, d, _ = synth.scene_rays(cfg)
    r = Renderer.from_config(cfg)
    r.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                 torch.from_numpy(sc.mlp).cuda())
    r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(sc.atlas).cuda(), sc.default)
    go, gd = to_gpu(o, d)
    out = r.render(go, gd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(len(o), size=1500, replace=False))
    ref = render(inputs_from_scene(sc, dist), o[sel], d[sel])
    assert np.array_equal(_np(out["n_samples"])[sel], ref.n_samples)
    assert np.array_equal(_np(out["n_reads"])[sel], ref.n_reads)
    assert np.abs(_np(out["rgb"])[sel].astype(np.float64) - ref.rgb).max() < COLOUR_TOL
    assert 5 < ref.n_samples.mean() < 40


@pytest.mark.parametrize("dtype", [0, 2])
def test_paper_configuration_render_parity_tiny(dtype):
    """Baked feature model + occupancy pyramid with the distance grid +
    view-dependent MLP together (the paper's rendering choices), tiny scale."""
    print(f"[paper configuration tiny dtype {dtype}]", flush=True)
    inp = oracle_inputs("paper_tiny", dtype)
    sc, _ = scene_and_dist("paper_tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("paper_tiny", dtype)
    go, gd = to_gpu(o, d)
    out = r.render(go, gd)
    ref = render(inp, o, d)
    assert ref.n_samples.mean() > 5
    _check_render(out, ref)


def test_baked_reload_coarse_reuse_and_realloc():
    """Re-loading the coarse grid: same block count (the allocations are
    kept, as in a training step), then another count (re-allocated), then
    the original again; every render matches the oracle of what is loaded."""
    import torch
    print("[baked coarse reload]", flush=True)
    sc, _ = scene_and_dist("baked_tiny")
    cfg = sc.cfg
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::7], d[::7]
    go, gd = to_gpu(o, d)
    r = gpu_renderer("baked_tiny")
    idx = torch.from_numpy(sc.block_index).cuda()
    first = _np(r.render(go, gd)["rgb"])
    inp = oracle_inputs("baked_tiny")
    scaled = (sc.atlas * np.float32(0.5)).astype(F32)
    r.load_coarse(idx, torch.from_numpy(scaled).cuda(), sc.default)          # same n_blocks
    inp.atlas = scaled
    _check_render(r.render(go, gd), render(inp, o, d))
    keep = sc.block_index >= 0
    fewer = np.where(keep & (sc.block_index < 100), sc.block_index, -1).astype(np.int32)
    r.load_coarse(torch.from_numpy(fewer).cuda(), torch.from_numpy(sc.atlas[:100].copy()).cuda(),
                  sc.default)                                                   # 100 blocks
    inp.block_index, inp.atlas = fewer, sc.atlas[:100]
    _check_render(r.render(go, gd), render(inp, o, d))
    r.load_coarse(idx, torch.from_numpy(sc.atlas).cuda(), sc.default)          # back to all
    again = _np(r.render(go, gd)["rgb"])
    assert np.array_equal(first.view(np.uint32), again.view(np.uint32))
