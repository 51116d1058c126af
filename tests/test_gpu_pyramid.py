"""GPU parity of the multi-level occupancy march (Sec. 4.3, Eq. 9 with its
s_O branch) through the C ABI: marching points, sample lattice indices and
transmittance bit-exact, colours within 1e-5 of the float64 oracle, with and
without the distance grid, in the box and the contracted domain."""
import numpy as np
import pytest

import synth
from oracle import pyramid
from oracle.distgrid import distance_grid_edt
from oracle.exact32 import F32
from oracle.render import CONTRACT, OracleInputs, inputs_from_scene, render, scene_occupancy

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu
COLOUR_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


def _sample_lists(ref, n, cap):
    exp = np.full((n, cap), -1, np.int32)
    starts = np.r_[0, np.cumsum(ref.n_samples)[:-1]]
    for i in range(n):
        exp[i, :ref.n_samples[i]] = ref.s_k[starts[i]:starts[i] + ref.n_samples[i]]
    return exp


@pytest.mark.parametrize("use_dist,naive", [(True, False), (False, False), (True, True)])
def test_pyramid_march_bit_exact_tiny(use_dist, naive):
    print(f"[pyramid march tiny G={use_dist} naive={naive}]", flush=True)
    inp = oracle_inputs("tiny_pyramid")
    inp.use_dist = use_dist
    sc, _ = scene_and_dist("tiny_pyramid")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("tiny_pyramid", use_distance=use_dist)
    go, gd = to_gpu(o, d)
    cap = 96
    sk, ns, nr = (_np(x) for x in r.march(go, gd, cap=cap, naive=naive))
    ref = render(inp, o, d, naive=naive)
    assert ref.n_samples.max() <= cap
    assert np.array_equal(ns, ref.n_samples)
    assert np.array_equal(nr, ref.n_reads)
    assert np.array_equal(sk, _sample_lists(ref, len(o), cap))


@pytest.mark.parametrize("use_dist", [True, False])
def test_pyramid_render_parity_tiny(use_dist):
    print(f"[pyramid render tiny G={use_dist}]", flush=True)
    inp = oracle_inputs("tiny_pyramid")
    inp.use_dist = use_dist
    sc, _ = scene_and_dist("tiny_pyramid")
    o, d, _ = synth.scene_rays(sc.cfg)
    r = gpu_renderer("tiny_pyramid", use_distance=use_dist)
    go, gd = to_gpu(o, d)
    out = r.render(go, gd)
    ref = render(inp, o, d)
    assert np.array_equal(_np(out["n_samples"]), ref.n_samples)
    assert np.array_equal(_np(out["n_reads"]), ref.n_reads)
    assert np.array_equal(_np(out["t_final"]).view(np.uint32), ref.t_final32.view(np.uint32))
    assert np.abs(_np(out["rgb"]).astype(np.float64) - ref.rgb).max() < COLOUR_TOL


@pytest.mark.parametrize("use_dist,jg", [(True, 1), (False, 1), (True, 2), (False, 2)])
def test_pyramid_march_contracted_random_grid(use_dist, jg):
    """Contracted domain, a random 128^3 .. 32^3 pyramid with the distance
    grid at 64^3 (one level above the finest: one word per marching point
    holds the finest level's bits) or at 32^3 (the finer levels read
    one by one)."""
    import torch
    from paper_2407_10482_amd.renderer import Renderer
    print(f"[pyramid march contracted G={use_dist} jg={jg}]", flush=True)
    rng = np.random.default_rng(7)
    fine = np.zeros((128, 128, 128), np.uint8)
    for _ in range(15):
        c = rng.integers(10, 118, size=3)
        h = rng.integers(2, 10, size=3)
        fine[c[2] - h[2]:c[2] + h[2], c[1] - h[1]:c[1] + h[1], c[0] - h[0]:c[0] + h[0]] = 1
    sc, _ = scene_and_dist("tiny")
    step = float(synth.CONTRACT_STEP)
    pyr = pyramid.build_pyramid(fine, 3)
    occ = pyr[jg]
    inp = OracleInputs(tables=sc.tables, occ=occ, dist=distance_grid_edt(occ), mlp=sc.mlp,
                       resolutions=sc.cfg.resolutions, domain=CONTRACT, roi_half=2.0, step=step,
                       max_samples=1024, t_threshold=1e-4, pyramid=pyr, use_dist=use_dist)
    n = 2000
    o = rng.uniform(-3, 3, size=(n, 3)).astype(F32)
    dd = rng.uniform(-1.5, 1.5, size=(n, 3)) - o
    d = (dd / np.linalg.norm(dd, axis=1, keepdims=True)).astype(F32)
    r = Renderer(sc.cfg.resolutions, sc.cfg.log2_table, 0, CONTRACT, 2.0, 128 >> jg, step, 1024, 1e-4,
                 occ_levels=3, occ_fine_res=128, use_distance=use_dist)
    r.load_tables(torch.from_numpy(sc.tables).cuda())
    r.load_occupancy_pyramid(torch.from_numpy(fine).cuda())
    r.load_mlp(torch.from_numpy(sc.mlp).cuda())
    assert np.array_equal(_np(r.export_distance()), inp.dist)
    go, gd = to_gpu(o, d)
    out = r.render(go, gd)
    ref = render(inp, o, d)
    assert ref.n_samples.sum() > 1000
    assert np.array_equal(_np(out["n_samples"]), ref.n_samples)
    assert np.array_equal(_np(out["n_reads"]), ref.n_reads)
    assert np.abs(_np(out["rgb"]).astype(np.float64) - ref.rgb).max() < COLOUR_TOL


def test_pyramid_api_errors():
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[pyramid api errors]", flush=True)
    sc, _ = scene_and_dist("tiny_pyramid")
    r = gpu_renderer("tiny_pyramid")
    with pytest.raises(NgprtError):                       # single-grid load on a pyramid context
        r.load_occupancy(torch.zeros((sc.cfg.occ_res,) * 3, dtype=torch.uint8, device="cuda"))
    h = gpu_renderer("tiny")
    h.occ_fine_res = 128
    with pytest.raises(NgprtError):                       # pyramid load on a single-grid context
        h.load_occupancy_pyramid(torch.from_numpy(sc.occ_fine).cuda())
    torch.cuda.synchronize()


def test_hd_pyramid_full_frame_sampled():
    """The 8-view 1080p workload marched with the 512^3 .. 32^3 pyramid and
    the 256^3 distance grid, in the benchmark's launch configuration: sampled
    rays against the oracle one by one; the distance grid cuts marching
    points (the paper's Table 4)."""
    import torch
    from paper_2407_10482_amd.renderer import Renderer
    print("[hd pyramid full frame]", flush=True)
    cfg = synth.hd_pyramid()
    sc = synth.make_scene(cfg)
    o, d, _ = synth.scene_rays(cfg)
    go, gd = to_gpu(o, d)
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(len(o), size=1500, replace=False))
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    reads = {}
    for use_dist in (True, False):
        r2 = Renderer.from_config(cfg, use_distance=use_dist)
        r2.load_tables(torch.from_numpy(sc.tables).cuda())
        r2.load_occupancy_pyramid(torch.from_numpy(sc.occ_fine).cuda())
        r2.load_mlp(torch.from_numpy(sc.mlp).cuda())
        out = r2.render(go, gd)
        torch.cuda.synchronize()
        inp.use_dist = use_dist
        ref = render(inp, o[sel], d[sel])
        assert np.array_equal(_np(out["n_samples"])[sel], ref.n_samples)
        assert np.array_equal(_np(out["n_reads"])[sel], ref.n_reads)
        assert np.abs(_np(out["rgb"])[sel].astype(np.float64) - ref.rgb).max() < COLOUR_TOL
        reads[use_dist] = float(_np(out["n_reads"]).mean())
        print(f"G={use_dist}: marching points/ray {reads[use_dist]:.2f}, "
              f"samples/ray {_np(out['n_samples']).mean():.2f}", flush=True)
        r2.close()
    assert reads[True] < reads[False]
