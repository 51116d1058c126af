"""A renderer built from a scene directory renders what the same scene
loaded array by array renders, bit for bit."""
import numpy as np
import pytest

import synth
from helpers import gpu_renderer, scene_and_dist, scene_assets, to_gpu

pytestmark = pytest.mark.gpu

FIELDS = ("rgb", "t_final", "n_samples", "n_reads", "depth")


def _same(a, b):
    for k in FIELDS:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), k


@pytest.mark.parametrize("name,with_dist", [("tiny", False), ("tiny", True), ("baked_tiny_pyramid", False),
                                            ("tiny_view", False), ("baked_tiny_shared_v", True)])
def test_from_assets_renders_bit_identically(tmp_path, name, with_dist):
    import torch
    from paper_2407_10482_amd.renderer import Renderer
    print(f"assets case {name} dist={with_dist}", flush=True)
    sc, _ = scene_and_dist(name)
    direct = gpu_renderer(name)
    path = str(tmp_path / name)
    direct.save_assets(path, **scene_assets(name, with_dist=with_dist))
    loaded = Renderer.from_assets(path)
    assert loaded.descriptor == direct.descriptor
    o, d, _ = synth.scene_rays(sc.cfg, cams=synth.camera_positions(sc.cfg)[:1], width=96, height=64)
    go, gd = to_gpu(o, d)
    a, b = direct.render(go, gd), loaded.render(go, gd)
    torch.cuda.synchronize()
    assert int(a["n_samples"].sum()) > 0
    _same(a, b)
    if with_dist and not sc.cfg.occ_levels:
        # the supplied distance grid is the one the library builds itself
        assert torch.equal(loaded.export_distance(), direct.export_distance())


def test_from_assets_loads_the_proposal_network(tmp_path):
    import torch
    from paper_2407_10482_amd.renderer import Renderer
    print("assets case tiny + proposal", flush=True)
    sc, _ = scene_and_dist("tiny")
    rng = np.random.default_rng(8)
    params = rng.normal(0.0, 0.05, size=7556).astype(np.float32)
    params[7552:7556] = np.array([0.0, 0.25, 0.2, 0.5], np.float32)
    direct = gpu_renderer("tiny")
    (gp,) = to_gpu(params)
    direct.load_proposal(gp)
    path = str(tmp_path / "tiny_prop")
    direct.save_assets(path, proposal=gp, **scene_assets("tiny"))
    loaded = Renderer.from_assets(path)
    o, d, _ = synth.scene_rays(sc.cfg, cams=synth.camera_positions(sc.cfg)[:1], width=96, height=64)
    go, gd = to_gpu(o, d)
    margin = 3.0 * sc.cfg.step
    a = direct.render_proposal(go, gd, 0.5, margin)
    b = loaded.render_proposal(go, gd, 0.5, margin)
    torch.cuda.synchronize()
    _same(a, b)
    assert np.array_equal(a["proposal"].cpu().numpy().view(np.uint32), b["proposal"].cpu().numpy().view(np.uint32))
