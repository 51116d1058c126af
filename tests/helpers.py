"""Shared test helpers: seeded scenes on the GPU and the oracle beside them."""
import functools

import numpy as np

import synth
from oracle.distgrid import distance_grid_edt
from oracle.render import inputs_from_scene, scene_occupancy


@functools.lru_cache(maxsize=4)
def scene_and_dist(name: str, dtype: int = 0):
    cfg = synth.CONFIGS[name](table_dtype=dtype)
    if cfg.model == synth.MODEL_BAKED:
        from synth.baked import make_baked_scene
        sc = make_baked_scene(cfg)
    else:
        sc = synth.make_scene(cfg)
    dist = distance_grid_edt(scene_occupancy(sc))
    return sc, dist


def oracle_inputs(name: str, dtype: int = 0):
    sc, dist = scene_and_dist(name, dtype)
    return inputs_from_scene(sc, dist, dtype)


def renderer_kwargs(name: str, dtype: int = 0, **overrides):
    """The Renderer arguments of a seeded scene."""
    cfg = scene_and_dist(name, dtype)[0].cfg
    kw = dict(resolutions=cfg.resolutions, log2_table_size=cfg.log2_table, table_dtype=dtype,
              domain=cfg.domain, roi_half=cfg.roi_half, occ_res=cfg.occ_res, step=cfg.step,
              max_samples=cfg.max_samples, t_threshold=cfg.t_threshold,
              feature_model=cfg.model, coarse_res=cfg.coarse_res, occ_levels=cfg.occ_levels,
              occ_fine_res=cfg.occ_fine_res, use_distance=True, mlp_dims=tuple(cfg.mlp_dims),
              aggregation=cfg.aggregation, gate_params=tuple(cfg.gate_params))
    kw.update(overrides)
    return kw


def scene_assets(name: str, dtype: int = 0, with_dist: bool = False):
    """A seeded scene as the asset arrays a scene directory holds."""
    sc, dist = scene_and_dist(name, dtype)
    cfg = sc.cfg
    a = {"tables": sc.tables, "mlp": sc.mlp}
    if cfg.occ_levels:
        a["occ_fine"] = sc.occ_fine
    else:
        a["occ"] = sc.occ
        if with_dist:
            a["dist"] = np.ascontiguousarray(dist, dtype=np.uint8)
    if cfg.model == synth.MODEL_BAKED:
        a.update(coarse_index=sc.block_index, coarse_atlas=sc.atlas,
                 coarse_default=np.asarray(sc.default, np.float32))
    return a


def gpu_renderer(name: str, dtype: int = 0, **overrides):
    import torch
    from paper_2407_10482_amd.renderer import Renderer
    sc, _ = scene_and_dist(name, dtype)
    cfg = sc.cfg
    kw = renderer_kwargs(name, dtype, **overrides)
    r = Renderer(**kw)
    r.load_tables(torch.from_numpy(sc.tables).cuda())
    if kw["occ_levels"]:
        r.load_occupancy_pyramid(torch.from_numpy(sc.occ_fine).cuda())
    else:
        r.load_occupancy(torch.from_numpy(sc.occ).cuda())
    r.load_mlp(torch.from_numpy(sc.mlp).cuda())
    if cfg.model == synth.MODEL_BAKED:
        r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(sc.atlas).cuda(),
                      sc.default)
    torch.cuda.synchronize()
    return r


def to_gpu(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]
