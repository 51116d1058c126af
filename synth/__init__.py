"""Seeded synthetic inputs shared by the renderer's tests, the benchmark and
the oracle: workload configs, scene assets and camera rays.  Holds no
rendering arithmetic."""
from .configs import (CONFIGS, CONTRACT_STEP, DOMAIN_BOX, DOMAIN_CONTRACT, DTYPE_BF16,
                      DTYPE_F32, DTYPE_FP8, MODEL_BAKED, MODEL_HASH, SceneConfig, baked_hd,
                      baked_tiny, baked_tiny_pyramid, geometric_resolutions, hd, hd_pyramid, hd_regime, tiny,
                      tiny_pyramid, train_large, AGGREGATIONS, with_aggregation)
from .scene import Scene, camera_positions, make_scene
from .cameras import pinhole_rays, random_sphere_cameras, scene_rays, tile_order

__all__ = [
    "CONFIGS", "CONTRACT_STEP", "DOMAIN_BOX", "DOMAIN_CONTRACT", "DTYPE_BF16", "DTYPE_F32",
    "DTYPE_FP8", "MODEL_BAKED", "MODEL_HASH", "baked_hd", "baked_tiny", "SceneConfig", "geometric_resolutions", "hd", "tiny", "train_large", "Scene",
    "camera_positions", "make_scene", "pinhole_rays", "random_sphere_cameras", "scene_rays",
    "tile_order", "baked_tiny_pyramid", "hd_pyramid", "hd_regime", "tiny_pyramid", "AGGREGATIONS", "with_aggregation",
]
