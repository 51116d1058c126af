"""Workload definitions for the synthetic NGP-RT scenes.

Five workloads are defined.  They are inputs to the renderer, not part of the
rendering arithmetic:

* ``tiny``      -- 8 hash levels (16..256), 2^14 entries, box ROI [-1,1]^3,
                   64^3 occupancy, one 64x64 camera on the unit sphere,
                   lattice step 1/256.  Small enough for the CPU oracle.
* ``hd``        -- 16 hash levels (16..4096), 2^19 entries, FP32, scene in
                   the contracted unbounded domain (radius 2), 256^3
                   occupancy, 8 cameras of 1920x1080 on a ring of radius 3,
                   at most 1024 samples per ray, termination at T < 1e-4.
* ``precision`` -- ``tiny`` with BF16 or FP8-E4M3 tables.
* ``train``     -- one differentiable step on the ``tiny`` grid shape.
* ``proposal``  -- the learned sample-interval proposal on the ``tiny`` scene.
* ``baked_tiny`` / ``baked_hd`` -- the paper's own feature construction: a
                   block-sparse coarse grid of resolution L_C holding the
                   density, colour, specular feature and per-level attention
                   parameters, plus L fine hash levels (8 channels) fused by
                   sigmoid-gated separate attention.  ``baked_tiny``: box ROI,
                   L_C = 64, fine levels 128 and 256, 2^14 entries;
                   ``baked_hd``: the hd geometry, L_C = 512, fine levels
                   1024 * 2^l (l < L, L = 2..4), 2^22 entries.

Level resolutions follow a geometric progression between the coarsest and
finest resolution (the multi-resolution hash encoding the method builds on,
Sec. 3 "Preliminaries", Eq. 3), rounded down after adding 1e-6 so that the
end points are exact; the integer list is handed to the renderer explicitly.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Tuple


def geometric_resolutions(n_min: int, n_max: int, n_levels: int) -> List[int]:
    """Integer per-level grid resolutions N_l = floor(n_min * b**l + 1e-6)."""
    if n_levels == 1:
        return [n_min]
    b = (n_max / n_min) ** (1.0 / (n_levels - 1))
    return [int(math.floor(n_min * b ** l + 1e-6)) for l in range(n_levels)]


DOMAIN_BOX = 0        # axis-aligned cube ROI, straight lattice t_k = t0 + k*step
DOMAIN_CONTRACT = 1   # unbounded scene contracted into the ball of radius 2

DTYPE_F32 = 0
DTYPE_BF16 = 1
DTYPE_FP8 = 2

MODEL_HASH = 0        # every level a hash level, softmax attention over levels
MODEL_BAKED = 1       # coarse baked grid + fine hash levels with sigmoid gates
BLOCK = 8             # coarse grid: vertices per block edge


@dataclass
class SceneConfig:
    name: str
    n_levels: int
    n_min: int
    n_max: int
    log2_table: int
    domain: int
    roi_half: float            # grid covers [-roi_half, roi_half]^3
    occ_res: int
    step: float                # lattice step (world units for the box, contracted units otherwise)
    max_samples: int
    t_threshold: float
    n_blobs: int
    blob_sigma: Tuple[float, float]
    blob_centre_half: float    # box: centres ~ U[-h, h]^3 ; contract: radius of the ball of centres
    density_scale: float       # s_sigma of the density channel
    cam_width: int
    cam_height: int
    n_cams: int
    cam_radius: float
    fov_deg: float = 60.0
    table_dtype: int = DTYPE_F32
    seed: int = 0
    mlp_dims: Tuple[int, int, int, int] = (7, 16, 16, 3)
    resolutions: List[int] = field(default_factory=list)
    model: int = MODEL_HASH
    coarse_res: int = 0        # L_C of the baked model (vertex lattice L_C + 1 per axis)
    occ_levels: int = 0        # > 0: occupancy pyramid of this many levels, finest occ_fine_res
    occ_fine_res: int = 0
    aggregation: int = 0       # baked model: fusion of the fine levels (0 = Separate-Att (V))
    gate_params: Tuple[float, ...] = ()   # constant gates of the (Inv) aggregations

    def __post_init__(self):
        if not self.resolutions:
            self.resolutions = geometric_resolutions(self.n_min, self.n_max, self.n_levels)

    @property
    def coarse_channels(self) -> int:
        """8 feature channels + (omega, beta) per fine level (one a per
        level for Shared-Att (V); none for constant gates and SUM)."""
        return 8 + {0: 2 * self.n_levels, 1: self.n_levels}.get(self.aggregation, 0)

    @property
    def table_size(self) -> int:
        return 1 << self.log2_table

    @property
    def n_mlp_params(self) -> int:
        i, h1, h2, o = self.mlp_dims
        return h1 * i + h1 + h2 * h1 + h2 + o * h2 + o


# Lattice step of the contracted domain: 2*sqrt(3)/512, the base marching step
# the paper uses inside its [-1,1]^3 ROI (supplement, "Auto-tuning of Marching
# Step Size").  Rounded to fp32 once here.
CONTRACT_STEP = 2.0 * math.sqrt(3.0) / 512.0


def tiny(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    return SceneConfig(
        name="tiny", n_levels=8, n_min=16, n_max=256, log2_table=14,
        domain=DOMAIN_BOX, roi_half=1.0, occ_res=64, step=1.0 / 256.0,
        max_samples=1024, t_threshold=1e-4, n_blobs=3, blob_sigma=(0.1, 0.3),
        blob_centre_half=0.5, density_scale=600.0,
        cam_width=64, cam_height=64, n_cams=1, cam_radius=1.0,
        table_dtype=table_dtype, seed=seed)


def hd(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    return SceneConfig(
        name="hd", n_levels=16, n_min=16, n_max=4096, log2_table=19,
        domain=DOMAIN_CONTRACT, roi_half=2.0, occ_res=256, step=CONTRACT_STEP,
        max_samples=1024, t_threshold=1e-4, n_blobs=200, blob_sigma=(0.03, 0.12),
        blob_centre_half=1.9, density_scale=400.0,
        cam_width=1920, cam_height=1080, n_cams=8, cam_radius=3.0,
        table_dtype=table_dtype, seed=seed)


def hd_regime(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The hd workload on a scene calibrated to the paper's Table 4 regime
    (about 18 evaluated samples and 46 marching points per ray; the band
    15-20 samples, 40-55 grid reads): 400 smaller blobs, s_sigma = 350,
    which gives 17.3 samples and 42.6 grid reads per ray over the 8 views.
    The hd scene itself (15.2 / 34.8) stays the headline's."""
    cfg = hd(seed, table_dtype)
    cfg.name = "hd_regime"
    cfg.n_blobs, cfg.blob_sigma, cfg.density_scale = 400, (0.02, 0.08), 350.0
    return cfg


def train_large(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The tiny scene's geometry with the hd hash grid (16 levels 16..4096,
    2^19 entries): the large-table training measurement."""
    cfg = tiny(seed, table_dtype)
    cfg.name = "train_large"
    cfg.n_levels, cfg.n_max, cfg.log2_table = 16, 4096, 19
    cfg.resolutions = geometric_resolutions(cfg.n_min, cfg.n_max, cfg.n_levels)
    return cfg


def baked_tiny(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The tiny scene with the paper's feature construction: L_C = 64, fine
    hash levels 128 and 256 with 2^14 entries."""
    cfg = tiny(seed, table_dtype)
    cfg.name = "baked_tiny"
    cfg.model, cfg.coarse_res = MODEL_BAKED, 64
    cfg.density_scale = 1e4       # ~18 evaluated samples per ray
    cfg.n_levels, cfg.n_min, cfg.n_max = 2, 128, 256
    cfg.resolutions = [128, 256]
    return cfg


def baked_tiny_levels(n_fine: int, seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """baked_tiny with n_fine (1..4) fine levels 128 * 2^l (the paper doubles
    the fine resolution per level; supplement "Multi-level Hash Features")."""
    if not 1 <= n_fine <= 4:
        raise ValueError("n_fine must be 1..4")
    cfg = baked_tiny(seed, table_dtype)
    cfg.name = f"baked_tiny_l{n_fine}"
    cfg.n_levels = n_fine
    cfg.resolutions = [128 << l for l in range(n_fine)]
    cfg.n_min, cfg.n_max = cfg.resolutions[0], cfg.resolutions[-1]
    return cfg


def baked_hd(seed: int = 0, table_dtype: int = DTYPE_F32, n_fine: int = 2) -> SceneConfig:
    """The hd geometry with the paper's feature construction (supplement,
    "Multi-level Hash Features"): L_C = 512, fine levels 1024 * 2^l for
    l < n_fine, 2^22 entries per fine level."""
    if not 1 <= n_fine <= 4:
        raise ValueError("n_fine must be 1..4")
    cfg = hd(seed, table_dtype)
    cfg.name = f"baked_hd_l{n_fine}"
    cfg.model, cfg.coarse_res = MODEL_BAKED, 512
    cfg.density_scale = 4000.0    # ~14 evaluated samples and ~35 grid reads per ray
    cfg.n_levels, cfg.log2_table = n_fine, 22
    cfg.resolutions = [1024 << l for l in range(n_fine)]
    cfg.n_min, cfg.n_max = cfg.resolutions[0], cfg.resolutions[-1]
    return cfg


def tiny_pyramid(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The tiny scene marched with a 3-level occupancy pyramid 128^3 .. 32^3
    (samples where the 128^3 level is occupied) and the distance grid at 64^3."""
    cfg = tiny(seed, table_dtype)
    cfg.name = "tiny_pyramid"
    cfg.occ_levels, cfg.occ_fine_res = 3, 128
    return cfg


def hd_pyramid(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The hd scene marched as in the paper's renderer (supplement "Real-time
    Rendering" item 1; Sec. 4.3): occupancy pyramid 512^3 .. 32^3 (5 levels)
    plus the 256^3 distance grid."""
    cfg = hd(seed, table_dtype)
    cfg.name = "hd_pyramid"
    cfg.occ_levels, cfg.occ_fine_res = 5, 512
    return cfg


def tiny_view(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """The tiny scene with the view-dependent MLP_psi (23 -> 64 -> 64 -> 3 of
    C_d, F and the degree-0..3 spherical harmonics of the view direction)."""
    cfg = tiny(seed, table_dtype)
    cfg.name = "tiny_view"
    cfg.mlp_dims = (23, 64, 64, 3)
    return cfg


AGGREGATIONS = {"separate_v": 0, "shared_v": 1, "separate_inv": 2, "shared_inv": 3, "sum": 4}
# constant attention parameters of the (Inv) variants (fixed, spread over the
# sigmoid's useful range)
_GATE_CONSTANTS = (0.6, -0.4, -0.9, 1.3, 0.2, 0.8, -1.2, 0.5)


def with_aggregation(cfg: SceneConfig, name: str) -> SceneConfig:
    """The same scene fused by another of Table 3's aggregations."""
    agg = AGGREGATIONS[name]
    cfg = dataclasses.replace(cfg, aggregation=agg)
    L = cfg.n_levels
    cfg.gate_params = {2: _GATE_CONSTANTS[:2 * L], 3: _GATE_CONSTANTS[:L]}.get(agg, ())
    if agg:
        cfg.name = f"{cfg.name}_{name}"
    return cfg


def baked_tiny_pyramid(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """baked_tiny marched through the occupancy pyramid 128^3 .. 32^3 (the
    plain deferred MLP: a training configuration of the baked model)."""
    cfg = baked_tiny(seed, table_dtype)
    cfg.name = "baked_tiny_pyramid"
    cfg.occ_levels, cfg.occ_fine_res = 3, 128
    return cfg


def paper_tiny(seed: int = 0, table_dtype: int = DTYPE_F32) -> SceneConfig:
    """All of the paper's rendering choices at the tiny scale: the baked
    feature model (L_C = 64, fine levels 128 and 256), the occupancy pyramid
    128^3 .. 32^3 with the 64^3 distance grid, and the view-dependent MLP."""
    cfg = baked_tiny(seed, table_dtype)
    cfg.name = "paper_tiny"
    cfg.occ_levels, cfg.occ_fine_res = 3, 128
    cfg.mlp_dims = (23, 64, 64, 3)
    return cfg


def paper_hd(seed: int = 0, table_dtype: int = DTYPE_F32, n_fine: int = 2) -> SceneConfig:
    """All of the paper's rendering choices on the hd geometry: baked feature
    model (L_C = 512, n_fine fine levels), occupancy pyramid 512^3 .. 32^3 +
    256^3 distance grid, view-dependent MLP."""
    cfg = baked_hd(seed, table_dtype, n_fine)
    cfg.name = f"paper_hd_l{n_fine}"
    cfg.occ_levels, cfg.occ_fine_res = 5, 512
    cfg.mlp_dims = (23, 64, 64, 3)
    return cfg


CONFIGS = {"paper_tiny": paper_tiny, "paper_hd": paper_hd, "tiny_view": tiny_view, "tiny": tiny, "hd": hd, "hd_regime": hd_regime, "train_large": train_large, "baked_tiny": baked_tiny,
           "baked_tiny_pyramid": baked_tiny_pyramid,
           "baked_tiny_shared_v": lambda **k: with_aggregation(baked_tiny(**k), "shared_v"),
           "baked_tiny_separate_inv": lambda **k: with_aggregation(baked_tiny(**k), "separate_inv"),
           "baked_tiny_shared_inv": lambda **k: with_aggregation(baked_tiny(**k), "shared_inv"),
           "baked_tiny_sum": lambda **k: with_aggregation(baked_tiny(**k), "sum"),
           "baked_tiny_pyramid_shared_inv":
               lambda **k: with_aggregation(baked_tiny_pyramid(**k), "shared_inv"),
           "baked_tiny_l3": lambda **k: baked_tiny_levels(3, **k),
           "baked_tiny_l4": lambda **k: baked_tiny_levels(4, **k),
           "baked_hd": baked_hd, "tiny_pyramid": tiny_pyramid, "hd_pyramid": hd_pyramid}
