"""Seeded assets of the baked feature model (the paper's own construction,
Sec. 4.1 Eq. 6: a coarse grid holding the deferred features and per-level
attention parameters, plus fine hash levels).

Coarse grid: vertex lattice (L_C + 1)^3 over the grid domain, stored
block-sparse in blocks of 8^3 vertices.
* ``block_index`` int32 [nb][nb][nb] (z, y, x; nb = ceil((L_C + 1) / 8)):
  the block's row in the atlas, or -1 for an empty block;
* ``atlas`` float32 [n_blocks][8][8][8][C] (z, y, x within the block), with
  C = 8 + 2L channels [sigma~, r, g, b, s0..s3, omega_1, beta_1, ...,
  omega_L, beta_L] (attention parameters before their sigmoid);
* ``default`` float32 [C]: the value of every vertex of an empty block.

Value recipe (seeded): sigma~ = ln(s_sigma * rho(x) + 1e-4) with rho the
blob mixture density at the vertex (each blob truncated at 4 standard
deviations); colour ~ U[0, 1]; specular features ~ N(0, 0.5^2); omega, beta
~ N(0, 1).  A block is stored when rho exceeds 1e-3 at one of its vertices.
The default row is [ln(1e-4), 0, ..., 0].
Fine levels: float32 [L][T][9] in the hash-table layout of the hash model,
channel 8 unused (0): sigma^ ~ N(0, 0.5^2), colour ~ N(0, 0.2^2), specular
~ N(0, 0.5^2).  Occupancy and MLP as in the hash model's scenes.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from .configs import BLOCK, MODEL_BAKED, SceneConfig
from .scene import _blobs, make_mlp, occupancy_from_blobs


@dataclass
class BakedScene:
    cfg: SceneConfig
    tables: np.ndarray         # float32 [L, T, 9] fine hash levels (channel 8 unused)
    occ: np.ndarray            # uint8 [R, R, R]
    mlp: np.ndarray            # float32 [451]
    block_index: np.ndarray    # int32 [nb, nb, nb]
    atlas: np.ndarray          # float32 [n_blocks, 8, 8, 8, C]
    default: np.ndarray        # float32 [C]
    blob_mu: np.ndarray
    blob_sigma: np.ndarray
    occ_fine: np.ndarray = None   # uint8 [F, F, F] finest pyramid level (occ_levels > 0)

    @property
    def n_blocks(self) -> int:
        return self.atlas.shape[0]


def n_blocks_per_axis(coarse_res: int) -> int:
    return (coarse_res + 1 + BLOCK - 1) // BLOCK


def _block_density(cfg: SceneConfig, mu, sig, blocks: np.ndarray) -> np.ndarray:
    """Blob mixture density at the 8^3 vertices of the given blocks
    ([m, 3] block coordinates z, y, x) -> float64 [m, 8, 8, 8] (z, y, x)."""
    Lc = cfg.coarse_res
    lo = -cfg.roi_half
    h = 2.0 * cfg.roi_half / Lc                          # vertex spacing
    m = len(blocks)
    rho = np.zeros((m, BLOCK, BLOCK, BLOCK))
    off = np.arange(BLOCK)
    # vertex coordinates per block and axis: [m, 8]
    coords = [lo + (blocks[:, a:a + 1] * BLOCK + off[None, :]) * h for a in range(3)]   # z, y, x
    for b in range(len(sig)):
        r = 4.0 * sig[b]
        near = np.ones(m, bool)
        for a, ax in enumerate((2, 1, 0)):               # block axis a holds world axis ax
            c = coords[a]
            near &= (c.max(axis=1) >= mu[b, ax] - r) & (c.min(axis=1) <= mu[b, ax] + r)
        idx = np.nonzero(near)[0]
        if len(idx) == 0:
            continue
        g = []
        for a, ax in enumerate((2, 1, 0)):
            d = coords[a][idx] - mu[b, ax]
            gv = np.exp(-d * d / (2.0 * sig[b] ** 2))
            gv[np.abs(d) > r] = 0.0
            g.append(gv)
        rho[idx] += g[0][:, :, None, None] * g[1][:, None, :, None] * g[2][:, None, None, :]
    return rho


def make_baked_scene(cfg: SceneConfig, seed=None) -> BakedScene:
    if cfg.model != MODEL_BAKED:
        raise ValueError("config is not a baked-model config")
    rng_geo = np.random.default_rng(cfg.seed)
    mu, sig = _blobs(cfg, rng_geo)
    occ_fine = None
    if cfg.occ_levels > 0:
        occ_fine = occupancy_from_blobs(dataclasses.replace(cfg, occ_res=cfg.occ_fine_res), mu, sig)
        occ = None           # the coarser levels are the method's (OR pooling)
    else:
        occ = occupancy_from_blobs(cfg, mu, sig)
    nb = n_blocks_per_axis(cfg.coarse_res)
    # candidate blocks: within 4 standard deviations of some blob
    Lc = cfg.coarse_res
    h = 2.0 * cfg.roi_half / Lc
    cand = np.zeros((nb, nb, nb), bool)
    for b in range(len(sig)):
        r = 4.0 * sig[b]
        rng_ax = []
        for ax in (2, 1, 0):
            v0 = int(np.floor((mu[b, ax] - r + cfg.roi_half) / h)) // BLOCK
            v1 = int(np.floor((mu[b, ax] + r + cfg.roi_half) / h)) // BLOCK
            rng_ax.append((max(v0, 0), min(v1, nb - 1)))
        (z0, z1), (y0, y1), (x0, x1) = rng_ax
        if z1 >= z0 and y1 >= y0 and x1 >= x0:
            cand[z0:z1 + 1, y0:y1 + 1, x0:x1 + 1] = True
    blocks = np.argwhere(cand)                           # [m, 3] z, y, x, C order
    rho = np.zeros((0, BLOCK, BLOCK, BLOCK))
    chunks = []
    for s in range(0, len(blocks), 4096):
        chunks.append(_block_density(cfg, mu, sig, blocks[s:s + 4096]))
    if chunks:
        rho = np.concatenate(chunks)
    keep = rho.reshape(len(rho), -1).max(axis=1) > 1e-3 if len(rho) else np.zeros(0, bool)
    blocks, rho = blocks[keep], rho[keep]
    n_blocks = len(blocks)
    index = np.full((nb, nb, nb), -1, dtype=np.int32)
    index[blocks[:, 0], blocks[:, 1], blocks[:, 2]] = np.arange(n_blocks, dtype=np.int32)
    # every aggregation draws the same values (8 + 2L channels) and keeps its
    # own channels, so the variants share f~ and the fine tables
    C = 8 + 2 * cfg.n_levels
    rng_val = np.random.default_rng(2_000_003 + (cfg.seed if seed is None else seed))
    atlas = np.empty((n_blocks, BLOCK, BLOCK, BLOCK, C), dtype=np.float32)
    atlas[..., 0] = np.log(cfg.density_scale * rho + 1e-4)
    atlas[..., 1:4] = rng_val.uniform(0.0, 1.0, size=atlas[..., 1:4].shape)
    atlas[..., 4:8] = rng_val.normal(0.0, 0.5, size=atlas[..., 4:8].shape)
    atlas[..., 8:] = rng_val.normal(0.0, 1.0, size=atlas[..., 8:].shape)
    default = np.zeros(C, dtype=np.float32)
    default[0] = np.log(1e-4)
    L, T = cfg.n_levels, cfg.table_size
    tables = np.zeros((L, T, 9), dtype=np.float32)
    tables[:, :, 0] = rng_val.normal(0.0, 0.5, size=(L, T))
    tables[:, :, 1:4] = rng_val.normal(0.0, 0.2, size=(L, T, 3))
    tables[:, :, 4:8] = rng_val.normal(0.0, 0.5, size=(L, T, 4))
    mlp = make_mlp(cfg, rng_val)
    keep_ch = list(range(8))
    if cfg.aggregation == 0:
        keep_ch += list(range(8, C))
    elif cfg.aggregation == 1:                           # Shared-Att (V): a_l = the omega_l draw
        keep_ch += [8 + 2 * l for l in range(cfg.n_levels)]
    if len(keep_ch) != C:
        atlas = np.ascontiguousarray(atlas[..., keep_ch])
        default = np.ascontiguousarray(default[keep_ch])
    return BakedScene(cfg=cfg, tables=tables, occ=occ, mlp=mlp, block_index=index, atlas=atlas,
                      default=default, blob_mu=mu, blob_sigma=sig, occ_fine=occ_fine)
