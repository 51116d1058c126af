"""Seeded synthetic scene assets: hash tables, occupancy, deferred-MLP weights.

Everything here is scene construction.  It holds none of the rendering
arithmetic (no hashing, no marching, no distance transform): the renderer and
the oracle both receive these arrays as plain bytes.

Table layout: float32 [L][T][9], channels ordered
    [sigma_raw, r, g, b, s0, s1, s2, s3, logit]
i.e. the explicit deferred feature of a hash entry (density, diffuse colour,
4-D specular feature; Sec. 4.2 and the supplement's network design) plus one
attention logit per entry.

Value recipe (seeded):
* diffuse colour ~ U[0, 1]; specular features and logit ~ N(0, 0.5^2);
* sigma_raw = ln(s_sigma * exp(-|z|^2 / 2) + 1e-4), z ~ N(0, I_3): the
  log-density of a random point of a random isotropic Gaussian blob.  The
  density channel therefore follows the blob density distribution without the
  generator having to know where a hash entry lands in space.
Occupancy: voxel occupied (1) where the blob mixture density at the voxel
centre exceeds 0.01; each blob contributes within 4 of its standard
deviations of its centre.  uint8 [R][R][R], x fastest (index x + R*(y + R*z)).
MLP: Xavier-uniform weights, zero biases, flattened row-major as
W0[16][7], b0[16], W1[16][16], b1[16], W2[3][16], b2[3].
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .configs import DOMAIN_BOX, DOMAIN_CONTRACT, SceneConfig


@dataclass
class Scene:
    cfg: SceneConfig
    tables: np.ndarray        # float32 [L, T, 9]
    occ: np.ndarray           # uint8 [R, R, R] (z, y, x)
    mlp: np.ndarray           # float32 [n_params]
    blob_mu: np.ndarray       # float64 [B, 3]
    blob_sigma: np.ndarray    # float64 [B]
    occ_fine: Optional[np.ndarray] = None   # uint8 [F, F, F] finest pyramid level (occ_levels > 0)

    @property
    def grid_lo(self) -> float:
        return -self.cfg.roi_half


def _blobs(cfg: SceneConfig, rng: np.random.Generator):
    lo, hi = cfg.blob_sigma
    if cfg.domain == DOMAIN_BOX:
        mu = rng.uniform(-cfg.blob_centre_half, cfg.blob_centre_half, size=(cfg.n_blobs, 3))
        sig = rng.uniform(lo, hi, size=cfg.n_blobs)
        return mu, sig
    # contracted domain: centres uniform in the ball of radius blob_centre_half,
    # rejecting blobs that would swallow a camera's contracted position.
    cams = camera_positions(cfg)
    r_c = 2.0 - 1.0 / np.linalg.norm(cams, axis=1)
    cams_c = cams / np.linalg.norm(cams, axis=1, keepdims=True) * r_c[:, None]
    mus, sigs = [], []
    while len(mus) < cfg.n_blobs:
        p = rng.uniform(-cfg.blob_centre_half, cfg.blob_centre_half, size=3)
        s = rng.uniform(lo, hi)
        if np.linalg.norm(p) >= cfg.blob_centre_half:
            continue
        if np.min(np.linalg.norm(cams_c - p, axis=1)) < 3.0 * s:
            continue
        mus.append(p)
        sigs.append(s)
    return np.array(mus), np.array(sigs)


def camera_positions(cfg: SceneConfig, seed_offset: int = 0) -> np.ndarray:
    """Camera centres.  Box scenes: on the sphere of radius cam_radius, random
    direction from the seed.  Contracted scenes: evenly on the z = 0 ring."""
    if cfg.domain == DOMAIN_BOX:
        rng = np.random.default_rng(cfg.seed + 7919 + seed_offset)
        v = rng.normal(size=(cfg.n_cams, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True) * cfg.cam_radius
    th = 2.0 * np.pi * (np.arange(cfg.n_cams) + 0.0) / cfg.n_cams
    return np.stack([cfg.cam_radius * np.cos(th), cfg.cam_radius * np.sin(th),
                     np.zeros_like(th)], axis=1)


def occupancy_from_blobs(cfg: SceneConfig, mu: np.ndarray, sig: np.ndarray) -> np.ndarray:
    R = cfg.occ_res
    lo = -cfg.roi_half
    v = 2.0 * cfg.roi_half / R
    centres = lo + (np.arange(R) + 0.5) * v
    rho = np.zeros((R, R, R), dtype=np.float64)
    for b in range(len(sig)):
        r = 4.0 * sig[b]
        sl = []
        for a in range(3):
            i0 = max(int(np.floor((mu[b, a] - r - lo) / v)), 0)
            i1 = min(int(np.ceil((mu[b, a] + r - lo) / v)) + 1, R)
            sl.append((i0, i1))
        if any(i1 <= i0 for i0, i1 in sl):
            continue
        cx = centres[sl[0][0]:sl[0][1]] - mu[b, 0]
        cy = centres[sl[1][0]:sl[1][1]] - mu[b, 1]
        cz = centres[sl[2][0]:sl[2][1]] - mu[b, 2]
        d2 = cz[:, None, None] ** 2 + cy[None, :, None] ** 2 + cx[None, None, :] ** 2
        rho[sl[2][0]:sl[2][1], sl[1][0]:sl[1][1], sl[0][0]:sl[0][1]] += np.exp(-d2 / (2 * sig[b] ** 2))
    return (rho > 0.01).astype(np.uint8)


def make_tables(cfg: SceneConfig, rng: np.random.Generator) -> np.ndarray:
    L, T = cfg.n_levels, cfg.table_size
    tab = np.empty((L, T, 9), dtype=np.float32)
    for l in range(L):
        z2 = (rng.standard_normal((T, 3)) ** 2).sum(axis=1)
        tab[l, :, 0] = np.log(cfg.density_scale * np.exp(-0.5 * z2) + 1e-4)
        tab[l, :, 1:4] = rng.uniform(0.0, 1.0, size=(T, 3))
        tab[l, :, 4:9] = rng.normal(0.0, 0.5, size=(T, 5))
    return tab


def make_mlp(cfg: SceneConfig, rng: np.random.Generator) -> np.ndarray:
    i, h1, h2, o = cfg.mlp_dims
    parts = []
    for fin, fout in ((i, h1), (h1, h2), (h2, o)):
        a = np.sqrt(6.0 / (fin + fout))
        parts.append(rng.uniform(-a, a, size=(fout, fin)).ravel())
        parts.append(np.zeros(fout))
    return np.concatenate(parts).astype(np.float32)


def make_scene(cfg: SceneConfig, seed: Optional[int] = None) -> Scene:
    """Deterministic scene for ``cfg`` (``seed`` overrides cfg.seed for the
    table values and MLP; blob layout and occupancy always come from cfg.seed)."""
    rng_geo = np.random.default_rng(cfg.seed)
    mu, sig = _blobs(cfg, rng_geo)
    occ_fine = None
    if cfg.occ_levels > 0:
        # only the finest pyramid level, from the blobs: the coarser levels and
        # the grid behind the distance grid are the method's (OR pooling)
        fine_cfg = dataclasses.replace(cfg, occ_res=cfg.occ_fine_res)
        occ_fine = occupancy_from_blobs(fine_cfg, mu, sig)
        occ = None
    else:
        occ = occupancy_from_blobs(cfg, mu, sig)
    rng_val = np.random.default_rng(1_000_003 + (cfg.seed if seed is None else seed))
    tables = make_tables(cfg, rng_val)
    mlp = make_mlp(cfg, rng_val)
    return Scene(cfg=cfg, tables=tables, occ=occ, mlp=mlp, blob_mu=mu, blob_sigma=sig,
                 occ_fine=occ_fine)
