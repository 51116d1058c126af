"""Seeded pinhole cameras producing ray batches (origins, unit directions).

Pinhole model, horizontal field of view ``fov_deg``, pixel centres at
(i + 0.5, j + 0.5), world up +z (falls back to +y when the view axis is
vertical), camera looking at the origin.  Directions are normalised in
float64 and stored as float32.

Rays are emitted in 8x8-tile-major order (tiles row-major over the image,
pixels row-major inside a tile) so that 64 consecutive rays cover one compact
pixel tile; ``pix`` maps each ray back to ``row * width + col``.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

from .configs import SceneConfig
from .scene import camera_positions


def tile_order(width: int, height: int, tile: int = 8, group: int = 1) -> np.ndarray:
    """Pixel indices (row*W + col) in tile-major order; with group > 1 the
    tiles are taken in blocks of group x group tiles (row-major over blocks,
    row-major inside a block, blocks clipped at the image edge)."""
    if width % tile or height % tile:
        raise ValueError("image size must be a multiple of the tile size")
    if group < 1:
        raise ValueError("group must be >= 1")
    ty, tx = np.meshgrid(np.arange(height // tile), np.arange(width // tile), indexing="ij")
    ty, tx = ty.ravel(), tx.ravel()
    order = np.lexsort((tx % group, ty % group, tx // group, ty // group))
    ty, tx = ty[order], tx[order]
    py, px = np.meshgrid(np.arange(tile), np.arange(tile), indexing="ij")
    rows = ty[:, None] * tile + py.ravel()[None, :]
    cols = tx[:, None] * tile + px.ravel()[None, :]
    return (rows * width + cols).ravel()


def pinhole_rays(cam_pos: np.ndarray, width: int, height: int, fov_deg: float = 60.0,
                 tile: int = 8, target=(0.0, 0.0, 0.0), group: int = 1
                 ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    cam_pos = np.asarray(cam_pos, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - cam_pos
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    if abs(np.dot(fwd, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    cam_up = np.cross(right, fwd)
    tan_h = np.tan(np.deg2rad(fov_deg) * 0.5)
    pix = tile_order(width, height, tile, group)
    rows = pix // width
    cols = pix % width
    xn = (2.0 * (cols + 0.5) / width - 1.0) * tan_h
    yn = (1.0 - 2.0 * (rows + 0.5) / height) * tan_h * height / width
    d = fwd[None, :] + xn[:, None] * right[None, :] + yn[:, None] * cam_up[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(cam_pos, d.shape)
    return (np.ascontiguousarray(o, dtype=np.float32),
            np.ascontiguousarray(d, dtype=np.float32), pix)


def scene_rays(cfg: SceneConfig, cams=None, width=None, height=None, group: int = 1):
    """All rays of the config's cameras, concatenated camera-major."""
    pos = camera_positions(cfg) if cams is None else np.asarray(cams)
    W = cfg.cam_width if width is None else width
    H = cfg.cam_height if height is None else height
    os_, ds_, ps_ = [], [], []
    for c in pos:
        o, d, p = pinhole_rays(c, W, H, cfg.fov_deg, group=group)
        os_.append(o)
        ds_.append(d)
        ps_.append(p)
    return np.concatenate(os_), np.concatenate(ds_), np.concatenate(ps_)


def random_sphere_cameras(n: int, radius: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True) * radius
