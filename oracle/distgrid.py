"""Occupancy distance grid G (Sec. 4.3, Eq. 9 and the paragraph before it).

G_p is the distance from voxel p to the nearest occupied position, rounded
down to an integer number of voxels and stored as uint8.  The paper leaves
the metric open; the reading used here is the *box gap*: the smallest
Euclidean distance between any point of voxel p and any point of an
occupied voxel q,

    gap(p, q) = sqrt( sum_i max(|p_i - q_i| - 1, 0)^2 )     (voxel units)
    G_p = min(255, floor( min_{q occupied} gap(p, q) )),

which makes Eq. 9's skip conservative: a point within G_p voxels of any
point of voxel p cannot lie inside an occupied voxel.  Occupied voxels and
their 26 neighbours get 0; a grid with no occupied voxel is 255 everywhere.

Two independent routes: brute force over occupied voxels (small grids), and
the squared Euclidean distance transform of the 26-dilated occupied set
(gap^2 to q equals the squared distance from p to the 3x3x3 block around q),
followed by an integer square root.
"""
from __future__ import annotations

import math

import numpy as np


def distance_grid_bruteforce(occ: np.ndarray, voxels=None) -> np.ndarray:
    """Brute-force G for all voxels (or for a [m,3] (x,y,z) subset)."""
    occ = np.asarray(occ, dtype=np.uint8)
    R = occ.shape[0]
    oz, oy, ox = np.nonzero(occ)
    occ_pts = np.stack([ox, oy, oz], axis=1).astype(np.int64)
    if voxels is None:
        zz, yy, xx = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
        voxels = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    voxels = np.asarray(voxels, dtype=np.int64)
    out = np.full(len(voxels), 255, dtype=np.int64)
    if len(occ_pts) == 0:
        return out.astype(np.uint8)
    chunk = max(1, 2_000_000 // max(len(occ_pts), 1))
    for s in range(0, len(voxels), chunk):
        v = voxels[s:s + chunk]
        gap = np.maximum(np.abs(v[:, None, :] - occ_pts[None, :, :]) - 1, 0)
        g2 = (gap ** 2).sum(axis=2).min(axis=1)
        out[s:s + chunk] = np.minimum(255, np.array([math.isqrt(int(a)) for a in g2]))
    return out.astype(np.uint8)


def distance_grid_full_bruteforce(occ: np.ndarray) -> np.ndarray:
    R = occ.shape[0]
    return distance_grid_bruteforce(occ).reshape(R, R, R)


def dilate26(occ: np.ndarray) -> np.ndarray:
    occ = np.asarray(occ, dtype=bool)
    out = np.zeros_like(occ)
    R = occ.shape
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                src = occ[max(0, -dz):R[0] - max(0, dz), max(0, -dy):R[1] - max(0, dy),
                          max(0, -dx):R[2] - max(0, dx)]
                out[max(0, dz):R[0] - max(0, -dz), max(0, dy):R[1] - max(0, -dy),
                    max(0, dx):R[2] - max(0, -dx)] |= src
    return out


def distance_grid_edt(occ: np.ndarray) -> np.ndarray:
    """G via the exact Euclidean distance transform of the dilated set.

    scipy's EDT supplies, for every voxel, the index of a nearest dilated
    voxel; the squared distance to it is recomputed here in integers.
    """
    from scipy.ndimage import distance_transform_edt

    occ = np.asarray(occ, dtype=np.uint8)
    dil = dilate26(occ)
    if not dil.any():
        return np.full(occ.shape, 255, dtype=np.uint8)
    _, inds = distance_transform_edt(~dil, return_distances=True, return_indices=True)
    grid = np.indices(occ.shape)
    d2 = ((inds - grid).astype(np.int64) ** 2).sum(axis=0)
    root = np.floor(np.sqrt(d2.astype(np.float64))).astype(np.int64)
    # integer correction of the float root (exact isqrt)
    root -= (root * root > d2)
    root += ((root + 1) * (root + 1) <= d2)
    return np.minimum(root, 255).astype(np.uint8)
