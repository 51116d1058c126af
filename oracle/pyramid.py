"""Multi-level occupancy march (test infrastructure): the paper's full
marching rule, Sec. 4.3 Eq. 9 with its s_O branch.

Occupancy pyramid: O_0 is the finest grid (resolution R_0, a sample is
taken where the lattice point's O_0 voxel is occupied); O_j has resolution
R_0 / 2^j and a voxel of O_j is occupied when any of its 8 children in
O_{j-1} is (supplement "Real-time Rendering" item 1: five levels 512^3 ...
32^3).  The distance grid G has resolution R_G (256 in the paper) and is
built from the pyramid level of that resolution.

At a lattice point that is not known to be empty, the levels are read from
the coarsest to the finest; the first unoccupied level is the exiting
level j.  Its voxel is empty, so the march may skip to the voxel's exit
(s_O).  When R_j < R_G the distance grid is read as well and a value g > 0
proves every point within g voxels of G empty (v * G in Eq. 9).  The march
skips by the larger of the two proven-empty distances.  A marching point is
a lattice point where occupancy is checked (Table 4's "# Marching"); the
grid words read there (one per level visited, plus G) are counted apart.

Skip arithmetic (float32, one IEEE operation each; the same margins as the
single-level march):
* box domain, voxel q of level j with edge v_j = (2 h) / R_j: per axis with
  d_a != 0, b_a = lo + float(q_a + [d_a > 0]) * v_j, t_a = (b_a - o_a) / d_a;
  t_exit = min_a t_a; J_O = floor((t_exit - t_k) / step) clamped to
  [1, 2^16]; the G rule gives J_G = floor(g * ((v_G / step) / |d|)) as in the
  single-level march; the next read is at k + max(J_O, J_G);
* contracted domain: the known-empty ball around the contracted read point y
  has radius max(r_O, r_G) with r_O = min_a min(y_a - lower_a,
  upper_a - y_a) - v_0/1024 (the ball inscribed in the empty voxel) and
  r_G = g * v_G - v_G/1024.
"""
from __future__ import annotations

import numpy as np

from .exact32 import F32

N_LEVELS = 5


def build_pyramid(occ_fine: np.ndarray, n_levels: int = N_LEVELS):
    """[O_0, O_1, ...] uint8 grids (z, y, x), O_j of resolution R_0 / 2^j,
    by OR over 2x2x2 children."""
    levels = [(np.asarray(occ_fine) != 0).astype(np.uint8)]
    for _ in range(1, n_levels):
        a = levels[-1]
        R = a.shape[0] // 2
        levels.append(a.reshape(R, 2, R, 2, R, 2).max(axis=(1, 3, 5)).astype(np.uint8))
    return levels


def exit_level(pyr, u: np.ndarray):
    """Coarse-to-fine reads at float32 grid coordinates u [m, 3]: returns the
    exiting level (-1: occupied at every level), the number of reads, and the
    exiting level's voxel index [m, 3] (x, y, z)."""
    m = u.shape[0]
    lev = np.full(m, -1, dtype=np.int64)
    reads = np.zeros(m, dtype=np.int64)
    qx = np.zeros((m, 3), dtype=np.int64)
    open_ = np.ones(m, dtype=bool)
    for j in range(len(pyr) - 1, -1, -1):
        R = pyr[j].shape[0]
        q = np.clip(np.floor(u * F32(R)), 0, R - 1).astype(np.int64)
        occ = pyr[j][q[:, 2], q[:, 1], q[:, 0]] != 0
        reads[open_] += 1
        empty = open_ & ~occ
        lev[empty] = j
        qx[empty] = q[empty]
        open_ &= occ
    return lev, reads, qx


def voxel_exit_t(o, d, q, lo, vj):
    """Float32 slab exit t of voxel q (edge vj) along rays (o, d)."""
    t = np.full(o.shape[0], np.inf, dtype=F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            up = d[:, a] > 0
            b = F32(lo) + (q[:, a] + up.astype(np.int64)).astype(F32) * F32(vj)
            ta = (b - o[:, a]) / d[:, a]
            ta = np.where(d[:, a] != 0, ta, F32(np.inf)).astype(F32)
            t = np.minimum(t, ta)
    return t


def inscribed_radius(y, q, lo, vj):
    """Float32 distance from y to the nearest face of voxel q (edge vj)."""
    r = np.full(y.shape[0], np.inf, dtype=F32)
    for a in range(3):
        lower = F32(lo) + q[:, a].astype(F32) * F32(vj)
        upper = F32(lo) + (q[:, a] + 1).astype(F32) * F32(vj)
        r = np.minimum(r, np.minimum(y[:, a] - lower, upper - y[:, a]))
    return r
