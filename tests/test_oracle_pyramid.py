"""Pins of the multi-level occupancy march (Sec. 4.3, Eq. 9 with its s_O
branch): the pyramid against its definition by loops, the sample lists of
the skipping march (with and without the distance grid) against the
exhaustive march over the finest level (the paper's Table 4 invariant: the
occupied-point count does not change), and marching-point counts in closed
form on an empty scene."""
import numpy as np
import pytest

import synth
from oracle import pyramid
from oracle.distgrid import distance_grid_edt
from oracle.exact32 import F32
from oracle.render import BOX, CONTRACT, OracleInputs, inputs_from_scene, render, scene_occupancy


def test_pyramid_is_or_of_children():
    rng = np.random.default_rng(0)
    fine = (rng.random((64, 64, 64)) < 0.02).astype(np.uint8)
    pyr = pyramid.build_pyramid(fine, 3)
    assert [p.shape[0] for p in pyr] == [64, 32, 16]
    for j in (1, 2):
        R = pyr[j].shape[0]
        f = 1 << j
        for z in range(0, R, 3):
            for y in range(0, R, 5):
                for x in range(R):
                    want = fine[z * f:(z + 1) * f, y * f:(y + 1) * f, x * f:(x + 1) * f].any()
                    assert pyr[j][z, y, x] == want


def _inputs(fine, levels, R_g, domain=BOX, use_dist=True, roi_half=1.0, step=1.0 / 256):
    pyr = pyramid.build_pyramid(fine, levels)
    occ = next(p for p in pyr if p.shape[0] == R_g)
    L, T = 2, 1 << 10
    tab = np.zeros((L, T, 9), F32)
    tab[..., 0] = 2.0
    tab[..., 1:4] = 0.5
    return OracleInputs(tables=tab, occ=occ, dist=distance_grid_edt(occ), mlp=np.zeros(451, F32),
                        resolutions=[16, 32], domain=domain, roi_half=roi_half, step=step,
                        max_samples=1024, t_threshold=1e-4, pyramid=pyr, use_dist=use_dist)


def _rays(rng, n, domain):
    if domain == BOX:
        o = rng.uniform(-1.5, 1.5, size=(n, 3)).astype(F32)
        tgt = rng.uniform(-0.8, 0.8, size=(n, 3))
    else:
        o = rng.uniform(-3, 3, size=(n, 3)).astype(F32)
        tgt = rng.uniform(-1.5, 1.5, size=(n, 3))
    d = tgt - o
    return o, (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(F32)


@pytest.mark.parametrize("domain,use_dist", [(BOX, True), (BOX, False), (CONTRACT, True),
                                             (CONTRACT, False)])
def test_skip_march_equals_exhaustive_finest_level(domain, use_dist):
    rng = np.random.default_rng(1 + domain)
    fine = np.zeros((128, 128, 128), np.uint8)
    for _ in range(12):                                   # a few solid boxes
        c = rng.integers(10, 118, size=3)
        h = rng.integers(2, 10, size=3)
        fine[c[2] - h[2]:c[2] + h[2], c[1] - h[1]:c[1] + h[1], c[0] - h[0]:c[0] + h[0]] = 1
    if domain == BOX:
        inp = _inputs(fine, 3, 64, BOX, use_dist)
    else:
        inp = _inputs(fine, 3, 64, CONTRACT, use_dist, roi_half=2.0, step=2 * np.sqrt(3) / 512)
    inp.t_threshold = 0.0                                 # march every ray to its end
    o, d = _rays(rng, 300, domain)
    a = render(inp, o, d)
    b = render(inp, o, d, naive=True)
    assert np.array_equal(a.s_ray, b.s_ray) and np.array_equal(a.s_k, b.s_k)
    assert a.n_samples.sum() > 100
    assert a.n_reads.sum() < b.n_reads.sum()              # skipping visits fewer points


def test_distance_grid_reduces_marching_points_on_tiny_scene():
    cfg = synth.tiny_pyramid()
    sc = synth.make_scene(cfg)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    sel = slice(0, 4096, 5)
    with_g = render(inp, o[sel], d[sel])
    inp.use_dist = False
    without = render(inp, o[sel], d[sel])
    assert np.array_equal(with_g.s_k, without.s_k)
    assert with_g.n_reads.sum() < without.n_reads.sum()


def test_empty_scene_marching_points_closed_form():
    """Empty 128^3 .. 32^3 pyramid, ray along +z from the cube's face: each
    32^3 voxel spans 16 lattice steps, so without G the march checks one point
    per coarsest voxel (32 in all), one grid word each; with G (255
    everywhere) the first check jumps past the cube."""
    fine = np.zeros((128, 128, 128), np.uint8)
    o = np.array([[0.1, -0.3, -1.0]], F32)
    d = np.array([[0.0, 0.0, 1.0]], F32)
    inp = _inputs(fine, 3, 64, BOX, use_dist=False)
    r = render(inp, o, d)
    assert r.n_samples[0] == 0 and r.n_reads[0] == 32 and r.extra["n_mem"][0] == 32
    inp = _inputs(fine, 3, 64, BOX, use_dist=True)
    r = render(inp, o, d)
    assert r.n_reads[0] == 1 and r.extra["n_mem"][0] == 2
