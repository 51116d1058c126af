"""Pins of the CPU oracle against facts fixed outside it: the paper's
statements, closed forms, brute force and library routines.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import quant
from oracle.distgrid import (dilate26, distance_grid_bruteforce, distance_grid_edt,
                             distance_grid_full_bruteforce)
from oracle.exact32 import F32, exp32
from oracle.hashgrid import corners32, corners64, spatial_hash, spatial_hash_py
from oracle.render import (BOX, CONTRACT, OracleInputs, fused32, fused64, mlp64, render,
                           scene_occupancy)

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- hashing

def test_hash_golden_vectors():
    rows = [l.split() for l in open(os.path.join(GOLD, "hash_vectors.txt")) if not l.startswith("#")]
    for r in rows:
        x, y, z, h14, h19 = map(int, r)
        assert spatial_hash(x, y, z, 1 << 14) == h14
        assert spatial_hash(x, y, z, 1 << 19) == h19
        # hand check of the definition on the first non-trivial vector
    assert ((1 * 1) ^ ((2 * 2654435761) % 2 ** 32) ^ ((3 * 805459861) % 2 ** 32)) % (1 << 14) == 13788


def test_hash_numpy_matches_bigint_on_a_whole_level():
    N = 23
    c = np.arange(N + 1)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    h = spatial_hash(xx.ravel(), yy.ravel(), zz.ravel(), 1 << 14)
    ref = [spatial_hash_py(int(a), int(b), int(cz), 1 << 14)
           for a, b, cz in zip(xx.ravel(), yy.ravel(), zz.ravel())]
    assert np.array_equal(h, np.array(ref))


def test_corner_indices_are_hashes_of_the_enclosing_cell():
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 1, size=(500, 3)).astype(F32)
    N, T = 52, 1 << 14
    idx, w = corners32(u, N, T)
    for i in range(0, 500, 37):
        p = [float(u[i, a]) * N for a in range(3)]
        i0 = [min(max(int(math.floor(float(F32(u[i, a]) * F32(N)))), 0), N - 1) for a in range(3)]
        for c in range(8):
            b = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
            assert idx[i, c] == spatial_hash_py(i0[0] + b[0], i0[1] + b[1], i0[2] + b[2], T)
            wref = 1.0
            for a in range(3):
                f = p[a] - i0[a]
                wref *= f if b[a] else 1 - f
            assert abs(w[i, c] - wref) < 1e-5


# ---------------------------------------------------------------- trilinear

def test_trilinear_partition_of_unity():
    rng = np.random.default_rng(0)
    u = rng.uniform(0, 1, size=(2000, 3))
    for N in (16, 115, 4096):
        _, w = corners64(u, N, 1 << 19)
        assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
        _, w32 = corners32(u.astype(F32), N, 1 << 19)
        assert np.allclose(w32.astype(np.float64).sum(axis=1), 1.0, atol=1e-6)


def test_trilinear_reproduces_affine_field_on_injective_level():
    # N = 16, T = 2^19: 17^3 corners; check the hash is injective there, then store an
    # affine function of the corner coordinates and interpolate it.
    N, T = 16, 1 << 19
    c = np.arange(N + 1)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    h = spatial_hash(xx.ravel(), yy.ravel(), zz.ravel(), T)
    assert len(np.unique(h)) == h.size
    table = np.zeros(T)
    table[h] = 0.3 + 0.7 * xx.ravel() - 1.1 * yy.ravel() + 0.25 * zz.ravel()
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 1, size=(1000, 3))
    idx, w = corners64(u, N, T)
    val = (w * table[idx]).sum(axis=1)
    p = u * N
    assert np.allclose(val, 0.3 + 0.7 * p[:, 0] - 1.1 * p[:, 1] + 0.25 * p[:, 2], atol=1e-11)


def test_cell_decided_in_float32_below_an_integer():
    # u N within half an ulp below an integer k: the float32 product rounds
    # up to k, so the decided cell is k (not k - 1) with a negative fraction;
    # the float64 values use the same cell, and the trilinear formula there
    # equals the exact cell's value (the interpolant is continuous)
    N, T = 1351, 1 << 19
    found = []
    for k in range(300, 1300):
        u = np.nextafter(F32(k / N), F32(0.0))
        for _ in range(4):
            if float(u) * N < k and math.floor(float(F32(u) * F32(N))) == k:
                found.append((k, u))
                break
            u = np.nextafter(u, F32(0.0))
    assert found
    k, ux = found[0]
    u = np.array([[ux, F32(0.37), F32(0.61)]], dtype=F32)
    idx32, w32 = corners32(u, N, T)
    idx64, w64 = corners64(u, N, T)
    assert np.array_equal(idx32, idx64)
    f_exact = float(ux) * N - k
    assert f_exact < 0
    # corners 1, 3, 5, 7 (x + 1) carry the negative fraction
    assert np.all(w64[0, 1::2] < 0) and np.all(w32[0, 1::2] <= 0)
    assert abs(w64.sum() - 1.0) < 1e-14
    # an affine field is reproduced in the decided cell, as in the exact one
    c = np.array([[(k + (cc & 1)), 0, 0] for cc in range(8)], dtype=np.float64)
    val = (w64[0] * (0.5 + 2.0 * c[:, 0])).sum()
    assert abs(val - (0.5 + 2.0 * float(ux) * N)) < 1e-9


# ---------------------------------------------------------------- exp32 / sums

def test_exp32_accuracy_and_specials():
    x = np.linspace(-86.0, 88.0, 400001).astype(F32)
    y = exp32(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    rel = np.abs(y - ref) / ref
    assert rel.max() < 4.0 * 2.0 ** -23            # a few ulp
    assert exp32(F32(0.0)) == F32(1.0)
    assert exp32(F32(-87.0)) == 0.0 and exp32(F32(89.0)) == np.inf
    assert np.isnan(exp32(F32(np.nan)))
    # exp(a + b) ~ exp(a) exp(b) (no dropped scaling term)
    assert abs(float(exp32(F32(3.0))) - math.e ** 3) / math.e ** 3 < 5e-7


# ---------------------------------------------------------------- attention

def _tiny_inputs(tables, occ=None, dist=None, res=(16, 23, 35, 52), **kw):
    R = 16
    occ = np.zeros((R, R, R), np.uint8) if occ is None else occ
    dist = distance_grid_edt(occ) if dist is None else dist
    mlp = kw.pop("mlp", np.zeros(451, np.float32))
    args = dict(domain=BOX, roi_half=1.0, step=1.0 / 256.0, max_samples=1024, t_threshold=1e-4)
    args.update(kw)
    return OracleInputs(tables=tables, occ=occ, dist=dist, mlp=mlp, resolutions=list(res), **args)


def test_softmax_attention_properties():
    rng = np.random.default_rng(5)
    L, T = 4, 1 << 10
    tab = rng.normal(0, 0.5, size=(L, T, 9)).astype(F32)
    inp = _tiny_inputs(tab, res=(16, 23, 35, 52))
    u = rng.uniform(0, 1, size=(300, 3))
    fz, wl = fused64(inp, u)
    assert (wl > 0).all() and np.allclose(wl.sum(axis=1), 1.0, atol=1e-14)
    # equal logits -> uniform weights; fused = mean of levels
    tab2 = tab.copy()
    tab2[:, :, 8] = 0.37
    fz2, wl2 = fused64(_tiny_inputs(tab2), u)
    assert np.allclose(wl2, 1.0 / L)
    # shift invariance
    tab3 = tab.copy()
    tab3[:, :, 8] += 5.0
    _, wl3 = fused64(_tiny_inputs(tab3), u)
    assert np.allclose(wl3, wl, atol=1e-13)
    # all levels equal -> fused equals the common interpolated value
    tab4 = np.repeat(tab[:1], L, axis=0)
    tab4[:, :, 8] = rng.normal(size=(L, T))
    inp4 = _tiny_inputs(tab4, res=(16, 16, 16, 16))
    fz4, _ = fused64(inp4, u)
    idx, w = corners64(u, 16, T)
    common = np.einsum("mc,mcd->md", w, tab4[0][idx][:, :, :8].astype(np.float64))
    assert np.allclose(fz4, common, atol=1e-12)
    # float32 mirror (running-maximum softmax) agrees with the max-subtracted
    # float64 softmax to float32 rounding
    f32, w32, _ = fused32(inp, u.astype(F32))
    _, wref = fused64(inp, u.astype(F32).astype(np.float64))
    assert np.abs(w32 - wref).max() < 1e-6
    fz64, _ = fused64(inp, u.astype(F32).astype(np.float64))
    assert np.abs(f32 - fz64).max() < 1e-5


@pytest.mark.parametrize("case", ["outlier_entry", "all_very_negative", "all_very_positive", "ramp"])
def test_softmax_mirror_with_extreme_logits(case):
    """Eq. 8's softmax is invariant to a common shift of the logits, so the
    float32 mirror must return the softmax whatever their offset and spread:
    one table entry far above the rest (a shift by the table's largest
    logit would underflow every other sample's terms to 0), every logit far
    below or above 0 (exp of the raw logits would underflow or overflow),
    and levels whose logits differ by more than the float32 exponential's
    range (the weights of the lower levels are then exactly 0 and the fused
    value is the top level's own interpolated value)."""
    rng = np.random.default_rng(11)
    L, T = 4, 1 << 10
    res = (16, 23, 35, 52)
    tab = rng.normal(0, 0.5, size=(L, T, 9)).astype(F32)
    if case == "outlier_entry":
        tab[2, 17, 8] = 100.0
    elif case == "all_very_negative":
        tab[:, :, 8] -= 300.0
    elif case == "all_very_positive":
        tab[:, :, 8] += 200.0
    else:
        tab[:, :, 8] = (np.arange(L, dtype=F32) * 120.0)[:, None] + tab[:, :, 8]
    inp = _tiny_inputs(tab, res=res)
    u = rng.uniform(0, 1, size=(1000, 3)).astype(F32)
    f32, w32, _ = fused32(inp, u)
    fz64, w64 = fused64(inp, u.astype(np.float64))
    assert np.isfinite(f32).all() and np.isfinite(w32).all()
    # float32 interpolation rounds each logit a_l to within a few ulp of
    # its magnitude, which moves the weights by about that much: the
    # tolerance grows with the sample's largest |a_l| (2^-20 |a| is 8 ulp)
    amax = np.zeros(len(u))
    for l, N in enumerate(res):
        idx, w = corners64(u.astype(np.float64), N, T)
        amax = np.maximum(amax, np.abs(np.einsum("mc,mc->m", w, tab[l][idx][:, :, 8].astype(np.float64))))
    tol = 1e-6 + 2.0 ** -20 * amax
    assert (np.abs(w32 - w64).max(axis=1) <= tol).all()
    assert (np.abs(f32 - fz64).max(axis=1) <= 10 * tol).all()
    if case == "ramp":
        # the top level dominates: its interpolated channels, in closed form
        idx, w = corners64(u.astype(np.float64), res[-1], T)
        top = np.einsum("mc,mcd->md", w, tab[-1][idx][:, :, :8].astype(np.float64))
        assert np.array_equal(w32[:, :-1], np.zeros_like(w32[:, :-1]))
        assert np.abs(f32 - top).max() < 1e-5


# ---------------------------------------------------------------- distance grid

@pytest.mark.parametrize("seed,density", [(0, 0.002), (1, 0.01), (2, 0.05), (3, 0.0)])
def test_distance_grid_edt_equals_bruteforce(seed, density):
    rng = np.random.default_rng(seed)
    occ = (rng.uniform(size=(14, 14, 14)) < density).astype(np.uint8)
    assert np.array_equal(distance_grid_edt(occ), distance_grid_full_bruteforce(occ))


def test_distance_grid_single_voxel_closed_form():
    R = 20
    occ = np.zeros((R, R, R), np.uint8)
    occ[5, 9, 3] = 1                                   # (z, y, x)
    G = distance_grid_edt(occ)
    for (z, y, x) in [(5, 9, 3), (5, 9, 4), (6, 10, 4), (5, 9, 8), (19, 0, 19), (5, 1, 3)]:
        gap2 = max(abs(x - 3) - 1, 0) ** 2 + max(abs(y - 9) - 1, 0) ** 2 + max(abs(z - 5) - 1, 0) ** 2
        assert G[z, y, x] == min(255, math.isqrt(gap2))
    assert G[5, 9, 8] == 4 and G[5, 9, 4] == 0
    assert (distance_grid_edt(np.zeros((8, 8, 8), np.uint8)) == 255).all()


def test_distance_grid_conservative_and_tight_on_tiny_scene():
    from synth import make_scene, tiny
    sc = make_scene(tiny())
    G = distance_grid_edt(scene_occupancy(sc))
    rng = np.random.default_rng(11)
    vox = rng.integers(0, 64, size=(400, 3))
    bf = distance_grid_bruteforce(sc.occ, vox)
    assert np.array_equal(G[vox[:, 2], vox[:, 1], vox[:, 0]], bf)
    # clamp at 255 on a big empty grid
    occ = np.zeros((300, 4, 4), np.uint8)
    occ[0, 0, 0] = 1
    assert distance_grid_edt(occ)[299, 0, 0] == 255
    # occupied voxels and their neighbours are 0
    dil = dilate26(sc.occ)
    assert (G[dil] == 0).all() and (G[~dil] > 0).all()


# ---------------------------------------------------------------- march & compositing

def _slab_scene(sigma_raw, c0, v0, za, zb, R=64):
    L, T = 3, 1 << 10
    tab = np.zeros((L, T, 9), F32)
    tab[:, :, 0] = sigma_raw
    tab[:, :, 1:4] = c0
    tab[:, :, 4:8] = v0
    tab[:, :, 8] = np.random.default_rng(0).normal(size=(L, T))
    occ = np.zeros((R, R, R), np.uint8)
    occ[za:zb] = 1
    return _tiny_inputs(tab, occ=occ, res=(16, 23, 35))


@pytest.mark.parametrize("sigma_raw,expect_terminate", [(1.0, False), (3.0, False), (4.0, True), (8.0, True)])
def test_constant_density_slab_closed_form(sigma_raw, expect_terminate):
    za, zb = 20, 30
    c0 = np.array([0.2, 0.5, 0.9], F32)
    v0 = np.array([0.1, -0.3, 0.7, 0.05], F32)
    inp = _slab_scene(sigma_raw, c0, v0, za, zb)
    o = np.array([[0.1, 0.2, -1.0], [-0.37, 0.55, -1.0]], F32)
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]], F32)
    res = render(inp, o, d)
    res_naive = render(inp, o, d, naive=True)
    # lattice z_k = -1 + k/256 lies in voxel floor(k/8): slab holds k in [8 za, 8 zb)
    n_slab = 8 * (zb - za)
    sigma = math.exp(float(F32(sigma_raw)))
    dl = 1.0 / 256.0
    n_star = math.floor(math.log(1e-4) / (-sigma * dl)) + 1      # first n with T < 1e-4
    n = min(n_slab, n_star)
    assert (n < n_slab) == expect_terminate
    assert (res.n_samples == n).all() and np.array_equal(res.s_k, res_naive.s_k)
    assert np.array_equal(res.s_k[:n], np.arange(8 * za, 8 * za + n))
    Tf = math.exp(-sigma * n * dl)
    assert np.allclose(res.t_final, Tf, rtol=1e-12)
    assert np.allclose(res.c_d, c0.astype(np.float64)[None] * (1 - Tf), atol=1e-12)
    assert np.allclose(res.feat, v0.astype(np.float64)[None] * (1 - Tf), atol=1e-12)
    # the naive march reads every lattice point up to termination (512 inside the box)
    assert (res_naive.n_reads == (8 * za + n if expect_terminate else 512)).all()


def test_weights_telescope_to_one_minus_transmittance():
    from synth import make_scene, scene_rays, tiny
    sc = make_scene(tiny())
    tab = sc.tables.copy()
    tab[:, :, 1:4] = 1.0                          # unit colour everywhere
    inp = OracleInputs(tables=tab, occ=sc.occ, dist=distance_grid_edt(scene_occupancy(sc)), mlp=sc.mlp,
                       resolutions=sc.cfg.resolutions, domain=BOX, roi_half=1.0,
                       step=sc.cfg.step, max_samples=1024, t_threshold=1e-4)
    o, d, _ = scene_rays(sc.cfg)
    sel = slice(0, 4096, 9)
    r = render(inp, o[sel], d[sel])
    assert np.allclose(r.c_d, (1.0 - r.t_final)[:, None], atol=1e-12)
    # the float32 decision mirror tracks the float64 transmittance
    assert np.abs(r.t_final32 - r.t_final).max() < 1e-5


def test_skip_march_equals_naive_on_random_grids():
    rng = np.random.default_rng(21)
    for trial in range(3):
        R = 32
        occ = np.zeros((R, R, R), np.uint8)
        for _ in range(6):
            c = rng.integers(0, R, size=3)
            r = rng.integers(1, 5)
            occ[max(c[2] - r, 0):c[2] + r, max(c[1] - r, 0):c[1] + r, max(c[0] - r, 0):c[0] + r] = 1
        L, T = 4, 1 << 10
        tab = rng.normal(0, 0.5, size=(L, T, 9)).astype(F32)
        tab[:, :, 0] += 2.0
        inp = _tiny_inputs(tab, occ=occ)
        n = 400
        o = rng.uniform(-1.5, 1.5, size=(n, 3)).astype(F32)
        d = rng.normal(size=(n, 3))
        d[:40, 1:] = 0.0                          # axis-parallel rays
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d = d.astype(F32)
        a = render(inp, o, d)
        b = render(inp, o, d, naive=True)
        assert np.array_equal(a.s_ray, b.s_ray) and np.array_equal(a.s_k, b.s_k)
        assert np.array_equal(a.n_samples, b.n_samples)
        assert (a.n_reads <= b.n_reads).all()
        assert np.array_equal(a.t_final32, b.t_final32)


def test_skip_march_equals_naive_contracted():
    from synth.scene import occupancy_from_blobs
    from synth.configs import SceneConfig
    rng = np.random.default_rng(4)
    cfg = SceneConfig(name="c", n_levels=4, n_min=16, n_max=128, log2_table=12, domain=CONTRACT,
                      roi_half=2.0, occ_res=48, step=2 * math.sqrt(3) / 512 * 4, max_samples=1024,
                      t_threshold=1e-4, n_blobs=12, blob_sigma=(0.05, 0.15), blob_centre_half=1.8,
                      density_scale=50.0, cam_width=16, cam_height=16, n_cams=2, cam_radius=3.0)
    mu = rng.uniform(-1.2, 1.2, size=(12, 3))
    occ = occupancy_from_blobs(cfg, mu, rng.uniform(0.05, 0.15, size=12))
    L, T = 4, 1 << 12
    tab = rng.normal(0, 0.5, size=(L, T, 9)).astype(F32)
    tab[:, :, 0] += 1.0
    inp = OracleInputs(tables=tab, occ=occ, dist=distance_grid_edt(occ), mlp=np.zeros(451, F32),
                       resolutions=cfg.resolutions, domain=CONTRACT, roi_half=2.0, step=cfg.step,
                       max_samples=1024, t_threshold=1e-4)
    from synth.cameras import pinhole_rays
    o, d, _ = pinhole_rays(np.array([3.0, 0.2, 0.1]), 32, 32, 70.0)
    a = render(inp, o, d)
    b = render(inp, o, d, naive=True)
    assert a.n_samples.sum() > 0
    assert np.array_equal(a.s_ray, b.s_ray) and np.array_equal(a.s_k, b.s_k)
    assert (a.n_reads <= b.n_reads).all() and a.n_reads.sum() < b.n_reads.sum()


def test_contracted_lattice_has_equal_contracted_steps():
    from oracle.render import march
    step = 2 * math.sqrt(3) / 512
    tab = np.zeros((1, 16, 9), F32)
    occ = np.ones((8, 8, 8), np.uint8)            # everything occupied: every lattice point sampled
    inp = OracleInputs(tables=tab, occ=occ, dist=np.zeros_like(occ), mlp=np.zeros(451, F32),
                       resolutions=[4], domain=CONTRACT, roi_half=2.0, step=step,
                       max_samples=1024, t_threshold=0.0)
    o = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [0.3, -2.0, 0.5]], F32)
    d = np.array([[1.0, 0.0, 0.0], [-0.6, 0.8, 0.0], [0.0, 1.0, 0.0]], F32)
    m = march(inp, o, d)
    for r in range(3):
        p = m["s_pos"][m["s_ray"] == r].astype(np.float64)
        tw = m["s_t"][m["s_ray"] == r].astype(np.float64)
        rw = np.linalg.norm(o[r].astype(np.float64)[None] + tw[:-1, None] * d[r][None], axis=1)
        seg = np.linalg.norm(np.diff(p, axis=0), axis=1)
        # one Euler step of contracted arc length: exact (step) while |x| <= 1,
        # first-order accurate beyond, with relative error O(step * |x|)
        assert np.all(np.abs(seg / step - 1.0) <= 2.0 * step * np.maximum(rw, 1.0) + 1e-4)
        assert np.all(np.abs(seg[rw < 0.99] - step) < 1e-6)
        # contracted points stay inside the radius-2 ball
        assert np.linalg.norm(p, axis=1).max() < 2.0
    # radial ray from the origin ends where 1/r < step: contracted radius ~ 2 - step
    p0 = m["s_pos"][m["s_ray"] == 0]
    assert 2.0 - np.linalg.norm(p0[-1]) < 2 * step


def test_sample_coords64_closed_forms():
    """Float64 sample coordinates: a radial ray from the origin lands at
    contracted radius 2 - 1/t beyond the unit ball and at t inside it; every
    coordinate agrees with the float32 lattice position to float32 rounding;
    in the box domain the position is o + t d itself."""
    from oracle.render import march, sample_coords64
    step = 2 * math.sqrt(3) / 512
    tab = np.zeros((1, 16, 9), F32)
    occ = np.ones((8, 8, 8), np.uint8)
    for dom in (CONTRACT, BOX):
        half = 2.0 if dom == CONTRACT else 1.0
        inp = OracleInputs(tables=tab, occ=occ, dist=np.zeros_like(occ), mlp=np.zeros(451, F32),
                           resolutions=[4], domain=dom, roi_half=half, step=step,
                           max_samples=4096, t_threshold=0.0)
        o = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [0.2, -0.9, 0.5]], F32)
        d = np.array([[1.0, 0.0, 0.0], [-0.6, 0.8, 0.0], [0.0, 1.0, 0.0]], F32)
        m = march(inp, o, d)
        u = sample_coords64(inp, o, d, m["s_ray"], m["s_t"])
        x = (u * 2.0 * half) - half                          # back to positions
        t = m["s_t"].astype(np.float64)
        r0 = m["s_ray"] == 0
        if dom == CONTRACT:
            want = np.where(t[r0] > 1.0, 2.0 - 1.0 / np.maximum(t[r0], 1e-300), t[r0])
        else:
            want = t[r0]
        assert np.allclose(x[r0, 0], want, rtol=0, atol=1e-12)
        assert np.allclose(x[r0, 1:], 0.0, atol=1e-12)
        if dom == BOX:
            exact = o.astype(np.float64)[m["s_ray"]] + t[:, None] * d.astype(np.float64)[m["s_ray"]]
            assert np.allclose(x, exact, rtol=0, atol=1e-12)
        u32 = ((m["s_pos"].astype(np.float64)) + half) / (2.0 * half)
        assert np.abs(u - u32).max() < 1e-6
        assert len(t) > 100


def test_empty_rays_get_sigmoid_of_mlp_of_zero():
    rng = np.random.default_rng(2)
    tab = rng.normal(size=(3, 1 << 10, 9)).astype(F32)
    mlp = rng.normal(0, 0.3, size=451).astype(F32)
    inp = _tiny_inputs(tab, res=(16, 23, 35), mlp=mlp)
    o = np.array([[3.0, 3.0, 3.0], [0.0, 0.0, 0.0], [np.nan, 0, 0], [0.1, 0.1, 0.1]], F32)
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0, 0, 1], [0, 0, 0]], F32)
    r = render(inp, o, d)
    ref = 1.0 / (1.0 + np.exp(-mlp64(mlp, np.zeros((1, 7)))))
    assert (r.n_samples == 0).all()
    assert np.allclose(r.rgb, ref, atol=1e-15)


def test_mlp_matches_explicit_loops():
    rng = np.random.default_rng(8)
    p = rng.normal(size=451)
    x = rng.normal(size=(5, 7))
    W0 = p[:112].reshape(16, 7); b0 = p[112:128]
    W1 = p[128:384].reshape(16, 16); b1 = p[384:400]
    W2 = p[400:448].reshape(3, 16); b2 = p[448:451]
    for r in range(5):
        h1 = [max(0.0, sum(W0[j, i] * x[r, i] for i in range(7)) + b0[j]) for j in range(16)]
        h2 = [max(0.0, sum(W1[j, i] * h1[i] for i in range(16)) + b1[j]) for j in range(16)]
        out = [sum(W2[j, i] * h2[i] for i in range(16)) + b2[j] for j in range(3)]
        assert np.allclose(mlp64(p, x[r:r + 1])[0], out, atol=1e-12)


# ---------------------------------------------------------------- reduced precision

def test_bf16_exhaustive_decode_and_rne():
    codes = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    vals = quant.bf16_decode(codes)
    import struct
    for c in (0x0000, 0x3F80, 0xBF80, 0x7F7F, 0x0001, 0x4049):
        assert struct.unpack("<f", struct.pack("<I", c << 16))[0] == vals[c] or np.isnan(vals[c])
    finite = np.isfinite(vals)
    assert np.array_equal(quant.bf16_encode(vals[finite]), codes[finite])
    # halfway cases: ties to even
    x = np.array([0x3F808000, 0x3F818000, 0x3F808001, 0x3F807FFF], np.uint32).view(F32)
    assert list(quant.bf16_encode(x)) == [0x3F80, 0x3F82, 0x3F81, 0x3F80]


def test_fp8_e4m3fn_table_and_encoding():
    t = quant.FP8_TABLE
    assert t[0x7E] == 448.0 and t[0x38] == 1.0 and t[0x01] == 2.0 ** -9 and t[0x08] == 2.0 ** -6
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF]) and t[0xFE] == -448.0
    assert np.sum(np.isfinite(t)) == 254
    codes = np.array([c for c in range(256) if np.isfinite(t[c])], dtype=np.uint8)
    assert np.array_equal(quant.fp8_encode(t[codes].astype(F32)), codes)
    # ties to even: halfway between 1.0 (0x38) and 1.125 (0x39) -> 0x38;
    # between 1.125 and 1.25 (0x3A) -> 0x3A
    assert quant.fp8_encode(np.array([1.0625, 1.1875, 1000.0, -1000.0, np.nan], F32)).tolist() \
        == [0x38, 0x3A, 0x7E, 0xFE, 0x7F]
    # nearest: brute force over the table
    rng = np.random.default_rng(0)
    x = rng.normal(0, 50, size=3000).astype(F32)
    q = quant.fp8_encode(x)
    err = np.abs(t[q] - x.astype(np.float64))
    best = np.min(np.abs(t[codes][None, :] - np.clip(x, -448, 448)[:, None]), axis=1)
    assert np.allclose(err[np.abs(x) <= 448], best[np.abs(x) <= 448])


def test_fp8_scales_per_level_channel():
    rng = np.random.default_rng(1)
    tab = rng.normal(size=(3, 64, 9)).astype(F32)
    tab[1, :, 2] = 0.0
    q, s = quant.quantize_tables_fp8(tab)
    assert s[1, 2] == 1.0
    amax = np.abs(tab).max(axis=1)
    assert np.allclose(s[amax > 0], amax[amax > 0] / 448.0, rtol=1e-7)
    deq = quant.fp8_decode(q).astype(np.float64) * s[:, None, :]
    # 3 mantissa bits: half an ulp is 2^-4 relative for normals; below the
    # smallest normal (2^-6 in code units) the absolute error is 2^-10 * s
    floor = np.maximum(s[:, None, :].astype(np.float64) * 2.0 ** -6, 1e-30)
    rel = np.abs(deq - tab) / np.maximum(np.abs(tab), floor)
    assert rel.max() <= 2.0 ** -4 + 1e-6


def _round_to_f32_exact(q):
    """The float32 nearest to the rational q (ties to even), by exact
    comparison with its float32 neighbours."""
    from fractions import Fraction
    f = np.float32(float(q))                      # within an ulp of the answer
    best = None
    for cand in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - q)
        if best is None or d < best[0] or (d == best[0] and (int(np.array(cand).view(np.uint32)) & 1) == 0):
            best = (d, cand)
    return best[1]


def test_fma32_is_the_single_rounding_of_the_exact_value():
    """fma32 against exact rational arithmetic: random triples, cancellation
    (c close to -a b), and sums placed within float64 rounding of a float32
    halfway point, where a float64 sum rounded to float32 would round twice."""
    from fractions import Fraction
    from oracle.exact32 import fma32
    rng = np.random.default_rng(17)
    n = 4000
    a = (rng.normal(size=n) * np.exp2(rng.integers(-20, 20, n))).astype(np.float32)
    b = (rng.normal(size=n) * np.exp2(rng.integers(-20, 20, n))).astype(np.float32)
    c = (rng.normal(size=n) * np.exp2(rng.integers(-20, 20, n))).astype(np.float32)
    c[: n // 4] = (-(a[: n // 4].astype(np.float64) * b[: n // 4]) *
                   (1 + rng.normal(size=n // 4) * 1e-6)).astype(np.float32)
    # double-rounding traps: a = 1 + 2^-12 and b = (1 - 4095 2^-24) 2^-24 give
    # a b = 2^-24 + 2^-60 exactly; with c = t an even float32 in [1, 2), the
    # exact value lies 2^-60 above the halfway point t + 2^-24, the float64 sum
    # rounds onto that halfway point and a second rounding to float32 would
    # fall to t, while the single rounding goes up (signs flipped for half)
    m = n // 4
    t = (np.float32(1.0) + np.float32(2.0 ** -22) * rng.integers(0, 1 << 22, m).astype(np.float32))
    sign = np.where(np.arange(m) % 2 == 0, np.float32(1.0), np.float32(-1.0))
    a[-m:] = sign * np.float32(1.0 + 2.0 ** -12)
    b[-m:] = np.float32((1.0 - 4095 * 2.0 ** -24) * 2.0 ** -24)
    c[-m:] = sign * t
    got = fma32(a, b, c)
    for i in range(n):
        exact = Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i]))
        want = _round_to_f32_exact(exact)
        assert np.array(got[i]).view(np.uint32) == np.array(want).view(np.uint32), (i, a[i], b[i], c[i])
    # the trap cases really are ones where rounding the float64 sum differs
    naive = (a.astype(np.float64) * b + c).astype(np.float32)
    assert np.all(naive[-m:] != got[-m:])
