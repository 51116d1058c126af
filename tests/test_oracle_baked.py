"""Pins of the baked-model oracle (coarse grid + sigmoid-gated fine levels)
against facts it does not compute itself: a library trilinear interpolation
of the dense vertex array, affine reproduction, the closed forms of the
separate attention (Sec. 4.2 Eq. 8) at saturated gates, and the
constant-density slab render."""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

from oracle import baked
from oracle.distgrid import distance_grid_edt
from oracle.exact32 import F32
from oracle.render import BOX, OracleInputs, fused32, fused64, render, scene_occupancy

LC = 20            # 21 vertices per axis -> 3 blocks of 8 (the last one partial)


def _grid(rng, L=2, empty_frac=0.3, C=None):
    C = 8 + 2 * L if C is None else C
    nb = (LC + 1 + 7) // 8
    present = rng.random((nb, nb, nb)) >= empty_frac
    index = np.full((nb, nb, nb), -1, np.int32)
    index[present] = np.arange(present.sum(), dtype=np.int32)
    atlas = rng.normal(size=(int(present.sum()), 8, 8, 8, C)).astype(F32)
    default = rng.normal(size=C).astype(F32)
    return index, atlas, default


def _dense(index, atlas, default):
    """Dense vertex array [LC+1]^3 x C (z, y, x) expanded block by block."""
    C = atlas.shape[-1]
    V = LC + 1
    dense = np.empty((V, V, V, C), np.float64)
    for z in range(V):
        for y in range(V):
            for x in range(V):
                b = index[z >> 3, y >> 3, x >> 3]
                dense[z, y, x] = atlas[b, z & 7, y & 7, x & 7] if b >= 0 else default
    return dense


def _inputs(index, atlas, default, L=2, T=1 << 10, tables=None, occ=None, res=None):
    rng = np.random.default_rng(5)
    if tables is None:
        tables = np.zeros((L, T, 9), F32)
        tables[..., :8] = rng.normal(size=(L, T, 8))
    R = 8
    occ = np.ones((R, R, R), np.uint8) if occ is None else occ
    return OracleInputs(tables=tables, occ=occ, dist=distance_grid_edt(occ),
                        mlp=np.zeros(451, F32), resolutions=list(res or [32, 64][:L]),
                        domain=BOX, roi_half=1.0, step=1.0 / 256, max_samples=1024,
                        t_threshold=1e-4, coarse_res=LC, block_index=index, atlas=atlas,
                        coarse_default=default)


def test_sparse_lookup_equals_library_trilinear_on_dense_grid():
    rng = np.random.default_rng(0)
    index, atlas, default = _grid(rng)
    inp = _inputs(index, atlas, default)
    dense = _dense(index, atlas, default)
    u = rng.random((500, 3))
    u[:20] = rng.integers(0, LC + 1, size=(20, 3)) / LC          # on vertices, incl. u = 1
    got = baked.coarse64(inp, u)
    p = u * LC                                                     # (x, y, z) vertex coordinates
    for c in range(dense.shape[-1]):
        want = map_coordinates(dense[..., c], [p[:, 2], p[:, 1], p[:, 0]], order=1, mode="nearest")
        np.testing.assert_allclose(got[:, c], want, rtol=0, atol=1e-12)
    got32 = baked.coarse32(inp, u.astype(F32))
    np.testing.assert_allclose(got32, baked.coarse64(inp, u.astype(F32).astype(np.float64)),
                               rtol=0, atol=1e-5)


def test_coarse_reproduces_affine_field():
    rng = np.random.default_rng(1)
    nb = (LC + 1 + 7) // 8
    index = np.arange(nb ** 3, dtype=np.int32).reshape(nb, nb, nb)
    C = 12
    A = rng.normal(size=(3, C))
    b0 = rng.normal(size=C)
    atlas = np.empty((nb ** 3, 8, 8, 8, C), F32)
    for bz in range(nb):
        for by in range(nb):
            for bx in range(nb):
                lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
                v = np.stack([bx * 8 + lx, by * 8 + ly, bz * 8 + lz], axis=-1) / 4.0   # exact in float32
                atlas[index[bz, by, bx]] = (v @ A + b0).astype(F32)
    inp = _inputs(index, atlas.astype(np.float64).astype(F32), np.zeros(C, F32))
    u = rng.random((300, 3))
    got = baked.coarse64(inp, u)
    # stored values are the float32 roundings of the affine values; compare
    # against the float64 affine field within the rounding of the stored values
    want = (u * LC / 4.0) @ A + b0
    assert np.abs(got - want).max() < 1e-5 * (1 + np.abs(want).max())


@pytest.mark.parametrize("omega,beta", [(40.0, 40.0), (-40.0, -40.0), (40.0, -40.0), (0.0, 0.0)])
def test_separate_attention_closed_forms(omega, beta):
    rng = np.random.default_rng(2)
    index, atlas, default = _grid(rng, empty_frac=0.0)
    atlas[..., 8::2] = omega
    atlas[..., 9::2] = beta
    inp = _inputs(index, atlas, default)
    u = rng.random((200, 3))
    fused, gw = fused64(inp, u)
    coarse = baked.coarse64(inp, u)[:, :8]
    # fine levels: plain trilinear lookups written out here from the hash definition
    fine = np.zeros((len(u), 8))
    for l, N in enumerate(inp.resolutions):
        p = u * N
        i0 = np.clip(np.floor(p), 0, N - 1).astype(np.int64)
        f = p - i0
        for c in range(8):
            b = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
            w = np.prod([f[:, a] if b[a] else 1 - f[:, a] for a in range(3)], axis=0)
            cx, cy, cz = (i0[:, a] + b[a] for a in range(3))
            h = (cx ^ ((cy * 2654435761) % 2 ** 32) ^ ((cz * 805459861) % 2 ** 32)) % inp.T
            fine += w[:, None] * inp.tables[l][h, :8]
    g_o = 1.0 / (1.0 + math.exp(-omega))
    g_b = 1.0 / (1.0 + math.exp(-beta))
    want = coarse.copy()
    want[:, 0] += g_o * fine[:, 0]
    want[:, 1:] += g_b * fine[:, 1:]
    np.testing.assert_allclose(fused, want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(gw, g_o, rtol=0, atol=1e-15)
    if omega < 0 and beta < 0:                      # gates shut: the coarse grid alone
        np.testing.assert_allclose(fused, coarse, atol=1e-12)


def _fine_by_hand(inp, u):
    """Per-level trilinear values [L, m, 8] of the fine tables, written out
    from the hash definition (x * 1 ^ y * 2654435761 ^ z * 805459861 mod T)."""
    out = []
    for l, N in enumerate(inp.resolutions):
        p = u * N
        i0 = np.clip(np.floor(p), 0, N - 1).astype(np.int64)
        f = p - i0
        v = np.zeros((len(u), 8))
        for c in range(8):
            b = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
            w = np.prod([f[:, a] if b[a] else 1 - f[:, a] for a in range(3)], axis=0)
            cx, cy, cz = (i0[:, a] + b[a] for a in range(3))
            h = (cx ^ ((cy * 2654435761) % 2 ** 32) ^ ((cz * 805459861) % 2 ** 32)) % inp.T
            v += w[:, None] * inp.tables[l][h, :8]
        out.append(v)
    return out


@pytest.mark.parametrize("agg", [baked.SHARED_V, baked.SEPARATE_INV, baked.SHARED_INV, baked.SUM])
def test_aggregation_variants_closed_forms(agg):
    """Table 3's other aggregations against the coarse grid interpolated by
    scipy on the dense vertex array and fine values written out by hand:
    Shared-Att (V) gates both modalities with g(a_l) of the interpolated a_l;
    the (Inv) variants use constant parameters; SUM adds the levels."""
    rng = np.random.default_rng(7)
    L = 2
    C = 8 + (L if agg == baked.SHARED_V else 0)
    index, atlas, default = _grid(rng, L=L, C=C)
    inp = _inputs(index, atlas, default, L=L)
    consts = (0.7, -1.1, 0.3, 1.9)
    inp.aggregation = agg
    inp.gate_params = consts[:2 * L] if agg == baked.SEPARATE_INV else consts[:L]
    u = rng.random((300, 3))
    fused, _ = fused64(inp, u)
    dense = _dense(index, atlas, default)
    p = u * LC
    co = np.stack([map_coordinates(dense[..., c], [p[:, 2], p[:, 1], p[:, 0]], order=1, mode="nearest")
                   for c in range(C)], axis=1)
    sig = lambda a: 1.0 / (1.0 + np.exp(-np.asarray(a, np.float64)))
    want = co[:, :8].copy()
    for l, v in enumerate(_fine_by_hand(inp, u)):
        if agg == baked.SHARED_V:
            gw = gb = sig(co[:, 8 + l])
        elif agg == baked.SEPARATE_INV:
            gw, gb = sig(consts[2 * l]), sig(consts[2 * l + 1])
        elif agg == baked.SHARED_INV:
            gw = gb = sig(consts[l])
        else:
            gw = gb = 1.0
        want[:, 0] += gw * v[:, 0]
        want[:, 1:] += np.reshape(gb, (-1, 1)) * v[:, 1:]
    np.testing.assert_allclose(fused, want, rtol=0, atol=1e-9)
    # the float32 chain follows the same aggregation
    f32, _, _ = fused32(inp, u.astype(F32))
    assert np.abs(f32 - fused64(inp, u.astype(F32).astype(np.float64))[0]).max() < 2e-5


def test_sum_equals_saturated_separate_gates_in_float32():
    """SUM takes gates of exactly 1, which is what the float32 sigmoid of
    +40 rounds to: the two float32 chains agree bit for bit."""
    rng = np.random.default_rng(8)
    index, atlas, default = _grid(rng, empty_frac=0.0)
    atlas[..., 8:] = 40.0
    default[8:] = 40.0
    sep = _inputs(index, atlas, default)
    summ = _inputs(index, np.ascontiguousarray(atlas[..., :8]), np.ascontiguousarray(default[:8]))
    summ.aggregation = baked.SUM
    u = rng.random((500, 3)).astype(F32)
    a, _, _ = fused32(sep, u)
    b, _, _ = fused32(summ, u)
    assert np.array_equal(a, b)


def test_float32_chain_tracks_float64():
    rng = np.random.default_rng(3)
    index, atlas, default = _grid(rng)
    inp = _inputs(index, atlas, default)
    u = rng.random((1000, 3)).astype(F32)
    f32, g32, idx = fused32(inp, u)
    f64, g64 = fused64(inp, u.astype(np.float64))
    assert np.abs(f32 - f64).max() < 2e-5
    assert np.abs(g32 - g64).max() < 1e-6
    assert idx.shape == (1000, 2, 8)
    # the gates are the float32 sigmoid of the interpolated parameters
    co = baked.coarse32(inp, u)
    assert np.array_equal(g32[:, 1], baked.sigmoid32(co[:, 10]))


def test_constant_density_slab_closed_form():
    """Coarse grid of constant density and colour, fine levels zero: the
    render is the slab closed form C_d = c0 (1 - exp(-sigma n delta))."""
    nb = (LC + 1 + 7) // 8
    index = np.full((nb, nb, nb), -1, np.int32)
    C = 12
    default = np.zeros(C, F32)
    sigma_raw = 4.0
    c0 = np.array([0.2, 0.5, 0.9], F32)
    default[0] = sigma_raw
    default[1:4] = c0
    atlas = np.zeros((0, 8, 8, 8, C), F32)
    R = 64
    occ = np.zeros((R, R, R), np.uint8)
    za, zb = 20, 30
    occ[za:zb] = 1
    tables = np.zeros((2, 1 << 10, 9), F32)
    inp = _inputs(index, atlas, default, tables=tables, occ=occ)
    o = np.array([[0.1, 0.2, -1.0], [-0.37, 0.55, -1.0]], F32)
    d = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]], F32)
    res = render(inp, o, d)
    res_naive = render(inp, o, d, naive=True)
    sigma = math.exp(sigma_raw)
    dl = 1.0 / 256.0
    n_slab = 8 * (zb - za)
    n_star = math.floor(math.log(1e-4) / (-sigma * dl)) + 1
    n = min(n_slab, n_star)
    assert (res.n_samples == n).all() and np.array_equal(res.s_k, res_naive.s_k)
    Tf = math.exp(-sigma * n * dl)
    assert np.allclose(res.c_d, c0.astype(np.float64)[None] * (1 - Tf), atol=1e-12)


def test_baked_scene_march_skip_equals_naive():
    import synth
    from synth.baked import make_baked_scene
    from oracle.render import inputs_from_scene
    cfg = synth.CONFIGS["baked_tiny"]()
    sc = make_baked_scene(cfg)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    sel = slice(0, 4096, 13)
    a = render(inp, o[sel], d[sel])
    b = render(inp, o[sel], d[sel], naive=True)
    assert np.array_equal(a.s_ray, b.s_ray) and np.array_equal(a.s_k, b.s_k)
    assert 10 < a.n_samples.mean() < 30


def test_baked_gradient_matches_finite_differences():
    """The adjoint of the baked feature construction (coarse atlas rows,
    sigmoid gates, fine tables) through compositing and the MLP, against
    central differences of an MSE loss in float64."""
    import synth
    from synth.baked import make_baked_scene
    from oracle.grad import backward64, forward64, frozen_samples, mse_grad
    from oracle.render import inputs_from_scene
    cfg = synth.baked_tiny()
    sc = make_baked_scene(cfg)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::16], d[::16]
    s_ray, s_pos, _ = frozen_samples(inp, o, d)
    n = len(o)
    atlas = sc.atlas.astype(np.float64)
    fine = sc.tables.astype(np.float64)
    coarse = dict(atlas=atlas, default=sc.default.astype(np.float64), block_index=sc.block_index,
                  res=cfg.coarse_res)
    target = np.random.default_rng(0).random((n, 3))

    def loss():
        f = forward64(fine, sc.mlp, cfg.resolutions, cfg.step, n, s_ray, s_pos, coarse=coarse)
        return float(np.mean((f["rgb"] - target) ** 2))
    f = forward64(fine, sc.mlp, cfg.resolutions, cfg.step, n, s_ray, s_pos, coarse=coarse)
    (g_atlas, g_fine), _, _ = backward64(fine, sc.mlp, cfg.resolutions, cfg.step, n, s_ray, s_pos,
                                         mse_grad(f["rgb"], target), coarse=coarse)
    rng = np.random.default_rng(1)
    h = 1e-5
    checked = 0
    for arr, g in ((atlas, g_atlas), (fine, g_fine)):
        nz = np.argwhere(g != 0)
        for e in nz[rng.choice(len(nz), size=25, replace=False)]:
            e = tuple(e)
            orig = arr[e]
            arr[e] = orig + h
            lp = loss()
            arr[e] = orig - h
            lm = loss()
            arr[e] = orig
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[e]) <= 1e-4 * np.abs(g).max() + 1e-4 * abs(fd), (e, fd, g[e])
            checked += 1
    assert checked == 50
    assert np.all(g_fine[..., 8] == 0)
