"""Pins of the proposal-network oracle: Fourier features in closed form,
gradients against central finite differences, labels on a closed-form slab."""
import math

import numpy as np

from oracle import proposal as P
from oracle.exact32 import F32


def test_fourier_closed_form():
    o = np.array([[0.5, 0.0, 0.25]])
    d = np.array([[1.0, -0.5, 0.125]])
    enc = P.fourier(o, d)
    r = [0.5, 0.0, 0.25, 1.0, -0.5, 0.125]
    for j in range(6):
        for k in range(4):
            assert math.isclose(enc[0, 8 * j + 2 * k], math.sin(2 ** k * math.pi * r[j]), abs_tol=1e-12)
            assert math.isclose(enc[0, 8 * j + 2 * k + 1], math.cos(2 ** k * math.pi * r[j]), abs_tol=1e-12)
    assert enc[0, 0] == 1.0 and abs(enc[0, 1]) < 1e-15          # sin(pi/2), cos(pi/2)
    assert P.N_PARAMS == 7556 and P.init_params(0).size == 7556


def test_proposal_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = 40
    o = rng.normal(size=(n, 3)) * 0.3
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    enc = P.fourier(o, d)
    p = P.init_params(1).astype(np.float64)
    p[3072:3136] = rng.normal(size=64) * 0.1
    labels = rng.uniform(0, 2, size=(n, 4))
    valid = rng.uniform(size=n) < 0.8
    for phase in (1, 2):
        f = P.forward(p, enc, bf16_operands=False)
        loss, g = P.loss_and_grad_out(f["out"], labels, valid, phase, 0.05)
        grad = P.backward(p, f, g, bf16_operands=False)
        # finite differences with the confidence target held fixed (it is a
        # non-differentiable function of the outputs)
        tgt_valid = valid
        idx = list(range(0, P.N_PARAMS, 97)) + [P.N_PARAMS - 1, 7296, 7552]
        h = 1e-6
        for i in idx:
            def L(pp):
                ff = P.forward(pp, enc, bf16_operands=False)
                out = ff["out"]
                v = tgt_valid.astype(np.float64)
                # pinball losses written out from their definition
                r0 = labels[:, 0] - out[:, 0]
                r1 = labels[:, 1] - out[:, 1]
                pin = np.maximum(0.05 * r0, -0.95 * r0) + np.maximum(0.95 * r1, -0.05 * r1)
                val = np.sum(v * (pin + (out[:, 2] - labels[:, 2]) ** 2)) / n
                if phase >= 2:
                    tgt = P.conf_target(f["out"], labels, valid, 0.05)
                    s = 1 / (1 + np.exp(-out[:, 3]))
                    val += -np.sum(tgt * np.log(s + 1e-12) + (1 - tgt) * np.log(1 - s + 1e-12)) / n
                return val
            pp = p.copy(); pp[i] += h
            pm = p.copy(); pm[i] -= h
            fd = (L(pp) - L(pm)) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (phase, i, fd, grad[i])


def test_labels_from_decided_samples():
    s_ray = np.array([0, 0, 0, 2, 2])
    s_t = np.array([0.1, 0.2, 0.3, 1.0, 1.5], F32)
    s_T = np.array([0.9, 0.4, 0.0005, 0.8, 0.7], F32)
    lab, valid = P.labels_from_march(3, s_ray, s_t, s_T)
    assert valid.tolist() == [True, False, True]
    # ray 0: T < 0.5 after the 2nd sample, < 1e-3 after the 3rd
    assert np.allclose(lab[0], [0.1, 0.3, 0.2, 1]) and np.allclose(lab[2], [1.0, 1.5, 1.5, 1])
    s_T2 = np.array([0.0009, 0.0005, 0.0001, 0.8, 0.7], F32)
    lab2, _ = P.labels_from_march(3, s_ray, s_t, s_T2)
    assert np.allclose(lab2[0], [0.1, 0.1, 0.1, 1])
    assert np.all(lab[1] == 0)


def test_interval_march_with_exact_labels_equals_plain():
    import synth
    from oracle.distgrid import distance_grid_edt
    from oracle.render import inputs_from_scene, render, render_proposal, scene_occupancy
    cfg = synth.tiny()
    sc = synth.make_scene(cfg)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::9], d[::9]
    ref = render(inp, o, d)
    lab, valid = P.labels_from_march(len(o), ref.s_ray, ref.s_t, ref.extra["s_T"])
    # an interval from the first to the last sample holds every sample
    t_last = np.zeros(len(o), np.float32)
    t_last[ref.s_ray] = ref.s_t          # samples are sorted by (ray, k): the last write wins
    prop = np.stack([lab[:, 0], t_last, lab[:, 2], valid.astype(np.float32)], axis=1)
    res, fb = render_proposal(inp, o, d, prop, 0.9, 0.0)
    assert np.array_equal(res.s_k, ref.s_k) and np.array_equal(res.n_samples, ref.n_samples)
    assert np.array_equal(res.rgb, ref.rgb) and not fb.any()
    assert (res.n_reads <= ref.n_reads).all()
    # an end before any sample: the ray resumes, and is the plain march
    bad = prop.copy()
    bad[:, 1] = -1.0
    bad[:, 3] = 1.0
    res2, fb2 = render_proposal(inp, o, d, bad, 0.9, 0.0)
    assert fb2[ref.n_samples > 0].all()
    assert np.array_equal(res2.s_k, ref.s_k) and np.array_equal(res2.rgb, ref.rgb)
    assert np.array_equal(res2.n_reads, ref.n_reads)
    # ending where T first drops below 1e-3 drops the tail samples, which
    # carry at most 1e-3 of the colour weight
    cut = prop.copy()
    cut[:, 1] = lab[:, 1]
    res3, _ = render_proposal(inp, o, d, cut, 0.9, 0.0)
    assert (res3.n_samples <= ref.n_samples).all() and (res3.n_samples < ref.n_samples).any()
    assert np.abs(res3.c_d - ref.c_d).max() <= 1.05e-3 * np.abs(ref.c_d).max() + 1e-12
    assert np.all((res3.t_final <= 1e-3 + 1e-9) | (res3.n_samples == ref.n_samples))


def test_interval_render_is_a_filter_of_the_exhaustive_march():
    """With both ends used, a proposed ray's samples are the occupied lattice
    points of the exhaustive (naive, no termination) march whose t lies in
    [t_near - m, t_far + m], in order, cut where its own transmittance
    crosses the threshold; a ray whose padded interval holds none of them
    is the plain march, with the reads of both marches counted."""
    import synth
    from oracle.distgrid import distance_grid_edt
    from oracle.render import inputs_from_scene, march, ray_box32, render, render_proposal, scene_occupancy
    cfg = synth.tiny()
    sc = synth.make_scene(cfg)
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)))
    o, d, _ = synth.scene_rays(cfg)
    o, d = o[::11], d[::11]
    n = len(o)
    rng = np.random.default_rng(8)
    lo = rng.uniform(0.0, 0.4, n).astype(np.float32)
    hi = (lo + rng.uniform(0.0, 0.3, n)).astype(np.float32)
    margin = np.float32(2.0 / 256.0)
    prop = np.stack([lo, hi, lo, rng.uniform(0, 1, n)], axis=1).astype(np.float32)
    res, fb = render_proposal(inp, o, d, prop, 0.5, float(margin))
    plain = render(inp, o, d)
    full = march(inp, o, d, naive=True, terminate=False)
    t0, _, _ = ray_box32(o, d, inp.roi_half)
    conf = prop[:, 3] >= np.float32(0.5)
    assert fb.any() and (conf & ~fb).any() and (~conf).any()
    for i in range(n):
        got = res.s_k[res.s_ray == i]
        if not conf[i] or fb[i]:
            assert np.array_equal(got, plain.s_k[plain.s_ray == i])
            extra = 0
            if fb[i]:
                iv = np.array([[prop[i, 0] - margin, prop[i, 1] + margin]], np.float32)
                extra = march(inp, o[i:i + 1], d[i:i + 1], intervals=iv)["n_reads"][0]
                assert march(inp, o[i:i + 1], d[i:i + 1], intervals=iv)["n_samples"][0] == 0
            assert res.n_reads[i] == plain.n_reads[i] + extra
            continue
        sel = full["s_ray"] == i
        t, k = full["s_t"][sel], full["s_k"][sel]
        # box lattice: the march starts at the lattice point at or before t_near - m
        kstart = np.floor((np.float32(prop[i, 0] - margin) - t0[i]) / np.float32(inp.step))
        keep = (k >= max(kstart, 0)) & (t <= prop[i, 1] + margin)
        want = k[keep]
        assert len(got) >= 1
        assert np.array_equal(got, want[:len(got)])
        # cut short only by termination
        assert len(got) == len(want) or res.t_final32[i] < np.float32(inp.t_threshold)
