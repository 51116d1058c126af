"""Deterministic table gradients (ngprt_set_deterministic_gradients):
records sorted by entry and summed in a fixed order give the same
gradient bit for bit on every run, equal to the atomic backward up to
the order of its float adds; the modes and shapes it refuses."""
import numpy as np
import pytest

import synth

from helpers import gpu_renderer, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _rays(name, n, seed=3):
    sc, _ = scene_and_dist(name)
    cfg = sc.cfg
    if cfg.domain == synth.DOMAIN_CONTRACT:
        o, d, _ = synth.scene_rays(cfg, cams=synth.camera_positions(cfg)[:2], width=256, height=128)
    else:
        o, d, _ = synth.scene_rays(cfg)
    sel = np.sort(np.random.default_rng(seed).choice(len(o), size=n, replace=False))
    return o[sel], d[sel]


def _grads(r, go, gd, g_rgb, fwd=None):
    import torch
    gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
    gm = torch.zeros((451,), dtype=torch.float32, device="cuda")
    if fwd is None:
        r.backward(go, gd, g_rgb, gt, gm)
    else:
        r.backward_fwd(go, gd, fwd["c_d"], fwd["feat"], g_rgb, gt, gm)
    torch.cuda.synchronize()
    return gt.cpu().numpy(), gm.cpu().numpy()


@pytest.mark.parametrize("name,n", [("tiny", 2048), ("train_large", 1024), ("hd", 512)])
def test_deterministic_gradients_repeat_bit_for_bit(name, n):
    import torch
    print(f"[deterministic gradients {name}]", flush=True)
    o, d = _rays(name, n)
    go, gd = to_gpu(o, d)
    g_rgb = torch.from_numpy(np.random.default_rng(1).standard_normal((n, 3)).astype(np.float32)).cuda()
    r = gpu_renderer(name)
    t_atomic, m_atomic = _grads(r, go, gd, g_rgb)
    r.set_deterministic(True)
    t1, m1 = _grads(r, go, gd, g_rgb)
    t2, m2 = _grads(r, go, gd, g_rgb)
    out = {"rgb": torch.empty((n, 3), device="cuda"), "c_d": torch.empty((n, 3), device="cuda"),
           "feat": torch.empty((n, 4), device="cuda")}
    r.render(go, gd, out=out)
    t3, m3 = _grads(r, go, gd, g_rgb, fwd=out)
    for t in (t2, t3):
        assert np.array_equal(t1.view(np.uint32), t.view(np.uint32))
    for m in (m1, m2, m3):
        assert np.array_equal(m.view(np.uint32), m_atomic.view(np.uint32))
    assert np.abs(t1).max() > 0
    assert np.array_equal(t1 != 0, t_atomic != 0)
    assert np.allclose(t1, t_atomic, rtol=1e-5, atol=1e-6 * np.abs(t_atomic).max())
    r.set_deterministic(False)
    t4, _ = _grads(r, go, gd, g_rgb)
    assert np.allclose(t4, t_atomic, rtol=1e-5, atol=1e-6 * np.abs(t_atomic).max())


def test_deterministic_gradients_refusals():
    import torch
    from paper_2407_10482_amd._lib import DET_MAX_RECORDS, NgprtError
    print("[deterministic gradients: refusals]", flush=True)
    # too many contributions for one call: refused before any record is made
    r = gpu_renderer("train_large")
    sc, _ = scene_and_dist("train_large")
    o, d, _ = synth.scene_rays(sc.cfg)
    reps = 64
    o, d = np.tile(o, (reps, 1)), np.tile(d, (reps, 1))
    go, gd = to_gpu(o, d)
    g_rgb = torch.ones((len(o), 3), device="cuda")
    r.set_deterministic(True)
    gt = torch.zeros((r.L, r.T, 9), device="cuda")
    gm = torch.zeros((451,), device="cuda")
    ns = r.render(go, gd)["n_samples"].long().sum().item()
    assert ns * r.L * 8 > DET_MAX_RECORDS
    with pytest.raises(NgprtError) as ei:
        r.backward(go, gd, g_rgb, gt, gm)
    assert ei.value.code == -2
    torch.cuda.synchronize()
    assert float(gt.abs().max()) == 0.0
    # the allocation-free entry point cannot make the records
    with pytest.raises(NgprtError) as ei:
        r.backward_noalloc(go[:64], gd[:64], g_rgb[:64], gt, gm)
    assert ei.value.code == -7
    # the baked model's backward is not built for it
    rb = gpu_renderer("baked_tiny")
    sb, _ = scene_and_dist("baked_tiny")
    ob, db, _ = synth.scene_rays(sb.cfg)
    gob, gdb = to_gpu(ob[:256], db[:256])
    rb.set_deterministic(True)
    with pytest.raises(NgprtError) as ei:
        rb.backward_baked(gob, gdb, torch.ones((256, 3), device="cuda"), torch.zeros((rb.L, rb.T, 9), device="cuda"),
                          torch.zeros(sb.atlas.shape, device="cuda"), torch.zeros((451,), device="cuda"))
    assert ei.value.code == -7
