"""The allocation-free render backward (ngprt_render_backward_noalloc: its
workspace is the library's static device scratch) against the allocating
entry point it mirrors (ngprt_render_backward_reg), through the C ABI.

Two calls in a row on one context, the first at the largest batch the static
scratch holds and the second smaller and ragged, so the second call runs on a
scratch the first left full.  The MLP gradient is summed in a fixed order on
both paths, so it must agree bit for bit; the table gradient is summed with
float atomics in an order that varies from run to run, so it must agree to
float32 rounding of the sums and touch exactly the same entries."""
import numpy as np
import pytest

import synth

from helpers import gpu_renderer, to_gpu

pytestmark = pytest.mark.gpu


def _rays(n, seed):
    cfg = synth.tiny()
    cams = synth.random_sphere_cameras(32, 1.0, seed=seed)
    o, d, _ = synth.scene_rays(cfg, cams=cams, width=128, height=128)
    return o[:n], d[:n]


def _both(r, o, d, g_rgb, g_dist):
    import torch
    go, gd, gg = to_gpu(o, d, g_rgb)
    gdist = to_gpu(g_dist)[0] if g_dist is not None else None
    outs = []
    for fn in (r.backward, r.backward_noalloc):
        gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
        gm = torch.zeros((r.n_mlp,), dtype=torch.float32, device="cuda")
        fn(go, gd, gg, gt, gm, grad_dist=gdist)
        torch.cuda.synchronize()
        outs.append((gt.cpu().numpy(), gm.cpu().numpy()))
    return outs


def _check(outs):
    (t_ref, m_ref), (t_na, m_na) = outs
    assert np.array_equal(m_na, m_ref), np.abs(m_na - m_ref).max()
    assert np.array_equal(t_na == 0, t_ref == 0)
    scale = np.abs(t_ref).max()
    assert scale > 0
    err = np.abs(t_na - t_ref)
    assert np.all(err <= 1e-5 * scale + 1e-5 * np.abs(t_ref)), err.max() / scale


def test_noalloc_backward_matches_allocating_backward_twice():
    from paper_2407_10482_amd._lib import NOALLOC_MAX_RAYS
    print("[noalloc backward: tiny scene, 2 calls]", flush=True)
    r = gpu_renderer("tiny")
    rng = np.random.default_rng(5)
    # call 1: the largest batch the static scratch holds
    o, d = _rays(NOALLOC_MAX_RAYS, seed=11)
    assert len(o) == NOALLOC_MAX_RAYS
    g_rgb = rng.normal(0.0, 1e-3, (len(o), 3)).astype(np.float32)
    _check(_both(r, o, d, g_rgb, None))
    # call 2: smaller and ragged (not a multiple of 64), with the distortion term
    o2, d2 = _rays(3001, seed=12)
    g2 = rng.normal(0.0, 1e-2, (len(o2), 3)).astype(np.float32)
    gd2 = np.full((len(o2),), 0.01, dtype=np.float32)
    _check(_both(r, o2, d2, g2, gd2))
    r.close()


def test_noalloc_backward_rejects_batches_beyond_the_scratch():
    import torch
    from paper_2407_10482_amd._lib import NOALLOC_MAX_RAYS, NgprtError, check
    print("[noalloc backward: size limit]", flush=True)
    r = gpu_renderer("tiny")
    o, d = _rays(64, seed=13)
    go, gd, gg = to_gpu(o, d, np.zeros((64, 3), np.float32))
    gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device="cuda")
    gm = torch.zeros((r.n_mlp,), dtype=torch.float32, device="cuda")
    # the size check comes first, so nothing is enqueued and no pointer is read
    rc = r.lib.ngprt_render_backward_noalloc(r.ctx, NOALLOC_MAX_RAYS + 1, go.data_ptr(), gd.data_ptr(),
                                             gg.data_ptr(), None, gt.data_ptr(), gm.data_ptr(), None)
    assert rc == -2
    assert b"NGPRT_NOALLOC_MAX_RAYS" in r.lib.ngprt_last_error(r.ctx)
    # a batch within the limit still runs after the rejection
    r.backward_noalloc(go, gd, gg, gt, gm)
    torch.cuda.synchronize()
    with pytest.raises(NgprtError):
        check(rc, r.ctx)
    r.close()
