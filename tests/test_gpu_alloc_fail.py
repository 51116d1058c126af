"""Allocation failures injected by the library's test hook
(ngprt_test_fail_alloc): the call that meets one returns NGPRT_E_ALLOC,
leaks nothing it would reuse, and leaves its context usable."""
import numpy as np
import pytest

import synth
from oracle.render import render

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu
E_ALLOC = -5


def _lib():
    from paper_2407_10482_amd._lib import load_library
    return load_library()


@pytest.fixture(autouse=True)
def _disarm():
    yield
    _lib().ngprt_test_fail_alloc(-1)


def test_create_fails_at_each_allocation_then_succeeds():
    from paper_2407_10482_amd._lib import NgprtError
    print("[alloc fail: create]", flush=True)
    failures = 0
    for k in range(16):
        _lib().ngprt_test_fail_alloc(k)
        try:
            r = gpu_renderer("tiny")
        except NgprtError as e:
            assert e.code == E_ALLOC, e
            failures += 1
            continue
        _lib().ngprt_test_fail_alloc(-1)
        break
    else:
        pytest.fail("no allocation count let the context come up")
    assert failures >= 5      # tables, logits, scales, grid, MLP at least
    # the context that came up renders like any other
    inp = oracle_inputs("tiny")
    sc, _ = scene_and_dist("tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    o, d = o[::16], d[::16]
    out = r.render(*to_gpu(o, d))
    ref = render(inp, o, d)
    assert np.array_equal(out["n_samples"].cpu().numpy(), ref.n_samples)
    assert np.abs(out["rgb"].cpu().numpy() - ref.rgb).max() < 1e-5


def test_backward_workspace_failure_then_recovery():
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[alloc fail: backward workspace]", flush=True)
    sc, _ = scene_and_dist("tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    o, d = o[::4], d[::4]
    go, gd = to_gpu(o, d)
    g_rgb = torch.from_numpy(np.random.default_rng(0).standard_normal((len(o), 3)).astype(np.float32)).cuda()
    ref = gpu_renderer("tiny")
    gt0 = torch.zeros((ref.L, ref.T, 9), device="cuda")
    gm0 = torch.zeros((451,), device="cuda")
    ref.backward(go, gd, g_rgb, gt0, gm0)
    r = gpu_renderer("tiny")          # a fresh context: its workspace is not there yet
    gt = torch.zeros_like(gt0)
    gm = torch.zeros_like(gm0)
    _lib().ngprt_test_fail_alloc(0)
    with pytest.raises(NgprtError) as ei:
        r.backward(go, gd, g_rgb, gt, gm)
    assert ei.value.code == E_ALLOC
    torch.cuda.synchronize()
    assert float(gt.abs().max()) == 0.0 and float(gm.abs().max()) == 0.0
    r.backward(go, gd, g_rgb, gt, gm)
    torch.cuda.synchronize()
    assert np.array_equal(gm.cpu().numpy(), gm0.cpu().numpy())
    a, b = gt.cpu().numpy(), gt0.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(b).max())


def test_pyramid_load_failure_then_recovery():
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[alloc fail: pyramid]", flush=True)
    sc, _ = scene_and_dist("tiny_pyramid")
    r = gpu_renderer("tiny_pyramid")
    o, d, _ = synth.scene_rays(sc.cfg)
    o, d = o[::16], d[::16]
    go, gd = to_gpu(o, d)
    want = r.render(go, gd)
    occ = torch.from_numpy(sc.occ_fine).cuda()
    for k in (0, 1):                   # the scratch of the grid build, then its EDT buffers
        _lib().ngprt_test_fail_alloc(k)
        with pytest.raises(NgprtError) as ei:
            r.load_occupancy_pyramid(occ)
        assert ei.value.code == E_ALLOC
        _lib().ngprt_test_fail_alloc(-1)
        with pytest.raises(NgprtError):
            r.render(go, gd)           # the occupancy is not loaded after a failed load
    r.load_occupancy_pyramid(occ)
    got = r.render(go, gd)
    for key in ("rgb", "n_samples", "n_reads"):
        assert np.array_equal(got[key].cpu().numpy(), want[key].cpu().numpy()), key
