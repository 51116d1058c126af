"""GPU proposal path against the oracle: training labels, interval-restricted
marching with fallback, and the proposal network's kernels."""
import numpy as np
import pytest

import synth
from oracle import proposal as P
from oracle.exact32 import F32
from oracle.render import render, render_proposal

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rays(stride=3):
    sc, _ = scene_and_dist("tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    return o[::stride], d[::stride]


def test_label_outputs_bit_exact():
    print("[labels]", flush=True)
    inp = oracle_inputs("tiny")
    o, d = _rays(1)
    r = gpu_renderer("tiny")
    go, gd = to_gpu(o, d)
    out = r.render(go, gd, out=r.alloc_outputs(len(o), labels=True))
    ref = render(inp, o, d)
    lab, valid = P.labels_from_march(len(o), ref.s_ray, ref.s_t, ref.extra["s_T"])
    for j, k in enumerate(("t_first", "t_far", "t_half")):
        assert np.array_equal(_np(out[k]).view(np.uint32), lab[:, j].view(np.uint32)), k


@pytest.mark.parametrize("mode", ["exact", "random"])
def test_render_proposal_matches_oracle(mode):
    print(f"[render proposal {mode}]", flush=True)
    inp = oracle_inputs("tiny")
    o, d = _rays(3)
    ref = render(inp, o, d)
    lab, valid = P.labels_from_march(len(o), ref.s_ray, ref.s_t, ref.extra["s_T"])
    rng = np.random.default_rng(5)
    if mode == "exact":
        t_last = np.zeros(len(o), F32)
        t_last[ref.s_ray] = ref.s_t          # the last sample of each ray
        prop = np.stack([lab[:, 0], t_last, lab[:, 2], valid.astype(F32)], axis=1).astype(F32)
    else:
        t0 = rng.uniform(0.0, 1.5, size=len(o))
        prop = np.stack([t0, t0 + rng.uniform(0.0, 1.0, size=len(o)), t0,
                         rng.uniform(0.0, 1.0, size=len(o))], axis=1).astype(F32)
    r = gpu_renderer("tiny")
    go, gd, gp = to_gpu(o, d, prop)
    out = r.render_intervals(go, gd, gp, 0.9, 2.0 / 256.0)
    res, fb = render_proposal(inp, o, d, prop, 0.9, 2.0 / 256.0)
    assert np.array_equal(_np(out["n_samples"]), res.n_samples)
    assert np.array_equal(_np(out["n_reads"]), res.n_reads)
    assert np.array_equal(_np(out["fallback"]).astype(bool), fb)
    assert np.array_equal(_np(out["t_final"]).view(np.uint32), res.t_final32.view(np.uint32))
    assert np.abs(_np(out["rgb"]) - res.rgb).max() < 1e-5
    if mode == "exact":
        plain = r.render(go, gd)
        assert np.array_equal(_np(out["rgb"]).view(np.uint32), _np(plain["rgb"]).view(np.uint32))
        assert (_np(out["n_reads"]) <= _np(plain["n_reads"])).all()


@pytest.mark.parametrize("name,use_near,far_guard", [("tiny", True, 0.0), ("tiny", False, 1e-3),
                                                     ("tiny", True, 1e-3), ("hd_sub", True, 0.0)])
def test_render_with_loaded_network_matches_oracle(name, use_near, far_guard):
    """The network run inside the render kernel gives the stand-alone
    inference kernel's outputs bit for bit (same products in the same
    order) and the oracle's bf16-operand forward to rounding; given those
    outputs the oracle's interval render has the same sample counts, reads,
    fallbacks and transmittance bits, and colours within 1e-5."""
    import torch
    from paper_2407_10482_amd.renderer import Proposal
    print(f"[render with the loaded proposal network: {name} near={use_near} guard={far_guard}]", flush=True)
    if name == "tiny":
        inp = oracle_inputs("tiny")
        o, d = _rays(3)
        r = gpu_renderer("tiny")
        margin = 2.0 / 256.0
    else:
        # the contracted domain: the near end is a no-read prefix of the lattice
        inp = oracle_inputs("hd")
        sc, _ = scene_and_dist("hd")
        o, d, _ = synth.scene_rays(sc.cfg, cams=synth.camera_positions(sc.cfg)[:1], width=96, height=64)
        r = gpu_renderer("hd")
        margin = 3.0 * sc.cfg.step
    params = P.init_params(21)
    rng = np.random.default_rng(4)
    # output biases that give both proposed rays with samples in their
    # interval and proposed rays that fall back (checked with the oracle)
    params[7552:7556] = np.array([0.0, 0.25, 0.2, 0.5] if name == "tiny" else [0.6, 1.4, 1.0, 0.5], np.float32)
    params[7296:7552] += rng.normal(0, 0.05, size=256).astype(np.float32)
    go, gd, gp = to_gpu(o, d, params)
    net = Proposal(gp, r)
    alone = _np(net.infer(go, gd))
    r.load_proposal(gp)
    out = r.render_proposal(go, gd, 0.5, margin, use_near=use_near, far_guard=far_guard)
    torch.cuda.synchronize()
    prop = _np(out["proposal"])
    assert np.array_equal(prop.view(np.uint32), alone.view(np.uint32))
    f = P.forward(params, P.fourier(o, d), bf16_operands=True)["out"]
    ref = np.concatenate([f[:, :3], 1 / (1 + np.exp(-f[:, 3:4]))], axis=1)
    assert np.all(np.abs(prop - ref) <= 2e-3 * (1 + np.abs(ref))), np.abs(prop - ref).max()
    conf = prop[:, 3] >= 0.5
    assert 0.05 < conf.mean() < 0.95, conf.mean()
    res, fb = render_proposal(inp, o, d, prop, 0.5, margin, use_near=use_near, far_guard=far_guard)
    assert np.array_equal(_np(out["n_samples"]), res.n_samples)
    assert np.array_equal(_np(out["n_reads"]), res.n_reads)
    assert np.array_equal(_np(out["fallback"]).astype(bool), fb)
    assert fb.any() and (conf & ~fb).any()
    assert np.array_equal(_np(out["t_final"]).view(np.uint32), res.t_final32.view(np.uint32))
    assert np.abs(_np(out["rgb"]) - res.rgb).max() < 1e-5


def test_render_proposal_needs_a_loaded_network():
    import torch
    from paper_2407_10482_amd._lib import NgprtError
    print("[render proposal: not loaded]", flush=True)
    r = gpu_renderer("tiny")
    o, d = _rays(50)
    go, gd = to_gpu(o, d)
    with pytest.raises(NgprtError, match="NOT_LOADED"):
        r.render_proposal(go, gd, 0.9, 0.0)
    with pytest.raises(NgprtError, match="INVALID_ARG"):
        r.load_proposal(torch.zeros((7556,), dtype=torch.float32, device="cuda"))
        r.render_proposal(go, gd, 0.9, -1.0)


def _prop_problem(n=1000, seed=3):
    rng = np.random.default_rng(seed)
    cams = synth.random_sphere_cameras(4, 1.0, seed)
    o, d, _ = synth.scene_rays(synth.tiny(), cams=cams, width=32, height=32)
    sel = rng.choice(len(o), size=n, replace=False)
    o, d = o[sel], d[sel]
    inp = oracle_inputs("tiny")
    ref = render(inp, o, d)
    lab, valid = P.labels_from_march(len(o), ref.s_ray, ref.s_t, ref.extra["s_T"])
    return o, d, lab


def test_proposal_forward_matches_oracle():
    import torch
    from paper_2407_10482_amd.renderer import Proposal
    print("[proposal forward]", flush=True)
    o, d, lab = _prop_problem(777)
    params = P.init_params(11)
    params[3072:3136] = np.random.default_rng(1).normal(0, 0.1, size=64)
    r = gpu_renderer("tiny")
    go, gd, gp = to_gpu(o, d, params)
    net = Proposal(gp, r)
    out = _np(net.infer(go, gd))
    f = P.forward(params, P.fourier(o, d), bf16_operands=True)["out"]
    ref = np.concatenate([f[:, :3], 1 / (1 + np.exp(-f[:, 3:4]))], axis=1)
    assert np.all(np.abs(out - ref) <= 2e-3 * (1 + np.abs(ref))), np.abs(out - ref).max()


@pytest.mark.parametrize("phase", [1, 2])
def test_proposal_gradient_matches_oracle(phase):
    from paper_2407_10482_amd.renderer import Proposal
    print(f"[proposal gradient phase {phase}]", flush=True)
    o, d, lab = _prop_problem(1000)
    params = P.init_params(5)
    r = gpu_renderer("tiny")
    go, gd, gp, gl = to_gpu(o, d, params, lab)
    net = Proposal(gp, r)
    g, loss = net.grad(go, gd, gl, phase=phase, margin=2.0 / 256)
    g = _np(g).astype(np.float64)
    fwd = P.forward(params, P.fourier(o, d), bf16_operands=True)
    l64, gout = P.loss_and_grad_out(fwd["out"], lab.astype(np.float64), lab[:, 3] > 0, phase, 2.0 / 256)
    g64 = P.backward(params, fwd, gout, bf16_operands=True)
    scale = np.abs(g64).max()
    assert np.abs(g - g64).max() <= 1e-2 * scale
    assert np.linalg.norm(g - g64) <= 1e-2 * np.linalg.norm(g64)
    assert abs(_np(loss)[0] - l64) <= 1e-3 * abs(l64) + 1e-6


def test_proposal_training_reduces_loss():
    import torch
    from paper_2407_10482_amd.renderer import Proposal
    print("[proposal training]", flush=True)
    o, d, lab = _prop_problem(4096, seed=9)
    r = gpu_renderer("tiny")
    go, gd, gp, gl = to_gpu(o, d, P.init_params(2), lab)
    net = Proposal(gp, r)
    losses = []
    for it in range(300):
        loss = torch.zeros((1,), dtype=torch.float32, device="cuda")
        net.train_step(go, gd, gl, 3e-3, phase=1, loss=loss)
        losses.append(loss.item())
    print("proposal loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.2 * losses[0]


def test_trained_proposal_quality_and_gain():
    """Train on the plain renderer's labels, then on unseen views with the
    network run inside the render kernel (far end only, cut where the
    transmittance is below 1e-3): PSNR against a float64 reference (step / 4,
    no termination) within 0.1 dB of the plain render's, and no more samples.
    The most any proposal can save is what a perfect one saves (the plain
    render's own labels of these rays), and that is exactly a plain render
    terminated at T < 1e-3: same samples, same colours, no network."""
    import torch
    from oracle.render import OracleInputs
    from paper_2407_10482_amd.renderer import Proposal, Renderer, proposal_init
    print("[trained proposal]", flush=True)
    sc, dist = scene_and_dist("tiny")
    cfg = sc.cfg
    r = gpu_renderer("tiny")
    to, td, _ = synth.scene_rays(cfg, cams=synth.random_sphere_cameras(512, 1.0, 1000), width=32,
                                 height=32)
    to, td = to_gpu(to, td)
    lo = r.render(to, td, out=r.alloc_outputs(len(to), labels=True))
    labels = torch.stack([lo["t_first"], lo["t_far"], lo["t_half"],
                          (lo["n_samples"] > 0).float()], dim=1).contiguous()
    net = Proposal(proposal_init(7), r)
    n, bs = len(to), 1 << 13
    gen = torch.Generator(device="cuda").manual_seed(0)
    margin = 2.0 * cfg.step
    for ep in range(40):
        phase = 1 if ep < 20 else 2
        perm = torch.randperm(n, generator=gen, device="cuda")
        for b in range(0, n, bs):
            idx = perm[b:b + bs]
            net.train_step(to[idx].contiguous(), td[idx].contiguous(), labels[idx].contiguous(),
                           3e-3 if phase == 1 else 1e-3, phase=phase, margin=4.0 * cfg.step)
    eo, ed, _ = synth.scene_rays(cfg, cams=synth.random_sphere_cameras(2, 1.0, 2000), width=128,
                                 height=128)
    go, gd = to_gpu(eo, ed)
    plain = r.render(go, gd)
    r.load_proposal(net.params)
    withp = r.render_proposal(go, gd, 0.99, margin, use_near=False, far_guard=1e-3)
    prop = withp["proposal"]
    rp, rq = _np(plain["rgb"]).astype(np.float64), _np(withp["rgb"]).astype(np.float64)
    conf = (_np(prop)[:, 3] >= 0.99).mean()
    sp_plain, sp_prop = _np(plain["n_samples"]).mean(), _np(withp["n_samples"]).mean()
    print(f"confident {conf:.3f} fallback {_np(withp['fallback']).mean():.3f} "
          f"samples/ray {sp_plain:.2f} -> {sp_prop:.2f}", flush=True)
    # float64 reference on a subsample: step / 4, no termination
    rng = np.random.default_rng(0)
    sel = rng.choice(len(eo), size=400, replace=False)
    fine = OracleInputs(tables=sc.tables, occ=sc.occ, dist=dist, mlp=sc.mlp,
                        resolutions=cfg.resolutions, domain=cfg.domain, roi_half=cfg.roi_half,
                        step=cfg.step / 4, max_samples=1 << 16, t_threshold=0.0)
    ref = render(fine, eo[sel], ed[sel], terminate=False).rgb

    def psnr(a):
        return 10 * np.log10(1.0 / np.mean((a[sel] - ref) ** 2))
    p_plain, p_prop = psnr(rp), psnr(rq)
    print(f"PSNR vs reference: plain {p_plain:.3f} dB, proposal {p_prop:.3f} dB", flush=True)
    assert p_plain - p_prop <= 0.1
    assert sp_prop <= sp_plain
    # a perfect proposal: the plain render's own labels (first sample .. the
    # sample after which T < 1e-3), both ends, margin 0
    lab = r.render(go, gd, out=r.alloc_outputs(len(eo), labels=True))
    perfect = torch.stack([lab["t_first"], lab["t_far"], lab["t_half"],
                           (lab["n_samples"] > 0).float()], dim=1).contiguous()
    best = r.render_intervals(go, gd, perfect, 0.5, 0.0)
    sp_best = _np(best["n_samples"]).mean()
    print(f"perfect proposal: samples/ray {sp_best:.2f} reads/ray {_np(best['n_reads']).mean():.2f}", flush=True)
    assert sp_best <= sp_prop
    # ... is the plain render terminated at T < 1e-3
    r3 = gpu_renderer("tiny", t_threshold=1e-3)
    term3 = r3.render(go, gd)
    assert np.array_equal(_np(term3["n_samples"]), _np(best["n_samples"]))
    assert np.array_equal(_np(term3["rgb"]).view(np.uint32), _np(best["rgb"]).view(np.uint32))
