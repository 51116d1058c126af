"""Benchmark of the NGP-RT render path on one MI355X.

One step = one render of the full 'hd' workload: 8 views of 1920x1080 rays
(16,588,800 rays) through 16 hash levels (16..4096, 2^19 entries each), a
256^3 occupancy/distance grid in the contracted domain, <= 1024 samples per
ray, termination at T < 1e-4, and the deferred MLP per ray.  Scene, rays and
outputs are resident in HBM before the timed region.

Prints one JSON line (metric = frames/s of 1080p views; Msamples/s beside it),
with the dominant kernel's roofline figure and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources whose change invalidates hardware counters taken on the render kernel
KERNEL_SOURCES = ["paper_2407_10482_amd/csrc/" + f for f in
                  ("render.hip", "device.h", "march.h", "internal.h")] + ["paper_2407_10482_amd/build.py"]
BYTES_PER_ENTRY = {0: 36, 1: 18, 2: 9}     # 8 feature channels + 1 logit per entry
DTYPE_NAME = {0: "f32", 1: "bf16", 2: "fp8"}
AGG_NAME = {"separate_v": "sigmoid-gated separate attention (Separate-Att (V))",
            "shared_v": "Shared-Att (V)", "separate_inv": "Separate-Att (Inv)",
            "shared_inv": "Shared-Att (Inv)", "sum": "SUM aggregation"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=120)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--dtype", choices=["f32", "bf16", "fp8"], default="f32")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="approximate CPU time for the oracle baseline (0 skips it)")
    p.add_argument("--views", type=int, default=8)
    p.add_argument("--group", type=int, default=1,
                   help="ray order: 8x8-pixel tiles taken in blocks of group x group tiles")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="run one device copy of this many MiB first (hardware-counter calibration)")
    p.add_argument("--probe-points", type=int, default=1 << 24,
                   help="points of the random-gather ceiling probe (0 skips it)")
    p.add_argument("--model", choices=["hash", "baked"], default="hash",
                   help="hash: 16 hash levels fused by softmax attention (the headline); baked: "
                        "the paper's coarse grid + sigmoid-gated fine levels")
    p.add_argument("--fine-levels", type=int, default=2, help="baked model: fine levels (1..4)")
    p.add_argument("--agg", choices=["separate_v", "shared_v", "separate_inv", "shared_inv", "sum"],
                   default="separate_v",
                   help="baked model: fusion of the fine levels (Table 3's variants; separate_v is the "
                        "paper's sigmoid-gated separate attention)")
    p.add_argument("--scene", choices=["hd", "hd_regime"], default="hd",
                   help="hash model: hd (the headline scene: 15.2 samples, 34.8 grid reads per ray) or "
                        "hd_regime (calibrated to the paper's Table 4 regime: 17.3 samples, 42.6 reads)")
    p.add_argument("--occ", choices=["single", "pyramid"], default="single",
                   help="single: one 256^3 occupancy grid + distance grid (the headline); pyramid: "
                        "the paper's 512^3..32^3 occupancy pyramid + 256^3 distance grid")
    p.add_argument("--mlp", choices=["plain", "view"], default="plain",
                   help="plain: deferred MLP 7-16-16-3 of (C_d, F) (the headline); view: the "
                        "view-dependent MLP_psi 23-64-64-3 of (C_d, F, SH(d))")
    p.add_argument("--no-dist", action="store_true",
                   help="pyramid only: march without the distance grid (the ablation of Table 4)")
    p.add_argument("--mode", choices=["render", "train", "proposal", "cache"], default="render",
                   help="render: the headline; train: forward+backward+Adam steps; "
                        "proposal: learned sample-interval proposal vs plain marching; "
                        "cache: the random-gather probe over table sizes")
    p.add_argument("--train-size", choices=["tiny", "train_large"], default="tiny")
    p.add_argument("--prop-epochs", type=int, default=12)
    p.add_argument("--paper-steps", type=int, default=20,
                   help="default line: timed steps of the paper's rendering choices together (baked L = 2, "
                        "pyramid + G, MLP_psi) on the hd workload (0 skips it)")
    p.add_argument("--regime-steps", type=int, default=20,
                   help="timed renders of the scene calibrated to the paper's regime in the default "
                        "line (0 = skip)")
    p.add_argument("--prop-steps", type=int, default=20,
                   help="timed renders per side of the plain-vs-proposal comparison (0 skips it)")
    return p.parse_args()


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def copy_probe(mb: int):
    """One device copy of mb MiB: the plain copy kernel whose FETCH_SIZE and
    WRITE_SIZE calibrate the counter passes of the same command."""
    if mb <= 0:
        return
    import torch
    nbytes = mb << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"# copy probe: {nbytes} bytes read + {nbytes} bytes written", file=sys.stderr, flush=True)
    del src, dst


def bench_train(args):
    """One step = render 2^18 rays (16 cameras x 128^2) with the student
    tables, mean-squared colour loss against a teacher (tables of seed 1),
    hand-written backward, Adam on tables and MLP."""
    import torch

    import synth
    from paper_2407_10482_amd.renderer import (Renderer, adam_step, render_differentiable,
                                               render_differentiable_baked, render_differentiable_view)

    baked = args.model == "baked"
    if baked:
        from synth.baked import make_baked_scene
        if args.train_size != "tiny":
            raise SystemExit("--mode train --model baked trains the baked model of the tiny scene only")
        cfg = synth.baked_tiny()
        if args.mlp == "view":
            cfg.mlp_dims = (23, 64, 64, 3)
        sc, teacher = make_baked_scene(cfg), make_baked_scene(cfg, seed=1)
    else:
        cfg = synth.CONFIGS[args.train_size]()
        if args.mlp == "view":
            cfg.mlp_dims = (23, 64, 64, 3)
        sc, teacher = synth.make_scene(cfg), synth.make_scene(cfg, seed=1)
    view = args.mlp == "view"
    cams = synth.random_sphere_cameras(16, 1.0, seed=123)
    o, d, _ = synth.scene_rays(cfg, cams=cams, width=128, height=128)
    torch.cuda.set_device(0)
    copy_probe(args.copy_probe_mb)
    r = Renderer.from_config(cfg)
    r.load_scene(torch.from_numpy(teacher.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                 torch.from_numpy(sc.mlp).cuda())
    if baked:
        r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(teacher.atlas).cuda(),
                      teacher.default)
    go, gd = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    target = r.render(go, gd, aux=False)["rgb"].clone()
    params = [torch.from_numpy(sc.tables).cuda().requires_grad_(True)]
    if baked:
        params.append(torch.from_numpy(sc.atlas).cuda().requires_grad_(True))
    params.append(torch.from_numpy(sc.mlp).cuda().requires_grad_(True))
    moments = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    state = {"step": 0, "loss": []}

    def step():
        if view:
            rgb = render_differentiable_view(r, params[0], params[-1], go, gd,
                                             atlas=params[1] if baked else None)
        elif baked:
            rgb = render_differentiable_baked(r, *params, go, gd)
        else:
            rgb = render_differentiable(r, *params, go, gd)
        loss = torch.mean((rgb - target) ** 2)
        loss.backward()
        state["step"] += 1
        with torch.no_grad():
            for p, (m, v) in zip(params, moments):
                adam_step(p, p.grad, m, v, state["step"], 0.01)
                p.grad = None
        return loss

    first = step().item()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, end = _events()
    start.record()
    for _ in range(args.steps):
        loss = step()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    n_params = sum(p.numel() for p in params)
    return {
        "metric": "training steps/s (render + backward + Adam)",
        "value": round(1e3 / ms, 3),
        "unit": "steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: "
                               + (f"coarse grid L_C = {cfg.coarse_res} ({sc.atlas.shape[0]} blocks of 8^3) + "
                                  if baked else "")
                               + f"{cfg.n_levels} levels {cfg.n_min}..{cfg.n_max}, "
                               f"2^{cfg.log2_table} entries, "
                               + ("view-dependent MLP 23-64-64-3, " if view else "")
                               + "2^18 rays from 16 cameras x 128^2, MSE vs a seed-1 teacher, Adam lr 0.01",
                   "rays_per_step": len(o), "parameters": n_params},
        "loss_first": first, "loss_last": loss.item(),
    }


# proposal settings of the comparison: rays with confidence >= 0.99 stop at
# t_far + 2 steps, and only once their transmittance is below 1e-3 (the near
# end is not used: at this scale its misses cost up to 10 dB)
CONF = 0.99
MARGIN_STEPS = 2
USE_NEAR = False
FAR_GUARD = 1e-3


def regime_scene(steps: int) -> dict:
    """The same render on the scene calibrated to the paper's marching regime
    (hd_regime: about 17 samples and 43 grid reads per ray against hd's 15
    and 35), timed like the headline: 8 views x 1080p, HIP events."""
    import torch
    import synth
    from paper_2407_10482_amd.renderer import Renderer
    cfg = synth.hd_regime()
    sc = synth.make_scene(cfg)
    o, d, _ = synth.scene_rays(cfg, cams=synth.camera_positions(cfg)[:8])
    r = Renderer.from_config(cfg, 0)
    r.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                 torch.from_numpy(sc.mlp).cuda())
    go, gd = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    counts = r.render(go, gd)
    n_samples = int(counts["n_samples"].long().sum().item())
    n_reads = int(counts["n_reads"].long().sum().item())
    del counts
    out = {"rgb": torch.empty((len(o), 3), dtype=torch.float32, device="cuda")}
    for _ in range(2):
        r.render(go, gd, out=out)
    a, b = _events()
    a.record()
    for _ in range(steps):
        r.render(go, gd, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {"workload": "hd_regime: the hd render on 400 blobs (sigma 0.02-0.08), calibrated to the paper's "
                        "Table 4 regime of samples and marching points per ray",
            "fps": round(8 / (ms / 1e3), 3), "ms": round(ms, 4), "steps": steps,
            "samples_per_ray": round(n_samples / len(o), 3), "reads_per_ray": round(n_reads / len(o), 3),
            "msamples_per_s": round(n_samples / (ms / 1e3) / 1e6, 1)}


def paper_configuration(steps: int) -> dict:
    """The paper's rendering choices together on the hd workload: baked coarse
    grid (L_C = 512) + two sigmoid-gated fine levels, the 512^3..32^3
    occupancy pyramid with the 256^3 distance grid, and the view-dependent
    MLP as a second pass; F32 tables, timed like the headline (8 views x
    1080p, HIP events around render + MLP_psi)."""
    import torch
    import synth
    from synth.baked import make_baked_scene
    from paper_2407_10482_amd.renderer import Renderer
    cfg = synth.with_aggregation(synth.baked_hd(table_dtype=0, n_fine=2), "separate_v")
    cfg.occ_levels, cfg.occ_fine_res = 5, 512
    cfg.mlp_dims = (23, 64, 64, 3)
    sc = make_baked_scene(cfg)
    o, d, _ = synth.scene_rays(cfg, cams=synth.camera_positions(cfg)[:8])
    r = Renderer.from_config(cfg, 0)
    r.load_tables(torch.from_numpy(sc.tables).cuda())
    r.load_occupancy_pyramid(torch.from_numpy(sc.occ_fine).cuda())
    r.load_mlp(torch.from_numpy(sc.mlp).cuda())
    r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(sc.atlas).cuda(), sc.default)
    go, gd = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    counts = r.render(go, gd)
    n_samples = int(counts["n_samples"].long().sum().item())
    n_reads = int(counts["n_reads"].long().sum().item())
    del counts
    n = len(o)
    out = {k: torch.empty((n, c), dtype=torch.float32, device="cuda") for k, c in (("rgb", 3), ("c_d", 3), ("feat", 4))}
    for _ in range(2):
        r.render(go, gd, out=out)
    a, b = _events()
    a.record()
    for _ in range(steps):
        r.render(go, gd, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    return {"workload": "paper_hd: baked coarse grid L_C=512 + 2 sigmoid-gated fine levels (1024, 2048; 2^22 "
                        "entries, f32), occupancy pyramid 512^3..32^3 + 256^3 distance grid, view-dependent MLP "
                        "23-64-64-3 with SH(d); 8 views x 1920x1080",
            "fps": round(8 / (ms / 1e3), 3), "ms": round(ms, 4), "steps": steps,
            "samples_per_ray": round(n_samples / n, 3), "marching_points_per_ray": round(n_reads / n, 3),
            "msamples_per_s": round(n_samples / (ms / 1e3) / 1e6, 1)}


def proposal_comparison(steps: int, warmup: int, epochs: int):
    """Plain distance-grid marching against the learned sample-interval
    proposal on the same GPU: train the proposal network on 2^22 rays of the
    tiny scene (1024 cameras x 64^2, labels from the plain renderer), load it
    into the library, then render 8 unseen 1920x1080 views both ways (the
    network runs inside the render kernel).  The quality bar is the PSNR of
    each render against a reference rendered at a quarter of the step
    without termination (by the same GPU renderer), on every 16th ray."""
    import torch

    import synth
    from paper_2407_10482_amd.renderer import Proposal, Renderer, proposal_init

    cfg = synth.tiny()
    sc = synth.make_scene(cfg)
    torch.cuda.set_device(0)
    r = Renderer.from_config(cfg)
    r.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                 torch.from_numpy(sc.mlp).cuda())
    tcams = synth.random_sphere_cameras(1024, 1.0, seed=1000)
    to, td, _ = synth.scene_rays(cfg, cams=tcams, width=64, height=64)
    to, td = torch.from_numpy(to).cuda(), torch.from_numpy(td).cuda()
    lab_out = r.render(to, td, out=r.alloc_outputs(len(to), labels=True))
    labels = torch.stack([lab_out["t_first"], lab_out["t_far"], lab_out["t_half"],
                          (lab_out["n_samples"] > 0).float()], dim=1).contiguous()
    net = Proposal(proposal_init(7), r)
    n = len(to)
    bs = 1 << 14
    g = torch.Generator(device="cuda").manual_seed(0)
    margin = MARGIN_STEPS * cfg.step
    loss = torch.zeros((1,), dtype=torch.float32, device="cuda")
    history = []
    torch.cuda.synchronize()
    t0 = time.time()
    for ep in range(epochs):
        phase = 1 if ep < epochs // 2 else 2
        lr = 3e-3 if phase == 1 else 1e-3
        perm = torch.randperm(n, generator=g, device="cuda")
        loss.zero_()
        for b in range(0, n, bs):
            idx = perm[b:b + bs]
            net.train_step(to[idx].contiguous(), td[idx].contiguous(), labels[idx].contiguous(), lr,
                           phase=phase, margin=4.0 * cfg.step, loss=loss)
        history.append(round(loss.item() / (n // bs), 6))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    r.load_proposal(net.params)
    ecams = synth.random_sphere_cameras(8, 1.0, seed=2000)
    eo, ed, _ = synth.scene_rays(cfg, cams=ecams, width=1920, height=1080)
    eo, ed = torch.from_numpy(eo).cuda(), torch.from_numpy(ed).cuda()
    ne = len(eo)
    plain = r.render(eo, ed)
    withp = r.render_proposal(eo, ed, CONF, margin, use_near=USE_NEAR, far_guard=FAR_GUARD)
    torch.cuda.synchronize()

    def timed(fn):
        outp = {"rgb": torch.empty((ne, 3), dtype=torch.float32, device="cuda")}
        for _ in range(warmup):
            fn(outp)
        torch.cuda.synchronize()
        a, b = _events()
        a.record()
        for _ in range(steps):
            fn(outp)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    # the bound on any proposal: a perfect one, the plain render's own labels
    # of these rays (first sample .. the sample after which T < 1e-3), margin 0
    lab = r.render(eo, ed, out=r.alloc_outputs(ne, labels=True))
    perfect = torch.stack([lab["t_first"], lab["t_far"], lab["t_half"],
                           (lab["n_samples"] > 0).float()], dim=1).contiguous()
    del lab
    best = r.render_intervals(eo, ed, perfect, 0.5, 0.0)
    ms_plain = timed(lambda outp: r.render(eo, ed, out=outp))
    ms_prop = timed(lambda outp: r.render_proposal(eo, ed, CONF, margin, out=outp, use_near=USE_NEAR,
                                                   far_guard=FAR_GUARD))
    # the perfect proposal is the plain render terminated at T < 1e-3
    r3 = Renderer(resolutions=cfg.resolutions, log2_table_size=cfg.log2_table, table_dtype=0, domain=cfg.domain,
                  roi_half=cfg.roi_half, occ_res=cfg.occ_res, step=cfg.step, max_samples=cfg.max_samples,
                  t_threshold=1e-3)
    r3.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                  torch.from_numpy(sc.mlp).cuda())
    term3 = r3.render(eo, ed)
    ms_term3 = timed(lambda outp: r3.render(eo, ed, out=outp))
    ms_best = timed(lambda outp: r.render_intervals(eo, ed, perfect, 0.5, 0.0, out=outp))
    # quality: both renders against a quarter-step reference without termination
    sub = slice(0, ne, 16)
    fine = Renderer(resolutions=cfg.resolutions, log2_table_size=cfg.log2_table, table_dtype=0,
                    domain=cfg.domain, roi_half=cfg.roi_half, occ_res=cfg.occ_res, step=cfg.step / 4,
                    max_samples=1 << 15, t_threshold=0.0)
    fine.load_scene(torch.from_numpy(sc.tables).cuda(), torch.from_numpy(sc.occ).cuda(),
                    torch.from_numpy(sc.mlp).cuda())
    ref = fine.render(eo[sub].contiguous(), ed[sub].contiguous(), aux=False)["rgb"].double()
    torch.cuda.synchronize()

    def psnr(x, y):
        mse = torch.mean((x.double() - y) ** 2).item()
        return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)

    p_plain, p_prop = psnr(plain["rgb"][sub], ref), psnr(withp["rgb"][sub], ref)
    p_best = psnr(best["rgb"][sub], ref)
    p_term3 = psnr(term3["rgb"][sub], ref)
    views = 8

    def side(ms, out):
        ns = int(out["n_samples"].sum().item())
        nr = int(out["n_reads"].sum().item())
        return {"fps": round(views / (ms / 1e3), 3), "ms": round(ms, 4),
                "msamples_per_s": round(ns / (ms / 1e3) / 1e6, 1),
                "samples_per_ray": round(ns / ne, 3), "reads_per_ray": round(nr / ne, 3)}

    return {
        "workload": "tiny scene (8 levels 16..256, 2^14 entries, box ROI, 64^3 grid); proposal "
                    "48-64-64-4 trained on 2^22 rays (1024 cameras x 64^2, labels from the plain "
                    f"renderer, {epochs} epochs); 8 unseen 1920x1080 views; conf >= {CONF}, margin "
                    f"{MARGIN_STEPS} steps, near end {'used' if USE_NEAR else 'not used'}, far end cut only "
                    f"below T = {FAR_GUARD}; network run inside the render kernel",
        "plain": side(ms_plain, plain),
        "proposal": side(ms_prop, withp),
        "speedup": round(ms_plain / ms_prop, 4),
        "perfect_proposal_bound": dict(side(ms_best, best), speedup=round(ms_plain / ms_best, 4),
                                       psnr_loss_db=round(p_plain - p_best, 4)),
        "plain_terminated_at_1e-3": dict(side(ms_term3, term3), speedup=round(ms_plain / ms_term3, 4),
                                         psnr_loss_db=round(p_plain - p_term3, 4),
                                         same_samples_as_perfect=bool(torch.equal(term3["n_samples"],
                                                                                  best["n_samples"]))),
        "psnr_vs_reference_db": {"plain": round(p_plain, 3), "proposal": round(p_prop, 3)},
        "psnr_loss_db": round(p_plain - p_prop, 4),
        "psnr_proposal_vs_plain_db": round(psnr(withp["rgb"], plain["rgb"].double()), 3),
        "confident_fraction": round((withp["proposal"][:, 3] >= CONF).float().mean().item(), 4),
        "fallback_fraction": round(withp["fallback"].float().mean().item(), 4),
        "train_seconds": round(train_s, 1),
        "train_loss_per_epoch": history,
    }


def bench_proposal(args):
    """The plain-vs-proposal comparison as its own line (metric: frames/s of
    the proposal render)."""
    c = proposal_comparison(args.steps, args.warmup, args.prop_epochs)
    return {
        "metric": "1080p frames/s, learned proposal vs plain distance-grid marching",
        "value": c["proposal"]["fps"],
        "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": c["proposal"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": c["workload"], "rays_per_step": 8 * 1920 * 1080},
        "proposal_comparison": c,
    }


_POOL = {}


def _pool_init():
    from threadpoolctl import threadpool_limits
    _POOL["limit"] = threadpool_limits(1)       # one thread per worker process


def _oracle_chunk(bounds):
    from oracle.render import render
    a, b = bounds
    res = render(_POOL["inp"], _POOL["o"][a:b], _POOL["d"][a:b])
    return int(res.n_samples.sum())


def cpu_baseline(sc, o, d, dtype, seconds):
    """The oracle, as it stands, on a deterministic strided subsample of the
    rays, split over the host's cores (fork workers, one thread each).  Must
    run before this process touches the GPU (the workers are forks)."""
    import multiprocessing as mp
    from oracle.distgrid import distance_grid_edt
    from oracle.render import inputs_from_scene, render, scene_occupancy
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    inp = inputs_from_scene(sc, distance_grid_edt(scene_occupancy(sc)), dtype)
    n_total = len(o)
    # per-ray cost on one core, then a sample that keeps every core busy for
    # about `seconds`
    n1 = 4096
    st = max(1, n_total // n1)
    t0 = time.perf_counter()
    render(inp, o[::st][:n1], d[::st][:n1])
    per_ray = (time.perf_counter() - t0) / n1
    n2 = int(min(n_total, max(n1, seconds * cores / per_ray)))
    stride = max(1, n_total // n2)
    so, sd = np.ascontiguousarray(o[::stride][:n2]), np.ascontiguousarray(d[::stride][:n2])
    _POOL.update(inp=inp, o=so, d=sd)
    chunk = -(-len(so) // cores)                 # one lock-step march per worker
    bounds = [(a, min(a + chunk, len(so))) for a in range(0, len(so), chunk)]
    with mp.get_context("fork").Pool(cores, initializer=_pool_init) as pool:
        t0 = time.perf_counter()
        counts = pool.map(_oracle_chunk, bounds, chunksize=1)
        dt = time.perf_counter() - t0
    rays_per_s = len(so) / dt
    return {
        "value": rays_per_s / (1920 * 1080),
        "unit": "frames/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(so)} rays (every {stride}th ray of the 8 views) on {cores} worker processes, "
                  f"{dt:.1f} s, {sum(counts) / dt / 1e6:.4f} Msamples/s",
    }


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_PEAK_G = 256 * 4 * 2.4 / 4     # wave64 VALU instructions per ns: 256 CUs x 4 SIMDs x 2.4 GHz,
                                   # one wave64 instruction per 4 cycles on a 16-lane SIMD


def committed_counters(dtype_name: str, scene: str = "hd"):
    """Per-launch hardware counters of the render kernel from the committed
    summary, or None when it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"render_kernel_{scene}_{dtype_name}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256/16") != kernel_source_hash():
        return None
    out = {}
    for key, name in (("HBM bytes per launch", "hbm_bytes"), ("VALU instructions per launch", "valu"),
                      ("L2 requests per launch", "l2_req"), ("L2 hits per launch", "l2_hit"),
                      ("vector memory reads per launch", "vmem_rd")):
        try:
            # the figure leads the value; a parenthesised note may follow
            out[name] = int(vals[key].split()[0].replace(",", ""))
        except (KeyError, ValueError, IndexError):
            out[name] = None
    for key, name in (("TA busy fraction per CU", "ta_busy"), ("TD busy fraction per CU", "td_busy")):
        try:
            out[name] = float(vals[key])
        except (KeyError, ValueError):
            out[name] = None
    return out


def bench_cache(args) -> dict:
    """The random-gather probe over table sizes: 16 levels of 2^13..2^21
    entries in F32, BF16 and FP8 rows, uniform random entries per level (no
    reuse but what the caches hold).  Where the whole table outgrows the
    256 MB Infinity Cache the achieved rate drops; this locates that knee
    for the gather pattern of the render."""
    import torch
    import synth
    from paper_2407_10482_amd.renderer import Renderer
    torch.cuda.set_device(0)
    curve = []
    for dt in (0, 1, 2):
        for log2t in range(13, 22):
            cfg = synth.hd(table_dtype=dt)
            cfg.log2_table = log2t
            r = Renderer.from_config(cfg, dt)
            T = 1 << log2t
            g = torch.Generator(device="cuda").manual_seed(log2t)
            r.load_tables(torch.randn((cfg.n_levels, T, 9), generator=g, device="cuda") * 0.5)
            gbs = gather_probe(r, args.probe_points, 5, False)
            curve.append({"dtype": DTYPE_NAME[dt], "entries_per_level": T,
                          "table_mb": round(cfg.n_levels * T * BYTES_PER_ENTRY[dt] / 1e6, 1),
                          "requested_gbs": round(gbs, 1),
                          "g_rows_per_s": round(gbs / BYTES_PER_ENTRY[dt], 2)})
            print(json.dumps(curve[-1]), file=sys.stderr, flush=True)
            del r
            torch.cuda.empty_cache()
    return {"metric": "random-gather probe over table sizes (G corner rows/s)", "points": args.probe_points,
            "levels": 16, "unit": "G rows/s", "higher_is_better": True, "curve": curve}


def gather_probe(r, n_points: int, reps: int, pairs: bool) -> float:
    """Requested-gather GB/s of the random-gather probe (mean over reps)."""
    import torch
    buf = torch.empty((n_points,), dtype=torch.float32, device="cuda")
    r.gather_probe(n_points, seed=99, pairs=pairs, out=buf)
    a, b = _events()
    a.record()
    for i in range(reps):
        r.gather_probe(n_points, seed=i, pairs=pairs, out=buf)
    b.record()
    torch.cuda.synchronize()
    s = a.elapsed_time(b) / reps / 1e3
    return n_points * r.L * 8 * BYTES_PER_ENTRY[r.table_dtype] / s / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.mode == "train":
        print(json.dumps(bench_train(args)), flush=True)
        return
    if args.mode == "proposal":
        print(json.dumps(bench_proposal(args)), flush=True)
        return
    if args.mode == "cache":
        print(json.dumps(bench_cache(args)), flush=True)
        return
    import torch

    import synth
    from paper_2407_10482_amd.renderer import Renderer

    dtype = {"f32": 0, "bf16": 1, "fp8": 2}[args.dtype]
    baked = args.model == "baked"
    t0 = time.time()
    pyr = args.occ == "pyramid"
    if baked and args.scene != "hd":
        raise SystemExit("--scene applies to the hash model")
    if baked:
        from synth.baked import make_baked_scene
        cfg = synth.with_aggregation(synth.baked_hd(table_dtype=dtype, n_fine=args.fine_levels), args.agg)
        if pyr:
            cfg.occ_levels, cfg.occ_fine_res = 5, 512
        if args.mlp == "view":
            cfg.mlp_dims = (23, 64, 64, 3)
        sc = make_baked_scene(cfg)
    else:
        if args.scene == "hd_regime":
            if pyr:
                raise SystemExit("--scene hd_regime marches the single distance grid")
            cfg = synth.hd_regime(table_dtype=dtype)
        else:
            cfg = synth.hd_pyramid(table_dtype=dtype) if pyr else synth.hd(table_dtype=dtype)
        if args.mlp == "view":
            cfg.mlp_dims = (23, 64, 64, 3)
        sc = synth.make_scene(cfg)
    assert (args.mlp == "view") == (tuple(cfg.mlp_dims) == (23, 64, 64, 3))
    cams = synth.camera_positions(cfg)[: args.views]
    o, d, _ = synth.scene_rays(cfg, cams=cams, group=args.group)
    print(f"# scene + rays generated in {time.time() - t0:.1f} s ({len(o)} rays)", file=sys.stderr,
          flush=True)
    # the CPU oracle leg forks worker processes: run it before any GPU call
    cpu = cpu_baseline(sc, o, d, dtype, args.cpu_seconds) if args.cpu_seconds > 0 else None
    torch.cuda.set_device(0)
    copy_probe(args.copy_probe_mb)
    r = Renderer.from_config(cfg, dtype, use_distance=not args.no_dist)
    r.load_tables(torch.from_numpy(sc.tables).cuda())
    if pyr:
        r.load_occupancy_pyramid(torch.from_numpy(sc.occ_fine).cuda())
    else:
        r.load_occupancy(torch.from_numpy(sc.occ).cuda())
    r.load_mlp(torch.from_numpy(sc.mlp).cuda())
    if baked:
        r.load_coarse(torch.from_numpy(sc.block_index).cuda(), torch.from_numpy(sc.atlas).cuda(),
                      sc.default)
    go = torch.from_numpy(o).cuda()
    gd = torch.from_numpy(d).cuda()
    n = len(o)
    # one render with every output, outside the timed region: sample and read counts
    aux = r.render(go, gd)
    torch.cuda.synchronize()
    n_samples = int(aux["n_samples"].sum().item())
    n_reads = int(aux["n_reads"].sum().item())
    out = {"rgb": torch.empty((n, 3), dtype=torch.float32, device="cuda")}
    if r.view_mlp:      # MLP_psi runs as a second pass over the C_d and F outputs
        out.update(c_d=torch.empty((n, 3), dtype=torch.float32, device="cuda"),
                   feat=torch.empty((n, 4), dtype=torch.float32, device="cuda"))
    for _ in range(args.warmup):
        r.render(go, gd, out=out)
    torch.cuda.synchronize()
    # events on the stream the render kernel is launched on (torch's current
    # stream): one pair around the whole timed region, one per step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for i in range(args.steps):
        r.render(go, gd, out=out)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    probe = {}
    if args.probe_points > 0:
        for pairs in (False, True):
            probe["pairs" if pairs else "uniform"] = round(gather_probe(r, args.probe_points, 5, pairs), 1)
    views = len(cams)
    fps = views / (ms / 1e3)
    L = cfg.n_levels
    if baked:
        # per sample: 8 coarse vertices (4 B block index + 4 B per coarse
        # channel) and 8 corner rows per fine level (no logit)
        per_sample = 8 * (4 + 4 * cfg.coarse_channels) + L * 8 * (BYTES_PER_ENTRY[dtype] * 8 // 9)
    else:
        per_sample = L * 8 * BYTES_PER_ENTRY[dtype]
    gather = n_samples * per_sample
    alg_bytes = gather + 2 * n_reads + n * (24 + 12)
    sec = ms / 1e3
    ctr = None if (baked or pyr or args.mlp == "view") else committed_counters(DTYPE_NAME[dtype], args.scene)
    levels = {
        # what the method asks for: every corner row of every level of every
        # sample; most of it is served by the L1 and L2 caches, so this is no
        # fraction of any one peak
        "requested_gather": {"achieved_gbs": round(alg_bytes / sec / 1e9, 1), "bytes": alg_bytes},
    }
    if ctr:
        if ctr["valu"]:
            v = ctr["valu"] / sec / 1e9
            levels["valu_issue"] = {"achieved": round(v, 1), "peak": VALU_PEAK_G,
                                    "unit": "G wave64 VALU instructions/s", "frac": round(v / VALU_PEAK_G, 4),
                                    "instructions_per_launch": ctr["valu"]}
        if ctr["hbm_bytes"]:
            h = ctr["hbm_bytes"] / sec / 1e9
            levels["hbm_fabric"] = {"achieved_gbs": round(h, 1), "peak_gbs": HBM_PEAK_GBS,
                                    "frac": round(h / HBM_PEAK_GBS, 4), "bytes_per_launch": ctr["hbm_bytes"],
                                    "requested_over_fabric": round(alg_bytes / ctr["hbm_bytes"], 2)}
        if ctr["l2_req"] and ctr["l2_hit"] is not None:
            levels["l2"] = {"requests_per_launch": ctr["l2_req"],
                            "hit_rate": round(ctr["l2_hit"] / ctr["l2_req"], 4)}
        if ctr["ta_busy"] is not None:
            # busy cycles of the texture address / data units per CU; they
            # include cycles stalled on the caches, and taking half of the
            # load instructions off the TA (coarse levels by scalar loads)
            # gained 2 %, so this is occupancy of the path, not its limit
            levels["vmem_pipeline"] = {"ta_busy": ctr["ta_busy"], "td_busy": ctr["td_busy"],
                                       "load_instructions_per_launch": ctr["vmem_rd"]}
    # the binding level is the one closest to its peak
    cands = [(lv["frac"], name) for name, lv in levels.items() if "frac" in lv]
    if cands:
        frac, bname = max(cands)
        lv = levels[bname]
        roof = {"bound": "alu" if bname == "valu_issue" else "hbm", "level": bname,
                "achieved": lv.get("achieved", lv.get("achieved_gbs")),
                "peak": lv.get("peak", lv.get("peak_gbs")),
                "unit": lv.get("unit", "GB/s"), "frac": frac}
    else:
        roof = {"bound": None, "level": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "note": "no counter summary of these kernel sources: re-profile (profiles/)"}
    roof.update({
        "kernel": "render_kernel",
        "traffic": ctr["hbm_bytes"] if ctr else None,
        "levels": levels,
        "algorithmic_bytes_per_launch": alg_bytes,
        "algorithmic_bytes_per_sample": per_sample,
        "uniform_random_gather_probe_gbs": probe or None,
        "kernel_sources": kernel_source_hash(),
    })
    if baked:
        workload = (f"baked_hd: 8 views x 1920x1080 rays, coarse grid L_C=512 block-sparse "
                    f"({sc.n_blocks} of {sc.block_index.size} blocks of 8^3 vertices), {L} fine hash levels "
                    f"{cfg.resolutions[0]}..{cfg.resolutions[-1]}, 2^22 entries, {DTYPE_NAME[dtype]} fine "
                    f"tables, {AGG_NAME[args.agg]}, contracted scene of 200 blobs, 256^3 "
                    "occupancy + distance grid, <=1024 samples/ray, T<1e-4")
    elif args.scene == "hd_regime":
        workload = ("hd_regime: 8 views x 1920x1080 rays, 16 hash levels 16..4096, 2^19 entries, "
                    f"{DTYPE_NAME[dtype]} tables, contracted scene of 400 blobs (sigma 0.02-0.08, "
                    "calibrated to the paper's Table 4 regime), 256^3 occupancy + distance grid, "
                    "<=1024 samples/ray, T<1e-4")
    else:
        workload = ("hd: 8 views x 1920x1080 rays, 16 hash levels 16..4096, 2^19 entries, "
                    f"{DTYPE_NAME[dtype]} tables, contracted scene of 200 blobs, 256^3 "
                    "occupancy + distance grid, <=1024 samples/ray, T<1e-4")
    if pyr:
        workload += (", occupancy pyramid 512^3..32^3" +
                     (" without the distance grid" if args.no_dist else " + 256^3 distance grid"))
    march_name = ("occupancy pyramid" + ("" if args.no_dist else " + distance grid")) if pyr \
        else "plain distance-grid marching"
    if args.mlp == "view":
        march_name += ", view-dependent MLP"
        workload += ", view-dependent MLP 23-64-64-3 with SH(d) as a second pass"
    res = {
        "metric": f"1080p frames/s ({'baked model, ' if baked else ''}{march_name})",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[dtype],
        "data": "synthetic",
        "config": {
            "workload": workload,
            "rays_per_step": n,
            "views": views,
        },
        "ms_median": round(float(np.median(per_step)), 4),
        "ms_p90": round(float(np.percentile(per_step, 90)), 4),
        "msamples_per_s": round(n_samples / (ms / 1e3) / 1e6, 1),
        "mreads_per_s": round(n_reads / (ms / 1e3) / 1e6, 1),
        "samples_per_ray": round(n_samples / n, 3),
        "reads_per_ray": round(n_reads / n, 3),
        "roofline": roof,
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    headline = not (baked or pyr or args.mlp == "view" or args.dtype != "f32" or args.scene != "hd")
    if args.prop_steps > 0 and headline:
        # the metric's second half: the learned proposal against plain marching
        del r, go, gd, aux, out
        torch.cuda.empty_cache()
        res["proposal_comparison"] = proposal_comparison(args.prop_steps, 3, args.prop_epochs)
    if args.regime_steps > 0 and headline:
        torch.cuda.empty_cache()
        res["regime_scene"] = regime_scene(args.regime_steps)
    if args.paper_steps > 0 and headline:
        torch.cuda.empty_cache()
        res["paper_configuration"] = paper_configuration(args.paper_steps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
