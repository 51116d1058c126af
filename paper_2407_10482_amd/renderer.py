"""PyTorch-facing wrapper of the C ABI.  PyTorch supplies device memory and
the current stream; every step of the render path runs in libngprt.so."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib, assets
from ._lib import (BF16, F32, FP8E4M3, MODEL_BAKED, MODEL_HASH, ROI_BOX, ROI_CONTRACT, NgprtOutputs,
                   check, load_library)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, shape=None, name="tensor") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Renderer:
    """One library context (one scene) on the current device."""

    def __init__(self, resolutions: Sequence[int], log2_table_size: int, table_dtype: int = F32,
                 domain: int = ROI_BOX, roi_half: float = 1.0, occ_res: int = 64,
                 step: float = 1.0 / 256.0, max_samples: int = 1024, t_threshold: float = 1e-4,
                 feature_model: int = MODEL_HASH, coarse_res: int = 0, occ_levels: int = 0,
                 occ_fine_res: int = 0, use_distance: bool = True, mlp_dims=(7, 16, 16, 3),
                 aggregation: int = _lib.AGG_SEPARATE_V, gate_params=()):
        self.lib = load_library()
        self.resolutions = list(resolutions)
        self.L = len(self.resolutions)
        self.T = 1 << log2_table_size
        self.R = occ_res
        self.table_dtype = table_dtype
        self.feature_model = feature_model
        self.coarse_res = coarse_res
        self.occ_fine_res = occ_fine_res
        self.aggregation = int(aggregation)
        self.mlp_dims = tuple(mlp_dims)
        self.view_mlp = self.mlp_dims[1] == 64
        self.n_mlp = _lib.mlp_param_count(self.mlp_dims)
        # the constructor's arguments: the descriptor a scene's manifest records
        self.descriptor = assets.normalise_descriptor(dict(
            resolutions=self.resolutions, log2_table_size=log2_table_size, table_dtype=table_dtype,
            domain=domain, roi_half=roi_half, occ_res=occ_res, step=step, max_samples=max_samples,
            t_threshold=t_threshold, feature_model=feature_model, coarse_res=coarse_res,
            occ_levels=occ_levels, occ_fine_res=occ_fine_res, use_distance=use_distance,
            mlp_dims=self.mlp_dims, aggregation=aggregation, gate_params=gate_params))
        self.desc = _lib.make_desc(resolutions, log2_table_size, table_dtype, domain, roi_half,
                                   occ_res, step, max_samples, t_threshold,
                                   feature_model=feature_model, coarse_res=coarse_res,
                                   occ_levels=occ_levels, occ_fine_res=occ_fine_res,
                                   use_distance=int(bool(use_distance)),
                                   mlp=(self.mlp_dims[0], self.mlp_dims[1], self.mlp_dims[3]),
                                   aggregation=aggregation, gate_params=gate_params)
        ctx = ctypes.c_void_p()
        check(self.lib.ngprt_create(ctypes.byref(self.desc), ctypes.byref(ctx)))
        self.ctx = ctx
        # bumped by every call that changes what a render of this context
        # computes (loads, step changes): the autograd backward checks that
        # the scene its forward rendered is still the loaded one
        self.load_gen = 0

    @classmethod
    def from_config(cls, cfg, table_dtype: Optional[int] = None, use_distance: bool = True) -> "Renderer":
        return cls(cfg.resolutions, cfg.log2_table, cfg.table_dtype if table_dtype is None else table_dtype,
                   cfg.domain, cfg.roi_half, cfg.occ_res, cfg.step, cfg.max_samples, cfg.t_threshold,
                   getattr(cfg, "model", MODEL_HASH), getattr(cfg, "coarse_res", 0),
                   getattr(cfg, "occ_levels", 0), getattr(cfg, "occ_fine_res", 0), use_distance,
                   tuple(cfg.mlp_dims), getattr(cfg, "aggregation", _lib.AGG_SEPARATE_V),
                   tuple(getattr(cfg, "gate_params", ())))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ngprt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- loading
    def load_tables(self, tables: torch.Tensor):
        self.load_gen += 1
        _dev(tables, torch.float32, (self.L, self.T, 9), "tables")
        check(self.lib.ngprt_load_tables(self.ctx, _ptr(tables), _stream()), self.ctx)

    def load_occupancy(self, occ: torch.Tensor, dist: Optional[torch.Tensor] = None):
        self.load_gen += 1
        _dev(occ, torch.uint8, (self.R, self.R, self.R), "occ")
        if dist is not None:
            _dev(dist, torch.uint8, (self.R, self.R, self.R), "dist")
        check(self.lib.ngprt_load_occupancy(self.ctx, _ptr(occ), _ptr(dist), _stream()), self.ctx)

    def load_occupancy_pyramid(self, occ_fine: torch.Tensor):
        self.load_gen += 1
        F = self.occ_fine_res
        _dev(occ_fine, torch.uint8, (F, F, F), "occ_fine")
        check(self.lib.ngprt_load_occupancy_pyramid(self.ctx, _ptr(occ_fine), _stream()), self.ctx)

    def load_mlp(self, params: torch.Tensor):
        self.load_gen += 1
        _dev(params, torch.float32, (self.n_mlp,), "mlp params")
        check(self.lib.ngprt_load_mlp(self.ctx, _ptr(params), _stream()), self.ctx)

    def load_coarse(self, block_index: torch.Tensor, atlas: torch.Tensor, default):
        """Baked model: block index grid int32 [nb]^3, atlas float32
        [n_blocks, 8, 8, 8, C], default vector (C floats, host); C = 8 + 2L
        (8 + L for Shared-Att (V), 8 for constant gates and SUM)."""
        self.load_gen += 1
        nb = (self.coarse_res + 1 + 7) // 8
        C = _lib.coarse_channels(self.L, self.aggregation)
        _dev(block_index, torch.int32, (nb, nb, nb), "block_index")
        n_blocks = atlas.shape[0]
        if n_blocks:
            _dev(atlas, torch.float32, (n_blocks, 8, 8, 8, C), "atlas")
        dflt = (ctypes.c_float * C)(*[float(x) for x in default])
        self.n_blocks = int(n_blocks)
        self._coarse_index = block_index
        self._coarse_default = [float(x) for x in default]
        check(self.lib.ngprt_load_coarse(self.ctx, n_blocks, _ptr(block_index),
                                         _ptr(atlas) if n_blocks else None, dflt, _stream()), self.ctx)

    def load_scene(self, tables, occ, mlp, dist=None):
        self.load_tables(tables)
        self.load_occupancy(occ, dist)
        self.load_mlp(mlp)

    # ------------------------------------------------------------ scene files
    @classmethod
    def from_assets(cls, path: str) -> "Renderer":
        """A renderer built from a scene directory's descriptor with all of
        its assets loaded (every file verified against the manifest first)."""
        desc, arrays = assets.read_scene(path)
        kw = dict(desc)
        kw["mlp_dims"] = tuple(kw["mlp_dims"])
        kw["gate_params"] = tuple(kw["gate_params"])
        r = cls(**kw)
        r.load_assets(arrays)
        return r

    def load_assets(self, arrays: Dict[str, np.ndarray]):
        """Load verified host arrays (the names of ``assets.DTYPES``) into this
        context: tables, occupancy (pyramid or single grid), MLP, coarse
        grid and proposal network, each through its C-ABI loader."""
        assets.check_assets(self.descriptor, arrays)
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in arrays.items()
               if k != "coarse_default"}
        self.load_tables(dev["tables"])
        if "occ_fine" in dev:
            self.load_occupancy_pyramid(dev["occ_fine"])
        else:
            self.load_occupancy(dev["occ"], dev.get("dist"))
        self.load_mlp(dev["mlp"])
        if "coarse_index" in dev:
            self.load_coarse(dev["coarse_index"], dev["coarse_atlas"], arrays["coarse_default"].tolist())
        if "proposal" in dev:
            self.load_proposal(dev["proposal"])
        torch.cuda.current_stream().synchronize()

    def save_assets(self, path: str, **arrays) -> Dict:
        """Write a scene directory for this renderer's descriptor from the
        caller's arrays (numpy or torch, already in the asset dtypes; device
        tensors are copied to the host).  Returns the manifest."""
        host = {k: (v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else np.asarray(v))
                for k, v in arrays.items()}
        return assets.save_scene(path, self.descriptor, host)

    # ---------------------------------------------------------------- export
    def export_tables(self):
        dt = {F32: torch.float32, BF16: torch.int16, FP8E4M3: torch.uint8}[self.table_dtype]
        codes = torch.empty((self.L, self.T, 9), dtype=dt, device="cuda")
        scales = torch.empty((self.L, 9), dtype=torch.float32, device="cuda")
        check(self.lib.ngprt_export_tables(self.ctx, _ptr(codes), _ptr(scales), _stream()), self.ctx)
        return codes, scales

    def export_distance(self) -> torch.Tensor:
        out = torch.empty((self.R, self.R, self.R), dtype=torch.uint8, device="cuda")
        check(self.lib.ngprt_export_distance(self.ctx, _ptr(out), _stream()), self.ctx)
        return out

    # ---------------------------------------------------------------- render
    def render(self, origins: torch.Tensor, dirs: torch.Tensor, aux: bool = True,
               out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        n = origins.shape[0]
        _dev(origins, torch.float32, (n, 3), "origins")
        _dev(dirs, torch.float32, (n, 3), "dirs")
        if out is None:
            out = self.alloc_outputs(n) if aux else {"rgb": torch.empty((n, 3), dtype=torch.float32,
                                                                        device="cuda")}
        self._view_buffers(out, n)
        o = self._outputs(out)
        check(self.lib.ngprt_render(self.ctx, n, _ptr(origins), _ptr(dirs), ctypes.byref(o),
                                    _stream()), self.ctx)
        return out

    def _view_buffers(self, out, n):
        """The view-dependent MLP runs over the C_d and F outputs: make sure
        the caller's output dict has them."""
        if self.view_mlp:
            if "c_d" not in out:
                out["c_d"] = torch.empty((n, 3), dtype=torch.float32, device="cuda")
            if "feat" not in out:
                out["feat"] = torch.empty((n, 4), dtype=torch.float32, device="cuda")

    OUTPUT_FIELDS = ("rgb", "c_d", "feat", "t_final", "depth", "n_samples", "n_reads", "t_first",
                     "t_far", "t_half", "dist_loss", "proposal")

    @staticmethod
    def _outputs(out: Dict[str, torch.Tensor]) -> NgprtOutputs:
        o = NgprtOutputs()
        for k in Renderer.OUTPUT_FIELDS:
            setattr(o, k, out[k].data_ptr() if k in out else None)
        return o

    def alloc_outputs(self, n: int, labels: bool = False) -> Dict[str, torch.Tensor]:
        f = dict(device="cuda", dtype=torch.float32)
        out = dict(rgb=torch.empty((n, 3), **f), c_d=torch.empty((n, 3), **f),
                   feat=torch.empty((n, 4), **f), t_final=torch.empty((n,), **f),
                   depth=torch.empty((n,), **f),
                   n_samples=torch.empty((n,), dtype=torch.int32, device="cuda"),
                   n_reads=torch.empty((n,), dtype=torch.int32, device="cuda"))
        if labels:
            out.update(t_first=torch.empty((n,), **f), t_far=torch.empty((n,), **f),
                       t_half=torch.empty((n,), **f))
        return out

    def _proposal_outputs(self, origins, dirs, aux, out, with_net):
        n = origins.shape[0]
        _dev(origins, torch.float32, (n, 3), "origins")
        _dev(dirs, torch.float32, (n, 3), "dirs")
        if out is None:
            out = self.alloc_outputs(n) if aux else {"rgb": torch.empty((n, 3), dtype=torch.float32,
                                                                        device="cuda")}
            if aux and with_net:
                out["proposal"] = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        self._view_buffers(out, n)
        fb = out.get("fallback")
        if fb is None and aux:
            fb = out["fallback"] = torch.empty((n,), dtype=torch.int32, device="cuda")
        return n, out, fb

    @staticmethod
    def _proposal_cfg(conf_threshold, margin, use_near, far_guard):
        return _lib.NgprtProposalCfg(float(conf_threshold), float(margin), int(bool(use_near)),
                                     float(far_guard))

    def render_intervals(self, origins: torch.Tensor, dirs: torch.Tensor, proposal: torch.Tensor,
                         conf_threshold: float = 0.9, margin: float = 0.0, aux: bool = True,
                         out: Optional[Dict[str, torch.Tensor]] = None, use_near: bool = True,
                         far_guard: float = 0.0):
        """Render with per-ray proposals [n, 4] (t_near, t_far, t_term, confidence) given by the caller."""
        n, out, fb = self._proposal_outputs(origins, dirs, aux, out, False)
        _dev(proposal, torch.float32, (n, 4), "proposal")
        o = self._outputs(out)
        cfg = self._proposal_cfg(conf_threshold, margin, use_near, far_guard)
        check(self.lib.ngprt_render_intervals(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(proposal),
                                              ctypes.byref(cfg), ctypes.byref(o), _ptr(fb), _stream()), self.ctx)
        return out

    def load_proposal(self, params: torch.Tensor):
        """Load the proposal network's float32 master weights [7556] into the library."""
        _dev(params, torch.float32, (7556,), "proposal params")
        check(self.lib.ngprt_proposal_load(self.ctx, _ptr(params), _stream()), self.ctx)

    def render_proposal(self, origins: torch.Tensor, dirs: torch.Tensor, conf_threshold: float = 0.9,
                        margin: float = 0.0, aux: bool = True, out: Optional[Dict[str, torch.Tensor]] = None,
                        use_near: bool = True, far_guard: float = 0.0):
        """Render with the loaded proposal network run inside the render kernel
        (its per-ray outputs in out["proposal"] when aux)."""
        n, out, fb = self._proposal_outputs(origins, dirs, aux, out, True)
        o = self._outputs(out)
        cfg = self._proposal_cfg(conf_threshold, margin, use_near, far_guard)
        check(self.lib.ngprt_render_proposal(self.ctx, n, _ptr(origins), _ptr(dirs), ctypes.byref(cfg),
                                             ctypes.byref(o), _ptr(fb), _stream()), self.ctx)
        return out

    # ---------------------------------------------------------------- debug
    def eval_points(self, pos: torch.Tensor):
        n = pos.shape[0]
        _dev(pos, torch.float32, (n, 3), "pos")
        idx = torch.empty((n, self.L, 8), dtype=torch.int32, device="cuda")
        fused = torch.empty((n, 8), dtype=torch.float32, device="cuda")
        w = torch.empty((n, self.L), dtype=torch.float32, device="cuda")
        check(self.lib.ngprt_debug_eval_points(self.ctx, n, _ptr(pos), _ptr(idx), _ptr(fused), _ptr(w),
                                               _stream()), self.ctx)
        return idx, fused, w

    def gather_probe(self, n_points: int, seed: int = 0, pairs: bool = False, out: torch.Tensor = None):
        """Random-gather ceiling probe over the loaded tables (measurement aid)."""
        if out is None:
            out = torch.empty((n_points,), dtype=torch.float32, device="cuda")
        _dev(out, torch.float32, (n_points,), "out")
        check(self.lib.ngprt_gather_probe(self.ctx, n_points, seed & 0xFFFFFFFF, int(bool(pairs)), _ptr(out),
                                          _stream()), self.ctx)
        return out

    def march(self, origins: torch.Tensor, dirs: torch.Tensor, cap: int = 64, naive: bool = False):
        n = origins.shape[0]
        _dev(origins, torch.float32, (n, 3), "origins")
        _dev(dirs, torch.float32, (n, 3), "dirs")
        sk = torch.empty((n, cap), dtype=torch.int32, device="cuda")
        ns = torch.empty((n,), dtype=torch.int32, device="cuda")
        nr = torch.empty((n,), dtype=torch.int32, device="cuda")
        check(self.lib.ngprt_debug_march(self.ctx, n, _ptr(origins), _ptr(dirs), cap, _ptr(sk), _ptr(ns),
                                         _ptr(nr), 1 if naive else 0, _stream()), self.ctx)
        return sk, ns, nr


def _renderer_backward(self: Renderer, origins, dirs, grad_rgb, grad_tables, grad_mlp, grad_dist=None):
    """Accumulate dL/dtables [L, T, 9] and dL/dmlp [451] for dL/drgb and,
    optionally, dL/d(dist_loss) per ray (the distortion regulariser)."""
    n = origins.shape[0]
    _dev(grad_rgb, torch.float32, (n, 3), "grad_rgb")
    _dev(grad_tables, torch.float32, (self.L, self.T, 9), "grad_tables")
    _dev(grad_mlp, torch.float32, (self.n_mlp,), "grad_mlp")
    if grad_dist is not None:
        _dev(grad_dist, torch.float32, (n,), "grad_dist")
    check(self.lib.ngprt_render_backward_reg(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(grad_rgb),
                                             _ptr(grad_dist), _ptr(grad_tables), _ptr(grad_mlp), _stream()),
          self.ctx)


def _renderer_backward_noalloc(self: Renderer, origins, dirs, grad_rgb, grad_tables, grad_mlp, grad_dist=None):
    """_renderer_backward through the allocation-free entry point (workspace
    in the library's static device scratch; at most NOALLOC_MAX_RAYS rays)."""
    n = origins.shape[0]
    _dev(grad_rgb, torch.float32, (n, 3), "grad_rgb")
    _dev(grad_tables, torch.float32, (self.L, self.T, 9), "grad_tables")
    _dev(grad_mlp, torch.float32, (self.n_mlp,), "grad_mlp")
    if grad_dist is not None:
        _dev(grad_dist, torch.float32, (n,), "grad_dist")
    check(self.lib.ngprt_render_backward_noalloc(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(grad_rgb),
                                                 _ptr(grad_dist), _ptr(grad_tables), _ptr(grad_mlp),
                                                 _stream()), self.ctx)


def _renderer_backward_baked(self: Renderer, origins, dirs, grad_rgb, grad_tables, grad_atlas, grad_mlp,
                             grad_dist=None):
    """Baked model: accumulate dL/d(fine tables) [L, T, 9] (channel 8 not
    written), dL/d(atlas) [n_blocks, 8, 8, 8, 8 + 2L] and dL/dmlp [451]."""
    n = origins.shape[0]
    _dev(grad_rgb, torch.float32, (n, 3), "grad_rgb")
    _dev(grad_tables, torch.float32, (self.L, self.T, 9), "grad_tables")
    _dev(grad_mlp, torch.float32, (self.n_mlp,), "grad_mlp")
    nblk = getattr(self, "n_blocks", 0)
    if nblk:
        _dev(grad_atlas, torch.float32, (nblk, 8, 8, 8, 8 + 2 * self.L), "grad_atlas")
    if grad_dist is not None:
        _dev(grad_dist, torch.float32, (n,), "grad_dist")
    check(self.lib.ngprt_render_backward_baked(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(grad_rgb),
                                               _ptr(grad_dist), _ptr(grad_tables),
                                               _ptr(grad_atlas) if nblk else None, _ptr(grad_mlp), _stream()),
          self.ctx)


def _renderer_backward_fwd(self: Renderer, origins, dirs, c_d, feat, grad_rgb, grad_tables, grad_mlp,
                           grad_atlas=None):
    """backward (hash model) or backward_baked (baked model) without the
    regulariser, given the forward's c_d [n, 3] and feat [n, 4] from render()
    of the same scene and rays: the library skips its first re-march."""
    n = origins.shape[0]
    _dev(c_d, torch.float32, (n, 3), "c_d")
    _dev(feat, torch.float32, (n, 4), "feat")
    _dev(grad_rgb, torch.float32, (n, 3), "grad_rgb")
    _dev(grad_tables, torch.float32, (self.L, self.T, 9), "grad_tables")
    _dev(grad_mlp, torch.float32, (self.n_mlp,), "grad_mlp")
    nblk = getattr(self, "n_blocks", 0) if self.feature_model == MODEL_BAKED else 0
    if nblk:
        _dev(grad_atlas, torch.float32, (nblk, 8, 8, 8, 8 + 2 * self.L), "grad_atlas")
    check(self.lib.ngprt_render_backward_fwd(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(c_d), _ptr(feat),
                                             _ptr(grad_rgb), _ptr(grad_tables),
                                             _ptr(grad_atlas) if nblk else None, _ptr(grad_mlp), _stream()),
          self.ctx)


def _renderer_view_mlp_backward(self: Renderer, dirs, c_d, feat, grad_rgb, grad_mlp) -> torch.Tensor:
    """View-dependent MLP: dL/dC_d and dL/dF per ray [n, 7] for dL/drgb,
    accumulating dL/dpsi [5891] into grad_mlp."""
    n = dirs.shape[0]
    _dev(dirs, torch.float32, (n, 3), "dirs")
    _dev(c_d, torch.float32, (n, 3), "c_d")
    _dev(feat, torch.float32, (n, 4), "feat")
    _dev(grad_rgb, torch.float32, (n, 3), "grad_rgb")
    _dev(grad_mlp, torch.float32, (self.n_mlp,), "grad_mlp")
    grad_cf = torch.empty((n, 7), dtype=torch.float32, device=dirs.device)
    check(self.lib.ngprt_view_mlp_backward(self.ctx, n, _ptr(dirs), _ptr(c_d), _ptr(feat), _ptr(grad_rgb),
                                           _ptr(grad_cf), _ptr(grad_mlp), _stream()), self.ctx)
    return grad_cf


def _renderer_backward_features(self: Renderer, origins, dirs, grad_cf, grad_tables, grad_atlas=None,
                                grad_dist=None, c_d=None, feat=None):
    """Accumulate dL/dtables (and, baked model, dL/datlas) from dL/dC_d and
    dL/dF per ray [n, 7].  c_d [n, 3], feat [n, 4]: the forward's, if at
    hand (then the library skips its first re-march; not with grad_dist)."""
    n = origins.shape[0]
    _dev(grad_cf, torch.float32, (n, 7), "grad_cf")
    if c_d is not None or feat is not None:
        _dev(c_d, torch.float32, (n, 3), "c_d")
        _dev(feat, torch.float32, (n, 4), "feat")
    _dev(grad_tables, torch.float32, (self.L, self.T, 9), "grad_tables")
    if grad_dist is not None:
        _dev(grad_dist, torch.float32, (n,), "grad_dist")
    nblk = getattr(self, "n_blocks", 0) if self.feature_model == MODEL_BAKED else 0
    if nblk:
        _dev(grad_atlas, torch.float32, (nblk, 8, 8, 8, 8 + 2 * self.L), "grad_atlas")
    check(self.lib.ngprt_render_backward_features(self.ctx, n, _ptr(origins), _ptr(dirs), _ptr(grad_cf),
                                                  _ptr(grad_dist), _ptr(grad_tables),
                                                  _ptr(grad_atlas) if nblk else None, _ptr(c_d), _ptr(feat),
                                                  _stream()), self.ctx)


def _renderer_set_deterministic(self: Renderer, on: bool = True):
    """Table gradients by sorted, fixed-order sums instead of atomics (the
    same bits on every run; slower, for gradient checks; hash model)."""
    check(self.lib.ngprt_set_deterministic_gradients(self.ctx, 1 if on else 0), self.ctx)


def _renderer_set_step(self: Renderer, step: float):
    self.load_gen += 1
    check(self.lib.ngprt_set_step(self.ctx, float(step)), self.ctx)
    self.step = float(step)


Renderer.backward = _renderer_backward
Renderer.backward_noalloc = _renderer_backward_noalloc
Renderer.backward_baked = _renderer_backward_baked
Renderer.view_mlp_backward = _renderer_view_mlp_backward
Renderer.backward_features = _renderer_backward_features
Renderer.backward_fwd = _renderer_backward_fwd
Renderer.set_deterministic = _renderer_set_deterministic
Renderer.set_step = _renderer_set_step


class StepAutoTuner:
    """Marching-step auto-tuning of the paper's training (supplement Eq. S3),
    run by the library: update(n_samples) takes a batch's per-ray sample
    counts (int32 [n] on the GPU), updates gamma and sets the renderer's step
    to gamma * s0."""

    def __init__(self, renderer: Renderer, s0: float, n_min: float = 3.0, kappa: float = 0.001,
                 gamma_min: float = 0.2217, gamma: float = 1.0):
        self.r = renderer
        self.state = _lib.NgprtStepTuner(float(s0), float(n_min), float(kappa), float(gamma_min), float(gamma),
                                         0.0)

    @property
    def gamma(self) -> float:
        return self.state.gamma

    def update(self, n_samples: torch.Tensor) -> float:
        n = n_samples.shape[0]
        _dev(n_samples, torch.int32, (n,), "n_samples")
        self.r.load_gen += 1
        check(self.r.lib.ngprt_step_autotune(self.r.ctx, n, _ptr(n_samples), ctypes.byref(self.state), _stream()),
              self.r.ctx)
        self.r.step = float(np.float32(float(self.state.gamma) * float(self.state.s0)))
        return self.state.gamma


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
              lr: float, beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-8):
    """In-place Adam update on the GPU (library kernel)."""
    for t, name in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _dev(t, torch.float32, param.shape, name)
    check(load_library().ngprt_adam_step(param.numel(), _ptr(param), _ptr(grad), _ptr(m), _ptr(v), int(step),
                                         float(lr), float(beta1), float(beta2), float(eps), _stream()))


def _forward_outputs(n: int, device, with_dist: bool) -> dict:
    """Output buffers of a differentiable forward: rgb, and either the
    per-ray regulariser value or the composited C_d and F that the backward
    then takes instead of re-marching for them."""
    f = dict(dtype=torch.float32, device=device)
    out = {"rgb": torch.empty((n, 3), **f)}
    if with_dist:
        out["dist_loss"] = torch.empty((n,), **f)
    else:
        out["c_d"] = torch.empty((n, 3), **f)
        out["feat"] = torch.empty((n, 4), **f)
    return out


def _same_scene(renderer: Renderer, gen: int):
    """The library's backward recomputes the forward from the scene loaded in
    the renderer: refuse when it changed since the forward."""
    if renderer.load_gen != gen:
        raise RuntimeError("the renderer's tables, MLP, grids or step changed between this render's forward "
                           "and its backward; render again (or use one renderer per differentiable model)")


class RenderFunction(torch.autograd.Function):
    """rgb = render(tables, mlp; rays) with the library's hand-written backward.

    forward loads `tables` (float32 [L, T, 9]) and `mlp` (float32 [451]) into
    the renderer and renders; backward re-marches each ray inside the
    library (taking the forward's C_d and F when no regulariser is on) and
    returns dL/dtables and dL/dmlp."""

    @staticmethod
    def forward(ctx, tables, mlp, origins, dirs, renderer, with_dist):
        renderer.load_tables(tables.detach().contiguous())
        renderer.load_mlp(mlp.detach().contiguous())
        n = origins.shape[0]
        out = _forward_outputs(n, origins.device, with_dist)
        renderer.render(origins, dirs, out=out)
        ctx.renderer = renderer
        ctx.load_gen = renderer.load_gen
        ctx.with_dist = with_dist
        if not with_dist:
            # the backward takes the forward's C_d and F instead of re-marching for them
            ctx.save_for_backward(origins, dirs, out["c_d"], out["feat"])
            dist = torch.zeros((n,), dtype=torch.float32, device=origins.device)
            ctx.mark_non_differentiable(dist)
            return out["rgb"], dist
        ctx.save_for_backward(origins, dirs)
        return out["rgb"], out["dist_loss"]

    @staticmethod
    def backward(ctx, grad_rgb, grad_dist):
        saved = ctx.saved_tensors
        origins, dirs = saved[0], saved[1]
        r = ctx.renderer
        _same_scene(r, ctx.load_gen)
        gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device=origins.device)
        gm = torch.zeros((r.n_mlp,), dtype=torch.float32, device=origins.device)
        if grad_rgb is None:
            grad_rgb = torch.zeros((origins.shape[0], 3), dtype=torch.float32, device=origins.device)
        if not ctx.with_dist:
            r.backward_fwd(origins, dirs, saved[2], saved[3], grad_rgb.contiguous().float(), gt, gm)
            return gt, gm, None, None, None, None
        gdist = grad_dist.contiguous().float() if grad_dist is not None else None
        r.backward(origins, dirs, grad_rgb.contiguous().float(), gt, gm, gdist)
        return gt, gm, None, None, None, None


class BakedRenderFunction(torch.autograd.Function):
    """rgb = render(fine tables, atlas, mlp; rays) for the baked feature
    model, with the library's hand-written backward.  The block index grid
    and the default vector are those of the renderer's last load_coarse;
    forward re-loads the fine tables, the atlas and the MLP."""

    @staticmethod
    def forward(ctx, tables, atlas, mlp, origins, dirs, renderer, with_dist):
        renderer.load_tables(tables.detach().contiguous())
        renderer.load_coarse(renderer._coarse_index, atlas.detach().contiguous(), renderer._coarse_default)
        renderer.load_mlp(mlp.detach().contiguous())
        n = origins.shape[0]
        out = _forward_outputs(n, origins.device, with_dist)
        renderer.render(origins, dirs, out=out)
        ctx.renderer = renderer
        ctx.load_gen = renderer.load_gen
        ctx.with_dist = with_dist
        ctx.atlas_shape = tuple(atlas.shape)
        if not with_dist:
            ctx.save_for_backward(origins, dirs, out["c_d"], out["feat"])
            dist = torch.zeros((n,), dtype=torch.float32, device=origins.device)
            ctx.mark_non_differentiable(dist)
            return out["rgb"], dist
        ctx.save_for_backward(origins, dirs)
        return out["rgb"], out["dist_loss"]

    @staticmethod
    def backward(ctx, grad_rgb, grad_dist):
        saved = ctx.saved_tensors
        origins, dirs = saved[0], saved[1]
        r = ctx.renderer
        _same_scene(r, ctx.load_gen)
        gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device=origins.device)
        ga = torch.zeros(ctx.atlas_shape, dtype=torch.float32, device=origins.device)
        gm = torch.zeros((r.n_mlp,), dtype=torch.float32, device=origins.device)
        if grad_rgb is None:
            grad_rgb = torch.zeros((origins.shape[0], 3), dtype=torch.float32, device=origins.device)
        if not ctx.with_dist:
            r.backward_fwd(origins, dirs, saved[2], saved[3], grad_rgb.contiguous().float(), gt, gm, ga)
            return gt, ga, gm, None, None, None, None
        gdist = grad_dist.contiguous().float() if grad_dist is not None else None
        r.backward_baked(origins, dirs, grad_rgb.contiguous().float(), gt, ga, gm, gdist)
        return gt, ga, gm, None, None, None, None


class ViewRenderFunction(torch.autograd.Function):
    """rgb with the view-dependent MLP (either feature model) as a function
    of the tables, the coarse atlas (baked model; None otherwise) and psi:
    backward runs the MLP's adjoint, then the render adjoint from dL/dC_d
    and dL/dF."""

    @staticmethod
    def forward(ctx, tables, atlas, mlp, origins, dirs, renderer, with_dist):
        renderer.load_tables(tables.detach().contiguous())
        if atlas is not None:
            renderer.load_coarse(renderer._coarse_index, atlas.detach().contiguous(),
                                 renderer._coarse_default)
        renderer.load_mlp(mlp.detach().contiguous())
        n = origins.shape[0]
        dev = origins.device
        out = {"rgb": torch.empty((n, 3), dtype=torch.float32, device=dev),
               "c_d": torch.empty((n, 3), dtype=torch.float32, device=dev),
               "feat": torch.empty((n, 4), dtype=torch.float32, device=dev)}
        if with_dist:
            out["dist_loss"] = torch.empty((n,), dtype=torch.float32, device=dev)
        renderer.render(origins, dirs, out=out)
        ctx.renderer = renderer
        ctx.load_gen = renderer.load_gen
        ctx.with_dist = with_dist
        ctx.atlas_shape = None if atlas is None else tuple(atlas.shape)
        ctx.save_for_backward(origins, dirs, out["c_d"], out["feat"])
        if not with_dist:
            dist = torch.zeros((n,), dtype=torch.float32, device=dev)
            ctx.mark_non_differentiable(dist)
            return out["rgb"], dist
        return out["rgb"], out["dist_loss"]

    @staticmethod
    def backward(ctx, grad_rgb, grad_dist):
        origins, dirs, c_d, feat = ctx.saved_tensors
        r = ctx.renderer
        _same_scene(r, ctx.load_gen)
        dev = origins.device
        if grad_rgb is None:
            grad_rgb = torch.zeros((origins.shape[0], 3), dtype=torch.float32, device=dev)
        gm = torch.zeros((r.n_mlp,), dtype=torch.float32, device=dev)
        grad_cf = r.view_mlp_backward(dirs, c_d, feat, grad_rgb.contiguous().float(), gm)
        gt = torch.zeros((r.L, r.T, 9), dtype=torch.float32, device=dev)
        ga = None if ctx.atlas_shape is None else torch.zeros(ctx.atlas_shape, dtype=torch.float32, device=dev)
        if not ctx.with_dist:
            # the forward's C_d and F stand in for the backward's first re-march
            r.backward_features(origins, dirs, grad_cf, gt, ga, None, c_d, feat)
            return gt, ga, gm, None, None, None, None
        gdist = grad_dist.contiguous().float() if grad_dist is not None else None
        r.backward_features(origins, dirs, grad_cf, gt, ga, gdist)
        return gt, ga, gm, None, None, None, None


def render_differentiable_view(renderer: Renderer, tables, mlp, origins, dirs, atlas=None,
                               with_dist: bool = False):
    """View-dependent MLP: rgb (and, with_dist, the distortion regulariser)
    as differentiable functions of the tables, psi and, baked model, the
    coarse atlas."""
    rgb, dist = ViewRenderFunction.apply(tables, atlas, mlp, origins, dirs, renderer, with_dist)
    return (rgb, dist) if with_dist else rgb


def render_differentiable_baked(renderer: Renderer, tables, atlas, mlp, origins, dirs, with_dist: bool = False):
    """Baked model: rgb (and, with_dist, the distortion regulariser) as
    differentiable functions of the fine tables, the coarse atlas and the
    MLP (load_coarse must have set the block index grid first)."""
    rgb, dist = BakedRenderFunction.apply(tables, atlas, mlp, origins, dirs, renderer, with_dist)
    return (rgb, dist) if with_dist else rgb


def render_differentiable(renderer: Renderer, tables, mlp, origins, dirs, with_dist: bool = False):
    """rgb (and, with_dist, the per-ray distortion regulariser) as
    differentiable functions of the tables and the MLP."""
    rgb, dist = RenderFunction.apply(tables, mlp, origins, dirs, renderer, with_dist)
    return (rgb, dist) if with_dist else rgb


N_PROPOSAL_PARAMS = 7556


def proposal_init(seed: int) -> torch.Tensor:
    """He-uniform float32 weights and zero biases for the proposal network
    (W1[64][48], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]), on the GPU."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for fin, fout in ((48, 64), (64, 64), (64, 4)):
        a = (6.0 / fin) ** 0.5
        parts.append((torch.rand((fout * fin,), generator=g, dtype=torch.float64) * 2 - 1) * a)
        parts.append(torch.zeros(fout, dtype=torch.float64))
    return torch.cat(parts).float().cuda()


class Proposal:
    """Per-ray sample-interval proposal network on the GPU (library kernels).

    Holds float32 master weights and Adam moments as torch tensors; training
    and inference run in libngprt.so on bfloat16 operands."""

    def __init__(self, params: torch.Tensor, ctx_owner: Renderer):
        _dev(params, torch.float32, (N_PROPOSAL_PARAMS,), "proposal params")
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self.owner = ctx_owner          # supplies the library context (workspace)

    def infer(self, origins: torch.Tensor, dirs: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        n = origins.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        _dev(out, torch.float32, (n, 4), "out")
        check(self.owner.lib.ngprt_proposal_infer(self.owner.ctx, n, _ptr(origins), _ptr(dirs),
                                                  _ptr(self.params), _ptr(out), _stream()), self.owner.ctx)
        return out

    def grad(self, origins, dirs, labels, phase: int = 1, margin: float = 0.0):
        """Gradient and loss of one batch, no update."""
        g = torch.empty_like(self.params)
        loss = torch.zeros((1,), dtype=torch.float32, device="cuda")
        check(self.owner.lib.ngprt_proposal_train_step(
            self.owner.ctx, origins.shape[0], _ptr(origins), _ptr(dirs), _ptr(labels), int(phase),
            float(margin), _ptr(self.params), None, None, 0, 0.0, _ptr(loss), _ptr(g), _stream()),
            self.owner.ctx)
        return g, loss

    def train_step(self, origins, dirs, labels, lr: float, phase: int = 1, margin: float = 0.0,
                   loss: Optional[torch.Tensor] = None):
        _dev(labels, torch.float32, (origins.shape[0], 4), "labels")
        self.step += 1
        check(self.owner.lib.ngprt_proposal_train_step(
            self.owner.ctx, origins.shape[0], _ptr(origins), _ptr(dirs), _ptr(labels), int(phase),
            float(margin), _ptr(self.params), _ptr(self.m), _ptr(self.v), self.step, float(lr),
            _ptr(loss), None, _stream()), self.owner.ctx)
