"""ctypes declarations of libngprt.so (see include/ngprt.h).  Argument
marshalling only; no arithmetic of the render path lives here."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libngprt.so")

MAX_LEVELS = 16
NOALLOC_MAX_RAYS = 524288        # NGPRT_NOALLOC_MAX_RAYS
DET_MAX_RECORDS = 67108864       # NGPRT_DET_MAX_RECORDS
NGPRT_OK = 0
STATUS = {0: "NGPRT_OK", -1: "NGPRT_E_INVALID_ARG", -2: "NGPRT_E_SHAPE", -3: "NGPRT_E_DTYPE",
          -4: "NGPRT_E_NOT_LOADED", -5: "NGPRT_E_ALLOC", -6: "NGPRT_E_HIP", -7: "NGPRT_E_UNSUPPORTED"}

F32, BF16, FP8E4M3 = 0, 1, 2
ROI_BOX, ROI_CONTRACT = 0, 1
MODEL_HASH, MODEL_BAKED = 0, 1
AGG_SEPARATE_V, AGG_SHARED_V, AGG_SEPARATE_INV, AGG_SHARED_INV, AGG_SUM = 0, 1, 2, 3, 4


class NgprtDesc(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32),
        ("resolutions", ctypes.c_int32 * MAX_LEVELS),
        ("log2_table_size", ctypes.c_int32),
        ("table_dtype", ctypes.c_int32),
        ("domain", ctypes.c_int32),
        ("roi_half", ctypes.c_float),
        ("occ_res", ctypes.c_int32),
        ("step", ctypes.c_float),
        ("max_samples", ctypes.c_int32),
        ("t_threshold", ctypes.c_float),
        ("mlp_in", ctypes.c_int32),
        ("mlp_hidden", ctypes.c_int32),
        ("mlp_out", ctypes.c_int32),
        ("feature_model", ctypes.c_int32),
        ("coarse_res", ctypes.c_int32),
        ("occ_levels", ctypes.c_int32),
        ("occ_fine_res", ctypes.c_int32),
        ("use_distance", ctypes.c_int32),
        ("aggregation", ctypes.c_int32),
        ("gate_params", ctypes.c_float * 8),
    ]


class NgprtOutputs(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("rgb", "c_d", "feat", "t_final", "depth", "n_samples", "n_reads", "t_first",
                 "t_far", "t_half", "dist_loss", "proposal")]


class NgprtProposalCfg(ctypes.Structure):
    _fields_ = [("conf_threshold", ctypes.c_float), ("margin", ctypes.c_float), ("use_near", ctypes.c_int32),
                ("far_guard", ctypes.c_float)]


class NgprtStepTuner(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in ("s0", "n_min", "kappa", "gamma_min", "gamma", "mean_samples")]


# (name, restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
SIGNATURES = [
    ("ngprt_create", ctypes.c_int, [ctypes.POINTER(NgprtDesc), ctypes.POINTER(_P)]),
    ("ngprt_destroy", None, [_P]),
    ("ngprt_validate_desc", ctypes.c_int, [ctypes.POINTER(NgprtDesc)]),
    ("ngprt_load_tables", ctypes.c_int, [_P, _P, _P]),
    ("ngprt_export_tables", ctypes.c_int, [_P, _P, _P, _P]),
    ("ngprt_load_coarse", ctypes.c_int, [_P, _I64, _P, _P, _P, _P]),
    ("ngprt_load_occupancy", ctypes.c_int, [_P, _P, _P, _P]),
    ("ngprt_export_distance", ctypes.c_int, [_P, _P, _P]),
    ("ngprt_load_occupancy_pyramid", ctypes.c_int, [_P, _P, _P]),
    ("ngprt_load_mlp", ctypes.c_int, [_P, _P, _P]),
    ("ngprt_render", ctypes.c_int, [_P, _I64, _P, _P, ctypes.POINTER(NgprtOutputs), _P]),
    ("ngprt_debug_eval_points", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P]),
    ("ngprt_gather_probe", ctypes.c_int, [_P, _I64, ctypes.c_uint32, _I32, _P, _P]),
    ("ngprt_debug_march", ctypes.c_int, [_P, _I64, _P, _P, _I32, _P, _P, _P, _I32, _P]),
    ("ngprt_render_intervals", ctypes.c_int, [_P, _I64, _P, _P, _P, ctypes.POINTER(NgprtProposalCfg),
                                              ctypes.POINTER(NgprtOutputs), _P, _P]),
    ("ngprt_render_proposal", ctypes.c_int, [_P, _I64, _P, _P, ctypes.POINTER(NgprtProposalCfg),
                                             ctypes.POINTER(NgprtOutputs), _P, _P]),
    ("ngprt_proposal_load", ctypes.c_int, [_P, _P, _P]),
    ("ngprt_render_backward", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P]),
    ("ngprt_render_backward_reg", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_render_backward_noalloc", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_render_backward_baked", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_render_backward_fwd", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_test_fail_alloc", ctypes.c_int, [_I64]),
    ("ngprt_set_deterministic_gradients", ctypes.c_int, [_P, ctypes.c_int]),
    ("ngprt_view_mlp_backward", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_render_backward_features", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("ngprt_set_step", ctypes.c_int, [_P, ctypes.c_float]),
    ("ngprt_step_autotune", ctypes.c_int, [_P, _I64, _P, ctypes.POINTER(NgprtStepTuner), _P]),
    ("ngprt_adam_step", ctypes.c_int, [_I64, _P, _P, _P, _P, _I32, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, _P]),
    ("ngprt_proposal_infer", ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _P]),
    ("ngprt_proposal_train_step", ctypes.c_int, [_P, _I64, _P, _P, _P, _I32, ctypes.c_float, _P, _P, _P,
                                                 _I32, ctypes.c_float, _P, _P, _P]),
    ("ngprt_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("ngprt_last_error", ctypes.c_char_p, [_P]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libngprt.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # Load PyTorch's HIP runtime first so libngprt binds to the same
    # libamdhip64 instance (its SONAME satisfies libngprt's dependency);
    # loading libngprt first would bring in a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class NgprtError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code: int, ctx=None):
    if code != NGPRT_OK:
        msg = ""
        if ctx:
            m = load_library().ngprt_last_error(ctx)
            msg = m.decode() if m else ""
        raise NgprtError(code, msg)


def make_desc(resolutions, log2_table_size, table_dtype, domain, roi_half, occ_res, step,
              max_samples, t_threshold, mlp=(7, 16, 3), feature_model=MODEL_HASH,
              coarse_res=0, occ_levels=0, occ_fine_res=0, use_distance=1, aggregation=AGG_SEPARATE_V,
              gate_params=()) -> NgprtDesc:
    d = NgprtDesc()
    d.n_levels = len(resolutions)
    for i, r in enumerate(resolutions[:MAX_LEVELS]):
        d.resolutions[i] = int(r)
    d.log2_table_size = int(log2_table_size)
    d.table_dtype = int(table_dtype)
    d.domain = int(domain)
    d.roi_half = float(roi_half)
    d.occ_res = int(occ_res)
    d.step = float(step)
    d.max_samples = int(max_samples)
    d.t_threshold = float(t_threshold)
    d.mlp_in, d.mlp_hidden, d.mlp_out = mlp
    d.feature_model = int(feature_model)
    d.coarse_res = int(coarse_res)
    d.occ_levels = int(occ_levels)
    d.occ_fine_res = int(occ_fine_res)
    d.use_distance = int(use_distance)
    d.aggregation = int(aggregation)
    for i, g in enumerate(list(gate_params)[:8]):
        d.gate_params[i] = float(g)
    return d


def mlp_param_count(dims) -> int:
    """Parameters of an in -> h -> h -> out MLP with biases (weights, then biases, layer by layer)."""
    i, h, h2, o = dims
    return h * i + h + h2 * h + h2 + o * h2 + o


def coarse_channels(n_levels: int, aggregation: int = AGG_SEPARATE_V) -> int:
    """Channels per coarse vertex of the baked model under an aggregation."""
    return 8 + {AGG_SEPARATE_V: 2 * n_levels, AGG_SHARED_V: n_levels}.get(aggregation, 0)
