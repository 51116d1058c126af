"""C-ABI boundary tests that need no GPU: the library loads, exports what
include/ngprt.h declares, validates descriptors and rejects bad arguments
with the documented status codes."""
import ctypes
import os
import re

import pytest

import synth
from paper_2407_10482_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load_library()


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ngprt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ngprt_[a-z_]+)\s*\(", src)))


def test_header_symbols_are_exported(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound


def test_missing_library_fails_loudly(tmp_path):
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError):
            _lib.load_library(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def _good_desc():
    cfg = synth.tiny()
    return _lib.make_desc(cfg.resolutions, cfg.log2_table, 0, cfg.domain, cfg.roi_half, cfg.occ_res,
                          cfg.step, cfg.max_samples, cfg.t_threshold)


@pytest.mark.parametrize("field,value,code", [
    ("n_levels", 0, -2), ("n_levels", 17, -2), ("log2_table_size", 3, -2),
    ("log2_table_size", 25, -2), ("table_dtype", 3, -3), ("table_dtype", -1, -3),
    ("domain", 2, -1), ("roi_half", 1.5, -1), ("roi_half", 0.0, -1), ("roi_half", float("inf"), -1),
    ("occ_res", 1, -2), ("occ_res", 2048, -2), ("step", 0.0, -1), ("step", -0.1, -1),
    ("step", float("nan"), -1), ("step", 1e-6, -1), ("max_samples", 0, -1),
    ("t_threshold", -1.0, -1), ("t_threshold", float("nan"), -1), ("mlp_in", 8, -7),
    ("mlp_hidden", 64, -7), ("feature_model", 2, -1), ("feature_model", -1, -1),
])
def test_validate_desc_rejects(lib, field, value, code):
    d = _good_desc()
    setattr(d, field, value)
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == code


def test_validate_desc_baked_model(lib):
    cfg = synth.baked_hd(n_fine=4)
    d = _lib.make_desc(cfg.resolutions, cfg.log2_table, 0, cfg.domain, cfg.roi_half, cfg.occ_res,
                       cfg.step, cfg.max_samples, cfg.t_threshold, feature_model=_lib.MODEL_BAKED,
                       coarse_res=cfg.coarse_res)
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == 0
    d.coarse_res = 0
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -2
    d.coarse_res = 4096
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -2
    d.coarse_res = 512
    d.n_levels = 5                        # at most 4 fine levels (16 coarse channels)
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -2


def test_validate_desc_aggregation(lib):
    """Table 3's aggregations: baked model only, float32 tables, finite
    constant gates for the (Inv) variants."""
    cfg = synth.baked_hd(n_fine=4)

    def desc(agg, dtype=0, params=()):
        return _lib.make_desc(cfg.resolutions, cfg.log2_table, dtype, cfg.domain, cfg.roi_half,
                              cfg.occ_res, cfg.step, cfg.max_samples, cfg.t_threshold,
                              feature_model=_lib.MODEL_BAKED, coarse_res=cfg.coarse_res,
                              aggregation=agg, gate_params=params)
    for agg in range(5):
        assert lib.ngprt_validate_desc(ctypes.byref(desc(agg, params=[0.5] * 8))) == 0
    assert lib.ngprt_validate_desc(ctypes.byref(desc(5))) == -1
    assert lib.ngprt_validate_desc(ctypes.byref(desc(-1))) == -1
    assert lib.ngprt_validate_desc(ctypes.byref(desc(0, dtype=1))) == 0
    for agg in range(1, 5):
        assert lib.ngprt_validate_desc(ctypes.byref(desc(agg, dtype=1, params=[0.5] * 8))) == -7
    bad = [0.5] * 8
    bad[7] = float("nan")                 # Separate-Att (Inv) at L = 4 reads all 8
    assert lib.ngprt_validate_desc(ctypes.byref(desc(2, params=bad))) == -1
    assert lib.ngprt_validate_desc(ctypes.byref(desc(3, params=bad))) == 0    # reads 4
    bad[3] = float("inf")
    assert lib.ngprt_validate_desc(ctypes.byref(desc(3, params=bad))) == -1
    d = _good_desc()                      # hash model: aggregation must stay 0
    d.aggregation = 4
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -1
    assert _lib.coarse_channels(4, 0) == 16 and _lib.coarse_channels(4, 1) == 12
    assert all(_lib.coarse_channels(4, a) == 8 for a in (2, 3, 4))


def test_validate_desc_accepts_workloads(lib):
    assert lib.ngprt_validate_desc(ctypes.byref(_good_desc())) == 0
    cfg = synth.hd()
    d = _lib.make_desc(cfg.resolutions, cfg.log2_table, 2, cfg.domain, cfg.roi_half, cfg.occ_res,
                       cfg.step, cfg.max_samples, cfg.t_threshold)
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == 0
    d.roi_half = 1.0                      # the contracted domain needs roi_half = 2
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -1
    d = _good_desc()
    d.resolutions[3] = 0
    assert lib.ngprt_validate_desc(ctypes.byref(d)) == -2
    assert lib.ngprt_validate_desc(None) == -1


def test_null_context_and_arguments(lib):
    assert lib.ngprt_create(ctypes.byref(_good_desc()), None) == -1
    bad = _good_desc()
    bad.n_levels = 0
    out = ctypes.c_void_p()
    assert lib.ngprt_create(ctypes.byref(bad), ctypes.byref(out)) == -2
    assert out.value is None
    o = _lib.NgprtOutputs()
    assert lib.ngprt_render(None, 10, None, None, ctypes.byref(o), None) == -1
    assert lib.ngprt_load_tables(None, None, None) == -1
    assert lib.ngprt_load_occupancy(None, None, None, None) == -1
    assert lib.ngprt_load_mlp(None, None, None) == -1
    assert lib.ngprt_export_tables(None, None, None, None) == -1
    assert lib.ngprt_export_distance(None, None, None) == -1
    assert lib.ngprt_debug_eval_points(None, 1, None, None, None, None, None) == -1
    assert lib.ngprt_debug_march(None, 1, None, None, 0, None, None, None, 0, None) == -1
    lib.ngprt_destroy(None)
    assert lib.ngprt_last_error(None) == b""


def test_status_strings(lib):
    for code, name in _lib.STATUS.items():
        assert lib.ngprt_status_string(code).decode() == name
    assert lib.ngprt_status_string(-99) == b"NGPRT_E_UNKNOWN"
