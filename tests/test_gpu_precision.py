"""Reduced-precision tables: per-image error of the GPU render against the
float64 oracle with the unquantised tables (quantisation loss + kernel
error), and of the oracle on the quantised tables (quantisation loss alone).
The report is printed, and written as precision_report.json into the
directory named by NGPRT_REPORT_DIR when that is set."""
import json
import os

import numpy as np
import pytest

import synth
from oracle.render import render

from helpers import gpu_renderer, oracle_inputs, scene_and_dist, to_gpu

pytestmark = pytest.mark.gpu


def _psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def test_precision_report():
    sc, _ = scene_and_dist("tiny")
    o, d, _ = synth.scene_rays(sc.cfg)
    ref64 = render(oracle_inputs("tiny", 0), o, d).rgb
    go, gd = to_gpu(o, d)
    report = {}
    for dt, name in ((0, "f32"), (1, "bf16"), (2, "fp8")):
        print(f"[precision {name}]", flush=True)
        gpu = gpu_renderer("tiny", dt).render(go, gd)["rgb"].cpu().numpy().astype(np.float64)
        orq = render(oracle_inputs("tiny", dt), o, d).rgb
        report[name] = {
            "gpu_vs_fp64_f32tables": {"max_abs": float(np.abs(gpu - ref64).max()),
                                      "mean_abs": float(np.abs(gpu - ref64).mean()),
                                      "psnr_db": _psnr(gpu, ref64)},
            "oracle_q_vs_fp64_f32tables": {"max_abs": float(np.abs(orq - ref64).max()),
                                           "mean_abs": float(np.abs(orq - ref64).mean()),
                                           "psnr_db": _psnr(orq, ref64)},
            "kernel_error_max_abs": float(np.abs(gpu - orq).max()),
        }
        print(name, json.dumps(report[name]), flush=True)
        assert report[name]["kernel_error_max_abs"] < 1e-5
    assert report["f32"]["gpu_vs_fp64_f32tables"]["max_abs"] < 1e-5
    assert report["bf16"]["gpu_vs_fp64_f32tables"]["psnr_db"] > 40.0
    assert report["fp8"]["gpu_vs_fp64_f32tables"]["psnr_db"] > 25.0
    report_dir = os.environ.get("NGPRT_REPORT_DIR")
    if report_dir:
        os.makedirs(report_dir, exist_ok=True)
        with open(os.path.join(report_dir, "precision_report.json"), "w") as f:
            json.dump(report, f, indent=1)
