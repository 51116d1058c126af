"""The benchmark's host side: its command line, and the committed counter
summaries its roofline reads (they must have been taken on the kernel
sources as they are, or the roofline would be dropped)."""
import sys

import pytest

sys.path.insert(0, __file__.rsplit("/tests/", 1)[0])
import bench  # noqa: E402


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_committed_render_counters_match_the_sources(dtype):
    c = bench.committed_counters(dtype, "hd")
    assert c is not None, (f"profiles/render_kernel_hd_{dtype}_counters.md was taken on other kernel sources "
                           f"than {bench.kernel_source_hash()}: re-profile")
    for k in ("hbm_bytes", "valu", "l2_req", "l2_hit", "vmem_rd", "ta_busy", "td_busy"):
        assert c[k] is not None and c[k] > 0, k
    assert 0.0 < c["ta_busy"] <= 1.0 and 0.0 < c["td_busy"] <= 1.0


def test_regime_counters_match_the_sources():
    assert bench.committed_counters("f32", "hd_regime") is not None


def test_default_arguments_time_the_headline_over_five_seconds(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    args = bench.parse()
    assert args.gpus == 1 and args.steps * 0.0467 > 5.0
    assert args.regime_steps > 0 and args.paper_steps > 0 and args.prop_steps > 0
