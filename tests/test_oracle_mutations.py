"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of an oracle module (a textual change to its source, executed as
a fresh module), runs an existing pin with the mutated functions in place of
the real ones, and expects the pin to fail.  CPU only; the real oracle is
untouched."""
import importlib
import inspect
import sys
import types

import pytest

import test_oracle_baked as pins_baked
import test_oracle_distortion as pins_dist
import test_oracle_pins as pins


def _mutated(name, old, new, **inject):
    """A fresh copy of module `name` with `old` replaced by `new` once."""
    src = inspect.getsource(importlib.import_module(name))
    assert src.count(old) == 1, (name, old)
    mod = types.ModuleType(name + "_mutant")
    mod.__package__ = name.rpartition(".")[0]
    mod.__file__ = "<mutant of %s>" % name
    sys.modules[mod.__name__] = mod            # dataclasses resolve their module by name
    try:
        exec(compile(src.replace(old, new), mod.__file__, "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    for k, v in inject.items():
        setattr(mod, k, v)
    return mod


def _run(pin, *args, **rebind):
    """Run a pin test with some of its module-level names rebound."""
    g = dict(pin.__globals__)
    g.update(rebind)
    f = types.FunctionType(pin.__code__, g, pin.__name__, pin.__defaults__, pin.__closure__)
    f(*args)


def _fails(pin, *args, **rebind):
    with pytest.raises(AssertionError):
        _run(pin, *args, **rebind)


def test_unmutated_copies_pass():
    """The harness itself: unmodified copies pass the same pins."""
    hg = _mutated("oracle.hashgrid", "PRIMES = (", "PRIMES = (")
    _run(pins.test_hash_golden_vectors, spatial_hash=hg.spatial_hash)
    _run(pins.test_trilinear_reproduces_affine_field_on_injective_level, corners64=hg.corners64,
         spatial_hash=hg.spatial_hash)
    ex = _mutated("oracle.exact32", "def exp32(", "def exp32(")
    _run(pins.test_exp32_accuracy_and_specials, exp32=ex.exp32)


def test_swapped_hash_primes_are_caught():
    hg = _mutated("oracle.hashgrid", "PRIMES = (1, 2654435761, 805459861)", "PRIMES = (1, 805459861, 2654435761)")
    _fails(pins.test_hash_golden_vectors, spatial_hash=hg.spatial_hash)


def test_swapped_trilinear_weights_are_caught():
    hg = _mutated("oracle.hashgrid", "wa = [f[:, a] if b[a] else 1.0 - f[:, a] for a in range(3)]",
                  "wa = [1.0 - f[:, a] if b[a] else f[:, a] for a in range(3)]")
    _fails(pins.test_trilinear_reproduces_affine_field_on_injective_level, corners64=hg.corners64,
           spatial_hash=hg.spatial_hash)


def test_dropped_taylor_term_in_exp32_is_caught():
    ex = _mutated("oracle.exact32", "for j in range(6, -1, -1):", "for j in range(6, 0, -1):")
    _fails(pins.test_exp32_accuracy_and_specials, exp32=ex.exp32)


def test_wrong_opacity_in_compositing_is_caught():
    rd = _mutated("oracle.render", "alpha = 1.0 - np.exp(-sigma * float(F32(inp.step)))",
                  "alpha = np.exp(-sigma * float(F32(inp.step)))")
    _fails(pins.test_constant_density_slab_closed_form, 3.0, False, render=rd.render)


def test_transposed_mlp_weights_are_caught():
    rd = _mutated("oracle.render", "W1 = p[off:off + h2 * h1].reshape(h2, h1); off += h2 * h1",
                  "W1 = p[off:off + h2 * h1].reshape(h1, h2).T; off += h2 * h1")
    _fails(pins.test_mlp_matches_explicit_loops, mlp64=rd.mlp64)


def test_dropped_distortion_self_term_is_caught():
    dm = _mutated("oracle.distortion", "loss = float((w * pair).sum() + (w * w * dl).sum() / 3.0)",
                  "loss = float((w * pair).sum() + (w * w * dl).sum() / 2.0)")
    _fails(pins_dist.test_closed_forms, D=dm)


def test_swapped_attention_parameters_are_caught():
    bk = _mutated("oracle.baked", "return co[:, 8 + 2 * l], co[:, 9 + 2 * l]",
                  "return co[:, 9 + 2 * l], co[:, 8 + 2 * l]")
    rd = _mutated("oracle.render", "from . import baked, pyramid, quant, sh",
                  "from . import baked, pyramid, quant, sh", baked=bk)
    _fails(pins_baked.test_separate_attention_closed_forms, 40.0, -40.0, fused64=rd.fused64, baked=bk)


def test_shared_gate_on_the_wrong_channel_is_caught():
    bk = _mutated("oracle.baked", "return co[:, 8 + l], co[:, 8 + l]", "return co[:, 8], co[:, 8]")
    rd = _mutated("oracle.render", "from . import baked, pyramid, quant, sh",
                  "from . import baked, pyramid, quant, sh", baked=bk)
    _fails(pins_baked.test_aggregation_variants_closed_forms, bk.SHARED_V, fused64=rd.fused64,
           fused32=rd.fused32, baked=bk)


def test_scene_constant_softmax_shift_is_caught():
    """Shifting every sample's logits by a fixed constant instead of the
    running maximum (the softmax is unchanged by the shift in exact
    arithmetic, but every term underflows when the sample's logits lie far
    below the constant)."""
    rd = _mutated("oracle.render", "run_max = np.full(m, -np.inf, dtype=F32)",
                  "run_max = np.full(m, F32(100.0), dtype=F32)")
    _fails(pins.test_softmax_mirror_with_extreme_logits, "outlier_entry", fused32=rd.fused32)


def test_unrescaled_running_sums_are_caught():
    """A new running maximum that does not rescale the sums taken so far."""
    rd = _mutated("oracle.render", "esum = fma32(esum, scale, e)", "esum = esum + e")
    _fails(pins.test_softmax_mirror_with_extreme_logits, "ramp", fused32=rd.fused32)


def test_double_rounding_fma32_is_caught():
    """fma32 computed as the float64 sum rounded to float32 (two roundings)."""
    ex = _mutated("oracle.exact32", "    return np.asarray(s_odd).astype(F32)\n",
                  "    return np.asarray(s).astype(F32)\n")
    import oracle.exact32 as real
    real_fma = real.fma32
    real.fma32 = ex.fma32
    try:
        _fails(pins.test_fma32_is_the_single_rounding_of_the_exact_value)
    finally:
        real.fma32 = real_fma


def test_contraction_without_normalising_is_caught():
    """The float64 sample positions contracted as (2 - 1/r) x instead of
    (2 - 1/r) x / r."""
    rd = _mutated("oracle.render", "x[outer] = ((2.0 - 1.0 / r[outer]) / r[outer])[:, None] * x[outer]",
                  "x[outer] = (2.0 - 1.0 / r[outer])[:, None] * x[outer]")
    import oracle.render as real
    real_fn = real.sample_coords64
    real.sample_coords64 = rd.sample_coords64
    try:
        _fails(pins.test_sample_coords64_closed_forms)
    finally:
        real.sample_coords64 = real_fn
