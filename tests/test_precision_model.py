"""CPU checks of the operand-rounding model (tests/precision_model.py) and of
what it predicts for the collision path's precisions.

The model is pinned first (its unrounded mode is the FP64 oracle; its
roundings agree with torch's own float conversions), then used to state
which operand schemes can meet the accuracy target |f - f64| <= 1e-3,
normal angle <= 1e-2 rad (max over the sample) on the two 3->256x8->1 skip-5
networks of the cloth workload, and to derive the FP8 tolerances of the GPU
tests.  The GPU tests and the benchmark print the kernels' own errors; on
the cloth workload they match the model's to within a few percent.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2110_01614_amd import inputs as I

import precision_model as PM

BAR_F, BAR_A = 1e-3, 1e-2


@pytest.fixture(scope="module")
def cloth():
    """Both cloth-workload networks on 4096 of the cloth vertices (the benchmark's sample), with FP64 references."""
    spec, pn, pts, _ = I.workload_inputs("cloth1m")
    pg = I.workload_inputs("cloth1m", n=1, init="geometric")[1]
    P = pts[np.random.default_rng(3).choice(len(pts), 4096, replace=False)]
    return {name: (spec, prm, P, oracle.mlp_eval(spec, prm, P)) for name, prm in (("normal", pn), ("geometric", pg))}


def test_roundings_agree_with_torch_conversions():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 2000), rng.uniform(-400, 400, 2000)])
    x32 = x.astype(np.float32)
    t = torch.from_numpy(x32)
    assert np.array_equal(PM.round_bf16(x32), t.to(torch.bfloat16).double().numpy())
    assert np.array_equal(PM.round_fp16(x32), t.to(torch.float16).double().numpy())
    assert np.array_equal(PM.round_e4m3(x32), t.to(torch.float8_e4m3fn).double().numpy())
    assert PM.round_e4m3(np.array([1000.0, -500.0])).tolist() == [448.0, -448.0]  # saturating
    # pairs: hi + lo keeps about 16 bits
    hi, lo = PM.split(x, "bf16x2")
    assert np.all(np.abs(hi + lo - x) <= 2.0 ** -16 * np.abs(x) + 1e-300)


@pytest.mark.parametrize("name", ["normal", "geometric"])
def test_unrounded_model_is_the_oracle(cloth, name):
    spec, prm, P, (f64, g64) = cloth[name]
    f, g = PM.emulate(spec, prm, P, "exact")
    assert np.max(np.abs(f - f64)) <= 1e-12 * (1 + np.abs(f64).max())
    assert np.max(np.abs(g - g64)) <= 1e-11 * np.abs(g64).max()


def _err(cloth, name, fwd, rev=None):
    spec, prm, P, ref = cloth[name]
    return PM.scheme_errors(spec, prm, P, fwd, rev, ref=ref)


@pytest.mark.parametrize("scheme", ["bf16", "fp16", "bf16_w2", "bf16_x2", "fp16_w2", "fp16_x2"])
def test_one_or_two_products_miss_the_angle_bar_on_the_normal_init_net(cloth, scheme):
    """With N(0, 0.02) weights |grad f| ~ 2e-5 and the normal is ill-conditioned:
    any scheme that leaves one operand at 16-bit rounding misses 1e-2 rad."""
    e = _err(cloth, "normal", scheme)
    assert e["angle_max"] > BAR_A, e


def test_bf16x3_meets_the_bar_on_both_nets(cloth):
    for name in ("normal", "geometric"):
        e = _err(cloth, name, "bf16x3")
        assert e["sdf_max"] <= 1e-4 and e["angle_max"] <= 1e-3, (name, e)


def test_plain_bf16_misses_and_fp16_meets_the_bar_on_the_geometric_net(cloth):
    eb = _err(cloth, "geometric", "bf16")
    ef = _err(cloth, "geometric", "fp16")
    assert eb["sdf_max"] > BAR_F, eb
    assert ef["sdf_max"] <= BAR_F and ef["angle_max"] <= BAR_A, ef


@pytest.fixture(scope="module")
def cloth16k():
    """The same networks on 16,384 other cloth vertices: the target is a
    maximum over points, so claims that a scheme meets it are checked on a
    sample four times larger than the GPU tests use."""
    spec, pn, pts, _ = I.workload_inputs("cloth1m")
    pg = I.workload_inputs("cloth1m", n=1, init="geometric")[1]
    P = pts[np.random.default_rng(5).choice(len(pts), 16384, replace=False)]
    return {name: (spec, prm, P, oracle.mlp_eval(spec, prm, P)) for name, prm in (("normal", pn), ("geometric", pg))}


def test_cheapest_scheme_found_that_meets_the_bar(cloth16k):
    """FP16 main products plus both cross terms (W_lo x_hi + W_hi x_lo) on E4M3
    operands with a power-of-two scale per 32 elements of K, in both sweeps,
    with the activations kept for the reverse sweep as FP16 pairs: two 16-bit
    products per product (the FP8 pass has twice the K at twice the rate)."""
    for name in ("normal", "geometric"):
        e = _err(cloth16k, name, "fp16_c8p", "fp16_c8p")
        assert e["sdf_max"] <= BAR_F and e["angle_max"] <= 0.5 * BAR_A, (name, e)
    assert PM.SCHEMES["fp16_c8p"].cost == 2.0


def test_a_single_16_bit_stack_misses_the_angle_bar(cloth16k):
    """The sigmoids of the reverse sweep need more than 16 bits of the stored
    activation on the N(0, 0.02) network: with one FP16 copy of r - 1 kept,
    even BF16x3 contractions, or FP16 forward with FP8 cross terms in the
    reverse sweep, miss 1e-2 rad (on 4096 vertices the latter happens to
    pass)."""
    for fwd, rev in (("bf16x3_s16", "bf16x3_s16"), ("fp16m1", "fp16_c8")):
        e = _err(cloth16k, "normal", fwd, rev)
        assert e["angle_max"] > BAR_A, (fwd, rev, e)


@pytest.mark.parametrize("width", [256, 512])
def test_fp8_error_bound_of_the_gpu_tests(width):
    """The FP8 tolerances asserted by the GPU tests (|df| <= 0.15, angle p99
    <= 0.15, max <= 0.6 rad) cover the modelled E4M3 errors on geometric-init
    nets with a margin of at least 1.4."""
    spec = I.NetSpec((width,) * 8, 5)
    prm = I.init_geometric(spec, 0)
    P = I.uniform_points(2048, 1)
    ref = oracle.mlp_eval(spec, prm, P)
    e = PM.scheme_errors(spec, prm, P, "fp8", "fp8r", ref=ref)
    print("fp8 width %d: %s" % (width, e))
    assert e["sdf_max"] <= 0.15 / 1.4 and e["angle_p99"] <= 0.15 / 1.4 and e["angle_max"] <= 0.6 / 1.4, e
