"""Pins of the oracle's 16-bit rounding and rounded-input sketch (oracle/lowprec.py).

* BF16 rounding: hand-worked ties and carries, and agreement with torch's own
  float32 -> bfloat16 conversion (an independent implementation) on a million
  values spanning normal, subnormal and huge magnitudes.
* FP16 rounding: hand-worked ties, gradual underflow and overflow (IEEE 754
  binary16), and the defining property |x - r(x)| <= half an ulp of r(x).
* FP16 scale: the largest scaled entry lands in [2^14, 2^15).
* Rounded sketch: exact on inputs that are already 16-bit values, scaling undone
  exactly, and within the unit-roundoff bound of the unrounded product.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import lowprec

torch = pytest.importorskip("torch")


def test_bf16_hand_worked_values():
    one = 1.0
    cases = [
        (one, one),
        (one + 2.0**-8, one),                       # halfway, even significand below
        (one + 3 * 2.0**-8, one + 2.0**-6),         # halfway, even significand above
        (one + 2.0**-8 + 2.0**-20, one + 2.0**-7),  # just above halfway
        (one + 2.0**-7, one + 2.0**-7),             # representable
        (-(one + 3 * 2.0**-8), -(one + 2.0**-6)),   # sign symmetric
        (2.0 - 2.0**-9, 2.0),                       # carry into the exponent
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert lowprec.round_bf16(np.array([x]))[0] == want, x
    # the largest FP32 value rounds past the largest BF16 value to infinity
    assert np.isinf(lowprec.round_bf16(np.array([np.finfo(np.float32).max]))[0])


def test_bf16_matches_torch_conversion():
    g = synth.rng(1)
    x = np.concatenate([
        g.standard_normal(400_000),
        g.standard_normal(200_000) * 1e-40,          # FP32 subnormals
        g.standard_normal(200_000) * 1e30,
        (g.random(200_000) - 0.5) * 2.0**-10,
    ]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = lowprec.round_bf16(x)
    assert np.array_equal(got, want)


def test_fp16_hand_worked_values():
    cases = [
        (2049.0, 2048.0),               # tie, even significand below
        (2051.0, 2052.0),               # tie, even significand above
        (2.0**-24, 2.0**-24),           # smallest subnormal
        (2.0**-25, 0.0),                # half of it: tie to even (zero)
        (3 * 2.0**-26, 2.0**-24),       # above the tie
        (65504.0, 65504.0),             # largest finite
        (65519.0, 65504.0),             # below the overflow threshold
    ]
    for x, want in cases:
        assert lowprec.round_fp16(np.array([x]))[0] == want, x
    assert np.isinf(lowprec.round_fp16(np.array([65520.0]))[0])


def test_fp16_half_ulp_property():
    g = synth.rng(2)
    x = (g.standard_normal(100_000) * 100.0).astype(np.float32).astype(np.float64)
    r = lowprec.round_fp16(x)
    # ulp of a normal binary16 value r: 2^(exponent(r) - 10)
    e = np.floor(np.log2(np.abs(r)))
    ulp = 2.0 ** (np.maximum(e, -14) - 10)
    assert np.all(np.abs(x - r) <= ulp / 2)


@pytest.mark.parametrize("amax", [1.0, 0.75, 2.0**-20, 3.0e4, 7.4e-5, 65504.0 * 4])
def test_fp16_scale_lands_in_range(amax):
    A = np.array([[amax, -amax / 3], [0.0, amax / 7]])
    s = lowprec.fp16_scale(A)
    assert np.log2(s) == np.round(np.log2(s))           # a power of two
    assert 2.0**14 <= amax * s < 2.0**15


def test_fp16_scale_degenerate():
    assert lowprec.fp16_scale(np.zeros((3, 4))) == 1.0
    assert lowprec.fp16_scale(np.array([[np.inf, 1.0]])) == 1.0


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_sketch_exact_on_representable_inputs(prec):
    # small integers are exact in both formats, and the products and sums stay
    # exact in FP64: the rounded sketch is the exact product
    g = synth.rng(3)
    A = g.integers(-8, 9, size=(40, 30)).astype(np.float64)
    Om = g.integers(-4, 5, size=(6, 40)).astype(np.float64)
    assert np.array_equal(lowprec.sketch_rounded(A, Om, prec), Om @ A)


@pytest.mark.parametrize("prec,u", [("bf16", 2.0**-8), ("fp16", 2.0**-11)])
def test_sketch_within_rounding_bound(prec, u):
    # each input carries a relative error <= u, so each product term <= 2u + u^2:
    # |Y_r - Omega A| <= (2u + u^2) |Omega| |A| elementwise
    g = synth.rng(4)
    A = synth.lowrank(300, 200, synth.sigma_pow(200, 2.0), seed=5).astype(np.float32).astype(np.float64)
    Om = g.standard_normal((20, 300)).astype(np.float32).astype(np.float64)
    Y = lowprec.sketch_rounded(A, Om, prec)
    bound = (2 * u + u * u) * (np.abs(Om) @ np.abs(A))
    assert np.all(np.abs(Y - Om @ A) <= bound * (1 + 1e-12))
    # and the rounding is not a no-op
    assert np.abs(Y - Om @ A).max() > 0


def test_fp16_scaling_is_undone_exactly():
    # a power-of-two rescaling of A gives exactly the rescaled sketch: the scale
    # factor follows A, so the rounded significands are the same
    g = synth.rng(6)
    A = g.standard_normal((50, 40)).astype(np.float32).astype(np.float64)
    Om = g.standard_normal((8, 50)).astype(np.float32).astype(np.float64)
    Y1 = lowprec.sketch_rounded(A, Om, "fp16")
    Y2 = lowprec.sketch_rounded(A * 2.0**-20, Om, "fp16")
    assert np.array_equal(Y1 * 2.0**-20, Y2)
    # without the scale, entries of this size would land in the FP16 subnormals
    # and lose digits: the scaled sketch is far closer to the exact product
    tiny = A * 2.0**-20
    exact = Om @ tiny
    unscaled = lowprec.round_fp16(Om) @ lowprec.round_fp16(tiny)
    assert np.linalg.norm(Y2 - exact) < 0.1 * np.linalg.norm(unscaled - exact)
