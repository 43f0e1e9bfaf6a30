"""The sketch Y = Omega A (Section 5.1, eq. (Y=OmegaA)) with its inputs rounded to
16-bit floating point, as a mixed-precision sketch computes it: both factors
are rounded to BF16 or FP16 (round to nearest, ties to even) and the product of
the rounded values is the result, here formed in FP64 (the exact product up to
FP64 rounding; a matrix core that accumulates in FP32 differs from it by at
most K u32 |Omega_r| |A_r| elementwise).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Readings (the paper predates 16-bit matrix cores and is silent on them):

* BF16 keeps the FP32 exponent; an FP32 value is rounded to the nearest value
  with 8 significant bits (ties to the even significand).
* FP16 has 5 exponent bits: FP32 entries of the paper's test matrices sit near
  the FP16 minimum normal 2^-14, so A is first multiplied by 2^(15-e), where
  max|A| lies in [2^(e-1), 2^e), and the product is divided by the same power of
  two. J and T do not change when A is scaled (the pivoted QR and S11^{-1} S12
  are invariant to a positive scalar), so the scaling costs nothing in
  exactness. Omega and orthonormal bases are rounded unscaled.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values (given in any float dtype; they are first taken to FP32)
    to the nearest BF16 value, ties to even. Returns FP64 holding BF16 values.

    On the FP32 bit pattern: adding 0x7FFF plus the lowest kept bit and clearing
    the low 16 bits rounds to nearest with ties to even (a carry out of the
    significand steps the exponent, overflow reaches infinity)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    keep = (bits >> np.uint64(16)) & np.uint64(1)
    r = ((bits + np.uint64(0x7FFF) + keep) & np.uint64(0xFFFF0000)).astype(np.uint32)
    # NaN stays NaN (the rounding above could carry a NaN payload into infinity)
    r = np.where(np.isnan(f), np.uint32(0x7FC00000), r)
    return r.view(np.float32).astype(np.float64)


def round_fp16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest IEEE binary16 value (ties to even,
    gradual underflow, overflow to infinity). Returns FP64 holding FP16 values."""
    with np.errstate(over="ignore"):
        return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def fp16_scale(A: np.ndarray) -> float:
    """The power of two s = 2^(15-e) with max|A| in [2^(e-1), 2^e), so that
    max|s A| lies in [2^14, 2^15); 1 for a zero or non-finite maximum. The
    exponent 15 - e is clamped to the normal FP32 exponents [-126, 127]."""
    a = float(np.max(np.abs(np.asarray(A, dtype=np.float32)))) if np.size(A) else 0.0
    if not (a > 0.0) or not np.isfinite(a):
        return 1.0
    _, e = np.frexp(a)   # a = f 2^e, f in [0.5, 1)
    return float(np.ldexp(1.0, int(min(max(15 - int(e), -126), 127))))


def round16(x: np.ndarray, prec: str) -> np.ndarray:
    if prec == "bf16":
        return round_bf16(x)
    if prec == "fp16":
        return round_fp16(x)
    raise ValueError(prec)


def sketch_rounded(A: np.ndarray, omega: np.ndarray, prec: str) -> np.ndarray:
    """Y = round(Omega) round(s A) / s in FP64 (s = fp16_scale(A) for FP16, 1 for
    BF16): the sketch of Section 5.1 with 16-bit matrix-core inputs."""
    A32 = np.asarray(A, dtype=np.float32)
    s = fp16_scale(A32) if prec == "fp16" else 1.0
    Ar = round16(A32 * np.float32(s), prec)
    Or = round16(np.asarray(omega, dtype=np.float32), prec)
    return (Or @ Ar) / s
