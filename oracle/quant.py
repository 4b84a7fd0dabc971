"""Quantization of real vectors to non-negative integers and its inverse.

Test infrastructure only (see the package docstring).

Sec. III-A defines Gamma_2(u) = round(Delta (u - u_min) / (u_max - u_min)),
mapping reals to {0, ..., Delta}.  This build uses one common interval
[z_min, z_max] for every vector that is aggregated (the interval Theorem 1
assumes), with the scale s = Delta / (z_max - z_min) a power of two, 2^k, and
the offset o = -z_min s an integer.  Then Gamma_2 takes the affine form

    Gamma_2(x) = rint(x * 2^k) + o,

where rint rounds half to even (the paper writes only "rounding") and x * 2^k
is exact in float64, so there is exactly one rounding.  Gamma_2 maps the
interval onto {0, ..., Delta}; with z_min = -o / 2^k and z_max = (Delta - o) / 2^k
an input outside [z_min, z_max) is an error (Theorem 1 assumes every
quantized value lies in the common interval), never clamped.  The top of the
interval is open, so that adjacent intervals of the same scale do not share
a point; rounding can still reach Delta itself from just below z_max.

Inverse quantization (Sec. III-C, inverse-quantization formula): a decrypted
integer M that is the sum of W quantized addends (W = K for a K-way
homomorphic sum, W = k for Enc(a)^k, W = 1 for a round trip) carries W copies
of the offset, so

    x = (M - W o) / 2^k,

evaluated as float64(M - W o) (round to nearest even) followed by an exact
power-of-two division.  This replaces the paper's N = 1 cross terms, which do
not generalise to N > 1.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Sequence

U64 = 1 << 64


def quantize(x: float, log2_scale: int, offset: int, delta: int) -> int:
    """Gamma_2 in affine form: rint(x 2^k) + o for x in the common interval
    [-o / 2^k, (Delta - o) / 2^k), so that the result lies in {0, ..., Delta}.

    0 <= o <= Delta < 2^64 is required of the parameters."""
    if not (0 <= offset <= delta < U64):
        raise ValueError("quantizer needs 0 <= offset <= delta < 2^64")
    if not math.isfinite(x):
        raise ValueError("non-finite input")
    t = math.ldexp(x, log2_scale)  # exact: a power-of-two scale
    # -o <= t < Delta - o, compared exactly as rationals (t is a binary fraction)
    if not (-offset <= Fraction(t) < delta - offset):
        raise ValueError("input outside the quantizer's common interval")
    v = round(t)  # Python rounds floats half to even
    return v + offset


def dequantize(M: int, log2_scale: int, offset: int, weight: int) -> float:
    """Inverse of Gamma_2 for an aggregate of ``weight`` quantized addends."""
    d = M - weight * offset
    return math.ldexp(float(d), -log2_scale)


def quantize_vec(xs: Sequence[float], log2_scale: int, offset: int, delta: int) -> list[int]:
    return [quantize(float(x), log2_scale, offset, delta) for x in xs]


def dequantize_vec(Ms: Sequence[int], log2_scale: int, offset: int,
                   weight: int) -> list[float]:
    return [dequantize(int(M), log2_scale, offset, weight) for M in Ms]
