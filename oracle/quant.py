"""Quantization of real vectors to non-negative integers and its inverse.

Test infrastructure only (see the package docstring).

Sec. III-A defines Gamma_2(u) = round(Delta (u - u_min) / (u_max - u_min)),
mapping reals to {0, ..., Delta}.  This build uses one common interval
[z_min, z_max] for every vector that is aggregated (the interval Theorem 1
assumes), with the scale s = Delta / (z_max - z_min) a power of two, 2^k, and
the offset o = -z_min s an integer.  Then Gamma_2 takes the affine form

    Gamma_2(x) = rint(x * 2^k) + o,

where rint rounds half to even (the paper writes only "rounding") and x * 2^k
is exact in float64, so there is exactly one rounding.

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
from typing import Sequence

U64 = 1 << 64


def quantize(x: float, log2_scale: int, offset: int) -> int:
    """Gamma_2 in affine form: rint(x 2^k) + o, required to lie in [0, 2^64)."""
    if not math.isfinite(x):
        raise ValueError("non-finite input")
    v = round(math.ldexp(x, log2_scale))  # Python rounds floats half to even
    m = v + offset
    if not (0 <= m < U64):
        raise ValueError("quantized value outside [0, 2^64)")
    return m


def dequantize(M: int, log2_scale: int, offset: int, weight: int) -> float:
    """Inverse of Gamma_2 for an aggregate of ``weight`` quantized addends."""
    d = M - weight * offset
    return math.ldexp(float(d), -log2_scale)


def quantize_vec(xs: Sequence[float], log2_scale: int, offset: int) -> list[int]:
    return [quantize(float(x), log2_scale, offset) for x in xs]


def dequantize_vec(Ms: Sequence[int], log2_scale: int, offset: int,
                   weight: int) -> list[float]:
    return [dequantize(int(M), log2_scale, offset, weight) for M in Ms]
