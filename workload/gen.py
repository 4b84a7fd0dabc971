"""Seeded generators: primes, randomness r in Z*_n, data vectors, lengths, arrivals.

Seeds: ``numpy.random.SeedSequence(ROOT_SEED, spawn_key=(config, purpose))``
gives one independent stream per (configuration, purpose).  Prime search uses
``random.Random`` seeded from that stream so that keys are reproducible.
"""
from __future__ import annotations

import functools
import math
import random
from dataclasses import dataclass

import numpy as np
import sympy

from .limbs import to_limbs

ROOT_SEED = 260114980

# purposes
KEYS, DATA, RAND, LENGTHS, ARRIVALS, TYPES = range(6)

# Distinct odd prime pairs small enough to enumerate every (m, r) pair.
TINY_PRIME_PAIRS = [(3, 5), (5, 7), (7, 11), (11, 13), (251, 241), (65521, 65519)]


def seed_seq(config: int, purpose: int, extra: int = 0) -> np.random.SeedSequence:
    return np.random.SeedSequence(ROOT_SEED, spawn_key=(config, purpose, extra))


def rng_np(config: int, purpose: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng(seed_seq(config, purpose, extra))


def _prime_from(rng: random.Random, half: int) -> int:
    cand = rng.getrandbits(half) | (3 << (half - 2)) | 1
    while not sympy.isprime(cand):
        cand += 2
    return cand


def gen_primes(nbits: int, seed: int) -> tuple[int, int]:
    """Two distinct primes of nbits/2 bits each, top two bits set, so that
    n = p q has exactly nbits bits and gcd(n, (p-1)(q-1)) = 1."""
    if nbits % 2 or nbits < 16:
        raise ValueError("nbits must be even and >= 16")
    rng = random.Random(seed)
    half = nbits // 2
    p = _prime_from(rng, half)
    q = _prime_from(rng, half)
    while q == p:
        q = _prime_from(rng, half)
    n = p * q
    assert n.bit_length() == nbits
    assert math.gcd(n, (p - 1) * (q - 1)) == 1
    return p, q


@functools.lru_cache(maxsize=None)
def primes_for(config: int, nbits: int, extra: int = 0) -> tuple[int, int]:
    seed = int(seed_seq(config, KEYS, extra).generate_state(1)[0])
    return gen_primes(nbits, seed)


def gen_r(n: int, count: int, config: int, extra: int = 0) -> list[int]:
    """``count`` draws uniform on Z*_n by rejection (0 < r < n, gcd(r, n) = 1)."""
    rng = random.Random(int(seed_seq(config, RAND, extra).generate_state(1)[0]))
    out = []
    while len(out) < count:
        r = rng.randrange(1, n)
        if math.gcd(r, n) == 1:
            out.append(r)
    return out


def gen_r_limbs(n: int, count: int, nlimbs: int, config: int, extra: int = 0) -> np.ndarray:
    """As ``gen_r`` but drawn as uniform limb rows (fast for large n); rows
    with r = 0, r >= n or gcd(r, n) != 1 are redrawn."""
    if n.bit_length() <= 64:
        return to_limbs(gen_r(n, count, config, extra), nlimbs)
    rng = rng_np(config, RAND, extra)
    top_bits = n.bit_length() - 32 * (nlimbs - 1)
    out = np.empty((count, nlimbs), dtype=np.uint32)
    filled = 0
    while filled < count:
        need = count - filled
        blk = rng.integers(0, 1 << 32, size=(need, nlimbs), dtype=np.uint64).astype(np.uint32)
        blk[:, -1] &= np.uint32((1 << top_bits) - 1)
        raw = blk.astype("<u4").tobytes()
        nb = 4 * nlimbs
        keep = []
        for i in range(need):
            r = int.from_bytes(raw[i * nb:(i + 1) * nb], "little")
            if 0 < r < n and math.gcd(r, n) == 1:
                keep.append(i)
        out[filled:filled + len(keep)] = blk[keep]
        filled += len(keep)
    return out


@dataclass(frozen=True)
class QParams:
    """Affine quantizer m = rint(x 2^log2_scale) + offset on the common
    interval [-offset, delta - offset) / 2^log2_scale, onto {0, ..., delta}."""
    log2_scale: int
    offset: int
    delta: int


# Quantizer settings per workload (common interval, power-of-two scale).
Q_TINY = QParams(16, 1 << 19, 1 << 20)      # [-8, 8) -> {0, ..., 2^20}
Q_PLAIN = QParams(20, 1 << 23, 1 << 24)     # [-8, 8) -> {0, ..., 2^24}
Q_ADMM = QParams(44, 1 << 51, 1 << 52)      # [-128, 128) -> {0, ..., 2^52}


def uniform_vectors(config: int, k: int, length: int, lo: float = -1.0, hi: float = 1.0):
    rng = rng_np(config, DATA)
    return [rng.uniform(lo, hi, size=length) for _ in range(k)]


def normal_vectors(config: int, lengths, extra: int = 0):
    rng = rng_np(config, DATA, extra)
    return [rng.standard_normal(size=int(L)) for L in lengths]


def log_uniform_lengths(config: int, count: int, lo: int, hi: int, extra: int = 0) -> list[int]:
    rng = rng_np(config, LENGTHS, extra)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(round(math.exp(v))) for v in u]
