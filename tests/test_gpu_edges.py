"""Adversarial limb patterns in every tile the benchmark times (GPU tests).

Longest carry chains and boundary values -- r = 1 and r = n - 1, m = 0 and
m = n - 1, ciphertexts 1 and n^2 - 1, all-ones limbs below the modulus,
values at 2^(32 i) - 1 and 2^(32 i) -- fed to encryption in each limb tile of
the key's class (PC2_OPT_TILE forced, the own tiles included; the VALU
engine, and the matrix-core engine once per key size), and to
decryption, K-way aggregation and scalar powers, in the one-call path and in
a persistent batch.  Counts span two wavefront groups and a ragged tail;
every output is compared with the oracle element by element.
"""
from __future__ import annotations

import functools
import math
import random

import numpy as np
import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import dev, gpu_decrypt, gpu_encrypt, gpu_hom_sum, gpu_scalar_mul, host_ints
from workload import gen
from workload.limbs import to_limbs

pytestmark = pytest.mark.gpu

# (bits, lanes per ciphertext of each encryption tile: own first)
TILES = {1024: (2, 4), 2048: (4, 8), 3072: (8,), 4096: (8,)}
SEED = 31


@functools.lru_cache(maxsize=None)
def _oracle_key(nbits):
    p, q = gen.primes_for(SEED, nbits)
    return p, q, O.derive_keys(p, q)


@functools.lru_cache(maxsize=None)
def _enc_cases(nbits):
    """Distinct (m, r) pairs and their oracle ciphertexts."""
    p, q, (opk, _) = _oracle_key(nbits)
    n = p * q
    L = (nbits + 31) // 32
    ones = (1 << (32 * (L - 1))) - 1          # all-ones limbs below n
    rnd = random.Random(nbits)
    rs = gen.gen_r(n, 3, SEED, extra=nbits)
    pairs = [(0, 1), (0, n - 1), (n - 1, 1), (n - 1, n - 1), (ones, ones),
             ((1 << 32) - 1, (1 << 64) - 1), (1 << 32, 1 << (32 * (L - 1))),
             (1, rs[0]), (rnd.randrange(n), rs[1]), (rnd.randrange(n), rs[2])]
    pairs = [(m, r) for m, r in pairs if math.gcd(r, n) == 1]
    return tuple(pairs), tuple(O.encrypt(opk, m, r) for m, r in pairs)


@functools.lru_cache(maxsize=None)
def _cipher_cases(nbits):
    """Units below n^2 with long carry chains, and their oracle plaintexts."""
    p, q, (opk, osk) = _oracle_key(nbits)
    n = p * q
    n2 = n * n
    L = (nbits + 31) // 32
    cands = [1, n2 - 1, n2 - 2, (1 << (32 * (2 * L - 1))) - 1, (1 << (32 * L)) - 1,
             1 << (32 * L), (1 << 32) - 1, n2 - (1 << (32 * L)) + 1,
             _enc_cases(nbits)[1][-1]]
    cs = tuple(c for c in cands if 0 < c < n2 and math.gcd(c, n) == 1)
    return cs, tuple(O.decrypt(osk, c) for c in cs)


def _spread(values, count):
    """values repeated over count positions (every lane of every group sees several)."""
    return [values[i % len(values)] for i in range(count)]


@pytest.fixture(scope="module")
def keys(gpu_ctx):
    from paper_2601_14980_amd import pc2
    out = {}
    for nbits in TILES:
        p, q, (opk, osk) = _oracle_key(nbits)
        out[nbits] = (pc2.SecretKey(gpu_ctx, nbits, p, q), opk, osk)
    yield out
    for sk, _, _ in out.values():
        sk.close()


@pytest.mark.parametrize("nbits,lanes", [(b, t) for b, ts in TILES.items() for t in ts])
def test_encrypt_edges_in_each_tile(gpu_ctx, keys, nbits, lanes):
    from paper_2601_14980_amd import pc2
    sk, opk, _ = keys[nbits]
    pairs, want = _enc_cases(nbits)
    count = 2 * (64 // lanes) + 3
    idx = _spread(list(range(len(pairs))), count)
    gpu_ctx.set_option(pc2.PC2_OPT_TILE, lanes)
    # the VALU engine in this tile; once per key size also the matrix-core engine
    engines = [pc2.PC2_MODMUL_VALU] + ([pc2.PC2_MODMUL_MFMA] if lanes == TILES[nbits][0] else [])
    try:
        for eng in engines:
            gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, eng)
            got, st = gpu_encrypt(gpu_ctx, sk.public, [pairs[i][0] for i in idx],
                                  [pairs[i][1] for i in idx])
            assert st == 0
            for j, i in enumerate(idx):
                assert got[j] == want[i], \
                    f"{nbits}-bit, {lanes} lanes, engine {eng}, element {j}, (m, r) #{i}"
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)
        # the same inputs as one job of a persistent batch in this tile
        L = sk.L
        m = dev(to_limbs([pairs[i][0] for i in idx], L))
        r = dev(to_limbs([pairs[i][1] for i in idx], L))
        c = torch.zeros((count, 2 * L), dtype=torch.int32, device="cuda")
        b = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m, r=r, out=c)])
        b.run(0)
        assert gpu_ctx.sync() == 0
        assert host_ints(c) == [want[i] for i in idx]
        b.close()
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_TILE, 0)
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)


@pytest.mark.parametrize("nbits", list(TILES))
def test_decrypt_edges(gpu_ctx, keys, nbits):
    from paper_2601_14980_amd import pc2
    sk, _, _ = keys[nbits]
    cs, want = _cipher_cases(nbits)
    count = 2 * (64 // 2) + 3                 # two groups of the s^2 tile of most classes
    idx = _spread(list(range(len(cs))), count)
    got, st = gpu_decrypt(gpu_ctx, sk, [cs[i] for i in idx])
    assert st == 0
    assert got == [want[i] for i in idx]
    # a persistent batch decryption of the same ciphertexts (two launches)
    L = sk.L
    c = dev(to_limbs([cs[i] for i in idx], 2 * L))
    m = torch.zeros((count, L), dtype=torch.int32, device="cuda")
    b = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_DECRYPT, sk=sk, c=c, out=m)])
    b.run(0)
    assert gpu_ctx.sync() == 0
    assert host_ints(m) == [want[i] for i in idx]
    b.close()


@pytest.mark.parametrize("nbits", list(TILES))
def test_hom_sum_and_scalar_edges(gpu_ctx, keys, nbits):
    sk, opk, _ = keys[nbits]
    cs, _ = _cipher_cases(nbits)
    count = 2 * 16 + 3
    E = len(cs)
    K = 3
    cvs = [[cs[(j + k) % E] for j in range(count)] for k in range(K)]
    got, st = gpu_hom_sum(gpu_ctx, sk.public, cvs)
    assert st == 0
    assert got == [O.hom_sum(opk, [cv[j] for cv in cvs]) for j in range(count)]
    ks = [0, 1, 2, (1 << 32) - 1, 1 << 32, 1 << 63, (1 << 64) - 1,
          random.Random(nbits).getrandbits(64)]
    c1 = _spread(list(cs), count)
    k1 = [ks[(j // E + j) % len(ks)] for j in range(count)]
    got, st = gpu_scalar_mul(gpu_ctx, sk.public, c1, k1)
    assert st == 0
    assert got == [O.hom_scalar_mul(opk, c, k) for c, k in zip(c1, k1)]
