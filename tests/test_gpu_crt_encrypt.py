"""Key-holder encryption through p^2 and q^2 (GPU tests): pc2_encrypt_sk must
give the public-key ciphertext bit for bit, i.e. the oracle's Enc(m, r)."""
from __future__ import annotations

import math
import random

import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import dev, host_ints
from workload import gen
from workload.limbs import to_limbs

pytestmark = pytest.mark.gpu


def _enc_sk(ctx, sk, ms, rs, m_limbs=None):
    from paper_2601_14980_amd import pc2
    L = sk.L
    m = dev(to_limbs(ms, m_limbs or L))
    r = dev(to_limbs(rs, L))
    c = torch.zeros((len(ms), 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_encrypt_sk(sk, m, r, c)
    return host_ints(c), ctx.sync()


@pytest.mark.parametrize("p,q", [(5, 7), (11, 13)])
def test_crt_bruteforce_tiny(gpu_ctx, p, q):
    from paper_2601_14980_amd import pc2
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, n.bit_length(), p, q)
    opk, _ = O.derive_keys(p, q)
    pairs = [(m, r) for m in range(n) for r in range(1, n) if math.gcd(r, n) == 1]
    cs, st = _enc_sk(gpu_ctx, sk, [m for m, _ in pairs], [r for _, r in pairs])
    assert st == 0
    assert cs == [O.encrypt(opk, m, r) for m, r in pairs]


@pytest.mark.parametrize("nbits", [64, 256, 1024, 2048, 3072, 4096])
def test_crt_matches_public_encryption(gpu_ctx, nbits):
    from paper_2601_14980_amd import pc2
    from tests.gpu_helpers import gpu_encrypt
    p, q = gen.primes_for(1, nbits, extra=11)
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, nbits, p, q)
    opk, _ = O.derive_keys(p, q)
    count = 64 if nbits > 3072 else (200 if nbits >= 2048 else 333)
    rng = random.Random(nbits + 1)
    ms = [0, 1, n - 1] + [rng.randrange(n) for _ in range(count - 3)]
    rs = [1, n - 1, 2] + gen.gen_r(n, count - 3, 1, extra=nbits + 1)
    cs, st = _enc_sk(gpu_ctx, sk, ms, rs)
    assert st == 0
    cv, st = gpu_encrypt(gpu_ctx, sk.public, ms, rs)
    assert st == 0
    assert cs == cv
    for j in ((0, 1, 2, count // 3, count - 1) if nbits <= 3072 else (1, count - 1)):
        assert cs[j] == O.encrypt(opk, ms[j], rs[j])


def test_crt_range_errors(gpu_ctx):
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(1, 256, extra=12)
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, 256, p, q)
    opk, _ = O.derive_keys(p, q)
    cs, st = _enc_sk(gpu_ctx, sk, [9, n, 4, 4], [5, 5, 0, n])
    assert st != 0
    assert cs[0] == O.encrypt(opk, 9, 5) and cs[1:] == [0, 0, 0]
    assert gpu_ctx.sync() == 0


def test_crt_rejects_unbalanced_primes(gpu_ctx):
    from paper_2601_14980_amd import pc2
    p, q = 1000003, 101      # p > 2 q
    sk = pc2.SecretKey(gpu_ctx, (p * q).bit_length(), p, q)
    m = torch.zeros((1, sk.L), dtype=torch.int32, device="cuda")
    r = dev(to_limbs([3], sk.L))
    c = torch.zeros((1, 2 * sk.L), dtype=torch.int32, device="cuda")
    with pytest.raises(pc2.PC2Error):
        pc2.pc2_encrypt_sk(sk, m, r, c)
