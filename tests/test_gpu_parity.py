"""Bit-exact parity of the HIP path with the oracle (GPU tests).

Every ciphertext and plaintext the kernels produce is compared with the
oracle's plain-definition result for the same seeded (m, r, key).
"""
from __future__ import annotations

import math
import random

import numpy as np
import pytest
import torch

from oracle import paillier as O
from oracle import quant as Q
from tests.gpu_helpers import (dev, gpu_decrypt, gpu_enc_sum_dec, gpu_encrypt, gpu_hom_add,
                               gpu_hom_sum, gpu_scalar_mul, host_ints)
from workload import gen

pytestmark = pytest.mark.gpu

TINY = [(3, 5), (5, 7), (7, 11), (11, 13)]


def keys(ctx, p, q, nbits=None):
    from paper_2601_14980_amd import pc2
    n = p * q
    nbits = nbits or n.bit_length()
    sk = pc2.SecretKey(ctx, nbits, p, q)
    opk, osk = O.derive_keys(p, q)
    return sk, opk, osk


@pytest.mark.parametrize("p,q", TINY)
def test_bruteforce_tiny_keys(gpu_ctx, p, q):
    """Every (m, r) in Z_n x Z*_n: encryption matches the oracle and
    decryption inverts it (also covers injectivity of the GPU map)."""
    sk, opk, osk = keys(gpu_ctx, p, q)
    n = p * q
    pairs = [(m, r) for m in range(n) for r in range(1, n) if math.gcd(r, n) == 1]
    ms = [m for m, _ in pairs]
    rs = [r for _, r in pairs]
    cs, st = gpu_encrypt(gpu_ctx, sk.public, ms, rs)
    assert st == 0
    assert cs == [O.encrypt(opk, m, r) for m, r in pairs]
    assert len(set(cs)) == len(cs)
    dec, st = gpu_decrypt(gpu_ctx, sk, cs)
    assert st == 0
    assert dec == ms


@pytest.mark.parametrize("p,q", [(5, 7), (11, 13)])
def test_bruteforce_hom_ops_tiny(gpu_ctx, p, q):
    sk, opk, osk = keys(gpu_ctx, p, q)
    n = p * q
    rng = random.Random(p * 1000 + q)
    units = [r for r in range(1, n) if math.gcd(r, n) == 1]
    a = [i for i in range(n) for _ in range(n)]
    b = [j for _ in range(n) for j in range(n)]
    ra = [rng.choice(units) for _ in a]
    rb = [rng.choice(units) for _ in b]
    ca = [O.encrypt(opk, x, r) for x, r in zip(a, ra)]
    cb = [O.encrypt(opk, x, r) for x, r in zip(b, rb)]
    s, st = gpu_hom_add(gpu_ctx, sk.public, ca, cb)
    assert st == 0
    assert s == [O.hom_add(opk, x, y) for x, y in zip(ca, cb)]
    dec, _ = gpu_decrypt(gpu_ctx, sk, s)
    assert dec == [(x + y) % n for x, y in zip(a, b)]
    # multiply by every constant k < n
    ks = b
    sm, st = gpu_scalar_mul(gpu_ctx, sk.public, ca, ks)
    assert st == 0
    assert sm == [O.hom_scalar_mul(opk, c, k) for c, k in zip(ca, ks)]


SIZES = [64, 128, 256, 512, 1024, 2048, 3072, 4096]
COUNTS = {64: 200, 128: 150, 256: 130, 512: 100, 1024: 70, 2048: 21, 3072: 11, 4096: 4}


@pytest.fixture(scope="module", params=SIZES)
def sized(request, gpu_ctx):
    nbits = request.param
    p, q = gen.primes_for(99, nbits)
    sk, opk, osk = keys(gpu_ctx, p, q, nbits)
    count = COUNTS[nbits]
    rng = random.Random(nbits)
    n = p * q
    ms = [rng.randrange(0, n) for _ in range(count)]
    ms[0], ms[1], ms[2] = 0, n - 1, 1
    rs = gen.gen_r(n, count, 99, extra=nbits)
    rs[0], rs[1] = 1, n - 1
    return dict(nbits=nbits, sk=sk, opk=opk, osk=osk, ms=ms, rs=rs, n=n)


def test_encrypt_decrypt_sizes(gpu_ctx, sized):
    d = sized
    cs, st = gpu_encrypt(gpu_ctx, d["sk"].public, d["ms"], d["rs"])
    assert st == 0
    want = [O.encrypt(d["opk"], m, r) for m, r in zip(d["ms"], d["rs"])]
    assert cs == want
    dec, st = gpu_decrypt(gpu_ctx, d["sk"], cs)
    assert st == 0
    assert dec == d["ms"]
    # decryption against the oracle's plain definition on a few ciphertexts
    # that are not fresh encryptions
    n2 = d["n"] ** 2
    extra = [(c * c) % n2 for c in cs[:5]]
    dec2, st = gpu_decrypt(gpu_ctx, d["sk"], extra)
    assert dec2 == [O.decrypt(d["osk"], c) for c in extra]


def test_small_plaintext_limbs(gpu_ctx, sized):
    """Quantized plaintexts are passed with two limbs (m_limbs = 2)."""
    d = sized
    if d["sk"].L < 2:
        pytest.skip("key narrower than two limbs")
    ms = [m % (1 << 64) for m in d["ms"]]
    ms = [m if m < d["n"] else m % d["n"] for m in ms]
    cs, st = gpu_encrypt(gpu_ctx, d["sk"].public, ms, d["rs"], m_limbs=2)
    assert st == 0
    assert cs == [O.encrypt(d["opk"], m, r) for m, r in zip(ms, d["rs"])]


def test_hom_sum_and_scalar(gpu_ctx, sized):
    d = sized
    opk = d["opk"]
    count = len(d["ms"])
    K = 3
    cvs = []
    for k in range(K):
        rs = gen.gen_r(d["n"], count, 98, extra=d["nbits"] * 10 + k)
        cvs.append([O.encrypt(opk, m, r) for m, r in zip(d["ms"], rs)])
    s, st = gpu_hom_sum(gpu_ctx, d["sk"].public, cvs)
    assert st == 0
    assert s == O.hom_sum_vec(opk, cvs)
    rng = random.Random(d["nbits"] + 7)
    ks = [rng.getrandbits(64) for _ in range(count)]
    ks[0], ks[1], ks[2] = 0, 1, (1 << 64) - 1
    sm, st = gpu_scalar_mul(gpu_ctx, d["sk"].public, cvs[0], ks)
    assert st == 0
    assert sm == [O.hom_scalar_mul(opk, c, k) for c, k in zip(cvs[0], ks)]


def test_fused_enc_sum_dec(gpu_ctx, sized):
    d = sized
    count = len(d["ms"])
    K = 3
    rng = random.Random(d["nbits"] + 11)
    mvs = [[rng.randrange(0, d["n"]) for _ in range(count)] for _ in range(K)]
    rvs = [gen.gen_r(d["n"], count, 97, extra=d["nbits"] * 10 + k) for k in range(K)]
    out, st = gpu_enc_sum_dec(gpu_ctx, d["sk"], mvs, rvs)
    assert st == 0
    want = [O.enc_sum_dec(d["osk"], [mv[j] for mv in mvs], [rv[j] for rv in rvs])
            for j in range(count)]
    assert out == want


@pytest.mark.parametrize("engine", ["valu", "mfma"])
@pytest.mark.parametrize("nbits,K", [(1024, 1), (1024, 2), (1024, 9), (256, 128), (2048, 3)])
def test_fused_number_of_addends(gpu_ctx, nbits, K, engine):
    """The fused path runs one encrypt-and-accumulate step per addend, with
    either Montgomery engine: one addend (the first step is also the last),
    a few, and the most a call takes; a bad input in any step zeroes that
    element and latches the error, the others stay exact."""
    from paper_2601_14980_amd import pc2
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL,
                       pc2.PC2_MODMUL_MFMA if engine == "mfma" else pc2.PC2_MODMUL_VALU)
    try:
        _fused_addends(gpu_ctx, nbits, K)
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)


def _fused_addends(gpu_ctx, nbits, K):
    p, q = gen.primes_for(98, nbits)
    sk, _, osk = keys(gpu_ctx, p, q, nbits)
    n = p * q
    count = 3 * 32 + 7 if nbits > 256 else 37     # several element groups and a tail
    rng = random.Random(nbits * 1000 + K)
    mvs = [[rng.randrange(0, n) for _ in range(count)] for _ in range(K)]
    rvs = [gen.gen_r(n, count, 98, extra=K * 100 + k) for k in range(K)]
    bad = count // 2
    rvs[K - 1][bad] = 0                      # a data error in the last step
    if K > 1:
        mvs[0][bad + 1] = n                  # ... and one in the first
    out, st = gpu_enc_sum_dec(gpu_ctx, sk, mvs, rvs)
    assert st == pc2_range_error()
    for j in range(count):
        if j == bad or (K > 1 and j == bad + 1):
            assert out[j] == 0, f"element {j} with a bad input"
        else:
            assert out[j] == sum(mv[j] for mv in mvs) % n, f"element {j}"
    for j in (0, count - 1):
        assert out[j] == O.enc_sum_dec(osk, [mv[j] for mv in mvs], [rv[j] for rv in rvs])


def pc2_range_error():
    from paper_2601_14980_amd import pc2
    return pc2.PC2_E_RANGE


def test_range_errors(gpu_ctx):
    p, q = gen.primes_for(99, 256)
    sk, opk, _ = keys(gpu_ctx, p, q, 256)
    n = p * q
    ms = [5, n, 7, 9]
    rs = [3, 3, 0, n]
    cs, st = gpu_encrypt(gpu_ctx, sk.public, ms, rs)
    assert st == -2
    assert cs[0] == O.encrypt(opk, 5, 3)
    assert cs[1:] == [0, 0, 0]
    assert gpu_ctx.sync() == 0  # the latch was cleared
    good = O.encrypt(opk, 11, 13)
    dec, st = gpu_decrypt(gpu_ctx, sk, [good, n * n, n * n + 5])
    assert st == -2
    assert dec == [11, 0, 0]
    s, st = gpu_hom_add(gpu_ctx, sk.public, [good, good], [good, n * n])
    assert st == -2
    assert s == [O.hom_add(opk, good, good), 0]


def test_quantize_dequantize(gpu_ctx):
    from paper_2601_14980_amd import pc2
    rng = np.random.default_rng(5)
    x = rng.standard_normal(10000)
    x[:8] = [0.5 / 2**20, 1.5 / 2**20, -0.5 / 2**20, -2.5 / 2**20, 7.999, -8.0, 0.0, -0.0]
    k, o, dl = 20, 1 << 23, 1 << 24
    xt = torch.from_numpy(x).cuda()
    mt = torch.zeros(x.shape, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, k, o, dl, xt, mt)
    assert gpu_ctx.sync() == 0
    m = mt.cpu().numpy().view(np.uint64)
    assert [int(v) for v in m] == Q.quantize_vec(x, k, o, dl)
    # dequantize sums of W addends
    W = 8
    Ms = [int(v) * W + 12345 for v in m[:1000]]
    mlimbs = torch.from_numpy(np.array(Ms, dtype=np.uint64).view(np.int32).reshape(-1, 2)).cuda()
    xo = torch.zeros(len(Ms), dtype=torch.float64, device="cuda")
    pc2.pc2_dequantize(gpu_ctx, k, o, mlimbs, W, xo)
    assert gpu_ctx.sync() == 0
    got = xo.cpu().numpy()
    want = Q.dequantize_vec(Ms, k, o, W)
    assert np.array_equal(got, np.array(want))


def test_quantize_range_errors(gpu_ctx):
    from paper_2601_14980_amd import pc2
    k, o, dl = 20, 1 << 23, 1 << 24  # the common interval [-8, 8)
    inside = [1.0, -8.0, np.nextafter(8.0, 0.0), -8.0 + 2.0 ** -21, 7.5 + 2.0 ** -21]
    outside = [np.nan, np.inf, -np.inf, -20.0, 1e30, 8.0, np.nextafter(-8.0, -9.0),
               -8.0 - 2.0 ** -21]  # the last rounds to -8 * 2^20, i.e. m = 0, yet lies below z_min
    x = np.array(inside + outside)
    xt = torch.from_numpy(x).cuda()
    mt = torch.zeros(x.shape, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, k, o, dl, xt, mt)
    assert gpu_ctx.sync() == -2
    m = [int(v) for v in mt.cpu().numpy().view(np.uint64)]
    want = Q.quantize_vec(inside, k, o, dl)
    assert want[1:3] == [0, dl]
    assert m == want + [0] * len(outside)
    for x_bad in outside:
        with pytest.raises(ValueError):
            Q.quantize(float(x_bad), k, o, dl)
    # a full-interval call with no error latches nothing
    pc2.pc2_quantize(gpu_ctx, k, o, dl, torch.from_numpy(np.array(inside)).cuda(), mt[:5])
    assert gpu_ctx.sync() == 0
    # offset above delta is an argument error, reported at once
    with pytest.raises(pc2.PC2Error):
        pc2.pc2_quantize(gpu_ctx, k, dl + 1, dl, xt, mt)
