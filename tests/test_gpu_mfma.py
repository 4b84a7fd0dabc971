"""Encryption with the i8-MFMA Montgomery product (GPU tests).

With PC2_OPT_MODMUL = PC2_MODMUL_MFMA, pc2_encrypt runs its modular
products on the matrix cores.  Every ciphertext must equal the oracle's and
the VALU path's bit for bit; decryption must invert it.  The default
(PC2_MODMUL_AUTO) takes the matrix cores from 2048 bits on."""
from __future__ import annotations

import math
import random

import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import gpu_decrypt, gpu_encrypt
from workload import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mfma_ctx():
    from paper_2601_14980_amd import pc2
    ctx = pc2.Context(0)
    ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_MFMA)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.fixture(scope="module")
def valu_ctx():
    from paper_2601_14980_amd import pc2
    ctx = pc2.Context(0)
    ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_VALU)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _key(ctx, p, q, nbits=None):
    from paper_2601_14980_amd import pc2
    n = p * q
    sk = pc2.SecretKey(ctx, nbits or n.bit_length(), p, q)
    opk, osk = O.derive_keys(p, q)
    return sk, opk, osk


@pytest.mark.parametrize("p,q", [(3, 5), (7, 11), (11, 13)])
def test_mfma_bruteforce_tiny(mfma_ctx, p, q):
    sk, opk, _ = _key(mfma_ctx, p, q)
    n = p * q
    pairs = [(m, r) for m in range(n) for r in range(1, n) if math.gcd(r, n) == 1]
    cs, st = gpu_encrypt(mfma_ctx, sk.public, [m for m, _ in pairs], [r for _, r in pairs])
    assert st == 0
    assert cs == [O.encrypt(opk, m, r) for m, r in pairs]


@pytest.mark.parametrize("nbits", [64, 256, 1024, 2048, 3072, 4096])
def test_mfma_matches_oracle_and_valu(valu_ctx, mfma_ctx, nbits):
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(1, nbits, extra=7)
    n = p * q
    sk, opk, osk = _key(mfma_ctx, p, q, nbits)
    count = 40 if nbits > 3072 else (150 if nbits >= 2048 else 300)  # several waves plus a tail
    rng = random.Random(nbits)
    ms = [0, 1, n - 1] + [rng.randrange(n) for _ in range(count - 3)]
    rs = [1, n - 1, 2] + gen.gen_r(n, count - 3, 1, extra=nbits)
    cs, st = gpu_encrypt(mfma_ctx, sk.public, ms, rs)
    assert st == 0
    sk_v = pc2.SecretKey(valu_ctx, nbits, p, q)
    cv, st = gpu_encrypt(valu_ctx, sk_v.public, ms, rs)
    assert st == 0
    assert cs == cv, "MFMA and VALU ciphertexts differ"
    for j in (sorted({0, 1, 2, 3, count // 2, count - 1}) if nbits <= 3072 else (1, count - 1)):
        assert cs[j] == O.encrypt(opk, ms[j], rs[j]), f"element {j}"
    dec, st = gpu_decrypt(valu_ctx, sk_v, cs)
    assert st == 0 and dec == ms


def test_mfma_small_plaintext_limbs(mfma_ctx):
    """Quantized plaintexts arrive as two limbs."""
    p, q = gen.primes_for(1, 2048, extra=8)
    n = p * q
    sk, opk, _ = _key(mfma_ctx, p, q, 2048)
    rng = random.Random(5)
    ms = [rng.getrandbits(64) for _ in range(70)]
    rs = gen.gen_r(n, 70, 1, extra=99)
    cs, st = gpu_encrypt(mfma_ctx, sk.public, ms, rs, m_limbs=2)
    assert st == 0
    for j in (0, 33, 69):
        assert cs[j] == O.encrypt(opk, ms[j], rs[j])


def test_mfma_range_errors(mfma_ctx):
    p, q = gen.primes_for(1, 256, extra=9)
    n = p * q
    sk, opk, _ = _key(mfma_ctx, p, q, 256)
    ms = [5, n, 7, 8]
    rs = [3, 3, 0, n]
    cs, st = gpu_encrypt(mfma_ctx, sk.public, ms, rs)
    assert st != 0
    assert cs[0] == O.encrypt(opk, 5, 3)
    assert cs[1:] == [0, 0, 0]
    assert mfma_ctx.sync() == 0   # the error latch was cleared


@pytest.mark.parametrize("nbits", [1024, 2048, 3072])
def test_auto_engine(valu_ctx, nbits):
    """A fresh context defaults to PC2_MODMUL_AUTO; its ciphertexts (the MFMA
    engine from 2048 bits on, the VALU engine below) equal the VALU engine's."""
    from paper_2601_14980_amd import pc2
    ctx = pc2.Context(0)
    assert ctx.get_option(pc2.PC2_OPT_MODMUL) == pc2.PC2_MODMUL_AUTO
    with pytest.raises(pc2.PC2Error):
        ctx.set_option(pc2.PC2_OPT_MODMUL, 3)
    p, q = gen.primes_for(1, nbits, extra=11)
    n = p * q
    sk, opk, _ = _key(ctx, p, q, nbits)
    sk_v = pc2.SecretKey(valu_ctx, nbits, p, q)
    rng = random.Random(nbits + 1)
    ms = [n - 1, 0] + [rng.randrange(n) for _ in range(69)]
    rs = [n - 1, 1] + gen.gen_r(n, 69, 1, extra=nbits + 1)
    cs, st = gpu_encrypt(ctx, sk.public, ms, rs)
    cv, st_v = gpu_encrypt(valu_ctx, sk_v.public, ms, rs)
    assert st == 0 and st_v == 0 and cs == cv
    assert cs[0] == O.encrypt(opk, ms[0], rs[0])
    sk.close()
    sk_v.close()
    ctx.close()


@pytest.mark.parametrize("nbits", [256, 2048, 3072])
def test_mfma_workgroups_loop_over_elements(valu_ctx, mfma_ctx, nbits):
    """More elements than workgroups: every workgroup runs several elements
    in turn on the same LDS workspace, so whatever one element leaves there
    must not reach the next.  All ciphertexts equal the VALU engine's;
    elements from the first, second and last pass of the grid equal the
    oracle's."""
    import numpy as np
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(2, nbits, extra=11)
    n = p * q
    sk, opk, _ = _key(mfma_ctx, p, q, nbits)
    sk_v = pc2.SecretKey(valu_ctx, nbits, p, q)
    count = {256: 40000, 2048: 7001, 3072: 5003}[nbits]   # above two grids of workgroups
    L = sk.L
    rng = np.random.default_rng(nbits)
    m = torch.from_numpy(rng.integers(0, 1 << 31, size=(count, 1), dtype=np.int64)
                         .astype(np.int32)).cuda()
    r = pc2.to_device_limbs(gen.gen_r_limbs(n, count, L, 5))
    out = {}
    for ctx, key in ((mfma_ctx, sk), (valu_ctx, sk_v)):
        c = torch.zeros((count, 2 * L), dtype=torch.int32, device="cuda")
        pc2.pc2_encrypt(key.public, m, r, c)
        assert ctx.sync() == 0
        out[ctx] = c
    assert torch.equal(out[mfma_ctx], out[valu_ctx]), "MFMA and VALU ciphertexts differ"
    cm = out[mfma_ctx].cpu().numpy().view(np.uint32)
    rh = r.cpu().numpy().view(np.uint32)
    mh = m.cpu().numpy().view(np.uint32)
    for j in (0, 1, count // 3, count // 2 + 1, count - 2, count - 1):
        cj = sum(int(w) << (32 * k) for k, w in enumerate(cm[j]))
        rj = sum(int(w) << (32 * k) for k, w in enumerate(rh[j]))
        assert cj == O.encrypt(opk, int(mh[j, 0]), rj), f"element {j}"


@pytest.mark.parametrize("nbits", [256, 2048])
def test_mfma_every_window(valu_ctx, mfma_ctx, nbits):
    """Every window width the option allows (2..6): the matrix-core kernel's
    table holds 2^(w-1) odd powers, the square and g^m in its 2^w entries,
    so w = 2 fills it exactly.  Ciphertexts equal the VALU engine's and the
    oracle's."""
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(3, nbits, extra=13)
    n = p * q
    sk, opk, _ = _key(mfma_ctx, p, q, nbits)
    sk_v = pc2.SecretKey(valu_ctx, nbits, p, q)
    rng = random.Random(nbits + 7)
    count = 70
    ms = [n - 1, 0] + [rng.randrange(n) for _ in range(count - 2)]
    rs = [n - 1, 1] + gen.gen_r(n, count - 2, 1, extra=nbits + 7)
    cv, st = gpu_encrypt(valu_ctx, sk_v.public, ms, rs)
    assert st == 0
    try:
        for w in (2, 3, 4, 5, 6):
            mfma_ctx.set_option(pc2.PC2_OPT_WINDOW, w)
            cs, st = gpu_encrypt(mfma_ctx, sk.public, ms, rs)
            assert st == 0
            assert cs == cv, f"window {w}"
    finally:
        mfma_ctx.set_option(pc2.PC2_OPT_WINDOW, 0)
    for j in (0, 1, count - 1):
        assert cv[j] == O.encrypt(opk, ms[j], rs[j])
