"""Ciphertext matrix-vector product (pc2_matvec_*) on the GPU.

out_i = alpha_i * prod_j c_j^(B_ij) mod n^2 must equal the oracle's
hom_matvec bit for bit (several tiles and a ragged tail of rows, one and many
column chunks, window widths 1..12, exponent edges), data errors must zero
exactly the rows the contract names, and at larger sizes the outputs must
decrypt to the exact integer mat-vec of the plaintexts."""
from __future__ import annotations

import random

import numpy as np
import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import dev, gpu_decrypt, gpu_encrypt, host_ints
from workload import gen
from workload.limbs import to_limbs

pytestmark = pytest.mark.gpu


def _key(ctx, nbits, seed=8):
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(seed, nbits)
    opk, osk = O.derive_keys(p, q)
    return pc2.SecretKey(ctx, nbits, p, q), opk, osk


def _B_dev(B):
    a = np.array(B, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).cuda()


def _run(ctx, sk, B, cs, alpha=None, ebits=50, window=0, rows_hint=0):
    from paper_2601_14980_amd import pc2
    L2 = 2 * sk.L
    rows, cols = len(B), len(cs)
    mv = pc2.MatVec(sk.public, cols, ebits, window, rows_hint or rows)
    mv.load(dev(to_limbs(cs, L2)))
    out = torch.full((rows, L2), -1, dtype=torch.int32, device="cuda")
    a = dev(to_limbs(alpha, L2)) if alpha is not None else None
    mv.apply(_B_dev(B), out, a)
    st = ctx.sync()
    res = host_ints(out)
    w = mv.window
    mv.close()
    return res, st, w


@pytest.mark.parametrize("nbits,window,with_alpha", [
    (256, 1, True), (256, 5, False), (1024, 3, True), (2048, 4, True), (2048, 8, False),
])
def test_matvec_matches_oracle(gpu_ctx, nbits, window, with_alpha):
    sk, opk, _ = _key(gpu_ctx, nbits)
    n2 = opk.n2
    rng = random.Random(nbits * 10 + window)
    rows, cols = 37, 23                      # rows: two wavefront groups and a tail
    cs = [0, 1, n2 - 1] + [rng.randrange(n2) for _ in range(cols - 3)]
    B = [[rng.getrandbits(50) for _ in range(cols)] for _ in range(rows)]
    B[0] = [0] * cols
    B[1] = [(1 << 50) - 1] * cols
    B[2][5] = 1
    alpha = [rng.randrange(n2) for _ in range(rows)] if with_alpha else None
    got, st, w = _run(gpu_ctx, sk, B, cs, alpha, window=window)
    assert st == 0 and w == window
    assert got == O.hom_matvec(opk, B, cs, alpha)


@pytest.mark.parametrize("nbits,rows,cols", [(3072, 9, 4), (4096, 5, 3)])
def test_matvec_large_keys(gpu_ctx, nbits, rows, cols):
    """The 3072- and 4096-bit classes (28-bit digits on 8 lanes, renormalised
    products) with a ragged wavefront of rows."""
    sk, opk, _ = _key(gpu_ctx, nbits, seed=10)
    n2 = opk.n2
    rng = random.Random(nbits)
    cs = [rng.randrange(n2) for _ in range(cols)]
    B = [[rng.getrandbits(40) for _ in range(cols)] for _ in range(rows)]
    alpha = [rng.randrange(n2) for _ in range(rows)]
    got, st, _ = _run(gpu_ctx, sk, B, cs, alpha, ebits=40, window=5)
    assert st == 0
    assert got == O.hom_matvec(opk, B, cs, alpha)


def test_matvec_column_chunks_combine(gpu_ctx):
    """Few rows and many columns: the rows are split over column chunks whose
    partial products are multiplied afterwards."""
    sk, opk, _ = _key(gpu_ctx, 1024)
    n2 = opk.n2
    rng = random.Random(21)
    rows, cols = 5, 300
    cs = [rng.randrange(n2) for _ in range(cols)]
    B = [[rng.getrandbits(20) for _ in range(cols)] for _ in range(rows)]
    alpha = [rng.randrange(n2) for _ in range(rows)]
    got, st, _ = _run(gpu_ctx, sk, B, cs, alpha, ebits=20, window=6)
    assert st == 0
    assert got == O.hom_matvec(opk, B, cs, alpha)


@pytest.mark.parametrize("ebits,window", [(64, 7), (64, 12), (1, 1), (1, 4), (33, 11)])
def test_matvec_exponent_edges(gpu_ctx, ebits, window):
    sk, opk, _ = _key(gpu_ctx, 256)
    n2 = opk.n2
    rng = random.Random(ebits * 100 + window)
    rows, cols = 19, 3
    top = (1 << ebits) - 1
    cs = [rng.randrange(n2) for _ in range(cols)]
    B = [[rng.randrange(top + 1) for _ in range(cols)] for _ in range(rows)]
    B[0] = [top] * cols
    B[1] = [0, 1, top]
    B[2] = [1 << (ebits - 1)] * cols
    got, st, _ = _run(gpu_ctx, sk, B, cs, None, ebits=ebits, window=window)
    assert st == 0
    assert got == O.hom_matvec(opk, B, cs)


def test_matvec_range_errors(gpu_ctx):
    sk, opk, _ = _key(gpu_ctx, 256)
    n2 = opk.n2
    rng = random.Random(5)
    rows, cols, ebits = 20, 6, 40
    cs = [rng.randrange(n2) for _ in range(cols)]
    cs[3] = n2                               # not a residue: column 3's tables are zeroed
    B = [[rng.getrandbits(ebits) | 1 for _ in range(cols)] for _ in range(rows)]
    for i in range(0, rows, 2):
        B[i][3] = 0                          # even rows never use column 3
    B[4][1] = 1 << ebits                     # constant out of range
    alpha = [rng.randrange(n2) for _ in range(rows)]
    alpha[6] = n2 + 5                        # alpha out of range
    got, st, _ = _run(gpu_ctx, sk, B, cs, alpha, ebits=ebits, window=5)
    assert st != 0
    assert gpu_ctx.sync() == 0               # the latch was cleared
    cs_ok = cs[:3] + [1] + cs[4:]            # c^0 = 1 whatever c is
    want = O.hom_matvec(opk, B, cs_ok, [a % n2 for a in alpha])
    for i in range(rows):
        if i % 2 == 1 or i in (4, 6):
            assert got[i] == 0, f"row {i}"
        else:
            assert got[i] == want[i], f"row {i}"


def test_matvec_alias_and_argument_errors(gpu_ctx):
    from paper_2601_14980_amd import pc2
    sk, opk, _ = _key(gpu_ctx, 256)
    n2 = opk.n2
    L2 = 2 * sk.L
    rng = random.Random(6)
    rows, cols = 10, 4
    cs = [rng.randrange(n2) for _ in range(cols)]
    B = [[rng.getrandbits(16) for _ in range(cols)] for _ in range(rows)]
    alpha = [rng.randrange(n2) for _ in range(rows)]
    mv = pc2.MatVec(sk.public, cols, 16, 4)
    with pytest.raises(pc2.PC2Error):        # apply before any load
        mv.apply(_B_dev(B), torch.zeros((rows, L2), dtype=torch.int32, device="cuda"))
    mv.load(dev(to_limbs(cs, L2)))
    buf = dev(to_limbs(alpha, L2))
    mv.apply(_B_dev(B), buf, buf)            # out is alpha itself
    assert gpu_ctx.sync() == 0
    assert host_ints(buf) == O.hom_matvec(opk, B, cs, alpha)
    big = torch.zeros((rows + 1, L2), dtype=torch.int32, device="cuda")
    Bd = _B_dev(B)
    rc = pc2.lib.pc2_matvec_apply(mv.handle, Bd.data_ptr(), big[:rows].data_ptr(),
                                  big[1:].data_ptr(), rows, None)
    assert rc == -1                          # PC2_E_INVAL: alpha and out overlap in part
    mv.close()
    for bad in (dict(cols=0, ebits=8, window=0), dict(cols=2, ebits=0, window=0),
                dict(cols=2, ebits=65, window=0), dict(cols=2, ebits=8, window=13)):
        with pytest.raises(pc2.PC2Error):
            pc2.MatVec(sk.public, bad["cols"], bad["ebits"], bad["window"])


def test_matvec_auto_window(gpu_ctx):
    from paper_2601_14980_amd import pc2
    sk, _, _ = _key(gpu_ctx, 2048)
    a = pc2.MatVec(sk.public, 64, 50, 0)
    assert a.window == 8
    b = pc2.MatVec(sk.public, 64, 50, 0, rows_hint=9000)
    assert b.window == 10                    # ceil(50/w) (9000 + 2^w - 1) is least at w = 10
    assert b.table_bytes == 64 * 5 * 1023 * 640
    a.close()
    b.close()


def test_matvec_decrypts_to_integer_matvec(gpu_ctx):
    """2048-bit key, 300 x 700 quantized-scale data: every output decrypts to
    alpha's plaintext + sum_j B_ij m_j (exact integers on the host)."""
    from paper_2601_14980_amd import pc2
    sk, opk, _ = _key(gpu_ctx, 2048, seed=9)
    n = opk.n
    rng = random.Random(9)
    rows, cols = 300, 700
    m = [rng.getrandbits(24) for _ in range(cols)]
    a = [rng.getrandbits(24) for _ in range(rows)]
    r = gen.gen_r(n, cols + rows, 9, extra=1)
    cs, st = gpu_encrypt(gpu_ctx, sk.public, m, r[:cols], m_limbs=1)
    assert st == 0
    alpha, st = gpu_encrypt(gpu_ctx, sk.public, a, r[cols:], m_limbs=1)
    assert st == 0
    Bn = np.frombuffer(np.random.default_rng(9).bytes(rows * cols * 8), dtype=np.uint64)
    Bn = (Bn >> np.uint64(14)).reshape(rows, cols)       # 50-bit constants
    mv = pc2.MatVec(sk.public, cols, 50, 0, rows_hint=rows)
    mv.load(dev(to_limbs(cs, 2 * sk.L)))
    out = torch.zeros((rows, 2 * sk.L), dtype=torch.int32, device="cuda")
    mv.apply(torch.from_numpy(Bn.view(np.int64)).cuda(), out, dev(to_limbs(alpha, 2 * sk.L)))
    assert gpu_ctx.sync() == 0
    dec, st = gpu_decrypt(gpu_ctx, sk, host_ints(out))
    assert st == 0
    Bo = Bn.astype(object)
    for i in range(rows):
        assert dec[i] == (a[i] + sum(int(b) * mj for b, mj in zip(Bo[i], m))) % n, f"row {i}"
    mv.close()
