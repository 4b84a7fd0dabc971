"""Data calls under HIP graph capture, across streams, and without allocation
(GPU tests).

* encrypt -> hom_sum -> decrypt captured in one HIP graph on a fresh context
  and replayed, with the program's own eager work between replays: every
  replay equals the eager run and the oracle;
* calls sharing a context's scratch on two streams are ordered by the
  library, so their results equal the one-stream results;
* once the keys exist, no data call allocates device memory.
"""
from __future__ import annotations

import random

import numpy as np
import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import dev, host_ints
from workload import gen
from workload.limbs import to_limbs

pytestmark = pytest.mark.gpu

NBITS = 2048
K = 3
COUNT = 3 * 16 + 5   # three wavefront groups of the own tile and a ragged tail


def _inputs(n, L, seed):
    rng = random.Random(seed)
    ms = [[rng.getrandbits(24) for _ in range(COUNT)] for _ in range(K)]
    ms[0][0], ms[1][1] = n - 1, 0
    rs = [gen.gen_r(n, COUNT, 21, extra=seed * 10 + k) for k in range(K)]
    rs[0][2], rs[1][3] = 1, n - 1
    m = [dev(to_limbs(v, L)) for v in ms]
    r = [dev(to_limbs(v, L)) for v in rs]
    return ms, rs, m, r


def test_graph_encrypt_sum_decrypt_replays():
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(21, NBITS)
    n = p * q
    opk, osk = O.derive_keys(p, q)
    ctx = pc2.Context(0)                       # fresh context: nothing cached before the keys
    sk = pc2.SecretKey(ctx, NBITS, p, q)
    L = sk.L
    ms, rs, m, r = _inputs(n, L, 1)
    c = [torch.zeros((COUNT, 2 * L), dtype=torch.int32, device="cuda") for _ in range(K)]
    agg = torch.zeros((COUNT, 2 * L), dtype=torch.int32, device="cuda")
    dec = torch.zeros((COUNT, L), dtype=torch.int32, device="cuda")

    def step():
        for k in range(K):
            pc2.pc2_encrypt(sk.public, m[k], r[k], c[k])
        pc2.pc2_hom_sum(sk.public, c, agg)
        pc2.pc2_decrypt(sk, agg, dec)

    step()                                     # eager reference
    assert ctx.sync() == 0
    ref = [t.clone() for t in (*c, agg, dec)]
    cts = [host_ints(t) for t in c]
    for k in range(K):
        for j in (0, 1, 2, 3, COUNT // 2, COUNT - 1):
            assert cts[k][j] == O.encrypt(opk, ms[k][j], rs[k][j])
    got_agg, got_dec = host_ints(agg), host_ints(dec)
    for j in range(COUNT):
        assert got_dec[j] == sum(ms[k][j] for k in range(K)) % n
    for j in (0, 1, COUNT - 1):
        assert got_agg[j] == O.hom_sum(opk, [cts[k][j] for k in range(K)])
        assert got_dec[j] == O.decrypt(osk, got_agg[j])

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    for t in (*c, agg, dec):
        t.fill_(-1)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=side):
        step()
    for rep in range(3):
        for t in (*c, agg, dec):               # eager work between replays
            t.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ctx.sync() == 0
        for t, want in zip((*c, agg, dec), ref):
            assert torch.equal(t, want), f"replay {rep} differs from the eager run"
    del g
    sk.close()
    ctx.close()


def test_two_streams_share_the_scratch_in_order(gpu_ctx):
    """Encryptions and decryptions issued alternately on two streams of one
    context: each call's table slots are the context's scratch, so the library
    makes each stream wait for the previous call; results equal the
    one-stream results."""
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(22, NBITS)
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, NBITS, p, q)
    L = sk.L
    count = 8192
    rng = np.random.default_rng(22)
    mv = [torch.from_numpy(rng.integers(0, 1 << 24, size=(count, 1), dtype=np.int64)
                           .astype(np.int32)).cuda() for _ in range(2)]
    rv = [dev(gen.gen_r_limbs(n, count, L, 22, extra=i)) for i in range(2)]
    want = [torch.zeros((count, 2 * L), dtype=torch.int32, device="cuda") for _ in range(2)]
    want_m = [torch.zeros((count, L), dtype=torch.int32, device="cuda") for _ in range(2)]
    for i in range(2):
        pc2.pc2_encrypt(sk.public, mv[i], rv[i], want[i])
        pc2.pc2_decrypt(sk, want[i], want_m[i])
    assert gpu_ctx.sync() == 0
    for i in range(2):
        assert torch.equal(want_m[i][:, :1], mv[i]) and not want_m[i][:, 1:].any()
    s = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = [torch.full_like(w, -1) for w in want]
    got_m = [torch.full_like(w, -1) for w in want_m]
    torch.cuda.synchronize()
    for i in range(2):                          # issue everything before waiting
        pc2.pc2_encrypt(sk.public, mv[i], rv[i], got[i], stream=s[i])
    for i in range(2):
        pc2.pc2_decrypt(sk, want[1 - i], got_m[1 - i], stream=s[i])
    torch.cuda.synchronize()
    assert gpu_ctx.sync() == 0
    for i in range(2):
        assert torch.equal(got[i], want[i]), f"encryption on stream {i}"
        assert torch.equal(got_m[i], want_m[i]), f"decryption of vector {i}"
    sk.close()


def test_data_calls_allocate_nothing():
    """After the keys exist, every data call runs in memory sized at key
    creation: the device's free memory is the same before and after a
    round of every call (all kernels were loaded by a first round on
    another context)."""
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(23, NBITS)
    n = p * q
    Bm = torch.from_numpy(np.random.default_rng(23).integers(0, 1 << 20, size=(40, 32),
                                                             dtype=np.int64)).cuda()

    def round_of_calls(ctx, sk, bufs):
        m, r, c, c2, k, dec, agg, xo, mq, mvp, B, mv_out, xin = bufs
        pc2.pc2_quantize(ctx, 20, 1 << 23, 1 << 24, xin, mq)
        pc2.pc2_encrypt(sk.public, m, r, c)
        pc2.pc2_encrypt_sk(sk, m, r, c2)
        ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_MFMA)
        pc2.pc2_encrypt(sk.public, m[:64], r[:64], c2[:64])
        ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_VALU)
        pc2.pc2_hom_sum(sk.public, [c, c2, c], agg)
        pc2.pc2_hom_scalar_mul(sk.public, c, k, c2)
        pc2.pc2_decrypt(sk, agg, dec)
        pc2.pc2_enc_sum_dec(sk, [m, m], [r, r], dec)
        pc2.pc2_dequantize(ctx, 20, 1 << 23, dec, 2, xo)
        mvp.load(c[:32])
        mvp.apply(B, mv_out)
        assert ctx.sync() == 0

    def make(ctx):
        sk = pc2.SecretKey(ctx, NBITS, p, q)
        L = sk.L
        cnt = 4096
        m = torch.from_numpy(np.arange(cnt, dtype=np.int64).reshape(cnt, 1).astype(np.int32)).cuda()
        r = dev(gen.gen_r_limbs(n, cnt, L, 23))
        bufs = (m, r,
                torch.zeros((cnt, 2 * L), dtype=torch.int32, device="cuda"),
                torch.zeros((cnt, 2 * L), dtype=torch.int32, device="cuda"),
                torch.arange(cnt, dtype=torch.int64, device="cuda"),
                torch.zeros((cnt, L), dtype=torch.int32, device="cuda"),
                torch.zeros((cnt, 2 * L), dtype=torch.int32, device="cuda"),
                torch.zeros(cnt, dtype=torch.float64, device="cuda"),
                torch.zeros(cnt, dtype=torch.int64, device="cuda"),
                pc2.MatVec(sk.public, 32, 20, 4, rows_hint=8),
                Bm,
                torch.zeros((40, 2 * L), dtype=torch.int32, device="cuda"),
                torch.zeros(cnt, dtype=torch.float64, device="cuda"))
        return sk, bufs

    warm = pc2.Context(0)
    wsk, wbufs = make(warm)
    round_of_calls(warm, wsk, wbufs)          # loads every kernel's code
    ctx = pc2.Context(0)
    sk, bufs = make(ctx)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(2):
        round_of_calls(ctx, sk, bufs)         # rows 40 > the plan's hint of 8: fewer chunks
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(bufs[11], wbufs[11]) and torch.equal(bufs[5], wbufs[5])
    for b in (bufs, wbufs):
        b[9].close()
    sk.close()
    wsk.close()
    ctx.close()
    warm.close()
