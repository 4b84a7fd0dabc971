"""Serving loop on the GPU: requests of mixed type and length run through the
continuous-batching scheduler (persistent runner launches on three streams)
and each result must equal, bit for bit, the same request run alone through
the one-call entry points, and sampled elements must equal the oracle."""
from __future__ import annotations

import random

import pytest
import torch

from oracle import paillier as O
from workload import gen
from workload.limbs import ints_from_limbs, to_limbs

pytestmark = pytest.mark.gpu

NBITS = 1024


def test_mixed_requests_equal_alone(gpu_ctx):
    from paper_2601_14980_amd import pc2
    from paper_2601_14980_amd.serve import GpuExecutor, Request, Scheduler, percentile

    p, q = gen.primes_for(5, NBITS)
    n = p * q
    opk, osk = O.derive_keys(p, q)
    sk = pc2.SecretKey(gpu_ctx, NBITS, p, q)
    L = sk.L
    rng = random.Random(9)
    # resident ciphertext pool for aggregate / decrypt requests
    POOL, PLEN = 6, 700
    pool_m = [[rng.getrandbits(30) for _ in range(PLEN)] for _ in range(POOL)]
    pool_c = []
    for k in range(POOL):
        c = torch.zeros((PLEN, 2 * L), dtype=torch.int32, device="cuda")
        pc2.pc2_encrypt(sk.public, pc2.to_device_limbs(to_limbs(pool_m[k], 2)),
                        pc2.to_device_limbs(to_limbs(gen.gen_r(n, PLEN, 5, extra=k), L)), c)
        pool_c.append(c)
    assert gpu_ctx.sync() == 0

    reqs = []
    t = 0.0
    for i in range(18):
        op = ("encrypt", "aggregate", "decrypt")[i % 3]
        length = rng.randint(20, PLEN)
        t += rng.expovariate(4000.0)
        req = Request(rid=i, op=op, length=length, arrival=t)
        if op == "encrypt":
            ms = [rng.getrandbits(30) for _ in range(length)]
            rs = gen.gen_r(n, length, 6, extra=i)
            req.payload = dict(m=pc2.to_device_limbs(to_limbs(ms, 2)),
                               r=pc2.to_device_limbs(to_limbs(rs, L)), ms=ms, rs=rs)
        elif op == "aggregate":
            K = rng.randint(2, 5)
            idx = rng.sample(range(POOL), K)
            req.K = K
            req.payload = dict(inputs=[pool_c[j] for j in idx], idx=idx)
        else:
            j = rng.randrange(POOL)
            req.payload = dict(c=pool_c[j][:length], idx=j)
        reqs.append(req)

    ex = GpuExecutor(gpu_ctx, sk, max_groups=4096, max_jobs=64)
    sch = Scheduler(ex, hbm_budget=1 << 30, tick_groups=24)
    sch.run_trace(reqs)
    torch.cuda.synchronize()
    assert gpu_ctx.sync() == 0
    assert len(sch.finished) == len(reqs)
    assert sch.ticks > 3
    lat = [r.latency for r in reqs]
    assert percentile(lat, 50) <= percentile(lat, 99)

    for req in reqs:
        got = req.result
        alone = torch.zeros_like(got)
        if req.op == "encrypt":
            pc2.pc2_encrypt(sk.public, req.payload["m"], req.payload["r"], alone)
        elif req.op == "aggregate":
            pc2.pc2_hom_sum(sk.public, [c[:req.length].contiguous()
                                        for c in req.payload["inputs"]], alone)
        else:
            pc2.pc2_decrypt(sk, req.payload["c"].contiguous(), alone)
        assert gpu_ctx.sync() == 0
        assert torch.equal(got, alone), f"request {req.rid} ({req.op}) differs from alone"
        vals = ints_from_limbs(pc2.from_device_limbs(got))
        j = req.length - 1
        if req.op == "encrypt":
            assert vals[j] == O.encrypt(opk, req.payload["ms"][j], req.payload["rs"][j])
        elif req.op == "aggregate":
            assert O.decrypt(osk, vals[j]) == sum(pool_m[k][j] for k in req.payload["idx"])
        else:
            assert vals[j] == pool_m[req.payload["idx"]][j]
    ex.close()
