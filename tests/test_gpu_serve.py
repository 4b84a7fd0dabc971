"""Request server on the GPU (pc2_server_*, pc2_serve_*): requests of mixed
type and length arrive over time, run through continuous batching
(persistent runner launches on three streams, admission by an HBM budget),
and each result must equal, bit for bit, the same request run alone through
the one-call entry points; sampled elements must equal the oracle."""
from __future__ import annotations

import random

import pytest
import torch

from oracle import paillier as O
from workload import gen
from workload.limbs import ints_from_limbs, to_limbs

pytestmark = pytest.mark.gpu

NBITS = 1024


@pytest.fixture(scope="module")
def keyset(gpu_ctx):
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(5, NBITS)
    n = p * q
    opk, osk = O.derive_keys(p, q)
    sk = pc2.SecretKey(gpu_ctx, NBITS, p, q)
    rng = random.Random(9)
    POOL, PLEN = 6, 700
    pool_m = [[rng.getrandbits(30) for _ in range(PLEN)] for _ in range(POOL)]
    pool_c = []
    for k in range(POOL):
        c = torch.zeros((PLEN, 2 * sk.L), dtype=torch.int32, device="cuda")
        pc2.pc2_encrypt(sk.public, pc2.to_device_limbs(to_limbs(pool_m[k], 2)),
                        pc2.to_device_limbs(to_limbs(gen.gen_r(n, PLEN, 5, extra=k), sk.L)), c)
        pool_c.append(c)
    assert gpu_ctx.sync() == 0
    return dict(sk=sk, n=n, opk=opk, osk=osk, pool_m=pool_m, pool_c=pool_c, PLEN=PLEN)


def _requests(pc2, ks, count, seed, rate):
    from paper_2601_14980_amd.serve import Request
    sk, n, L = ks["sk"], ks["n"], ks["sk"].L
    rng = random.Random(seed)
    reqs, t = [], 0.0
    for i in range(count):
        op = ("encrypt", "aggregate", "decrypt")[i % 3]
        length = rng.randint(20, ks["PLEN"])
        t += rng.expovariate(rate)
        req = Request(rid=i, op=op, length=length, arrival=t)
        if op == "encrypt":
            ms = [rng.getrandbits(30) for _ in range(length)]
            rs = gen.gen_r(n, length, 6, extra=i)
            out = torch.full((length, 2 * L), -1, dtype=torch.int32, device="cuda")
            req.payload = dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public,
                               m=pc2.to_device_limbs(to_limbs(ms, 2)),
                               r=pc2.to_device_limbs(to_limbs(rs, L)), out=out)
            req.result = dict(ms=ms, rs=rs)
        elif op == "aggregate":
            K = rng.randint(2, 5)
            idx = rng.sample(range(len(ks["pool_c"])), K)
            out = torch.full((length, 2 * L), -1, dtype=torch.int32, device="cuda")
            req.K = K
            req.payload = dict(op=pc2.PC2_OP_HOM_SUM, pk=sk.public,
                               inputs=[ks["pool_c"][j] for j in idx], out=out)
            req.result = dict(idx=idx)
        else:
            j = rng.randrange(len(ks["pool_c"]))
            out = torch.full((length, L), -1, dtype=torch.int32, device="cuda")
            req.payload = dict(op=pc2.PC2_OP_DECRYPT, sk=sk, c=ks["pool_c"][j][:length], out=out)
            req.result = dict(idx=j)
        reqs.append(req)
    return reqs


def _check_alone(pc2, gpu_ctx, ks, req):
    job = req.payload
    got = job["out"]
    alone = torch.zeros_like(got)
    if req.op == "encrypt":
        pc2.pc2_encrypt(ks["sk"].public, job["m"], job["r"], alone)
    elif req.op == "aggregate":
        pc2.pc2_hom_sum(ks["sk"].public, [c[:req.length].contiguous() for c in job["inputs"]],
                        alone)
    else:
        pc2.pc2_decrypt(ks["sk"], job["c"].contiguous(), alone)
    assert gpu_ctx.sync() == 0
    assert torch.equal(got, alone), f"request {req.rid} ({req.op}) differs from alone"
    vals = ints_from_limbs(pc2.from_device_limbs(got))
    j = req.length - 1
    if req.op == "encrypt":
        assert vals[j] == O.encrypt(ks["opk"], req.result["ms"][j], req.result["rs"][j])
    elif req.op == "aggregate":
        assert O.decrypt(ks["osk"], vals[j]) == sum(ks["pool_m"][k][j] for k in req.result["idx"])
    else:
        assert vals[j] == ks["pool_m"][req.result["idx"]][j]


@pytest.mark.parametrize("engine", ["auto", "mfma"])
def test_mixed_requests_equal_alone(gpu_ctx, keyset, engine):
    """A mixed trace through the request server equals every request run
    alone; with the matrix-core engine the server's encryption launches run
    on the matrix cores (and the alone runs too)."""
    from paper_2601_14980_amd import pc2
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_MFMA if engine == "mfma"
                       else pc2.PC2_MODMUL_AUTO)
    try:
        _mixed_equal_alone(pc2, gpu_ctx, keyset)
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)


def _mixed_equal_alone(pc2, gpu_ctx, keyset):
    from paper_2601_14980_amd.serve import percentile, serve_trace
    reqs = _requests(pc2, keyset, 18, 9, 4000.0)
    budget = 2 << 20                    # holds a few requests at a time
    srv = pc2.Server(gpu_ctx, keyset["sk"], hbm_budget=budget, tick_groups=24, max_requests=64)
    serve_trace(srv, reqs)
    torch.cuda.synchronize()
    assert gpu_ctx.sync() == 0
    st = srv.stats()
    assert all(r.completed is not None for r in reqs)
    assert st["launches"] > 3
    assert 0 < st["max_bytes"] <= budget and st["used_bytes"] == 0
    lat = [r.latency for r in reqs]
    assert percentile(lat, 50) <= percentile(lat, 99)
    for req in reqs:
        _check_alone(pc2, gpu_ctx, keyset, req)
    srv.close()


def test_poll_one_request_and_drain(gpu_ctx, keyset):
    """poll() waits on one id; completed() drains the rest in finishing order,
    skipping the ids poll already reported."""
    from paper_2601_14980_amd import pc2
    reqs = _requests(pc2, keyset, 9, 21, 1e9)
    srv = pc2.Server(gpu_ctx, keyset["sk"], hbm_budget=1 << 30, tick_groups=4096,
                     max_requests=16)
    ids = [srv.submit(r.payload) for r in reqs]
    while not srv.poll(ids[4]):
        pass
    seen = []
    while len(seen) < len(ids) - 1:
        srv.progress()
        seen += srv.completed()
    assert sorted(seen) == sorted(i for i in ids if i != ids[4])
    assert srv.progress() == 0 and srv.completed() == []
    assert gpu_ctx.sync() == 0
    for req in reqs:
        _check_alone(pc2, gpu_ctx, keyset, req)
    srv.close()


def test_server_argument_errors(gpu_ctx, keyset):
    from paper_2601_14980_amd import pc2
    sk = keyset["sk"]
    L = sk.L
    p2, q2 = gen.primes_for(6, NBITS)
    other = pc2.SecretKey(gpu_ctx, NBITS, p2, q2)
    srv = pc2.Server(gpu_ctx, sk, hbm_budget=1 << 20, tick_groups=8, max_requests=2)
    m = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    r = torch.ones((4, L), dtype=torch.int32, device="cuda")
    out = torch.zeros((4, 2 * L), dtype=torch.int32, device="cuda")
    with pytest.raises(pc2.PC2Error) as e:      # another key
        srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=other.public, m=m, r=r, out=out))
    assert e.value.status == pc2.PC2_E_INVAL
    big = torch.zeros((4096, 2 * L), dtype=torch.int32, device="cuda")
    with pytest.raises(pc2.PC2Error) as e:      # 4096 x 392 B > 1 MiB: never admissible
        srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=big[:, :2].contiguous(),
                        r=big[:, :L].contiguous(), out=big))
    assert e.value.status == pc2.PC2_E_NOMEM
    flat = torch.zeros(8 * L * 2, dtype=torch.int32, device="cuda")
    with pytest.raises(pc2.PC2Error) as e:      # output over its randomness, one row apart
        srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m,
                        r=flat[:4 * L].view(4, L), out=flat[L:L + 8 * L].view(4, 2 * L)))
    assert e.value.status == pc2.PC2_E_INVAL
    empty = torch.zeros((0, 2 * L), dtype=torch.int32, device="cuda")
    z = srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m[:0], r=r[:0], out=empty))
    assert srv.poll(z)                          # nothing to compute: done at once
    with pytest.raises(pc2.PC2Error) as e:      # forgotten once reported
        srv.poll(z)
    assert e.value.status == pc2.PC2_E_INVAL
    a = srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m, r=r, out=out))
    out2 = torch.zeros_like(out)
    b = srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m, r=r, out=out2))
    with pytest.raises(pc2.PC2Error) as e:      # max_requests tracked
        srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m, r=r,
                        out=torch.zeros_like(out)))
    assert e.value.status == pc2.PC2_E_BUSY
    for rid in (a, b):
        while not srv.poll(rid):
            pass
    assert gpu_ctx.sync() == 0
    assert torch.equal(out, out2)
    srv.close()
    other.close()


def test_tile_change_while_admitted_is_refused(gpu_ctx, keyset):
    """Groups are cut for the key's tile at admission: changing the tile while
    a request still has groups to launch is refused until it is restored."""
    from paper_2601_14980_amd import pc2
    sk, L, n = keyset["sk"], keyset["sk"].L, keyset["n"]
    count = 200
    rng = random.Random(33)
    ms = [rng.getrandbits(30) for _ in range(count)]
    m = pc2.to_device_limbs(to_limbs(ms, 2))
    r = pc2.to_device_limbs(to_limbs(gen.gen_r(n, count, 8), L))
    out = torch.full((count, 2 * L), -1, dtype=torch.int32, device="cuda")
    srv = pc2.Server(gpu_ctx, sk, hbm_budget=1 << 30, tick_groups=2, max_requests=4)
    rid = srv.submit(dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m, r=r, out=out))
    other = 4 if pc2.runner_group_size(sk.public, pc2.PC2_OP_ENCRYPT) == 32 else 2
    try:
        gpu_ctx.set_option(pc2.PC2_OPT_TILE, other)  # 1024-bit keys: 2 or 4 lanes
        with pytest.raises(pc2.PC2Error) as e:
            srv.poll(rid)
        assert e.value.status == pc2.PC2_E_UNSUPPORTED
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_TILE, 0)
    while not srv.poll(rid):
        pass
    assert gpu_ctx.sync() == 0
    alone = torch.zeros_like(out)
    pc2.pc2_encrypt(sk.public, m, r, alone)
    assert gpu_ctx.sync() == 0
    assert torch.equal(out, alone)
    srv.close()


@pytest.mark.parametrize("policy", ["shortest_aging", "fair"])
def test_policies_equal_alone(gpu_ctx, keyset, policy):
    """The default is shortest remaining first; here with an age limit short
    enough that aged requests lead most launches, and the fair-share policy."""
    from paper_2601_14980_amd import pc2
    from paper_2601_14980_amd.serve import serve_trace
    reqs = _requests(pc2, keyset, 15, 17, 4000.0)
    srv = pc2.Server(gpu_ctx, keyset["sk"], hbm_budget=2 << 20, tick_groups=24, max_requests=64)
    for bad in ((7, 1.0), (pc2.PC2_SERVE_SHORTEST, -1.0)):
        with pytest.raises(pc2.PC2Error):
            srv.set_policy(*bad)
    if policy == "fair":
        srv.set_policy(pc2.PC2_SERVE_FAIR, 1.0)
    else:
        srv.set_policy(pc2.PC2_SERVE_SHORTEST, 0.001)
    serve_trace(srv, reqs)
    torch.cuda.synchronize()
    assert gpu_ctx.sync() == 0
    assert all(r.completed is not None for r in reqs)
    for req in reqs:
        _check_alone(pc2, gpu_ctx, keyset, req)
    srv.close()
