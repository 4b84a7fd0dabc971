"""Persistent batch launches: mixed 1024/2048-bit keys, ragged vector lengths,
HIP-graph replay, and the autotuner (GPU tests).

Batch results must equal the one-call entry points bit for bit, and sampled
elements must equal the oracle."""
from __future__ import annotations

import random

import numpy as np
import pytest
import torch

from oracle import paillier as O
from workload import gen
from workload.limbs import ints_from_limbs, to_limbs

pytestmark = pytest.mark.gpu

LENGTHS = [300, 1000, 77, 513, 64, 129]   # node i uses key i % 2
BITS = [1024, 2048]


@pytest.fixture(scope="module")
def setup(gpu_ctx):
    from paper_2601_14980_amd import pc2
    keys = []
    for b in BITS:
        p, q = gen.primes_for(3, b)
        opk, osk = O.derive_keys(p, q)
        keys.append(dict(bits=b, sk=pc2.SecretKey(gpu_ctx, b, p, q), opk=opk, osk=osk, n=p * q))
    nodes = []
    for i, L in enumerate(LENGTHS):
        k = keys[i % 2]
        rng = random.Random(i)
        ms = [rng.getrandbits(40) for _ in range(L)]
        rs = gen.gen_r(k["n"], L, 3, extra=i)
        nodes.append(dict(key=k, ms=ms, rs=rs,
                          m=pc2.to_device_limbs(to_limbs(ms, 2)),
                          r=pc2.to_device_limbs(to_limbs(rs, k["sk"].L)),
                          c=torch.zeros((L, 2 * k["sk"].L), dtype=torch.int32, device="cuda")))
    return dict(keys=keys, nodes=nodes)


def _sample(L):
    return sorted({0, 1, L // 2, L - 2, L - 1})


def test_batch_encrypt_mixed_keys(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    nodes = setup["nodes"]
    jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"], r=nd["r"],
                 out=nd["c"]) for nd in nodes]
    b = pc2.Batch(gpu_ctx, jobs)
    b.run(0)
    assert gpu_ctx.sync() == 0
    for nd in nodes:
        k = nd["key"]
        ref = torch.zeros_like(nd["c"])
        pc2.pc2_encrypt(k["sk"].public, nd["m"], nd["r"], ref)
        assert gpu_ctx.sync() == 0
        assert torch.equal(ref, nd["c"])
        got = ints_from_limbs(pc2.from_device_limbs(nd["c"]))
        for j in _sample(len(nd["ms"])):
            assert got[j] == O.encrypt(k["opk"], nd["ms"][j], nd["rs"][j])
    b.close()


def test_batch_ragged_sum_and_decrypt(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    nodes = setup["nodes"]
    # ciphertexts from the one-call path
    for nd in nodes:
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], nd["c"])
    assert gpu_ctx.sync() == 0
    groups = []
    for g, k in enumerate(setup["keys"]):
        members = [nd for i, nd in enumerate(nodes) if i % 2 == g]
        maxlen = max(len(nd["ms"]) for nd in members)
        groups.append(dict(key=k, members=members, maxlen=maxlen,
                           agg=torch.zeros((maxlen, 2 * k["sk"].L), dtype=torch.int32,
                                           device="cuda"),
                           dec=torch.zeros((maxlen, k["sk"].L), dtype=torch.int32,
                                           device="cuda")))
    sum_jobs = [dict(op=pc2.PC2_OP_HOM_SUM, pk=g["key"]["sk"].public,
                     inputs=[nd["c"] for nd in g["members"]],
                     lengths=[len(nd["ms"]) for nd in g["members"]], out=g["agg"])
                for g in groups]
    dec_jobs = [dict(op=pc2.PC2_OP_DECRYPT, sk=g["key"]["sk"], c=g["agg"], out=g["dec"])
                for g in groups]
    bs, bd = pc2.Batch(gpu_ctx, sum_jobs), pc2.Batch(gpu_ctx, dec_jobs)
    bs.run(0)
    bd.run(0)
    assert gpu_ctx.sync() == 0
    for g in groups:
        k = g["key"]
        cts = [ints_from_limbs(pc2.from_device_limbs(nd["c"])) for nd in g["members"]]
        agg = ints_from_limbs(pc2.from_device_limbs(g["agg"]))
        dec = ints_from_limbs(pc2.from_device_limbs(g["dec"]))
        for j in range(g["maxlen"]):
            terms = [ct[j] for ct in cts if j < len(ct)]
            assert agg[j] == O.hom_sum(k["opk"], terms)
            # exact end-to-end: Dec(prod) == sum of the plaintexts reaching j
            assert dec[j] == sum(nd["ms"][j] for nd in g["members"] if j < len(nd["ms"]))
        for j in _sample(g["maxlen"])[:3]:
            assert dec[j] == O.decrypt(k["osk"], agg[j])
    bs.close()
    bd.close()


def test_batch_sum_and_decrypt_graph_replays(gpu_ctx, setup):
    """The ragged aggregation batch and the two-launch decryption batch (queue
    reset, per-prime items, recombination) on a non-null stream: the first run
    captures each in a HIP graph, the next two replay it; with the program's
    own eager work between runs, every run equals the null-stream run, which
    equals the oracle on sampled elements and the plaintext sums on all."""
    from paper_2601_14980_amd import pc2
    nodes = setup["nodes"]
    for nd in nodes:
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], nd["c"])
    assert gpu_ctx.sync() == 0
    groups = []
    for g, k in enumerate(setup["keys"]):
        members = [nd for i, nd in enumerate(nodes) if i % 2 == g]
        maxlen = max(len(nd["ms"]) for nd in members)
        groups.append(dict(key=k, members=members, maxlen=maxlen,
                           agg=torch.zeros((maxlen, 2 * k["sk"].L), dtype=torch.int32,
                                           device="cuda"),
                           dec=torch.zeros((maxlen, k["sk"].L), dtype=torch.int32,
                                           device="cuda")))
    bs = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_HOM_SUM, pk=g["key"]["sk"].public,
                                  inputs=[nd["c"] for nd in g["members"]],
                                  lengths=[len(nd["ms"]) for nd in g["members"]], out=g["agg"])
                             for g in groups])
    bd = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_DECRYPT, sk=g["key"]["sk"], c=g["agg"],
                                  out=g["dec"]) for g in groups])
    bs.run(0)
    bd.run(0)
    assert gpu_ctx.sync() == 0
    ref = [(g["agg"].clone(), g["dec"].clone()) for g in groups]
    for g in groups:
        k = g["key"]
        cts = [ints_from_limbs(pc2.from_device_limbs(nd["c"])) for nd in g["members"]]
        agg = ints_from_limbs(pc2.from_device_limbs(g["agg"]))
        dec = ints_from_limbs(pc2.from_device_limbs(g["dec"]))
        for j in range(g["maxlen"]):
            assert dec[j] == sum(nd["ms"][j] for nd in g["members"] if j < len(nd["ms"]))
        for j in _sample(g["maxlen"]):
            assert agg[j] == O.hom_sum(k["opk"], [ct[j] for ct in cts if j < len(ct)])
            assert dec[j] == O.decrypt(k["osk"], agg[j])
    side = torch.cuda.Stream()
    for rep in range(3):
        for g in groups:        # the program's own eager work between runs
            g["agg"].fill_(-1)
            g["dec"].fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            bs.run()            # the first run captures, later runs replay
            bd.run()
        side.synchronize()
        assert gpu_ctx.sync(side) == 0
        for g, (ra, rd) in zip(groups, ref):
            assert torch.equal(g["agg"], ra), f"aggregation, run {rep}"
            assert torch.equal(g["dec"], rd), f"decryption, run {rep}"
    bs.close()
    bd.close()


def test_batch_graph_replays_match_eager(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    nodes = setup["nodes"]
    eager = []
    for nd in nodes:
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], nd["c"])
    assert gpu_ctx.sync() == 0
    eager = [nd["c"].clone() for nd in nodes]
    jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"], r=nd["r"],
                 out=nd["c"]) for nd in nodes]
    b = pc2.Batch(gpu_ctx, jobs)
    side = torch.cuda.Stream()
    for rep in range(3):
        for nd in nodes:        # the program's own eager work between replays
            nd["c"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.run()             # first run captures the graph, later runs replay it
        side.synchronize()
        assert gpu_ctx.sync(side) == 0
        for nd, ref in zip(nodes, eager):
            assert torch.equal(nd["c"], ref), f"replay {rep} differs from the eager result"
    b.close()


def test_batch_rejects_bad_jobs(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    nd = setup["nodes"][0]
    with pytest.raises(pc2.PC2Error):
        pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"],
                                 r=nd["r"], out=nd["c"]),
                            dict(op=pc2.PC2_OP_DECRYPT, sk=nd["key"]["sk"], c=nd["c"],
                                 out=nd["m"])])


def test_autotune_keeps_results(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    k = setup["keys"][0]
    we, wd, te = pc2.pc2_autotune(k["sk"])
    assert we in (4, 5, 6) and wd in (4, 5, 6) and te in (2, 4)
    nd = setup["nodes"][0]
    out = torch.zeros_like(nd["c"])
    pc2.pc2_encrypt(k["sk"].public, nd["m"], nd["r"], out)
    assert gpu_ctx.sync() == 0
    got = ints_from_limbs(pc2.from_device_limbs(out))
    for j in _sample(len(nd["ms"])):
        assert got[j] == O.encrypt(k["opk"], nd["ms"][j], nd["rs"][j])


@pytest.mark.parametrize("engine", ["valu", "mfma", "auto"])
def test_batch_encrypt_engines(gpu_ctx, setup, engine):
    """Encryption batches under each Montgomery engine setting: the VALU
    kernel alone, the matrix cores for both key classes (two matrix-core
    launches) and the automatic choice (the VALU kernel for the 1024-bit
    jobs, the matrix cores for the 2048-bit ones).  Eager on the null
    stream and graph-captured on a side stream (replayed twice), every run
    equal to the VALU one-call results."""
    from paper_2601_14980_amd import pc2
    nodes = setup["nodes"]
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_VALU)
    refs = []
    for nd in nodes:
        ref = torch.zeros_like(nd["c"])
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], ref)
        refs.append(ref)
    assert gpu_ctx.sync() == 0
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, {"valu": pc2.PC2_MODMUL_VALU,
                                            "mfma": pc2.PC2_MODMUL_MFMA,
                                            "auto": pc2.PC2_MODMUL_AUTO}[engine])
    try:
        jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"], r=nd["r"],
                     out=nd["c"]) for nd in nodes]
        b = pc2.Batch(gpu_ctx, jobs)
        side = torch.cuda.Stream()
        for rep in range(3):
            for nd in nodes:
                nd["c"].zero_()
            torch.cuda.synchronize()
            if rep == 0:
                b.run(0)
                assert gpu_ctx.sync() == 0
            else:
                with torch.cuda.stream(side):
                    b.run()
                side.synchronize()
                assert gpu_ctx.sync(side) == 0
            for nd, ref in zip(nodes, refs):
                assert torch.equal(nd["c"], ref), f"{engine}, run {rep}"
        b.close()
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)
    k = nodes[1]["key"]
    got = ints_from_limbs(pc2.from_device_limbs(nodes[1]["c"]))
    for j in _sample(len(nodes[1]["ms"])):
        assert got[j] == O.encrypt(k["opk"], nodes[1]["ms"][j], nodes[1]["rs"][j])
