"""The paper-sized workloads at full size, in the launch shapes bench.py times
(GPU tests).  The oracle checks sampled elements one by one; every element is
checked through the exact identity Dec(prod_k Enc(m_k)) = sum_k m_k; and
every eighth ciphertext of the 2048-bit encryption launch (every 32nd at
3072 bits) is compared with the oracle's through digests written from
oracle/ alone.

* 2048-bit key, 8 nodes x 65536 quantized N(0,1) values: one encryption
  launch of 524288, an 8-way aggregation, one decryption launch of 65536.
* 16 nodes of log-uniform lengths in [1024, 65536] under alternating
  1024/2048-bit keys: one persistent batch launch per phase.
* 3072-bit key, 32 x 16384 quantized values (one lasso iteration's
  crypto): encryption of 524288, 32-way aggregation, decryption of 16384.
* The request server as the benchmark runs it (2048-bit key, launches of 2048
  groups, 4 GiB budget) on requests of up to 65536 elements."""
from __future__ import annotations

import hashlib
import json
from pathlib import Path

import numpy as np
import pytest
import torch

from oracle import paillier as O
from oracle import quant as Q
from workload import gen
from workload.limbs import ints_from_limbs

pytestmark = pytest.mark.gpu

GOLDEN = Path(__file__).resolve().parent / "golden"


def _sums_exact(pc2, dec: torch.Tensor, mq: np.ndarray) -> bool:
    """dec: [len][L] plaintexts; mq: [K][len] uint64 quantized addends."""
    d = pc2.from_device_limbs(dec)
    got = d[:, 0].astype(object) + (d[:, 1].astype(object) << 32)
    want = mq.astype(object).sum(axis=0)
    return bool(np.all(d[:, 2:] == 0)) and bool(np.all(got == want))


@pytest.mark.parametrize("nbits,nodes,length,seed", [(2048, 8, 65536, 2), (3072, 32, 16384, 4)],
                         ids=["2048bit_8x65536", "3072bit_32x16384"])
def test_full_size_encrypt_aggregate_decrypt(gpu_ctx, nbits, nodes, length, seed):
    from paper_2601_14980_amd import pc2
    p, q = gen.primes_for(seed, nbits)
    n = p * q
    opk, osk = O.derive_keys(p, q)
    sk = pc2.SecretKey(gpu_ctx, nbits, p, q)
    L = sk.L
    qp = gen.Q_PLAIN
    xs = gen.normal_vectors(seed, [length] * nodes)
    rs = np.concatenate([gen.gen_r_limbs(n, length, L, seed, extra=k) for k in range(nodes)])
    total = nodes * length
    m = torch.empty(total, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta, torch.from_numpy(np.concatenate(xs)).cuda(),
                     m)
    c = torch.empty((total, 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_encrypt(sk.public, m.view(torch.int32).reshape(total, 2), pc2.to_device_limbs(rs), c)
    agg = torch.empty((length, 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_hom_sum(sk.public, [c[k * length:(k + 1) * length] for k in range(nodes)], agg)
    dec = torch.empty((length, L), dtype=torch.int32, device="cuda")
    pc2.pc2_decrypt(sk, agg, dec)
    xo = torch.empty(length, dtype=torch.float64, device="cuda")
    pc2.pc2_dequantize(gpu_ctx, qp.log2_scale, qp.offset, dec, nodes, xo)
    assert gpu_ctx.sync() == 0
    mq = m.cpu().numpy().view(np.uint64).reshape(nodes, length)
    assert _sums_exact(pc2, dec, mq), "a decrypted aggregate differs from the integer sum"
    # sampled elements against the oracle, one by one
    rng = np.random.default_rng(nbits)
    for node, j in zip(rng.integers(0, nodes, 3), rng.integers(0, length, 3)):
        e = int(node) * length + int(j)
        mv = Q.quantize(float(xs[node][j]), qp.log2_scale, qp.offset, qp.delta)
        assert int(mq[node, j]) == mv
        r = int(ints_from_limbs(rs[e:e + 1])[0])
        want = O.encrypt(opk, mv, r)
        assert ints_from_limbs(pc2.from_device_limbs(c[e:e + 1]))[0] == want, f"element {e}"
    j = int(rng.integers(0, length))
    cts = [ints_from_limbs(pc2.from_device_limbs(c[k * length + j:k * length + j + 1]))[0]
           for k in range(nodes)]
    want_agg = O.hom_sum(opk, cts)
    assert ints_from_limbs(pc2.from_device_limbs(agg[j:j + 1]))[0] == want_agg
    assert ints_from_limbs(pc2.from_device_limbs(dec[j:j + 1]))[0] == O.decrypt(osk, want_agg)
    want_x = Q.dequantize(int(mq[:, j].astype(object).sum()), qp.log2_scale, qp.offset, nodes)
    assert float(xo[j].item()) == want_x


def test_full_size_batches(gpu_ctx):
    """16 nodes, lengths log-uniform in [1024, 65536], keys alternating
    1024/2048-bit: encryptions, ragged aggregation and decryptions, one
    persistent launch each."""
    from paper_2601_14980_amd import pc2
    seed = 3
    lengths = gen.log_uniform_lengths(seed, 16, 1024, 65536)
    keys = []
    for bits in (1024, 2048):
        p, q = gen.primes_for(seed, bits)
        keys.append(dict(sk=pc2.SecretKey(gpu_ctx, bits, p, q), opk=O.derive_keys(p, q)[0],
                         n=p * q))
    xs = gen.normal_vectors(seed, lengths)
    qp = gen.Q_PLAIN
    nodes = []
    for i, Ln in enumerate(lengths):
        k = keys[i % 2]
        m = torch.empty(Ln, dtype=torch.int64, device="cuda")
        pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta, torch.from_numpy(xs[i]).cuda(), m)
        rl = gen.gen_r_limbs(k["n"], Ln, k["sk"].L, seed, extra=i)
        nodes.append(dict(k=k, L=Ln, m=m, rl=rl, r=pc2.to_device_limbs(rl),
                          c=torch.empty((Ln, 2 * k["sk"].L), dtype=torch.int32, device="cuda")))
    groups = []
    for g, k in enumerate(keys):
        mem = [nd for i, nd in enumerate(nodes) if i % 2 == g]
        mx = max(nd["L"] for nd in mem)
        groups.append(dict(k=k, mem=mem, mx=mx,
                           agg=torch.empty((mx, 2 * k["sk"].L), dtype=torch.int32, device="cuda"),
                           dec=torch.empty((mx, k["sk"].L), dtype=torch.int32, device="cuda")))
    assert gpu_ctx.sync() == 0
    enc = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["k"]["sk"].public,
                                   m=nd["m"].view(torch.int32).reshape(nd["L"], 2), r=nd["r"],
                                   out=nd["c"]) for nd in nodes])
    agg = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_HOM_SUM, pk=g["k"]["sk"].public,
                                   inputs=[nd["c"] for nd in g["mem"]],
                                   lengths=[nd["L"] for nd in g["mem"]], out=g["agg"])
                              for g in groups])
    dec = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_DECRYPT, sk=g["k"]["sk"], c=g["agg"],
                                   out=g["dec"]) for g in groups])
    for b in (enc, agg, dec):
        b.run(0)
    assert gpu_ctx.sync() == 0
    for g in groups:
        want = np.zeros(g["mx"], dtype=object)
        for nd in g["mem"]:
            want[:nd["L"]] += nd["m"].cpu().numpy().view(np.uint64).astype(object)
        d = pc2.from_device_limbs(g["dec"])
        got = d[:, 0].astype(object) + (d[:, 1].astype(object) << 32)
        assert bool(np.all(d[:, 2:] == 0)) and bool(np.all(got == want))
    rng = np.random.default_rng(5)
    for i in (0, 1, 15):
        nd = nodes[i]
        j = int(rng.integers(0, nd["L"]))
        mv = int(nd["m"][j].item())
        r = int(ints_from_limbs(nd["rl"][j:j + 1])[0])
        got = ints_from_limbs(pc2.from_device_limbs(nd["c"][j:j + 1]))[0]
        assert got == O.encrypt(nd["k"]["opk"], mv, r), f"node {i}, element {j}"
    for b in (enc, agg, dec):
        b.close()


def test_full_size_serving(gpu_ctx):
    """The request server in the benchmark's configuration (2048-bit key,
    launches of 2048 groups, a 4 GiB budget) on requests of up to 65536
    elements of each operation: every result equals the same request run
    alone; sampled elements equal the oracle."""
    from paper_2601_14980_amd import pc2
    from paper_2601_14980_amd.serve import Request, serve_trace
    seed, PL = 6, 65536
    p, q = gen.primes_for(seed, 2048)
    n = p * q
    opk, osk = O.derive_keys(p, q)
    sk = pc2.SecretKey(gpu_ctx, 2048, p, q)
    L = sk.L
    qp = gen.Q_PLAIN
    m = torch.empty(PL, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta,
                     torch.from_numpy(gen.normal_vectors(seed, [PL])[0]).cuda(), m)
    m2 = m.view(torch.int32).reshape(PL, 2)
    rl = gen.gen_r_limbs(n, PL, L, seed)
    r = pc2.to_device_limbs(rl)
    pool = [torch.empty((PL, 2 * L), dtype=torch.int32, device="cuda") for _ in range(3)]
    pc2.pc2_encrypt(sk.public, m2, r, pool[0])
    for k in (1, 2):
        pc2.pc2_hom_scalar_mul(sk.public, pool[0],
                               torch.full((PL,), k + 1, dtype=torch.int64, device="cuda"), pool[k])
    assert gpu_ctx.sync() == 0
    specs = [("encrypt", PL), ("aggregate", PL), ("decrypt", PL),
             ("encrypt", 300), ("aggregate", 4097), ("decrypt", 1000)]
    reqs = []
    for i, (op, ln) in enumerate(specs):
        req = Request(rid=i, op=op, length=ln, arrival=0.002 * i)
        width = L if op == "decrypt" else 2 * L
        out = torch.full((ln, width), -1, dtype=torch.int32, device="cuda")
        if op == "encrypt":
            req.payload = dict(op=pc2.PC2_OP_ENCRYPT, pk=sk.public, m=m2[:ln], r=r[:ln], out=out)
        elif op == "aggregate":
            req.payload = dict(op=pc2.PC2_OP_HOM_SUM, pk=sk.public, inputs=pool, out=out)
        else:
            req.payload = dict(op=pc2.PC2_OP_DECRYPT, sk=sk, c=pool[1][:ln], out=out)
        reqs.append(req)
    srv = pc2.Server(gpu_ctx, sk, hbm_budget=4 << 30, tick_groups=2048, max_requests=64)
    serve_trace(srv, reqs)
    assert gpu_ctx.sync() == 0
    srv.close()
    mh = m.cpu().numpy().view(np.uint64)
    for req in reqs:
        job, ln = req.payload, req.length
        alone = torch.empty_like(job["out"])
        if req.op == "encrypt":
            pc2.pc2_encrypt(sk.public, job["m"], job["r"], alone)
        elif req.op == "aggregate":
            pc2.pc2_hom_sum(sk.public, [c[:ln] for c in pool], alone)
        else:
            pc2.pc2_decrypt(sk, job["c"], alone)
        assert gpu_ctx.sync() == 0
        assert torch.equal(job["out"], alone), f"request {req.rid} ({req.op}, {ln})"
        j = ln - 1
        got = ints_from_limbs(pc2.from_device_limbs(job["out"][j:j + 1]))[0]
        if req.op == "encrypt":
            assert got == O.encrypt(opk, int(mh[j]), int(ints_from_limbs(rl[j:j + 1])[0]))
        elif req.op == "aggregate":
            assert O.decrypt(osk, got) == 6 * int(mh[j])   # (1 + 2 + 3) m_j
        else:
            assert got == 2 * int(mh[j])


@pytest.mark.parametrize("engine", ["mfma", "valu"])
@pytest.mark.parametrize("config", ["2048bit_8x65536", "3072bit_32x16384", "4096bit_1x32768"])
def test_full_size_ciphertexts_match_the_oracle_digests(gpu_ctx, config, engine):
    """Elements 0, 8, 16, ... of the 2048-bit 8 x 65536 encryption launch
    (65536 ciphertexts), 0, 32, 64, ... of the 3072-bit 32 x 16384 one
    (16384) and 0, 8, 16, ... of a 4096-bit launch of 32768 (4096), over every
    node and every position of the launch, with each Montgomery engine,
    against the oracle's ciphertexts of the same seeded inputs: SHA-256 per
    chunk of 4096, as tests/golden/make_fullsize_digests.py wrote them from
    oracle/ alone; then the aggregates over the nodes at the sampled
    positions against the oracle's products."""
    from paper_2601_14980_amd import pc2
    doc = json.loads((GOLDEN / f"fullsize_{config}.json").read_text())
    w = doc["workload"]
    nbits, nodes, length, seed = w["nbits"], w["nodes"], w["length"], w["key_seed"]
    stride, chunk = doc["stride"], doc["chunk"]
    p, q = gen.primes_for(seed, nbits)
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, nbits, p, q)
    L = sk.L
    qp = gen.Q_PLAIN
    assert w["quantizer"] == {"log2_scale": qp.log2_scale, "offset": qp.offset,
                              "delta": qp.delta}
    xs = gen.normal_vectors(seed, [length] * nodes)
    rs = np.concatenate([gen.gen_r_limbs(n, length, L, seed, extra=k) for k in range(nodes)])
    total = nodes * length
    m = torch.empty(total, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta,
                     torch.from_numpy(np.concatenate(xs)).cuda(), m)
    c = torch.empty((total, 2 * L), dtype=torch.int32, device="cuda")
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL,
                       pc2.PC2_MODMUL_MFMA if engine == "mfma" else pc2.PC2_MODMUL_VALU)
    try:
        pc2.pc2_encrypt(sk.public, m.view(torch.int32).reshape(total, 2), pc2.to_device_limbs(rs),
                        c)
        assert gpu_ctx.sync() == 0
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)
    bad = _digest_mismatches(c[::stride], doc["samples"], chunk, doc["digests"])
    assert not bad, \
        f"{config}, {engine}: chunks {bad} of {chunk} sampled elements differ from the oracle"
    if nodes > 1:
        # the element-wise products over the nodes, at the sampled positions
        agg = torch.empty((length, 2 * L), dtype=torch.int32, device="cuda")
        pc2.pc2_hom_sum(sk.public, [c[k * length:(k + 1) * length] for k in range(nodes)], agg)
        assert gpu_ctx.sync() == 0
        bad = _digest_mismatches(agg[::stride], length // stride, doc["agg_chunk"],
                                 doc["agg_digests"])
        assert not bad, f"{config}, {engine}: aggregate chunks {bad} differ from the oracle"


def _digest_mismatches(rows_dev: torch.Tensor, count: int, chunk: int,
                       digests: list[str]) -> list[int]:
    """SHA-256 per chunk of `chunk` rows (little-endian limbs) against the
    stored digests; the indices of the chunks that differ."""
    rows = rows_dev.cpu().numpy().view(np.uint32)
    assert rows.shape[0] == count and count == chunk * len(digests)
    blob = rows.astype("<u4").tobytes()
    nb = chunk * rows.shape[1] * 4
    return [i for i, e in enumerate(digests)
            if hashlib.sha256(blob[i * nb:(i + 1) * nb]).hexdigest() != e]


@pytest.mark.parametrize("engine", ["mfma", "valu"])
def test_full_size_batches_match_the_oracle_digests(gpu_ctx, engine):
    """The batching workload (16 nodes of log-uniform lengths, 1024-bit key
    on even nodes, 2048-bit on odd ones) through one persistent encryption
    launch and one ragged aggregation launch, with the 2048-bit encryptions
    on either engine: every eighth ciphertext of every node, and the ragged
    products at the same positions, against the digests that
    tests/golden/make_fullsize_digests.py wrote from oracle/ alone."""
    from paper_2601_14980_amd import pc2
    doc = json.loads((GOLDEN / "fullsize_batch_16nodes.json").read_text())
    w, stride = doc["workload"], doc["stride"]
    seed, lengths, key_bits = w["seed"], w["lengths"], w["key_bits"]
    assert lengths == gen.log_uniform_lengths(seed, w["nodes"], 1024, 65536)
    qp = gen.Q_PLAIN
    assert w["quantizer"] == {"log2_scale": qp.log2_scale, "offset": qp.offset,
                              "delta": qp.delta}
    keys = []
    for bits in key_bits:
        p, q = gen.primes_for(seed, bits)
        keys.append(dict(sk=pc2.SecretKey(gpu_ctx, bits, p, q), n=p * q))
    xs = gen.normal_vectors(seed, lengths)
    nodes = []
    for i, Ln in enumerate(lengths):
        k = keys[i % 2]
        m = torch.empty(Ln, dtype=torch.int64, device="cuda")
        pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta,
                         torch.from_numpy(xs[i]).cuda(), m)
        rl = gen.gen_r_limbs(k["n"], Ln, k["sk"].L, seed, extra=i)
        nodes.append(dict(k=k, L=Ln, m=m, r=pc2.to_device_limbs(rl),
                          c=torch.empty((Ln, 2 * k["sk"].L), dtype=torch.int32, device="cuda")))
    groups = []
    for g, k in enumerate(keys):
        mem = [nd for i, nd in enumerate(nodes) if i % 2 == g]
        mx = max(nd["L"] for nd in mem)
        groups.append(dict(k=k, mem=mem, mx=mx,
                           agg=torch.empty((mx, 2 * k["sk"].L), dtype=torch.int32, device="cuda")))
    assert gpu_ctx.sync() == 0
    gpu_ctx.set_option(pc2.PC2_OPT_MODMUL,
                       pc2.PC2_MODMUL_MFMA if engine == "mfma" else pc2.PC2_MODMUL_VALU)
    try:
        enc = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["k"]["sk"].public,
                                       m=nd["m"].view(torch.int32).reshape(nd["L"], 2),
                                       r=nd["r"], out=nd["c"]) for nd in nodes])
    finally:
        gpu_ctx.set_option(pc2.PC2_OPT_MODMUL, pc2.PC2_MODMUL_AUTO)
    agg = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_HOM_SUM, pk=g["k"]["sk"].public,
                                   inputs=[nd["c"] for nd in g["mem"]],
                                   lengths=[nd["L"] for nd in g["mem"]], out=g["agg"])
                              for g in groups])
    enc.run(0)
    agg.run(0)
    assert gpu_ctx.sync() == 0
    for i, nd in enumerate(nodes):
        rows = nd["c"][::stride]
        assert rows.shape[0] == (nd["L"] + stride - 1) // stride
        assert not _digest_mismatches(rows, rows.shape[0], rows.shape[0],
                                      [doc["node_digests"][i]]), f"{engine}: node {i}"
    for g, grp in enumerate(groups):
        rows = grp["agg"][::stride]
        assert not _digest_mismatches(rows, rows.shape[0], rows.shape[0],
                                      [doc["agg_digests"][g]]), f"{engine}: aggregate of key {g}"
    enc.close()
    agg.close()
