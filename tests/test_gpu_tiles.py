"""Limb tiles of the encryption kernels (PC2_OPT_TILE) and their autotuning
(GPU tests).

1024-bit keys encrypt with 2 or 4 lanes per ciphertext and 2048-bit keys with
4 or 8.  Every tile must give the same ciphertexts bit for bit, in one-call
encryption, in persistent batches that mix the two key sizes (every pair of
tiles) and in runner launches; sampled elements must equal the oracle."""
from __future__ import annotations

import random

import pytest
import torch

from oracle import paillier as O
from tests.gpu_helpers import dev
from workload import gen
from workload.limbs import ints_from_limbs, to_limbs

pytestmark = pytest.mark.gpu

LENGTHS = [333, 257, 64, 1029, 5, 700]   # node i uses key i % 2; ragged tails
BITS = [1024, 2048]


@pytest.fixture(scope="module")
def tctx():
    """A context of its own: the tile option and tuned choices stay here."""
    from paper_2601_14980_amd import pc2
    ctx = pc2.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.fixture(scope="module")
def setup(tctx):
    from paper_2601_14980_amd import pc2
    keys = []
    for b in BITS:
        p, q = gen.primes_for(4, b)
        opk, _ = O.derive_keys(p, q)
        keys.append(dict(bits=b, sk=pc2.SecretKey(tctx, b, p, q), opk=opk, n=p * q))
    nodes = []
    for i, L in enumerate(LENGTHS):
        k = keys[i % 2]
        rng = random.Random(100 + i)
        ms = [0, k["n"] - 1] + [rng.getrandbits(48) for _ in range(L - 2)] if L > 2 else \
            [rng.getrandbits(48) for _ in range(L)]
        rs = gen.gen_r(k["n"], L, 4, extra=i)
        nodes.append(dict(key=k, ms=ms, rs=rs, m=dev(to_limbs(ms, k["sk"].L)),
                          r=dev(to_limbs(rs, k["sk"].L))))
    # reference ciphertexts: each class's own tile, one call per node
    tctx.set_option(pc2.PC2_OPT_TILE, 2)
    for nd in nodes:
        nd["ref"] = torch.zeros((len(nd["ms"]), 2 * nd["key"]["sk"].L), dtype=torch.int32,
                                device="cuda")
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], nd["ref"])
    assert tctx.sync() == 0
    tctx.set_option(pc2.PC2_OPT_TILE, 0)
    for nd in nodes:
        got = ints_from_limbs(pc2.from_device_limbs(nd["ref"]))
        L = len(nd["ms"])
        for j in sorted({0, 1, L // 2, L - 1}):
            assert got[j] == O.encrypt(nd["key"]["opk"], nd["ms"][j], nd["rs"][j]), j
    return dict(keys=keys, nodes=nodes)


def _out(nd):
    return torch.full_like(nd["ref"], -1)


@pytest.mark.parametrize("tile", [4, 8, 1])   # 1 = PC2_TILE_WIDE
def test_tile_one_call_identical(tctx, setup, tile):
    from paper_2601_14980_amd import pc2
    tctx.set_option(pc2.PC2_OPT_TILE, tile)
    try:
        assert tctx.get_option(pc2.PC2_OPT_TILE) == tile
        for nd in setup["nodes"]:
            out = _out(nd)
            pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], out)
            assert tctx.sync() == 0
            assert torch.equal(out, nd["ref"]), f"tile {tile}, {len(nd['ms'])} elements"
    finally:
        tctx.set_option(pc2.PC2_OPT_TILE, 0)


@pytest.mark.parametrize("tile", [2, 4, 8, 1])  # geometry pairs (5,6), (6,9), (5,10), (9,10)
def test_tile_batch_mixed_identical(tctx, setup, tile):
    from paper_2601_14980_amd import pc2
    tctx.set_option(pc2.PC2_OPT_TILE, tile)
    try:
        nodes = setup["nodes"]
        outs = [_out(nd) for nd in nodes]
        jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"], r=nd["r"],
                     out=o) for nd, o in zip(nodes, outs)]
        b = pc2.Batch(tctx, jobs)
        side = torch.cuda.Stream()
        for rep in range(3):    # null stream (no graph), then capture, then replay
            for o in outs:
                o.fill_(-1)
            torch.cuda.synchronize()
            if rep == 0:
                b.run(0)
            else:
                with torch.cuda.stream(side):
                    b.run()
                side.synchronize()
            assert tctx.sync(side if rep else None) == 0
            for nd, o in zip(nodes, outs):
                assert torch.equal(o, nd["ref"]), f"tile {tile}, run {rep}, {len(nd['ms'])}"
        b.close()
    finally:
        tctx.set_option(pc2.PC2_OPT_TILE, 0)


def test_tile_runner_groups(tctx, setup):
    """A runner launch over element-group ranges; group sizes follow the tile."""
    from paper_2601_14980_amd import pc2
    nodes = [nd for nd in setup["nodes"] if nd["key"]["bits"] == 2048]
    sizes = {}
    for tile in (4, 8):
        tctx.set_option(pc2.PC2_OPT_TILE, tile)
        try:
            pk = nodes[0]["key"]["sk"].public
            epg = pc2.runner_group_size(pk, pc2.PC2_OP_ENCRYPT)
            sizes[tile] = epg
            r = pc2.Runner(tctx, pc2.PC2_OP_ENCRYPT, 2048, len(nodes), 4096)
            outs = [_out(nd) for nd in nodes]
            jobs = [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"],
                         r=nd["r"], out=o) for nd, o in zip(nodes, outs)]
            ng = [(len(nd["ms"]) + epg - 1) // epg for nd in nodes]
            # two launches: the first half of each job's groups, then the rest
            half = [g // 2 for g in ng]
            r.launch(jobs, [0] * len(jobs), half)
            r.launch(jobs, half, [g - h for g, h in zip(ng, half)])
            assert tctx.sync() == 0
            for nd, o in zip(nodes, outs):
                assert torch.equal(o, nd["ref"]), f"tile {tile}"
            r.close()
        finally:
            tctx.set_option(pc2.PC2_OPT_TILE, 0)
    assert sizes == {4: 16, 8: 8}


def test_tile_option_validation(tctx):
    from paper_2601_14980_amd import pc2
    for bad in (-1, 3, 16):
        with pytest.raises(pc2.PC2Error):
            tctx.set_option(pc2.PC2_OPT_TILE, bad)
    assert tctx.get_option(pc2.PC2_OPT_TILE) == 0


@pytest.mark.parametrize("bits", BITS)
def test_tile_auto_latency_threshold(tctx, setup, bits):
    """Automatic tile: a call of at most one wavefront per SIMD of the wider
    tile (4 * CUs * 64 / lanes elements) runs in the wider tile, one element
    more in the class's own; both sides of the threshold must give the own
    tile's ciphertexts."""
    from paper_2601_14980_amd import pc2
    k = setup["keys"][BITS.index(bits)]
    L = k["sk"].L
    wide = {1024: 4, 2048: 8}[bits]
    edge = 4 * torch.cuda.get_device_properties(0).multi_processor_count * (64 // wide)
    count = edge + 1
    g = torch.Generator().manual_seed(bits)
    m = torch.randint(0, 2**31, (count, 2), generator=g, dtype=torch.int64).to(torch.int32).cuda()
    rl = gen.gen_r_limbs(k["n"], count, L, 6)
    r = pc2.to_device_limbs(rl)
    ref = torch.full((count, 2 * L), -1, dtype=torch.int32, device="cuda")
    tctx.set_option(pc2.PC2_OPT_TILE, {1024: 2, 2048: 4}[bits])
    try:
        pc2.pc2_encrypt(k["sk"].public, m, r, ref)
        assert tctx.sync() == 0
    finally:
        tctx.set_option(pc2.PC2_OPT_TILE, 0)
    for n in (edge, count):
        out = torch.full((n, 2 * L), -1, dtype=torch.int32, device="cuda")
        pc2.pc2_encrypt(k["sk"].public, m[:n], r[:n], out)
        assert tctx.sync() == 0
        assert torch.equal(out, ref[:n]), f"{bits}-bit, {n} elements"
    mh = m.cpu().numpy().view("uint32").astype(object)
    for j in (0, edge - 1, edge):
        mv = int(mh[j, 0]) + (int(mh[j, 1]) << 32)
        rv = int(ints_from_limbs(rl[j:j + 1])[0])
        assert _ct(ref, j) == O.encrypt(k["opk"], mv, rv), j


def _ct(t, j):
    from paper_2601_14980_amd import pc2
    return ints_from_limbs(pc2.from_device_limbs(t[j:j + 1]))[0]


def test_autotune_picks_a_tile(tctx, setup):
    from paper_2601_14980_amd import pc2
    for k, lanes in zip(setup["keys"], ((2, 4), (4, 8))):
        we, wd, te = pc2.pc2_autotune(k["sk"])
        assert we in (4, 5, 6) and wd in (4, 5, 6)
        assert te in lanes
    # the tuned tiles and windows (option automatic) keep the results
    for nd in setup["nodes"]:
        out = _out(nd)
        pc2.pc2_encrypt(nd["key"]["sk"].public, nd["m"], nd["r"], out)
        assert tctx.sync() == 0
        assert torch.equal(out, nd["ref"])
    nodes = setup["nodes"]
    outs = [_out(nd) for nd in nodes]
    b = pc2.Batch(tctx, [dict(op=pc2.PC2_OP_ENCRYPT, pk=nd["key"]["sk"].public, m=nd["m"],
                              r=nd["r"], out=o) for nd, o in zip(nodes, outs)])
    b.run(0)
    assert tctx.sync() == 0
    for nd, o in zip(nodes, outs):
        assert torch.equal(o, nd["ref"])
    b.close()
