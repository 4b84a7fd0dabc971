"""Aliasing rules of the data calls (GPU tests): an output may be an input of
the same size exactly -- the in-place result equals the out-of-place one --
and any other overlap of an output with an input is refused with
PC2_E_INVAL before anything is enqueued."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from workload import gen
from workload.limbs import to_limbs

pytestmark = pytest.mark.gpu

COUNT = 300


@pytest.fixture(scope="module", params=[256, 2048], ids=["256bit", "2048bit"])
def setup(gpu_ctx, request):
    from paper_2601_14980_amd import pc2
    nbits = request.param
    p, q = gen.primes_for(7, nbits)
    n = p * q
    sk = pc2.SecretKey(gpu_ctx, nbits, p, q)
    L = sk.L
    rng = np.random.default_rng(nbits)
    ms = [int(v) for v in rng.integers(0, 2**40, COUNT)]
    m = pc2.to_device_limbs(to_limbs(ms, 2))
    r = pc2.to_device_limbs(gen.gen_r_limbs(n, COUNT, L, 7))
    cs = []
    for k in range(3):
        c = torch.empty((COUNT, 2 * L), dtype=torch.int32, device="cuda")
        pc2.pc2_encrypt(sk.public, m, r if k == 0 else torch.roll(r, k, 0).contiguous(), c)
        cs.append(c)
    assert gpu_ctx.sync() == 0
    return dict(sk=sk, L=L, m=m, r=r, cs=cs)


def test_exact_alias_equals_out_of_place(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    sk, cs = setup["sk"], setup["cs"]
    ref = torch.empty_like(cs[0])
    pc2.pc2_hom_add(sk.public, cs[0], cs[1], ref)
    inplace = cs[0].clone()
    pc2.pc2_hom_add(sk.public, inplace, cs[1], inplace)
    assert gpu_ctx.sync() == 0
    assert torch.equal(inplace, ref)
    ref = torch.empty_like(cs[0])
    pc2.pc2_hom_sum(sk.public, [cs[0], cs[1], cs[2]], ref)
    inplace = cs[1].clone()
    pc2.pc2_hom_sum(sk.public, [cs[0], inplace, cs[2]], inplace)
    assert gpu_ctx.sync() == 0
    assert torch.equal(inplace, ref)
    k = torch.arange(3, 3 + COUNT, dtype=torch.int64, device="cuda")
    ref = torch.empty_like(cs[0])
    pc2.pc2_hom_scalar_mul(sk.public, cs[2], k, ref)
    inplace = cs[2].clone()
    pc2.pc2_hom_scalar_mul(sk.public, inplace, k, inplace)
    assert gpu_ctx.sync() == 0
    assert torch.equal(inplace, ref)


def test_quantize_dequantize_in_place(gpu_ctx):
    from paper_2601_14980_amd import pc2
    qp = gen.Q_PLAIN
    x = torch.from_numpy(np.random.default_rng(3).standard_normal(COUNT)).cuda()
    ref = torch.empty(COUNT, dtype=torch.int64, device="cuda")
    pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta, x, ref)
    buf = x.clone()
    pc2.pc2_quantize(gpu_ctx, qp.log2_scale, qp.offset, qp.delta, buf, buf.view(torch.int64))
    assert gpu_ctx.sync() == 0
    assert torch.equal(buf.view(torch.int64), ref)
    back = torch.empty(COUNT, dtype=torch.float64, device="cuda")
    pc2.pc2_dequantize(gpu_ctx, qp.log2_scale, qp.offset, ref.view(torch.int32).reshape(COUNT, 2),
                       1, back)
    pc2.pc2_dequantize(gpu_ctx, qp.log2_scale, qp.offset,
                       buf.view(torch.int32).reshape(COUNT, 2), 1, buf)
    assert gpu_ctx.sync() == 0
    assert torch.equal(buf, back)


def test_partial_overlap_refused(gpu_ctx, setup):
    from paper_2601_14980_amd import pc2
    sk, L, m, r, cs = setup["sk"], setup["L"], setup["m"], setup["r"], setup["cs"]
    n = 64
    flat = torch.zeros((2 * n + 8) * 2 * L, dtype=torch.int32, device="cuda")
    cases = []
    # ciphertexts one row apart in the same buffer
    a = flat[:n * 2 * L].view(n, 2 * L)
    b = flat[2 * L:(n + 1) * 2 * L].view(n, 2 * L)
    a.copy_(cs[0][:n])
    b.copy_(cs[1][:n])
    cases.append(lambda: pc2.pc2_hom_add(sk.public, a, cs[1][:n], b))
    cases.append(lambda: pc2.pc2_hom_sum(sk.public, [cs[0][:n], a], b))
    cases.append(lambda: pc2.pc2_hom_scalar_mul(
        sk.public, a, torch.ones(n, dtype=torch.int64, device="cuda"), b))
    # an output over an input of another size, starting at the same address
    rr = flat[:n * L].view(n, L)
    rr.copy_(r[:n])
    cases.append(lambda: pc2.pc2_encrypt(sk.public, m[:n], rr, a))
    mm = flat[:n * L].view(n, L)
    cases.append(lambda: pc2.pc2_decrypt(sk, a, mm))
    for i, call in enumerate(cases):
        with pytest.raises(pc2.PC2Error) as e:
            call()
        assert e.value.status == pc2.PC2_E_INVAL, f"case {i}"
    assert gpu_ctx.sync() == 0


def test_batch_jobs_follow_the_aliasing_rule(gpu_ctx, setup):
    """Batches: an aggregation into one of its inputs gives the out-of-place
    result; an output over another job array is refused at planning."""
    from paper_2601_14980_amd import pc2
    sk, L, cs = setup["sk"], setup["L"], setup["cs"]
    ref = torch.empty_like(cs[0])
    pc2.pc2_hom_sum(sk.public, [cs[0], cs[1]], ref)
    inplace = cs[0].clone()
    b = pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_HOM_SUM, pk=sk.public, inputs=[inplace, cs[1]],
                                 out=inplace)])
    b.run(0)
    assert gpu_ctx.sync() == 0
    assert torch.equal(inplace, ref)
    b.close()
    n = 64
    flat = torch.zeros(n * 2 * L, dtype=torch.int32, device="cuda")
    with pytest.raises(pc2.PC2Error) as e:     # plaintexts over the first half of c
        pc2.Batch(gpu_ctx, [dict(op=pc2.PC2_OP_DECRYPT, sk=sk, c=flat.view(n, 2 * L),
                                 out=flat[:n * L].view(n, L))])
    assert e.value.status == pc2.PC2_E_INVAL
