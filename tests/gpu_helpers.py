"""Test-side helpers: run libpc2 calls on Python-int inputs and read results back."""
from __future__ import annotations

import numpy as np
import torch

from workload.limbs import ints_from_limbs, to_limbs


def dev(arr: np.ndarray) -> torch.Tensor:
    from paper_2601_14980_amd import pc2
    return pc2.to_device_limbs(arr)


def host_ints(t: torch.Tensor) -> list[int]:
    from paper_2601_14980_amd import pc2
    return ints_from_limbs(pc2.from_device_limbs(t))


def gpu_encrypt(ctx, pk, ms, rs, m_limbs=None):
    from paper_2601_14980_amd import pc2
    L = pk.L
    m_limbs = m_limbs or L
    m = dev(to_limbs(ms, m_limbs))
    r = dev(to_limbs(rs, L))
    c = torch.zeros((len(ms), 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_encrypt(pk, m, r, c)
    st = ctx.sync()
    return host_ints(c), st


def gpu_decrypt(ctx, sk, cs):
    from paper_2601_14980_amd import pc2
    L = sk.L
    c = dev(to_limbs(cs, 2 * L))
    m = torch.zeros((len(cs), L), dtype=torch.int32, device="cuda")
    pc2.pc2_decrypt(sk, c, m)
    st = ctx.sync()
    return host_ints(m), st


def gpu_hom_sum(ctx, pk, cvs):
    from paper_2601_14980_amd import pc2
    L = pk.L
    ts = [dev(to_limbs(cv, 2 * L)) for cv in cvs]
    out = torch.zeros((len(cvs[0]), 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_hom_sum(pk, ts, out)
    st = ctx.sync()
    return host_ints(out), st


def gpu_hom_add(ctx, pk, c1, c2):
    from paper_2601_14980_amd import pc2
    L = pk.L
    a, b = dev(to_limbs(c1, 2 * L)), dev(to_limbs(c2, 2 * L))
    out = torch.zeros((len(c1), 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_hom_add(pk, a, b, out)
    st = ctx.sync()
    return host_ints(out), st


def gpu_scalar_mul(ctx, pk, cs, ks):
    from paper_2601_14980_amd import pc2
    L = pk.L
    c = dev(to_limbs(cs, 2 * L))
    k = torch.from_numpy(np.array(ks, dtype=np.uint64).view(np.int64)).cuda()
    out = torch.zeros((len(cs), 2 * L), dtype=torch.int32, device="cuda")
    pc2.pc2_hom_scalar_mul(pk, c, k, out)
    st = ctx.sync()
    return host_ints(out), st


def gpu_enc_sum_dec(ctx, sk, mvs, rvs, m_limbs=None):
    from paper_2601_14980_amd import pc2
    L = sk.L
    m_limbs = m_limbs or L
    ms = [dev(to_limbs(mv, m_limbs)) for mv in mvs]
    rs = [dev(to_limbs(rv, L)) for rv in rvs]
    out = torch.zeros((len(mvs[0]), L), dtype=torch.int32, device="cuda")
    pc2.pc2_enc_sum_dec(sk, ms, rs, out)
    st = ctx.sync()
    return host_ints(out), st
