"""Privacy-preserving consensus-lasso driver on one GPU.

K simulated nodes each hold a block of rows of A.  Every iteration:

    node k (FP64 kernels):  x_k, and xu_k = x_k + u_k          pc2_admm_local
    node k:                 m_k = Gamma_2(xu_k)                  pc2_quantize
    node k:                 c_k = Enc(m_k)                       pc2_encrypt (one launch, all nodes)
    master:                 C = prod_k c_k mod n^2               pc2_hom_sum
    master:                 M = Dec(C)                           pc2_decrypt
    master:                 sum = (M - K o) / 2^s                pc2_dequantize
    master:                 z, u_k update                        pc2_admm_consensus

Every step runs in libpc2's kernels; this module only allocates tensors and
sequences the calls.  The encryption randomness is drawn once from a seeded
pool and reused across iterations (a benchmark simplification: the work of
an encryption does not depend on r; a deployment draws a fresh r per
encryption).
"""
from __future__ import annotations

from ctypes import byref, c_void_p

import torch

from . import pc2

_lib = pc2.lib


def _f64(t: torch.Tensor, what: str) -> int:
    return pc2._dev_ptr(t, torch.float64, what)


class EncryptedConsensusLasso:
    def __init__(self, ctx: pc2.Context, sk: pc2.SecretKey, A: torch.Tensor, y: torch.Tensor,
                 K: int, rho: float, lam: float, log2_scale: int, offset: int, delta: int,
                 r_pool: torch.Tensor):
        M, N = A.shape
        self.ctx, self.sk, self.K, self.N = ctx, sk, K, N
        self.rho, self.lam, self.k, self.o, self.delta = rho, lam, log2_scale, offset, delta
        self.A, self.y = A, y
        h = c_void_p()
        pc2._check(_lib.pc2_admm_create(ctx.handle, _f64(A, "A"), _f64(y, "y"), M, N, K, rho,
                                        pc2._stream(None), byref(h)), "pc2_admm_create")
        self.handle = h
        L = sk.L
        dev = A.device
        self.x = torch.empty((K, N), dtype=torch.float64, device=dev)
        self.xu = torch.empty((K, N), dtype=torch.float64, device=dev)
        self.m = torch.empty(K * N, dtype=torch.int64, device=dev)
        self.c = torch.empty((K * N, 2 * L), dtype=torch.int32, device=dev)
        self.agg = torch.empty((N, 2 * L), dtype=torch.int32, device=dev)
        self.msum = torch.empty((N, L), dtype=torch.int32, device=dev)
        self.total = torch.empty(N, dtype=torch.float64, device=dev)
        if r_pool.shape != (K * N, L):
            raise ValueError("r_pool must be [K*N, L]")
        self.r = r_pool
        self.parts = [self.c[i * N:(i + 1) * N] for i in range(K)]

    def close(self):
        if self.handle:
            _lib.pc2_admm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def local(self, z: torch.Tensor, u: torch.Tensor) -> None:
        pc2._check(_lib.pc2_admm_local(self.handle, _f64(z, "z"), _f64(u, "u"), _f64(self.x, "x"),
                                       _f64(self.xu, "xu"), pc2._stream(None)), "pc2_admm_local")

    def aggregate(self) -> None:
        """total = sum_k x_k + u_k through quantize -> encrypt -> product -> decrypt."""
        K, N = self.K, self.N
        pc2.pc2_quantize(self.ctx, self.k, self.o, self.delta, self.xu.reshape(-1), self.m)
        pc2.pc2_encrypt(self.sk.public, self.m.view(torch.int32).reshape(K * N, 2), self.r, self.c)
        pc2.pc2_hom_sum(self.sk.public, self.parts, self.agg)
        pc2.pc2_decrypt(self.sk, self.agg, self.msum)
        pc2.pc2_dequantize(self.ctx, self.k, self.o, self.msum, K, self.total)

    def consensus(self, z: torch.Tensor, u: torch.Tensor) -> None:
        pc2._check(_lib.pc2_admm_consensus(self.handle, _f64(self.total, "total"),
                                           _f64(self.x, "x"), self.lam, _f64(z, "z"),
                                           _f64(u, "u"), pc2._stream(None)), "pc2_admm_consensus")

    def step(self, z: torch.Tensor, u: torch.Tensor) -> None:
        self.local(z, u)
        self.aggregate()
        self.consensus(z, u)
