"""Column-split 3P-ADMM-PC2 (Algorithm 1) on one GPU.

A is split by columns over K simulated edge nodes.  At set-up each node's
B_k = (A_k^T A_k + rho I)^-1, the quantized matrix Gamma_2(rho B_k) and the
master's Enc(Gamma_1(B_k A_k^T y)) are computed on the device
(pc2_colsplit_create; pc2_colsplit_set_scale quantizes again at another
scale).  Every iteration (pc2_colsplit_iterate):

    master:  Enc(Gamma_2(z_k)), Enc(Gamma_2(-v_k))          pc2_encrypt
    node k:  alpha_k (+) Gamma_2(rho B_k) (x) (z_k (+) -v_k)   pc2_hom_add, pc2_matvec_*
    master:  Dec, inverse quantization (N > 1 cross terms)   pc2_decrypt + a float64 kernel
    master:  z = S_{lambda/rho}(v + x), v = v + x - z        a float64 kernel

Every step runs in libpc2's kernels; this module only allocates tensors and
calls the library.  The randomness comes from a caller-provided pool that the
iterations walk through cyclically (a benchmark simplification: the work of an
encryption does not depend on r).
"""
from __future__ import annotations

from ctypes import byref, c_void_p

import torch

from . import pc2

_lib = pc2.lib


class ColumnSplitLasso:
    def __init__(self, ctx: pc2.Context, sk: pc2.SecretKey, A: torch.Tensor, y: torch.Tensor,
                 K: int, rho: float, log2_scale: int, r_pool: torch.Tensor, stream=None):
        M, N = A.shape
        if y.shape != (M,):
            raise ValueError("y must have one entry per row of A")
        self.ctx, self.sk, self.K, self.N, self.rho = ctx, sk, K, N, rho
        self._keep = (A, y, r_pool)      # the library reads them while it lives
        pc2._rows(r_pool, sk.L, "r_pool")
        h = c_void_p()
        pc2._check(_lib.pc2_colsplit_create(
            sk.handle, pc2._dev_ptr(A, torch.float64, "A"), pc2._dev_ptr(y, torch.float64, "y"),
            M, N, K, rho, log2_scale, pc2._dev_ptr(r_pool, torch.int32, "r_pool"),
            r_pool.shape[0], pc2._stream(stream), byref(h)), "pc2_colsplit_create")
        self.handle = h
        dev = A.device
        self.x = torch.zeros(N, dtype=torch.float64, device=dev)
        self.z = torch.zeros(N, dtype=torch.float64, device=dev)
        self.v = torch.zeros(N, dtype=torch.float64, device=dev)

    def set_scale(self, log2_scale: int, stream=None) -> None:
        """Quantize again at scale 2^log2_scale (the float64 setup is kept)."""
        pc2._check(_lib.pc2_colsplit_set_scale(self.handle, log2_scale, pc2._stream(stream)),
                   "pc2_colsplit_set_scale")

    def iterate(self, lam: float, quantized: bool = True, stream=None) -> None:
        pc2._check(_lib.pc2_colsplit_iterate(
            self.handle, lam, 1 if quantized else 0, pc2._dev_ptr(self.x, torch.float64, "x"),
            pc2._dev_ptr(self.z, torch.float64, "z"), pc2._dev_ptr(self.v, torch.float64, "v"),
            pc2._stream(stream)), "pc2_colsplit_iterate")

    def close(self) -> None:
        if self.handle:
            _lib.pc2_colsplit_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
