"""Consensus-lasso ADMM in float64, the update the master runs around the
encrypted aggregation.  Test infrastructure only.

Sec. II states the lasso problem, its ADMM iterates (x-update with
(A^T A + rho I)^-1, z = S_{lambda/rho}(v + x), v += x - z with v = u/rho) and
the split of the work over K nodes.  With A split by ROWS over K nodes (each
node k holds A_k, y_k), the same iteration in global-consensus form is

    node k:  x_k = argmin 1/2 ||A_k x - y_k||^2 + rho/2 ||x - z + u_k||^2
                 = (A_k^T A_k + rho I)^-1 (A_k^T y_k + rho (z - u_k))
    master:  z   = S_{lambda/(rho K)}( (1/K) sum_k (x_k + u_k) )
    node k:  u_k = u_k + x_k - z

The x-update is evaluated with the Woodbury identity
(A_k^T A_k + rho I)^-1 w = (w - A_k^T (rho I + A_k A_k^T)^-1 A_k w) / rho,
which replaces an N x N solve by a B x B one (B rows per node).  In the
encrypted protocol the master only sees sum_k (x_k + u_k) through
Dec(prod_k Enc(Gamma_2(x_k + u_k))) = sum_k Gamma_2(x_k + u_k) (exact while
the sum stays below n), dequantized with weight K.
"""
from __future__ import annotations

import numpy as np


def soft_threshold(a: np.ndarray, kappa: float) -> np.ndarray:
    """S_kappa(a) = sign(a) max(|a| - kappa, 0)."""
    return np.sign(a) * np.maximum(np.abs(a) - kappa, 0.0)


def quantize_exact(x: np.ndarray, log2_scale: int, offset: int) -> np.ndarray:
    """Gamma_2 in affine form, element-wise, as exact int64 (values must stay
    below 2^62 so that sums of a few dozen are exact)."""
    v = np.rint(np.ldexp(x, log2_scale))          # exact: power-of-two scale
    if not np.all(np.isfinite(v)) or np.any(np.abs(v) >= 2.0 ** 62):
        raise ValueError("value outside the quantizer's range")
    m = v.astype(np.int64) + np.int64(offset)
    if np.any(m < 0):
        raise ValueError("quantized value below 0")
    return m


class ConsensusLasso:
    def __init__(self, A: np.ndarray, y: np.ndarray, K: int, rho: float, lam: float):
        M, N = A.shape
        if M % K:
            raise ValueError("rows must split evenly over the nodes")
        B = M // K
        self.K, self.N, self.B, self.rho, self.lam = K, N, B, rho, lam
        self.A = [A[k * B:(k + 1) * B] for k in range(K)]
        self.y = [y[k * B:(k + 1) * B] for k in range(K)]
        self.W = [rho * np.eye(B) + Ak @ Ak.T for Ak in self.A]
        self.aty = [Ak.T @ yk for Ak, yk in zip(self.A, self.y)]

    def local(self, z: np.ndarray, u: np.ndarray) -> np.ndarray:
        """x_k for every node (K x N)."""
        x = np.empty((self.K, self.N))
        for k in range(self.K):
            w = self.aty[k] + self.rho * (z - u[k])
            s = np.linalg.solve(self.W[k], self.A[k] @ w)
            x[k] = (w - self.A[k].T @ s) / self.rho
        return x

    def consensus(self, total: np.ndarray, x: np.ndarray, u: np.ndarray):
        z = soft_threshold(total / self.K, self.lam / (self.rho * self.K))
        return z, u + x - z

    def step(self, z, u, quant: tuple[int, int] | None = None):
        """One iteration.  quant = (log2_scale, offset): the master's total is
        the dequantized exact sum of the nodes' quantized x_k + u_k (what the
        encrypted aggregation delivers); None: the float64 sum."""
        x = self.local(z, u)
        xu = x + u
        if quant is None:
            total = xu.sum(axis=0)
        else:
            k, o = quant
            M = sum(quantize_exact(xu[i], k, o) for i in range(self.K))  # exact int64
            total = np.ldexp((M - np.int64(self.K * o)).astype(np.float64), -k)
        z, u = self.consensus(total, x, u)
        return x, z, u, total
