"""Column-split 3P-ADMM-PC2 (Algorithm 1) in float64 and exact integers.

Test infrastructure only (see the package docstring).

Sec. II splits the lasso matrix by COLUMNS, A = (A_1, ..., A_K), and iterates
(eqs. (sldi231), (sldo34), (iu43))

    node k:  x_k = (A_k^T A_k + rho I)^-1 (A_k^T y + rho (z_k - v_k))
    master:  z   = S_{lambda/rho}(v + x),      v = v + x - z,

with x = (x_1; ...; x_K).  Algorithm 1 runs the node step on ciphertexts: the
node keeps B_k = (A_k^T A_k + rho I)^-1 (initialisation phase) and the
quantized matrix Gamma_2(rho B_k); the master sends alpha_k =
Enc(Gamma_1(B_k A_k^T y)) once and Enc(Gamma_2(z_k)), Enc(Gamma_2(-v_k)) every
iteration; the node returns alpha_k (+) Gamma_2(rho B_k) (x) (z_k (+) -v_k)
(eq. (itq2)); the master decrypts it and inverts the quantization.

Quantizers (the affine, power-of-two reading of Sec. III-A used throughout,
on the common interval [-8, 8)):

    Gamma_2(u) = rint(u 2^k) + o,        o  = 2^(k+3)
    Gamma_1(u) = rint(u 2^(2k)) + o1,    o1 = 2^(2k+3)

The decrypted node result is, exactly (no wrap mod n),

    P_i = Gamma_1(alpha)_i + sum_j G_ij W_j,   G = Gamma_2(rho B_k),
                                               W = Gamma_2(z_k) + Gamma_2(-v_k).

Inverse quantization for a row of N_k terms (the N > 1 form of Theorem 1's
cross terms, with R_i = sum_j G_ij and S = sum_j W_j):

    X_i = P_i - o1 - 2 o R_i - o S + 2 N_k o^2
        = rint(alpha_i 2^(2k)) + sum_j (G_ij - o)(W_j - 2 o),
    x_i = float64(X_i) 2^(-2k)            (one rounding, to nearest even).

The master knows R_i because the node returns B_k in the initialisation
phase and the quantization is deterministic.

Every floating-point step is written in a fixed order so that it can be
compared with the device bit for bit: the Gram matrix sums over the rows of
A in ascending order, B_k comes from Gauss-Jordan elimination without
pivoting on [A_k^T A_k + rho I | I] (the matrix is symmetric positive
definite), and matrix-vector products sum over the columns in ascending order.
"""
from __future__ import annotations

import math

import numpy as np

ZMAX_LOG2 = 3   # the common quantization interval is [-2^3, 2^3)


def soft_threshold(a: np.ndarray, kappa: float) -> np.ndarray:
    """S_kappa(a) = sign(a) max(|a| - kappa, 0)."""
    return np.sign(a) * np.maximum(np.abs(a) - kappa, 0.0)


def gram(Ak: np.ndarray, rho: float) -> np.ndarray:
    """A_k^T A_k + rho I, summing the rows of A_k in ascending order."""
    M, Nk = Ak.shape
    G = np.zeros((Nk, Nk))
    for m in range(M):
        G += np.outer(Ak[m], Ak[m])
    G[np.diag_indices(Nk)] += rho
    return G


def gauss_jordan_inverse(G: np.ndarray) -> np.ndarray:
    """G^-1 by Gauss-Jordan elimination on [G | I], pivots in order, no row
    exchanges: the pivot row is divided by its pivot, then every other row
    subtracts (its entry in the pivot column) x (the scaled pivot row)."""
    Nk = G.shape[0]
    T = np.hstack([G, np.eye(Nk)])
    for p in range(Nk):
        rp = T[p] / T[p, p]
        f = T[:, p].copy()
        T -= np.outer(f, rp)
        T[p] = rp
    return T[:, Nk:].copy()


def matvec_ordered(Bm: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Bm x summing over the columns in ascending order."""
    acc = np.zeros(Bm.shape[0])
    for j in range(Bm.shape[1]):
        acc += Bm[:, j] * x[j]
    return acc


def aty_ordered(Ak: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A_k^T y summing over the rows in ascending order."""
    acc = np.zeros(Ak.shape[1])
    for m in range(Ak.shape[0]):
        acc += Ak[m] * y[m]
    return acc


def gamma2(u: np.ndarray, k: int) -> np.ndarray:
    """Gamma_2 as exact int64: rint(u 2^k) + 2^(k+3); u must lie in [-8, 8)."""
    if np.any(u < -(2.0 ** ZMAX_LOG2)) or np.any(u >= 2.0 ** ZMAX_LOG2):
        raise ValueError("value outside the quantization interval")
    return np.rint(np.ldexp(u, k)).astype(np.int64) + np.int64(1 << (k + ZMAX_LOG2))


def gamma1(u: float, k: int) -> int:
    """Gamma_1 as an exact integer: rint(u 2^(2k)) + 2^(2k+3)."""
    if not (-(2.0 ** ZMAX_LOG2) <= u < 2.0 ** ZMAX_LOG2):
        raise ValueError("value outside the quantization interval")
    return int(round(math.ldexp(u, 2 * k))) + (1 << (2 * k + ZMAX_LOG2))


class ColumnSplitLasso:
    """Algorithm 1 on one process: the plain float64 iteration (quantized =
    False) and the quantized one, whose homomorphic node step is evaluated by
    its exact plaintext equivalent (the ciphertext operations are pinned
    separately)."""

    def __init__(self, A: np.ndarray, y: np.ndarray, K: int, rho: float, k: int):
        M, N = A.shape
        if N % K:
            raise ValueError("columns must split evenly over the nodes")
        Nk = N // K
        self.K, self.N, self.Nk, self.rho, self.k = K, N, Nk, rho, k
        self.B, self.rhoB, self.alpha, self.G, self.R, self.g1 = [], [], [], [], [], []
        for kk in range(K):
            Ak = A[:, kk * Nk:(kk + 1) * Nk]
            Bk = gauss_jordan_inverse(gram(Ak, rho))
            rhoB = rho * Bk
            alpha = matvec_ordered(Bk, aty_ordered(Ak, y))
            G = gamma2(rhoB, k)
            self.B.append(Bk)
            self.rhoB.append(rhoB)
            self.alpha.append(alpha)
            self.G.append(G)
            self.R.append([int(r) for r in G.sum(axis=1, dtype=np.int64)])
            self.g1.append([gamma1(float(a), k) for a in alpha])

    def node_plain(self, kk: int, z: np.ndarray, v: np.ndarray) -> np.ndarray:
        """x_k = alpha_k + (rho B_k)(z_k - v_k) in float64."""
        sl = slice(kk * self.Nk, (kk + 1) * self.Nk)
        return self.alpha[kk] + matvec_ordered(self.rhoB[kk], z[sl] - v[sl])

    def node_plaintext(self, kk: int, z: np.ndarray, v: np.ndarray) -> tuple[list, list]:
        """P = Gamma_1(alpha_k) + Gamma_2(rho B_k) (Gamma_2(z_k) + Gamma_2(-v_k)),
        the plaintext of the node's returned ciphertext vector (eq. (itq2)), and W."""
        sl = slice(kk * self.Nk, (kk + 1) * self.Nk)
        W = [int(a) + int(b) for a, b in zip(gamma2(z[sl], self.k), gamma2(-v[sl], self.k))]
        G = self.G[kk]
        return [self.g1[kk][i] + sum(int(G[i, j]) * W[j] for j in range(self.Nk))
                for i in range(self.Nk)], W

    def dequantize(self, kk: int, P: list[int], W: list[int]) -> np.ndarray:
        """x_i = float64(P_i - o1 - 2 o R_i - o S + 2 N_k o^2) 2^(-2k)."""
        k, Nk = self.k, self.Nk
        o, o1 = 1 << (k + ZMAX_LOG2), 1 << (2 * k + ZMAX_LOG2)
        S = sum(W)
        out = np.empty(Nk)
        for i in range(Nk):
            X = P[i] - o1 - 2 * o * self.R[kk][i] - o * S + 2 * Nk * o * o
            out[i] = math.ldexp(float(X), -2 * k)
        return out

    def iterate(self, z: np.ndarray, v: np.ndarray, lam: float, quantized: bool):
        """One iteration: every node's x_k, then z = S_{lambda/rho}(v + x),
        v = v + x - z.  Returns (x, z, v)."""
        x = np.empty(self.N)
        for kk in range(self.K):
            sl = slice(kk * self.Nk, (kk + 1) * self.Nk)
            if quantized:
                P, W = self.node_plaintext(kk, z, v)
                x[sl] = self.dequantize(kk, P, W)
            else:
                x[sl] = self.node_plain(kk, z, v)
        t = v + x
        z_new = soft_threshold(t, lam / self.rho)
        v_new = t - z_new
        return x, z_new, v_new
