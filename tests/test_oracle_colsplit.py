"""Pins of the column-split ADMM oracle (oracle/colsplit.py) against facts
that do not come from it: LAPACK's inverse, least squares, the optimality
conditions of the soft threshold, the quantization error bound of Theorem 1
(in its N > 1 form), and the plain expansion of the inverse quantization."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import colsplit as C


def _data(M, N, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    x = np.zeros(N)
    x[rng.choice(N, size=max(1, N // 20), replace=False)] = rng.standard_normal(max(1, N // 20))
    y = A @ x + 1e-3 * rng.standard_normal(M)
    return A, y


def test_gram_and_gauss_jordan_against_lapack():
    A, _ = _data(50, 30, 1)
    G = C.gram(A, 1.5)
    assert np.allclose(G, A.T @ A + 1.5 * np.eye(30), rtol=1e-13, atol=1e-13)
    Binv = C.gauss_jordan_inverse(G)
    assert np.allclose(Binv, np.linalg.inv(G), rtol=1e-10, atol=1e-12)
    assert np.allclose(Binv @ G, np.eye(30), atol=1e-12)


def test_single_node_converges_to_least_squares():
    """K = 1, lambda = 0: the iteration is the proximal point method on the
    least-squares objective, whose limit is the lstsq solution."""
    A, y = _data(60, 20, 2)
    cs = C.ColumnSplitLasso(A, y, 1, 1.0, 40)
    z = np.zeros(20)
    v = np.zeros(20)
    for _ in range(400):
        x, z, v = cs.iterate(z, v, 0.0, quantized=False)
    ls = np.linalg.lstsq(A, y, rcond=None)[0]
    assert np.allclose(x, ls, rtol=0, atol=1e-9)
    assert np.allclose(v, 0.0, atol=1e-12)


@pytest.mark.parametrize("rho,lam", [(1.0, 0.05), (2.5, 0.3)])
def test_master_update_is_the_soft_threshold_prox(rho, lam):
    """z minimises lambda |z|_1 + rho/2 ||z - (v + x)||^2: element-wise,
    rho (t - z) = lambda sign(z) where z != 0 and |rho t| <= lambda where z = 0."""
    A, y = _data(40, 24, 3)
    cs = C.ColumnSplitLasso(A, y, 3, rho, 40)
    rng = np.random.default_rng(4)
    z0, v0 = rng.uniform(-1, 1, 24), rng.uniform(-0.2, 0.2, 24)
    x, z, v = cs.iterate(z0, v0, lam, quantized=False)
    t = v0 + x
    nz = z != 0
    assert np.allclose(rho * (t[nz] - z[nz]), lam * np.sign(z[nz]), atol=1e-12)
    assert np.all(np.abs(rho * t[~nz]) <= lam + 1e-12)
    assert np.array_equal(v, t - z)


@pytest.mark.parametrize("k", [12, 20, 30, 44])
def test_quantized_node_within_theorem_bound(k):
    """|x_q - x| <= 1/s^2 + N_k (max|rho B| + max|w|/2) / s + N_k / s^2 +
    |x| 2^-52 with s = 2^k and w = z - v: Theorem 1's error for rint
    quantizers, summed over a row."""
    A, y = _data(48, 36, 5)
    cs = C.ColumnSplitLasso(A, y, 3, 1.0, k)
    rng = np.random.default_rng(k)
    z, v = rng.uniform(-2, 2, 36), rng.uniform(-0.5, 0.5, 36)
    s = 2.0 ** k
    for kk in range(3):
        sl = slice(kk * 12, (kk + 1) * 12)
        xp = cs.node_plain(kk, z, v)
        P, W = cs.node_plaintext(kk, z, v)
        xq = cs.dequantize(kk, P, W)
        w = z[sl] - v[sl]
        bound = (1 / s ** 2 + 12 * (np.max(np.abs(cs.rhoB[kk])) + np.max(np.abs(w)) / 2) / s
                 + 12 / s ** 2 + np.abs(xp) * 2.0 ** -52 + 1e-300)
        assert np.all(np.abs(xq - xp) <= bound)
        if k >= 30:
            assert np.max(np.abs(xq - xp)) < 1e-6


def test_inverse_quantization_expands_to_centered_sums():
    """P - o1 - 2 o R - o S + 2 N o^2 equals rint(alpha 2^2k) +
    sum_j (G_ij - o)(W_j - 2 o), term by term."""
    A, y = _data(30, 18, 6)
    k = 20
    cs = C.ColumnSplitLasso(A, y, 2, 1.0, k)
    rng = np.random.default_rng(7)
    z, v = rng.uniform(-1, 1, 18), rng.uniform(-1, 1, 18)
    o = 1 << (k + 3)
    for kk in range(2):
        P, W = cs.node_plaintext(kk, z, v)
        x = cs.dequantize(kk, P, W)
        for i in range(cs.Nk):
            direct = int(round(math.ldexp(float(cs.alpha[kk][i]), 2 * k))) + sum(
                (int(cs.G[kk][i, j]) - o) * (W[j] - 2 * o) for j in range(cs.Nk))
            assert x[i] == math.ldexp(float(direct), -2 * k)


def test_fixed_order_loop_equals_plain_definition():
    """The oracle's float64 loop (summation in a fixed order, Gauss-Jordan
    without row exchanges, x_k = alpha_k + rho B_k (z_k - v_k) with alpha_k =
    B_k A_k^T y) against the iteration written from its definition with
    LAPACK's solver and numpy's products: x_k = solve(A_k^T A_k + rho I,
    A_k^T y + rho (z_k - v_k)), z = t - clip(t, -lambda/rho, lambda/rho) for
    t = v + x (the soft threshold), v = t - z.  50 iterations, 1e-12 relative
    at every one of them."""
    M, N, K, rho, lam = 150, 120, 3, 1.0, 0.02
    A, y = _data(M, N, 8)
    cs = C.ColumnSplitLasso(A, y, K, rho, 40)
    Nk = N // K
    z, v = np.zeros(N), np.zeros(N)
    zp, vp = np.zeros(N), np.zeros(N)
    for _ in range(50):
        x, z, v = cs.iterate(z, v, lam, quantized=False)
        xp = np.concatenate([
            np.linalg.solve(A[:, k * Nk:(k + 1) * Nk].T @ A[:, k * Nk:(k + 1) * Nk]
                            + rho * np.eye(Nk),
                            A[:, k * Nk:(k + 1) * Nk].T @ y
                            + rho * (zp[k * Nk:(k + 1) * Nk] - vp[k * Nk:(k + 1) * Nk]))
            for k in range(K)])
        t = vp + xp
        zp = t - np.clip(t, -lam / rho, lam / rho)
        vp = t - zp
        for got, want in ((x, xp), (z, zp), (v, vp)):
            assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    assert np.count_nonzero(z) not in (0, N)  # the threshold is active on both sides


def test_quantizer_range():
    with pytest.raises(ValueError):
        C.gamma2(np.array([8.0]), 10)
    with pytest.raises(ValueError):
        C.gamma1(-8.5, 10)
    assert C.gamma2(np.array([-8.0]), 10)[0] == 0
    assert C.gamma1(0.0, 10) == 1 << 23
