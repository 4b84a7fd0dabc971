"""Pins of the ADMM oracle (CPU): least squares at lambda = 0, scikit-learn's
Lasso for one node, the Woodbury x-update against a direct solve, the soft
threshold's closed form, and the quantized aggregate against the float sum."""
from __future__ import annotations

import numpy as np
import pytest

from oracle.admm import ConsensusLasso, quantize_exact, soft_threshold


def problem(M, N, seed=0, sparse=0.2):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, N)) / np.sqrt(M)
    xs = np.where(rng.random(N) < sparse, rng.standard_normal(N), 0.0)
    y = A @ xs + 1e-3 * rng.standard_normal(M)
    return A, y, xs


def run(cl, iters, quant=None):
    z = np.zeros(cl.N)
    u = np.zeros((cl.K, cl.N))
    for _ in range(iters):
        _, z, u, _ = cl.step(z, u, quant)
    return z


def test_soft_threshold():
    a = np.array([-3.0, -0.5, 0.0, 0.5, 2.0])
    assert np.array_equal(soft_threshold(a, 1.0), np.array([-2.0, 0.0, 0.0, 0.0, 1.0]))


def test_lambda_zero_reaches_least_squares():
    A, y, _ = problem(64, 8)
    cl = ConsensusLasso(A, y, K=4, rho=1.0, lam=0.0)
    z = run(cl, 400)
    ls, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert np.allclose(z, ls, atol=1e-9)


def test_single_node_matches_sklearn_lasso():
    sk = pytest.importorskip("sklearn.linear_model")
    A, y, _ = problem(80, 20, seed=1)
    lam = 0.05
    cl = ConsensusLasso(A, y, K=1, rho=1.0, lam=lam)
    z = run(cl, 3000)
    # sklearn minimises 1/(2M) ||y - Ax||^2 + alpha ||x||_1
    ref = sk.Lasso(alpha=lam / A.shape[0], fit_intercept=False, tol=1e-14,
                   max_iter=1_000_000).fit(A, y).coef_
    assert np.allclose(z, ref, atol=1e-7)


def test_woodbury_local_update_equals_direct_solve():
    A, y, _ = problem(24, 20, seed=2)
    cl = ConsensusLasso(A, y, K=3, rho=0.7, lam=0.1)
    rng = np.random.default_rng(3)
    z, u = rng.standard_normal(20), rng.standard_normal((3, 20))
    x = cl.local(z, u)
    for k in range(3):
        Ak, yk = cl.A[k], cl.y[k]
        direct = np.linalg.solve(Ak.T @ Ak + 0.7 * np.eye(20), Ak.T @ yk + 0.7 * (z - u[k]))
        assert np.allclose(x[k], direct, rtol=1e-12, atol=1e-12)


def test_quantized_aggregate_close_to_float_sum():
    A, y, _ = problem(64, 32, seed=4)
    cl = ConsensusLasso(A, y, K=8, rho=1.0, lam=0.05)
    k, o = 44, 1 << 51
    z = np.zeros(32)
    u = np.zeros((8, 32))
    _, zq, _, tq = cl.step(z, u, (k, o))
    _, zf, _, tf = cl.step(z, u, None)
    # each addend is rounded once to a multiple of 2^-44
    assert np.max(np.abs(tq - tf)) <= 8 * 2.0 ** -45 + 1e-15
    assert np.max(np.abs(zq - zf)) <= 2.0 ** -44


def test_quantize_exact_range():
    with pytest.raises(ValueError):
        quantize_exact(np.array([np.nan]), 44, 1 << 51)
    with pytest.raises(ValueError):
        quantize_exact(np.array([-1000.0]), 44, 1 << 51)
    assert quantize_exact(np.array([0.0, 1.0]), 4, 16).tolist() == [16, 32]
