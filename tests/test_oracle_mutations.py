"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
of test_oracle_pins catch every one of them."""
from __future__ import annotations

import math

import pytest

import oracle.paillier as O
import oracle.quant as Q
from tests import test_oracle_pins as pins

PINS_CRYPTO = [
    pins.test_golden_hand_worked_example,
    lambda: pins.test_bruteforce_bijection(5, 7),
    lambda: pins.test_bruteforce_homomorphisms(3, 5),
    pins.test_pow_plain_vs_builtin,
    lambda: pins.test_matvec_bruteforce_tiny(3, 5),
]
PINS_QUANT = [
    pins.test_quantize_error_bound_and_aggregate,
    pins.test_quantize_ties_round_half_even,
    pins.test_quantize_range,
    pins.test_quantize_common_interval,
    pins.test_dequantize_rounding_above_2_53,
]


def _agg_identities_64():
    import random as _r
    from workload import gen as _g
    p, q = _g.primes_for(7, 64)
    pk, sk = O.derive_keys(p, q)
    pins._aggregate_identities(pk, sk, _r.Random(5))


PINS_AGG = [
    lambda: pins.test_hom_sum_bruteforce_tiny(3, 5, 3),
    _agg_identities_64,
]


def _caught(checks) -> bool:
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError, ArithmeticError, ZeroDivisionError, LookupError,
                pytest.fail.Exception):  # a pytest.raises block that did not raise
            return True
    return False


def _pow_square_first(base, exp, mod):
    t, g, e = 1 % mod, base % mod, exp
    while e > 0:
        g = (g * g) % mod          # mistake: squares before using the bit
        if e & 1:
            t = (t * g) % mod
        e >>= 1
    return t


def _pow_drop_last(base, exp, mod):
    t, g, e = 1 % mod, base % mod, exp
    while e > 1:                   # mistake: the top bit is never applied
        if e & 1:
            t = (t * g) % mod
        g = (g * g) % mod
        e >>= 1
    return t


def _enc_g_is_n(pk, m, r):
    n2 = pk.n2
    return (O.pow_plain(pk.n, m, n2) * O.pow_plain(r, pk.n, n2)) % n2  # mistake: g = n


def _enc_r_exp_m(pk, m, r):
    n2 = pk.n2
    return (O.pow_plain(pk.g, m, n2) * O.pow_plain(r, m, n2)) % n2  # mistake: r^m


def _L_no_division(x, n):
    return x - 1  # mistake: forgets the division by n


def _add_is_sum(pk, c1, c2):
    return (c1 + c2) % pk.n2  # mistake: + instead of *


def _smul_off_by_one(pk, c, k):
    return O.pow_plain(c, k + 1, pk.n2)  # mistake: wrong exponent


def _derive_phi_and_wrong_mu(p, q):
    pk, sk = ORIG_DERIVE(p, q)
    lam = (p - 1) * (q - 1)        # mistake: phi instead of lcm (and mu not recomputed)
    return pk, O.SecretKey(p=p, q=q, n=sk.n, lam=lam, mu=sk.mu)


ORIG_DERIVE = O.derive_keys


def _matvec_transposed(pk, B, cs, alpha=None):
    n2 = pk.n2
    out = []
    for i, row in enumerate(B):
        acc = 1 if alpha is None else alpha[i]
        for j, cj in enumerate(cs):
            acc = (acc * O.pow_plain(cj, B[j][i], n2)) % n2  # mistake: B transposed
        out.append(acc)
    return out


def _matvec_no_alpha(pk, B, cs, alpha=None):
    n2 = pk.n2
    out = []
    for row in B:
        acc = 1                                             # mistake: alpha dropped
        for bij, cj in zip(row, cs):
            acc = (acc * O.pow_plain(cj, bij, n2)) % n2
        out.append(acc)
    return out


def _matvec_skip_first(pk, B, cs, alpha=None):
    n2 = pk.n2
    out = []
    for i, row in enumerate(B):
        acc = 1 if alpha is None else alpha[i]
        for bij, cj in list(zip(row, cs))[1:]:             # mistake: column 0 skipped
            acc = (acc * O.pow_plain(cj, bij, n2)) % n2
        out.append(acc)
    return out


@pytest.mark.parametrize("name,target,mutant", [
    ("pow square-first", "pow_plain", _pow_square_first),
    ("pow drops top bit", "pow_plain", _pow_drop_last),
    ("g = n", "encrypt", _enc_g_is_n),
    ("r^m", "encrypt", _enc_r_exp_m),
    ("L without division", "L", _L_no_division),
    ("add as sum", "hom_add", _add_is_sum),
    ("scalar k+1", "hom_scalar_mul", _smul_off_by_one),
    ("phi for lcm", "derive_keys", _derive_phi_and_wrong_mu),
    ("mat-vec transposed", "hom_matvec", _matvec_transposed),
    ("mat-vec drops alpha", "hom_matvec", _matvec_no_alpha),
    ("mat-vec skips a column", "hom_matvec", _matvec_skip_first),
])
def test_crypto_mutants_caught(monkeypatch, name, target, mutant):
    monkeypatch.setattr(O, target, mutant)
    assert _caught(PINS_CRYPTO), f"mutant '{name}' survived the pins"


def _q_floor(x, k, o, dl):
    v = math.floor(math.ldexp(x, k))  # mistake: floor instead of round-half-even
    return v + o


def _q_half_up(x, k, o, dl):
    v = math.floor(math.ldexp(x, k) + 0.5)  # mistake: ties away from even
    return v + o


def _q_checks_result(x, k, o, dl):
    if not math.isfinite(x):
        raise ValueError("non-finite input")
    m = round(math.ldexp(x, k)) + o
    if not (0 <= m <= dl):            # mistake: the rounded result is checked, not x
        raise ValueError("out of range")
    return m


def _q_closed_top(x, k, o, dl):
    if not math.isfinite(x):
        raise ValueError("non-finite input")
    t = math.ldexp(x, k)
    if not (-o <= t <= dl - o):       # mistake: z_max itself accepted
        raise ValueError("out of range")
    return round(t) + o


def _q_no_interval(x, k, o, dl):
    if not math.isfinite(x):
        raise ValueError("non-finite input")
    m = round(math.ldexp(x, k)) + o   # mistake: only [0, 2^64) is enforced
    if not (0 <= m < 1 << 64):
        raise ValueError("out of range")
    return m


def _dq_no_weight(M, k, o, W):
    return math.ldexp(float(M - o), -k)  # mistake: one offset regardless of W


def _dq_truncating(M, k, o, W):
    d = M - W * o
    return math.ldexp(float(d >> 1 << 1), -k)  # mistake: drops the low bit


@pytest.mark.parametrize("name,target,mutant", [
    ("floor", "quantize", _q_floor),
    ("half up", "quantize", _q_half_up),
    ("result checked, not x", "quantize", _q_checks_result),
    ("closed top", "quantize", _q_closed_top),
    ("no interval", "quantize", _q_no_interval),
    ("no weight", "dequantize", _dq_no_weight),
    ("truncating", "dequantize", _dq_truncating),
])
def test_quant_mutants_caught(monkeypatch, name, target, mutant):
    monkeypatch.setattr(Q, target, mutant)
    assert _caught(PINS_QUANT), f"mutant '{name}' survived the pins"


# ------------------------------------------------------- K-way aggregation
def _sum_no_reduction(pk, cs):
    acc = 1
    for c in cs:
        acc = acc * c                  # mistake: the product is never reduced mod n^2
    return acc


def _sum_starts_at_zero(pk, cs):
    acc = 0                            # mistake: empty product taken as 0
    for c in cs:
        acc = (acc * c) % pk.n2
    return acc


def _sum_skips_first(pk, cs):
    acc = 1
    for c in list(cs)[1:]:             # mistake: the first addend is skipped
        acc = (acc * c) % pk.n2
    return acc


def _sum_skips_last(pk, cs):
    acc = 1
    for c in list(cs)[:-1] or list(cs):  # mistake: the last addend is skipped (K > 1)
        acc = (acc * c) % pk.n2
    return acc


def _sum_mod_n(pk, cs):
    acc = 1
    for c in cs:
        acc = (acc * c) % pk.n         # mistake: reduced mod n instead of n^2
    return acc


def _sum_vec_first_element(pk, cvs):
    return [O.hom_sum(pk, (cv[0] for cv in cvs)) for _ in range(len(cvs[0]))]  # mistake: index


def _sum_vec_transposed(pk, cvs):
    K, J = len(cvs), len(cvs[0])       # mistake: element j combines row j of every vector
    return [O.hom_sum(pk, (cvs[min(j, K - 1)][k] for k in range(J))) for j in range(J)]


def _esd_first_only(sk, ms, rs):
    pk = sk.public                     # mistake: only the first contribution is decrypted
    return O.decrypt(sk, O.encrypt(pk, ms[0], rs[0]))


def _esd_plain_sum(sk, ms, rs):
    return sum(ms)                     # mistake: no reduction mod n


@pytest.mark.parametrize("name,target,mutant", [
    ("sum without reduction", "hom_sum", _sum_no_reduction),
    ("sum starts at 0", "hom_sum", _sum_starts_at_zero),
    ("sum skips the first addend", "hom_sum", _sum_skips_first),
    ("sum skips the last addend", "hom_sum", _sum_skips_last),
    ("sum mod n", "hom_sum", _sum_mod_n),
    ("vector sum indexes element 0", "hom_sum_vec", _sum_vec_first_element),
    ("vector sum transposed", "hom_sum_vec", _sum_vec_transposed),
    ("fused keeps one contribution", "enc_sum_dec", _esd_first_only),
    ("fused sum not reduced", "enc_sum_dec", _esd_plain_sum),
])
def test_aggregation_mutants_caught(monkeypatch, name, target, mutant):
    monkeypatch.setattr(O, target, mutant)
    assert _caught(PINS_AGG), f"mutant '{name}' survived the pins"


# ------------------------------------------------- column-split ADMM oracle
import numpy as np  # noqa: E402

import oracle.colsplit as CS  # noqa: E402
from tests import test_oracle_colsplit as cpins  # noqa: E402

PINS_COLSPLIT = [
    cpins.test_gram_and_gauss_jordan_against_lapack,
    cpins.test_single_node_converges_to_least_squares,
    lambda: cpins.test_master_update_is_the_soft_threshold_prox(2.5, 0.3),
    lambda: cpins.test_quantized_node_within_theorem_bound(30),
    cpins.test_inverse_quantization_expands_to_centered_sums,
]


def _dq_single_row_terms(self, kk, P, W):
    k, Nk = self.k, self.Nk
    o, o1 = 1 << (k + 3), 1 << (2 * k + 3)
    S = sum(W)
    # mistake: the paper's N = 1 cross terms (2 N o^2 written as 2 o^2)
    return np.array([math.ldexp(float(P[i] - o1 - 2 * o * self.R[kk][i] - o * S + 2 * o * o),
                                -2 * k) for i in range(Nk)])


def _dq_sign(self, kk, P, W):
    k, Nk = self.k, self.Nk
    o, o1 = 1 << (k + 3), 1 << (2 * k + 3)
    S = sum(W)
    # mistake: + o S
    return np.array([math.ldexp(float(P[i] - o1 - 2 * o * self.R[kk][i] + o * S
                                      + 2 * Nk * o * o), -2 * k) for i in range(Nk)])


def _iterate_lambda_unscaled(self, z, v, lam, quantized):
    x = np.empty(self.N)
    for kk in range(self.K):
        x[kk * self.Nk:(kk + 1) * self.Nk] = self.node_plain(kk, z, v)
    t = v + x
    zn = CS.soft_threshold(t, lam)       # mistake: threshold lambda, not lambda / rho
    return x, zn, t - zn


def _gj_no_scaling(G):
    Nk = G.shape[0]
    T = np.hstack([G, np.eye(Nk)])
    for p in range(Nk):
        rp = T[p].copy()                   # mistake: the pivot row is not divided
        f = T[:, p].copy() / T[p, p]
        T -= np.outer(f, rp)
        T[p] = rp
    return T[:, Nk:].copy()


def _gamma2_wrong_offset(u, k):
    return np.rint(np.ldexp(u, k)).astype(np.int64) + np.int64(1 << (k + 2))  # mistake: o / 2


@pytest.mark.parametrize("name,target,mutant", [
    ("N = 1 cross terms", ("ColumnSplitLasso", "dequantize"), _dq_single_row_terms),
    ("sign of o S", ("ColumnSplitLasso", "dequantize"), _dq_sign),
    ("threshold lambda", ("ColumnSplitLasso", "iterate"), _iterate_lambda_unscaled),
    ("unscaled pivot row", ("gauss_jordan_inverse",), _gj_no_scaling),
    ("offset o / 2", ("gamma2",), _gamma2_wrong_offset),
])
def test_colsplit_mutants_caught(monkeypatch, name, target, mutant):
    if len(target) == 2:
        monkeypatch.setattr(getattr(CS, target[0]), target[1], mutant)
    else:
        monkeypatch.setattr(CS, target[0], mutant)
    assert _caught(PINS_COLSPLIT), f"mutant '{name}' survived the pins"
