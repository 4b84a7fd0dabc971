"""Pins of the oracle against facts that do not come from the oracle itself.

* hand-derived worked example (tests/golden/paillier_n15.txt)
* brute force over every (m, r) of tiny keys: Enc is a bijection
  Z_n x Z*_n -> Z*_{n^2} and Dec inverts it
* ciphertext identities that hold exactly at any size
* the closed form (n+1)^m = 1 + m n (mod n^2)
* CPython's built-in three-argument pow and sympy's primality/inverse
* the CRT route reaching the plain decryption
* Euler/Carmichael: (r^n)^lambda = 1 (mod n^2)
* the quantizer's exact error bound and exact aggregate dequantization, and
  its common interval checked on the input, not on the rounded result
* the K-way aggregation (Definition 1 applied K - 1 times) and the fused
  encrypt -> aggregate -> decrypt: brute force over every K-tuple of tiny
  keys, and the exact identity prod_k Enc(a_k, r_k) = Enc(sum a_k, prod r_k)
  at every key size
* the ciphertext mat-vec decrypting to the integer mat-vec, and its special
  cases (identity and zero matrices, one column against built-in pow)
"""
from __future__ import annotations

import itertools
import math
import random
from pathlib import Path

import numpy as np
import pytest
import sympy

from oracle import paillier as O
from oracle import quant as Q
from workload import gen

GOLDEN = Path(__file__).parent / "golden" / "paillier_n15.txt"
TINY = [(3, 5), (5, 7), (7, 11), (11, 13)]


def _golden_rows():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        op, *kv = line.split()
        vals = {}
        for k, v in (x.split("=") for x in kv):
            vals[k] = [int(t) for t in v.split(",")] if "," in v else int(v)
        rows.append((op, vals))
    return rows


def test_golden_hand_worked_example():
    rows = _golden_rows()
    key = [r for op, r in rows if op == "key"][0]
    pk, sk = O.derive_keys(key["p"], key["q"])
    assert (sk.n, sk.lam, sk.mu) == (key["n"], key["lam"], key["mu"])
    seen = set()
    for op, r in rows:
        seen.add(op)
        if op == "enc":
            assert O.encrypt(pk, r["m"], r["r"]) == r["c"]
        elif op == "dec":
            assert O.decrypt(sk, r["c"]) == r["m"]
        elif op == "add":
            assert O.hom_add(pk, r["c1"], r["c2"]) == r["c"]
        elif op == "smul":
            assert O.hom_scalar_mul(pk, r["c1"], r["k"]) == r["c"]
        elif op == "matvec":
            assert O.hom_matvec(pk, [r["b"]], r["c"], [r["alpha"]]) == [r["out"]]
    assert seen == {"key", "enc", "dec", "add", "smul", "matvec"}


@pytest.mark.parametrize("p,q", TINY)
def test_bruteforce_bijection(p, q):
    pk, sk = O.derive_keys(p, q)
    n, n2 = p * q, (p * q) ** 2
    units = [r for r in range(1, n) if math.gcd(r, n) == 1]
    cs = {}
    for m in range(n):
        for r in units:
            c = O.encrypt(pk, m, r)
            assert 0 < c < n2 and math.gcd(c, n) == 1
            assert c not in cs
            cs[c] = m
            assert O.decrypt(sk, c) == m
    # |Z_n x Z*_n| = n phi(n) = phi(n^2): the image is all of Z*_{n^2}
    phi_n2 = sum(1 for c in range(1, n2) if math.gcd(c, n) == 1)
    assert len(cs) == phi_n2 == n * len(units)


@pytest.mark.parametrize("p,q", TINY[:3])
def test_bruteforce_homomorphisms(p, q):
    pk, sk = O.derive_keys(p, q)
    n = p * q
    rng = random.Random(n)
    units = [r for r in range(1, n) if math.gcd(r, n) == 1]
    for a in range(n):
        ca = O.encrypt(pk, a, rng.choice(units))
        for b in range(n):
            cb = O.encrypt(pk, b, rng.choice(units))
            assert O.decrypt(sk, O.hom_add(pk, ca, cb)) == (a + b) % n
            assert O.decrypt(sk, O.hom_scalar_mul(pk, ca, b)) == (a * b) % n


@pytest.fixture(scope="module", params=[64, 256, 1024, 2048])
def key(request):
    p, q = gen.primes_for(7, request.param)
    pk, sk = O.derive_keys(p, q)
    return p, q, pk, sk


def test_primes_and_key_constants(key):
    p, q, pk, sk = key
    assert sympy.isprime(p) and sympy.isprime(q) and p != q
    assert (p * q).bit_length() == pk.nbits
    assert sk.lam == sympy.ilcm(p - 1, q - 1)
    # mu from the textbook closed form for g = n + 1: L(g^lam mod n^2) = lam mod n
    assert sk.mu == sympy.mod_inverse(sk.lam % pk.n, pk.n)


def test_ciphertext_identities(key):
    """Exact identities, independent of any single modexp being right."""
    p, q, pk, sk = key
    n, n2 = pk.n, pk.n2
    rng = random.Random(n % 1000)
    for _ in range(4):
        a, b = rng.randrange(n), rng.randrange(n)
        r1, r2 = gen.gen_r(n, 2, 7, extra=a % 997)
        k = rng.getrandbits(64)
        ea, eb = O.encrypt(pk, a, r1), O.encrypt(pk, b, r2)
        assert O.hom_add(pk, ea, eb) == O.encrypt(pk, (a + b) % n, (r1 * r2) % n)
        assert O.hom_scalar_mul(pk, ea, k) == O.encrypt(pk, (k * a) % n, pow(r1, k, n))
        assert O.encrypt(pk, a, 1) == (1 + a * n) % n2


def test_closed_form_g_power(key):
    """(n+1)^m = 1 + m n (mod n^2) by the binomial theorem."""
    _, _, pk, _ = key
    n, n2 = pk.n, pk.n2
    rng = random.Random(3)
    for m in [0, 1, 2, n - 1] + [rng.randrange(n) for _ in range(5)]:
        assert O.pow_plain(n + 1, m, n2) == (1 + m * n) % n2


def test_pow_plain_vs_builtin():
    rng = random.Random(11)
    for bits in (8, 64, 512, 2048, 4096):
        N = rng.getrandbits(bits) | 1 | (1 << (bits - 1))
        cases = [(0, 0), (0, 5), (1, rng.getrandbits(bits)), (N - 1, N - 1), (N - 1, 2),
                 ((1 << bits) - 1, (1 << 64) - 1), (N, 3)]
        cases += [(rng.getrandbits(bits), rng.getrandbits(bits)) for _ in range(3)]
        for b, e in cases:
            assert O.pow_plain(b, e, N) == pow(b, e, N)


def test_crt_route_equals_plain(key):
    _, _, pk, sk = key
    n, n2 = pk.n, pk.n2
    rng = random.Random(5)
    for _ in range(4):
        c = rng.randrange(1, n2)
        if math.gcd(c, n) != 1:
            continue
        assert O.decrypt_crt(sk, c) == O.decrypt(sk, c)


def test_euler_carmichael(key):
    """(r^n mod n^2)^lambda = 1 (mod n^2) for r in Z*_n: pins r^n on its own."""
    _, _, pk, sk = key
    for r in gen.gen_r(pk.n, 3, 8):
        rn = O.encrypt(pk, 0, r)  # Enc(0, r) = r^n mod n^2
        assert O.pow_plain(rn, sk.lam, pk.n2) == 1


def test_invariants_and_edges(key):
    _, _, pk, sk = key
    n = pk.n
    rs = gen.gen_r(n, 2, 9)
    for m in (0, 1, n - 1, n // 2):
        for r in (1, n - 1, *rs):
            assert O.decrypt(sk, O.encrypt(pk, m, r)) == m
    with pytest.raises(ValueError):
        O.encrypt(pk, n, 1)
    with pytest.raises(ValueError):
        O.encrypt(pk, 0, 0)
    assert O.hom_scalar_mul(pk, O.encrypt(pk, 5, rs[0]), 0) == 1


# ------------------------------------------------------------ quantization
def test_quantize_error_bound_and_aggregate():
    rng = np.random.default_rng(1)
    k, o, dl = 20, 1 << 23, 1 << 24
    s = 2.0 ** k
    xs = rng.standard_normal((8, 500))
    qs = [Q.quantize_vec(x, k, o, dl) for x in xs]
    for x, qv in zip(xs, qs):
        for xi, mi in zip(x, qv):
            assert abs(xi - Q.dequantize(mi, k, o, 1)) <= 0.5 / s
    # aggregate of K addends: exact sum of the rounded scaled values
    K = len(xs)
    for j in range(xs.shape[1]):
        M = sum(qv[j] for qv in qs)
        exact = sum(round(x[j] * s) for x in xs)  # integers, exact
        assert Q.dequantize(M, k, o, K) == exact / s


def test_quantize_ties_round_half_even():
    k, o = 1, 100
    # x * 2 = 0.5, 1.5, 2.5, -0.5, -1.5 -> 0, 2, 2, -0, -2
    assert [Q.quantize(x, k, o, 200) for x in (0.25, 0.75, 1.25, -0.25, -0.75)] == \
        [100, 102, 102, 100, 98]


def test_quantize_range():
    top = (1 << 64) - 1
    with pytest.raises(ValueError):
        Q.quantize(float("nan"), 10, 0, top)
    with pytest.raises(ValueError):
        Q.quantize(float("inf"), 10, 0, top)
    with pytest.raises(ValueError):
        Q.quantize(-1.0, 10, 5, top)
    with pytest.raises(ValueError):
        Q.quantize(2.0 ** 60, 10, 0, top)
    with pytest.raises(ValueError):
        Q.quantize(0.0, 0, 9, 8)  # offset above delta
    assert Q.quantize(-1.0, 10, 1024, 2048) == 0
    assert Q.quantize(0.0, 0, top - 1, top) == top - 1


def test_quantize_common_interval():
    """Sec. III-A maps [z_min, z_max] onto {0, ..., Delta}; with s = 2, o = 4,
    Delta = 8 the interval is [-2, 2): its ends, values that round back into
    it, and the largest value below z_max, which rounds to Delta itself."""
    k, o, dl = 1, 4, 8
    assert Q.quantize(-2.0, k, o, dl) == 0                  # z_min is in
    assert Q.quantize(1.75, k, o, dl) == 8                  # 3.5 rounds (to even) to 4: Delta
    assert Q.quantize(1.25, k, o, dl) == 6                  # 2.5 -> 2
    assert Q.quantize(math.nextafter(2.0, 0.0), k, o, dl) == 8
    for x in (2.0, 2.25, -2.25, math.nextafter(-2.0, -3.0), 1e300, -1e300):
        with pytest.raises(ValueError):                     # -2.25 would round to m = 0
            Q.quantize(x, k, o, dl)
    # the benchmark's quantizer: [-8, 8) at scale 2^20
    q = gen.Q_PLAIN
    assert Q.quantize(-8.0, q.log2_scale, q.offset, q.delta) == 0
    assert Q.quantize(math.nextafter(8.0, 0.0), q.log2_scale, q.offset, q.delta) == q.delta
    with pytest.raises(ValueError):
        Q.quantize(8.0, q.log2_scale, q.offset, q.delta)


def test_dequantize_rounding_above_2_53():
    # float(int) rounds to nearest even: 2^53 + 1 -> 2^53, 2^53 + 3 -> 2^53 + 4
    assert Q.dequantize((1 << 53) + 1, 0, 0, 1) == float(1 << 53)
    assert Q.dequantize((1 << 53) + 3, 0, 0, 1) == float((1 << 53) + 4)


# ------------------------------------------------------- K-way aggregation
def _units(n):
    return [r for r in range(1, n) if math.gcd(r, n) == 1]


@pytest.mark.parametrize("p,q,kmax", [(3, 5, 3), (5, 7, 3), (7, 11, 2)])
def test_hom_sum_bruteforce_tiny(p, q, kmax):
    """Every K-tuple of plaintexts (K = 1..kmax) under tiny keys: the K-way
    aggregate is exactly Enc(sum m_k mod n, prod r_k mod n) (since
    (x + j n)^n = x^n mod n^2), it decrypts to the sum mod n, and the fused
    encrypt -> aggregate -> decrypt returns that sum."""
    pk, sk = O.derive_keys(p, q)
    n = p * q
    units = _units(n)
    rng = random.Random(n * 31)
    for K in range(1, kmax + 1):
        for ms in itertools.product(range(n), repeat=K):
            rs = [rng.choice(units) for _ in ms]
            cs = [O.encrypt(pk, m, r) for m, r in zip(ms, rs)]
            agg = O.hom_sum(pk, cs)
            assert agg == O.encrypt(pk, sum(ms) % n, math.prod(rs) % n)
            assert O.decrypt(sk, agg) == sum(ms) % n
            assert O.enc_sum_dec(sk, ms, rs) == sum(ms) % n


def _aggregate_identities(pk, sk, rng):
    n = pk.n
    for K in (1, 2, 5):
        a = [rng.randrange(n) for _ in range(K)]
        r = gen.gen_r(n, K, 12, extra=K + pk.nbits)
        cs = [O.encrypt(pk, ai, ri) for ai, ri in zip(a, r)]
        assert O.hom_sum(pk, cs) == O.encrypt(pk, sum(a) % n, math.prod(r) % n)
    # element-wise over K vectors of length 3: element j combines only column j
    K, J = 3, 3
    a = [[rng.randrange(n) for _ in range(J)] for _ in range(K)]
    r = [gen.gen_r(n, J, 13, extra=k + pk.nbits) for k in range(K)]
    cvs = [O.encrypt_vec(pk, a[k], r[k]) for k in range(K)]
    got = O.hom_sum_vec(pk, cvs)
    assert got == [O.encrypt(pk, sum(a[k][j] for k in range(K)) % n,
                             math.prod(r[k][j] for k in range(K)) % n) for j in range(J)]
    # the fused form: plaintexts that wrap past n, and the largest plaintexts
    ms = [n - 1, n - 2, 1, rng.randrange(n)]
    rs = gen.gen_r(n, 4, 14, extra=pk.nbits)
    assert O.enc_sum_dec(sk, ms, rs) == sum(ms) % n
    assert O.enc_sum_dec(sk, [n - 1], [n - 1]) == n - 1


def test_aggregate_identities(key):
    _, _, pk, sk = key
    _aggregate_identities(pk, sk, random.Random(pk.nbits + 77))


# ------------------------------------------------------ ciphertext mat-vec
@pytest.mark.parametrize("p,q", TINY[:2])
def test_matvec_bruteforce_tiny(p, q):
    """Every 2 x 2 constant matrix with entries < 4 over two fixed
    ciphertexts: the product decrypts to alpha + B m mod n (Definitions 1-2)."""
    pk, sk = O.derive_keys(p, q)
    n = p * q
    units = [r for r in range(1, n) if math.gcd(r, n) == 1]
    m = [2, n - 1]
    cs = [O.encrypt(pk, m[0], units[0]), O.encrypt(pk, m[1], units[-1])]
    a = [1, 3]
    alpha = [O.encrypt(pk, a[0], units[1 % len(units)]), O.encrypt(pk, a[1], units[0])]
    for b00 in range(4):
        for b01 in range(4):
            for b10 in range(4):
                for b11 in range(4):
                    B = [[b00, b01], [b10, b11]]
                    out = O.hom_matvec(pk, B, cs, alpha)
                    for i in range(2):
                        want = (a[i] + B[i][0] * m[0] + B[i][1] * m[1]) % n
                        assert O.decrypt(sk, out[i]) == want


def test_matvec_decrypts_to_integer_matvec(key):
    """Rows of 50-bit constants (the quantized matrix of Sec. III-C) against
    the exact integer mat-vec of the plaintexts."""
    p, q, pk, sk = key
    n = pk.n
    rng = random.Random(n % 10007)
    rows, cols = (3, 5) if pk.nbits >= 1024 else (4, 9)
    m = [rng.randrange(n) for _ in range(cols)]
    rs = gen.gen_r(n, cols + rows, 11, extra=pk.nbits)
    cs = [O.encrypt(pk, mj, rj) for mj, rj in zip(m, rs)]
    a = [rng.randrange(n) for _ in range(rows)]
    alpha = [O.encrypt(pk, ai, ri) for ai, ri in zip(a, rs[cols:])]
    B = [[rng.getrandbits(50) for _ in range(cols)] for _ in range(rows)]
    B[0][0] = 0
    B[-1][-1] = (1 << 50) - 1
    out = O.hom_matvec(pk, B, cs, alpha)
    for i in range(rows):
        want = (a[i] + sum(bij * mj for bij, mj in zip(B[i], m))) % n
        assert O.decrypt(sk, out[i]) == want
    # without alpha the offset is the integer 1, an encryption of 0
    out0 = O.hom_matvec(pk, B[:1], cs)
    assert O.decrypt(sk, out0[0]) == sum(bij * mj for bij, mj in zip(B[0], m)) % n


def test_matvec_special_cases(key):
    _, _, pk, _ = key
    n, n2 = pk.n, pk.n2
    rng = random.Random(pk.nbits)
    cols = 4
    cs = [rng.randrange(1, n2) for _ in range(cols)]
    alpha = [rng.randrange(1, n2) for _ in range(cols)]
    ident = [[1 if i == j else 0 for j in range(cols)] for i in range(cols)]
    assert O.hom_matvec(pk, ident, cs, alpha) == [(x * c) % n2 for x, c in zip(alpha, cs)]
    zero = [[0] * cols for _ in range(2)]
    assert O.hom_matvec(pk, zero, cs, alpha[:2]) == alpha[:2]
    assert O.hom_matvec(pk, zero, cs) == [1, 1]
    ks = [rng.getrandbits(64) for _ in range(3)]
    one_col = O.hom_matvec(pk, [[k] for k in ks], cs[:1], alpha[:3])
    assert one_col == [(x * pow(cs[0], k, n2)) % n2 for x, k in zip(alpha, ks)]
    with pytest.raises(ValueError):
        O.hom_matvec(pk, [[1]], [n2])
    with pytest.raises(ValueError):
        O.hom_matvec(pk, [[1, 2]], cs[:1])
