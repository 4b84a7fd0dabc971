"""Paillier encryption, decryption and homomorphic operations as plain definitions.

Test infrastructure only (see the package docstring): no product code imports
this module.

Everything here is exact Python integer arithmetic.  Each function states the
passage of the paper it writes out:

* key derivation      -- Sec. III-B, the key-generation list (n = pq,
                         eps = lcm(p-1, q-1), L(x) = (x-1)/n,
                         mu = L(g^eps mod n^2)^-1 mod n).
* encryption          -- Sec. III-B, f_en: c = g^m r^n mod n^2, a fresh r per
                         element.
* homomorphic add     -- Sec. III-B, Definition 1: c1 c2 mod n^2.
* scalar multiply     -- Sec. III-B, Definition 2: c^k mod n^2.
* decryption          -- Sec. III-C, f_de: L(c^eps mod n^2) mu mod n.
* modular power       -- the bit-serial square-and-multiply skeleton of
                         Algorithm 2, with exact ``%`` in place of the FFT
                         product and Barrett reduction.
* ciphertext mat-vec  -- Definition 2 with a matrix of constants (eq. (hemul))
                         followed by Definition 1 with the encrypted offset
                         alpha: the edge-node update of Sec. III-C
                         (eq. (itq2)).
* CRT decryption      -- Lemma 1 / Lemma 2 of Sec. IV applied to the
                         decryption (the paper states the decryption EP can be
                         split the same way as the encryption).  Used only as a
                         pin that the split route reaches the plain result; the
                         parity tests compare against ``decrypt``.

Choice of g: the paper allows any g in Z*_{n^2}; this implementation fixes g = n + 1, so
no g is ever passed around.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import gcd
from typing import Iterable, Sequence


def pow_plain(base: int, exp: int, mod: int) -> int:
    """base^exp mod ``mod`` by right-to-left binary square-and-multiply.

    Follows the loop of Algorithm 2 (Sec. IV-A): the running product T starts
    at 1; for every exponent bit from the least significant one, T is
    multiplied by the current base power when the bit is set, and the base
    power is squared.  Products are reduced with an exact remainder.
    """
    if mod <= 0:
        raise ValueError("modulus must be positive")
    if exp < 0:
        raise ValueError("negative exponent")
    t = 1 % mod
    g = base % mod
    e = exp
    while e > 0:
        if e & 1:
            t = (t * g) % mod
        g = (g * g) % mod
        e >>= 1
    return t


def lcm(a: int, b: int) -> int:
    return a // gcd(a, b) * b


def L(x: int, n: int) -> int:
    """L(x) = (x - 1) / n, an exact division (Sec. III-B key generation)."""
    num = x - 1
    if num % n != 0:
        raise ArithmeticError("L(x): n does not divide x - 1")
    return num // n


@dataclass(frozen=True)
class PublicKey:
    n: int

    @property
    def n2(self) -> int:
        return self.n * self.n

    @property
    def g(self) -> int:
        return self.n + 1

    @property
    def nbits(self) -> int:
        return self.n.bit_length()


@dataclass(frozen=True)
class SecretKey:
    p: int
    q: int
    n: int
    lam: int  # eps = lcm(p-1, q-1)
    mu: int

    @property
    def n2(self) -> int:
        return self.n * self.n

    @property
    def public(self) -> PublicKey:
        return PublicKey(self.n)


def derive_keys(p: int, q: int) -> tuple[PublicKey, SecretKey]:
    """Public and private key from the two primes (Sec. III-B key generation).

    n = p q, eps = lcm(p - 1, q - 1), g = n + 1,
    mu = L(g^eps mod n^2)^{-1} mod n.
    """
    if p == q or p < 3 or q < 3 or p % 2 == 0 or q % 2 == 0:
        raise ValueError("p, q must be distinct odd primes")
    n = p * q
    if gcd(n, (p - 1) * (q - 1)) != 1:
        raise ValueError("gcd(n, (p-1)(q-1)) must be 1")
    lam = lcm(p - 1, q - 1)
    n2 = n * n
    u = L(pow_plain(n + 1, lam, n2), n)
    mu = pow(u, -1, n)  # modular inverse (library routine)
    return PublicKey(n), SecretKey(p=p, q=q, n=n, lam=lam, mu=mu)


def encrypt(pk: PublicKey, m: int, r: int) -> int:
    """f_en(m) = g^m r^n mod n^2 with g = n + 1 (Sec. III-B).

    Requires 0 <= m < n (the plaintext space of Remark 2) and 0 < r < n.
    """
    n, n2 = pk.n, pk.n2
    if not (0 <= m < n):
        raise ValueError("plaintext out of [0, n)")
    if not (0 < r < n):
        raise ValueError("randomness out of (0, n)")
    return (pow_plain(pk.g, m, n2) * pow_plain(r, n, n2)) % n2


def decrypt(sk: SecretKey, c: int) -> int:
    """f_de(c) = L(c^eps mod n^2) mu mod n (Sec. III-C)."""
    n, n2 = sk.n, sk.n2
    if not (0 <= c < n2):
        raise ValueError("ciphertext out of [0, n^2)")
    return (L(pow_plain(c, sk.lam, n2), n) * sk.mu) % n


def hom_add(pk: PublicKey, c1: int, c2: int) -> int:
    """Ciphertext addition, Definition 1: c1 c2 mod n^2."""
    return (c1 * c2) % pk.n2


def hom_sum(pk: PublicKey, cs: Iterable[int]) -> int:
    """K-way aggregation: Definition 1 applied K-1 times (product mod n^2)."""
    acc = 1
    for c in cs:
        acc = (acc * c) % pk.n2
    return acc


def hom_scalar_mul(pk: PublicKey, c: int, k: int) -> int:
    """Multiply-by-constant, Definition 2: c^k mod n^2."""
    if k < 0:
        raise ValueError("negative scalar")
    return pow_plain(c, k, pk.n2)


def hom_matvec(pk: PublicKey, B: Sequence[Sequence[int]], cs: Sequence[int],
               alpha: Sequence[int] | None = None) -> list[int]:
    """Ciphertext matrix-vector product of the edge-node update (Sec. III-C,
    eq. (itq2)): row i is alpha_i (+) (B_i (x) c), where (x) is Definition 2
    with the constants B_ij applied to the ciphertexts c_j (eq. (hemul)) and
    the results, then alpha_i, are combined by Definition 1:

        out_i = alpha_i * prod_j c_j^(B_ij) mod n^2     (alpha_i = 1 if absent)

    It decrypts to alpha's plaintext + sum_j B_ij m_j mod n.  Ciphertexts and
    alpha must lie in [0, n^2), the constants must be non-negative integers.
    """
    n2 = pk.n2
    for c in cs:
        if not (0 <= c < n2):
            raise ValueError("ciphertext out of [0, n^2)")
    out = []
    for i, row in enumerate(B):
        if len(row) != len(cs):
            raise ValueError("row length differs from the vector length")
        acc = 1
        if alpha is not None:
            if not (0 <= alpha[i] < n2):
                raise ValueError("alpha out of [0, n^2)")
            acc = alpha[i]
        for bij, cj in zip(row, cs):
            acc = hom_add(pk, acc, hom_scalar_mul(pk, cj, bij))
        out.append(acc)
    return out


def enc_sum_dec(sk: SecretKey, ms: Sequence[int], rs: Sequence[int]) -> int:
    """Dec(prod_k Enc(m_k, r_k) mod n^2): the aggregation the master performs
    on the K edge contributions of one vector element (Sec. III-C with
    Definition 1)."""
    pk = sk.public
    return decrypt(sk, hom_sum(pk, (encrypt(pk, m, r) for m, r in zip(ms, rs))))


def decrypt_crt(sk: SecretKey, c: int) -> int:
    """Decryption through the split Z_{n^2} -> Z_{p^2} x Z_{q^2} (Sec. IV,
    Lemmas 1-2, applied to decryption as the paper states it can be).

    For each prime s in {p, q}: x_s = c^{s-1} mod s^2, m_s = L_s(x_s) h_s mod s
    with L_s(x) = (x-1)/s and h_s = L_s(g^{s-1} mod s^2)^{-1} mod s; then the
    two residues are recombined by Lemma 1.  Used only as a pin of
    ``decrypt``.
    """
    p, q, n = sk.p, sk.q, sk.n
    g = n + 1
    res = []
    for s in (p, q):
        s2 = s * s
        hs = pow(L(pow_plain(g, s - 1, s2), s), -1, s)
        res.append((L(pow_plain(c, s - 1, s2), s) * hs) % s)
    mp, mq = res
    # Lemma 1 with moduli p, q: x = sum a_i e_i T_i mod T, T_i = T / t_i,
    # e_i = T_i^{-1} mod t_i.
    return (mp * q * pow(q, -1, p) + mq * p * pow(p, -1, q)) % n


# ---------------------------------------------------------------- vectors
def encrypt_vec(pk: PublicKey, ms: Sequence[int], rs: Sequence[int]) -> list[int]:
    return [encrypt(pk, m, r) for m, r in zip(ms, rs, strict=True)]


def decrypt_vec(sk: SecretKey, cs: Sequence[int]) -> list[int]:
    return [decrypt(sk, c) for c in cs]


def hom_sum_vec(pk: PublicKey, cvs: Sequence[Sequence[int]]) -> list[int]:
    """Element-wise K-way aggregation of K ciphertext vectors."""
    length = len(cvs[0])
    return [hom_sum(pk, (cv[j] for cv in cvs)) for j in range(length)]
