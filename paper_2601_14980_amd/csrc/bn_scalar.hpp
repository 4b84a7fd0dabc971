// Single-lane multi-precision helpers (32-bit limbs, runtime loops) for the
// few once-per-element steps around an exponentiation: range checks,
// digit <-> limb conversion, the final canonical reduction, the exact
// division of L(x) = (x - 1)/s and the CRT recombination.  They run in one
// lane of a tile and cost a few hundred instructions per element, next to
// the ~10^4-10^5 instructions per lane of the exponentiation itself.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc2d {

// -1 / 0 / 1 comparing a (na limbs) with b (nb limbs)
__device__ inline int sc_cmp(const uint32_t* a, int na, const uint32_t* b, int nb) {
  int n = na > nb ? na : nb;
  for (int i = n - 1; i >= 0; --i) {
    uint32_t x = i < na ? a[i] : 0u, y = i < nb ? b[i] : 0u;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

__device__ inline bool sc_is_zero(const uint32_t* a, int n) {
  uint32_t o = 0;
  for (int i = 0; i < n; ++i) o |= a[i];
  return o == 0;
}

// a -= b (a: na limbs, b: nb <= na limbs); returns the final borrow
__device__ inline uint32_t sc_sub(uint32_t* a, int na, const uint32_t* b, int nb) {
  uint32_t borrow = 0;
  for (int i = 0; i < na; ++i) {
    uint64_t y = (uint64_t)(i < nb ? b[i] : 0u) + borrow;
    uint64_t x = a[i];
    a[i] = (uint32_t)(x - y);
    borrow = x < y ? 1u : 0u;
  }
  return borrow;
}

// a += b (a: na limbs, b: nb <= na limbs); returns the final carry
__device__ inline uint32_t sc_add(uint32_t* a, int na, const uint32_t* b, int nb) {
  uint64_t c = 0;
  for (int i = 0; i < na; ++i) {
    c += (uint64_t)a[i] + (i < nb ? b[i] : 0u);
    a[i] = (uint32_t)c;
    c >>= 32;
  }
  return (uint32_t)c;
}

// r = a * b, r has na + nb limbs (r must not alias a or b)
__device__ inline void sc_mul(uint32_t* r, const uint32_t* a, int na, const uint32_t* b, int nb) {
  for (int i = 0; i < na + nb; ++i) r[i] = 0;
  for (int i = 0; i < na; ++i) {
    uint64_t c = 0;
    uint32_t ai = a[i];
    for (int j = 0; j < nb; ++j) {
      c += (uint64_t)ai * b[j] + r[i + j];
      r[i + j] = (uint32_t)c;
      c >>= 32;
    }
    r[i + nb] = (uint32_t)c;
  }
}

// r = a * b mod 2^(32 n) (r must not alias a or b)
__device__ inline void sc_mullo(uint32_t* r, const uint32_t* a, const uint32_t* b, int n) {
  for (int i = 0; i < n; ++i) r[i] = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t c = 0;
    uint32_t ai = a[i];
    for (int j = 0; i + j < n; ++j) {
      c += (uint64_t)ai * b[j] + r[i + j];
      r[i + j] = (uint32_t)c;
      c >>= 32;
    }
  }
}

// Montgomery product with 32-bit limbs: r = a b 2^(-32 n) mod m, canonical.
// a, b < m; t: scratch of n + 2 words; r may alias a or b.
__device__ inline void sc_montmul(uint32_t* r, const uint32_t* a, const uint32_t* b,
                                  const uint32_t* m, uint32_t n0, int n, uint32_t* t) {
  for (int i = 0; i < n + 2; ++i) t[i] = 0;
  for (int i = 0; i < n; ++i) {
    uint64_t c = 0;
    uint32_t bi = b[i];
    for (int j = 0; j < n; ++j) {
      c += (uint64_t)a[j] * bi + t[j];
      t[j] = (uint32_t)c;
      c >>= 32;
    }
    c += t[n];
    t[n] = (uint32_t)c;
    t[n + 1] = (uint32_t)(c >> 32);
    uint32_t q = t[0] * n0;
    c = ((uint64_t)q * m[0] + t[0]) >> 32;
    for (int j = 1; j < n; ++j) {
      c += (uint64_t)q * m[j] + t[j];
      t[j - 1] = (uint32_t)c;
      c >>= 32;
    }
    c += t[n];
    t[n - 1] = (uint32_t)c;
    t[n] = t[n + 1] + (uint32_t)(c >> 32);
    t[n + 1] = 0;
  }
  if (t[n] != 0 || sc_cmp(t, n, m, n) >= 0) sc_sub(t, n + 1, m, n);
  for (int i = 0; i < n; ++i) r[i] = t[i];
}

// In place: S semi-normalised D-bit digits -> nl little-endian limbs.
// Requires S >= nl and the value < 2^(32 nl).
template <int D>
__device__ inline void sc_digits_to_limbs(uint32_t* buf, int S, int nl) {
  const uint32_t MASK = (1u << D) - 1u;
  uint64_t c = 0;
  for (int g = 0; g < S; ++g) {
    uint64_t v = (uint64_t)buf[g] + c;
    buf[g] = (uint32_t)v & MASK;
    c = v >> D;
  }
  uint64_t acc = 0;
  int nb = 0, li = 0;
  for (int g = 0; g < S; ++g) {
    acc |= (uint64_t)buf[g] << nb;
    nb += D;
    while (nb >= 32) {
      if (li < nl) buf[li] = (uint32_t)acc;
      ++li;
      acc >>= 32;
      nb -= 32;
    }
  }
  while (li < nl) {
    buf[li++] = (uint32_t)acc;
    acc >>= 32;
  }
}

}  // namespace pc2d
