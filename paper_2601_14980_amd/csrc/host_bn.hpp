// Host-side multi-precision helpers used once per key to derive the constants
// the device kernels need.  Little-endian uint32 limbs in std::vector.
// Not on the data path: sizes are at most a few hundred limbs and every
// routine is a plain textbook loop.
#pragma once
#include <cstdint>
#include <vector>

namespace pc2h {

using Limbs = std::vector<uint32_t>;

inline void trim(Limbs& a) {
  while (a.size() > 1 && a.back() == 0) a.pop_back();
  if (a.empty()) a.push_back(0);
}

inline Limbs resized(const Limbs& a, size_t n) {
  Limbs r(n, 0);
  for (size_t i = 0; i < a.size() && i < n; ++i) r[i] = a[i];
  return r;
}

inline int bitlen(const Limbs& a) {
  for (size_t i = a.size(); i-- > 0;)
    if (a[i]) return (int)(32 * i + 32 - __builtin_clz(a[i]));
  return 0;
}

inline bool is_zero(const Limbs& a) {
  for (uint32_t x : a)
    if (x) return false;
  return true;
}

// compare a and b of any lengths
inline int cmp(const Limbs& a, const Limbs& b) {
  size_t n = a.size() > b.size() ? a.size() : b.size();
  for (size_t i = n; i-- > 0;) {
    uint32_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

// a - b, requires a >= b; result has a.size() limbs
inline Limbs sub(const Limbs& a, const Limbs& b) {
  Limbs r(a.size());
  uint64_t borrow = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t y = (i < b.size() ? b[i] : 0) + borrow;
    uint64_t x = a[i];
    r[i] = (uint32_t)(x - y);
    borrow = x < y ? 1 : 0;
  }
  return r;
}

inline Limbs add(const Limbs& a, const Limbs& b) {
  size_t n = (a.size() > b.size() ? a.size() : b.size()) + 1;
  Limbs r(n);
  uint64_t c = 0;
  for (size_t i = 0; i < n; ++i) {
    c += (uint64_t)(i < a.size() ? a[i] : 0) + (i < b.size() ? b[i] : 0);
    r[i] = (uint32_t)c;
    c >>= 32;
  }
  trim(r);
  return r;
}

inline Limbs mul(const Limbs& a, const Limbs& b) {
  Limbs r(a.size() + b.size(), 0);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t c = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      c += (uint64_t)a[i] * b[j] + r[i + j];
      r[i + j] = (uint32_t)c;
      c >>= 32;
    }
    r[i + b.size()] = (uint32_t)c;
  }
  trim(r);
  return r;
}

inline Limbs from_u64(uint64_t v) { Limbs r{(uint32_t)v, (uint32_t)(v >> 32)}; trim(r); return r; }

// x mod m for x < 2^(32*len) by binary long division (shift-subtract);
// used only on small setup values.
inline Limbs mod(const Limbs& x, const Limbs& m) {
  Limbs mm = m;
  trim(mm);
  size_t n = mm.size() + 1;
  Limbs r(n, 0);
  int nb = bitlen(x);
  for (int bit = nb - 1; bit >= 0; --bit) {
    // r = 2r + bit
    uint32_t carry = (x[bit / 32] >> (bit % 32)) & 1u;
    for (size_t i = 0; i < n; ++i) {
      uint32_t nc = r[i] >> 31;
      r[i] = (r[i] << 1) | carry;
      carry = nc;
    }
    if (cmp(r, mm) >= 0) r = sub(r, mm);
  }
  trim(r);
  return r;
}

// x = 2x mod m, with x < m, both sized m.size()
inline void dbl_mod(Limbs& x, const Limbs& m) {
  uint32_t carry = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    uint32_t nc = x[i] >> 31;
    x[i] = (x[i] << 1) | carry;
    carry = nc;
  }
  if (carry || cmp(x, m) >= 0) {
    // subtract m (the true value is < 2m, so one subtraction suffices and the
    // dropped carry bit is absorbed by the wrap-around)
    uint64_t borrow = 0;
    for (size_t i = 0; i < x.size(); ++i) {
      uint64_t y = (uint64_t)m[i] + borrow;
      uint64_t v = x[i];
      x[i] = (uint32_t)(v - y);
      borrow = v < y ? 1 : 0;
    }
  }
}

// 2^k mod m by repeated doubling (m > 1, odd)
inline Limbs pow2_mod(uint64_t k, const Limbs& m0) {
  Limbs m = m0;
  trim(m);
  Limbs x(m.size(), 0);
  x[0] = 1;
  if (cmp(x, m) >= 0) x = mod(x, m), x = resized(x, m.size());
  for (uint64_t i = 0; i < k; ++i) dbl_mod(x, m);
  return x;
}

// x * 2^k mod m for x < m
inline Limbs shl_mod(const Limbs& x0, uint64_t k, const Limbs& m0) {
  Limbs m = m0;
  trim(m);
  Limbs x = resized(mod(x0, m), m.size());
  for (uint64_t i = 0; i < k; ++i) dbl_mod(x, m);
  return x;
}

// inverse of odd a modulo 2^32 (Newton iteration)
inline uint32_t inv32(uint32_t a) {
  uint32_t x = a;  // correct to 3 bits for odd a
  for (int i = 0; i < 5; ++i) x *= 2u - a * x;
  return x;
}

// inverse of odd a modulo 2^(32*n) (Newton-Hensel lifting, limb arithmetic)
inline Limbs inv_pow2(const Limbs& a0, size_t n) {
  Limbs a = resized(a0, n);
  Limbs x(n, 0);
  x[0] = inv32(a[0]);
  // x <- x (2 - a x) mod 2^(32n), doubling precision each round
  for (size_t prec = 1; prec < n; prec *= 2) {
    Limbs ax = resized(mul(a, x), n);
    // t = 2 - ax mod 2^(32n)  ==  (~ax) + 3 (two's complement of ax, plus 2)
    Limbs t(n);
    uint64_t c = 2;
    for (size_t i = 0; i < n; ++i) {
      uint64_t v = (uint64_t)(uint32_t)~ax[i] + (i == 0 ? 1 : 0) + c;
      t[i] = (uint32_t)v;
      c = v >> 32;
    }
    x = resized(mul(x, t), n);
  }
  return x;
}

// Montgomery context with 32-bit limbs, R32 = 2^(32 n), for odd modulus m.
struct Mont32 {
  Limbs m;
  size_t n;
  uint32_t n0;  // -m^{-1} mod 2^32
  Limbs r2;     // R32^2 mod m

  explicit Mont32(const Limbs& mod_) : m(mod_) {
    trim(m);
    n = m.size();
    n0 = (uint32_t)(0u - inv32(m[0]));
    r2 = pow2_mod((uint64_t)64 * n, m);
  }
  // a b R32^{-1} mod m, inputs < m
  Limbs mm(const Limbs& a0, const Limbs& b0) const {
    Limbs a = resized(a0, n), b = resized(b0, n);
    std::vector<uint64_t> t(n + 2, 0);
    for (size_t i = 0; i < n; ++i) {
      uint64_t c = 0;
      for (size_t j = 0; j < n; ++j) {
        uint64_t v = (uint64_t)a[j] * b[i] + (uint32_t)t[j] + c;
        t[j] = (uint32_t)v;
        c = v >> 32;
      }
      uint64_t v = (uint32_t)t[n] + c;
      t[n] = (uint32_t)v;
      t[n + 1] = v >> 32;
      uint32_t q = (uint32_t)t[0] * n0;
      c = ((uint64_t)q * m[0] + (uint32_t)t[0]) >> 32;
      for (size_t j = 1; j < n; ++j) {
        uint64_t w = (uint64_t)q * m[j] + (uint32_t)t[j] + c;
        t[j - 1] = (uint32_t)w;
        c = w >> 32;
      }
      v = (uint32_t)t[n] + c;
      t[n - 1] = (uint32_t)v;
      t[n] = t[n + 1] + (v >> 32);
      t[n + 1] = 0;
    }
    Limbs r(n + 1);
    for (size_t i = 0; i <= n; ++i) r[i] = (uint32_t)t[i];
    if (cmp(r, m) >= 0) r = sub(r, m);
    return resized(r, n);
  }
  Limbs to(const Limbs& a) const {
    Limbs t = a;
    trim(t);
    if (cmp(t, m) >= 0) t = mod(t, m);
    return mm(resized(t, n), r2);
  }
  Limbs from(const Limbs& a) const {
    Limbs one(n, 0);
    one[0] = 1;
    return mm(a, one);
  }
  // a * b mod m
  Limbs mulmod(const Limbs& a, const Limbs& b) const { return from(mm(to(a), to(b))); }
  // base^e mod m
  Limbs pow(const Limbs& base, const Limbs& e) const {
    Limbs x = to(base);
    Limbs acc = to(Limbs{1});
    int nb = bitlen(e);
    for (int i = nb - 1; i >= 0; --i) {
      acc = mm(acc, acc);
      if ((e[i / 32] >> (i % 32)) & 1u) acc = mm(acc, x);
    }
    return from(acc);
  }
};

// inverse of a modulo prime p (Fermat): a^(p-2) mod p
inline Limbs inv_mod_prime(const Limbs& a, const Limbs& p) {
  Mont32 M(p);
  Limbs e = sub(resized(p, p.size()), Limbs{2});
  return M.pow(a, e);
}

}  // namespace pc2h
