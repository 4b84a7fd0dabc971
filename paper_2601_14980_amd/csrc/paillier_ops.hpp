// Device bodies of the Paillier operations, shared by the one-launch-per-call
// kernels (kernels_paillier.hip) and the persistent batch kernels
// (kernels_batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "bn_scalar.hpp"
#include "engine.hpp"
#include "mont_tile.hpp"
#include "pc2_types.hpp"

using namespace pc2d;
using pc2k::HalfConst;
using pc2k::ModConst;
using pc2k::PkConst;
using pc2k::PtrList;
using pc2k::SkConst;

namespace pc2ops {

// Lane 0 of a tile: the tile's LDS digits (value < 2N) -> canonical limbs of
// the residue mod N, in place in LDS (nl + 1 words are used).
template <class G>
__device__ __forceinline__ void lds_canonical(uint32_t* lds, const ModConst& M) {
  sc_digits_to_limbs<G::D>(lds, G::S, M.nl + 1);
  if (sc_cmp(lds, M.nl + 1, M.Nl, M.nl) >= 0) sc_sub(lds, M.nl + 1, M.Nl, M.nl);
}

// The sliding-window schedule of a wave-uniform exponent for window w
// (2 <= w <= 6, the range the context accepts).
__device__ __forceinline__ void use_schedule(Program& P, const pc2k::Sched& sc, int w) {
  const int i = w < pc2k::SCHED_WMIN ? 0 : (w > pc2k::SCHED_WMAX ? pc2k::SCHED_WMAX - pc2k::SCHED_WMIN
                                                                   : w - pc2k::SCHED_WMIN);
  P.sched = sc.p[i];
  P.nsched = sc.n[i];
}

// Encryption of one element (Sec. III-B, f_en with g = n + 1):
//   pre0:  MM(m, n R)      = m n  (exact: m n < n^2), + 1 -> g^m, kept in slot entry 0
//   pre1:  MM(R^2, r)      = r R  (Montgomery form of r)
//   pow:   (r R)^n         = r^n R
//   post0: MM(g^m, r^n R)  = g^m r^n mod n^2   (normal form)
// m and r are first converted to digits in slot entries 0 and 1.
template <class G>
__device__ __forceinline__ Program encrypt_program(const PkConst& pk, const uint32_t* me,
                                                   int m_limbs, const uint32_t* re,
                                                   uint32_t* slot, int tl, int w) {
  chunk_from_limbs<G>(slot, me, m_limbs, 0, tl);
  chunk_from_limbs<G>(slot + G::CH, re, pk.L, 0, tl);
  Program P = empty_program();
  P.npre = 2;
  P.pre0_a = op_chunk(slot);
  P.pre0_b = op_chunk(pk.nR);
  P.pre0_to_slot = true;
  P.pre0_add1 = 1;
  P.pre1_a = op_chunk(pk.n2.R2);
  P.pre1_b = op_chunk(slot + G::CH);
  P.e = pk.n;
  P.elimbs = pk.L;
  P.ebits = pk.nbits;
  P.uniform_e = true;
  use_schedule(P, pk.nsch, w);
  P.one = pk.n2.R1;
  P.npost = 1;
  P.post0_a = op_chunk(slot);
  P.post0_b = op_x();
  return P;
}

// One CRT half of a decryption (Sec. III-C f_de through the split of Sec. IV):
//   redc:  c R^-1 mod s^2      (Montgomery reduction of the 2L-limb ciphertext)
//   pre1:  MM(R^3, c R^-1)     = c R
//   pow:   (c R)^(s-1)         = c^(s-1) R
//   post0: MM(., 1)            = c^(s-1) mod s^2
// (uniform: the half is the same for the whole wavefront, so its sliding
// schedule applies)
template <class G>
__device__ __forceinline__ Program decrypt_program(const HalfConst& H, int ebits,
                                                   const uint32_t* ce, int L2, uint32_t* slot,
                                                   int tl, int w, bool uniform) {
  chunk_from_limbs<G>(slot, ce, L2, 0, tl);
  Program P = empty_program();
  P.npre = 2;
  P.redc = true;
  P.redc_lo = slot;
  P.redc_hi = ce;
  P.redc_hi_n = L2;
  P.pre1_a = op_chunk(H.s2.R3);
  P.pre1_b = op_x();
  P.e = H.e;
  P.elimbs = H.Ls;
  P.ebits = ebits;
  P.uniform_e = uniform;
  if (uniform) use_schedule(P, H.esch, w);
  P.one = H.s2.R1;
  P.npost = 1;
  P.post0_a = op_x();
  P.post0_b = op_chunk(H.s2.ONE);
  return P;
}

// Lane 0 of a half-tile, after decrypt_program: y = c^(s-1) mod s^2 in LDS
// digits -> m_s = L_s(y) h_s mod s into slot[4Ls+2 ..), flag at slot[5Ls+2].
// L_s(y) = (y - 1)/s is an exact division: u = (y - 1) s^-1 mod 2^(32 Ls),
// verified by u s == y - 1 (fails only for c not coprime to s).
template <class Gp>
__device__ __forceinline__ void decrypt_half_finish(const HalfConst& H, uint32_t* lds,
                                                    uint32_t* slot, uint32_t cvalid) {
  const int Ls = H.Ls, ny = H.s2.nl + 1;
  uint32_t* y = lds;
  lds_canonical<Gp>(lds, H.s2);
  uint32_t one = 1u;
  uint32_t bor = sc_sub(y, ny, &one, 1);
  uint32_t* u = slot;                 // Ls
  uint32_t* us = slot + Ls;           // 2 Ls
  uint32_t* tmp = slot + 3 * Ls;      // Ls + 2
  uint32_t* ms = slot + 4 * Ls + 2;   // Ls
  uint32_t* flag = slot + 5 * Ls + 2;
  sc_mullo(u, y, H.sinv, Ls);
  sc_mul(us, u, Ls, H.s, Ls);
  bool good = (bor == 0) && (sc_cmp(us, 2 * Ls, y, ny) == 0) && cvalid;
  sc_montmul(ms, u, H.H, H.s, H.s_n0, Ls, tmp);
  *flag = good ? 1u : 0u;
}


// Lane 0 of a tile: canonical limbs of the tile's LDS value to dst (nl limbs),
// zeros and the error latch if !ok.
template <class G>
__device__ __forceinline__ void store_canonical(uint32_t* lds, const ModConst& M, uint32_t* dst,
                                                bool live, uint32_t ok, int* err) {
  lds_canonical<G>(lds, M);
  if (live) {
    for (int i = 0; i < M.nl; ++i) dst[i] = ok ? lds[i] : 0u;
    if (!ok) atomicOr(err, pc2k::ERR_RANGE);
  }
}

__device__ __forceinline__ uint32_t encrypt_inputs_ok(const PkConst& pk, const uint32_t* me,
                                                      int m_limbs, const uint32_t* re) {
  const int L = pk.L;
  return (sc_cmp(me, m_limbs, pk.n, L) < 0) && !sc_is_zero(re, L) && (sc_cmp(re, L, pk.n, L) < 0);
}


// ------------------------------------------------------- per-group bodies
// Each processes one group of elements (one wavefront's worth) so that the
// one-launch-per-call kernels and the persistent batch kernel share them.
// lds_all: the workgroup's LDS; slots: the workgroup's first scratch slot.

template <class G>
__device__ __forceinline__ void enc_group(const PkConst& pk, const uint32_t* __restrict__ m,
                                          int m_limbs, const uint32_t* __restrict__ r,
                                          uint32_t* __restrict__ c, size_t count, size_t gi,
                                          uint32_t* lds_all, uint32_t* slots, size_t slot_words,
                                          int w, int* err) {
  constexpr int EPW = 64 / G::T;
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t* slot = slots + tile * slot_words;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const int L = pk.L, L2 = 2 * pk.L;
  size_t e = gi * EPW + tile;
  const bool live = e < count;
  if (!live) e = count - 1;
  const uint32_t* me = m + e * m_limbs;
  const uint32_t* re = r + e * L;
  uint32_t ok = 1;
  if (tl == 0) ok = encrypt_inputs_ok(pk, me, m_limbs, re);
  Program P = encrypt_program<G>(pk, me, m_limbs, re, slot, tl, w);
  uint32_t x[G::K];
  run_program<G, true>(P, x, lds, slot, w, N, np, tl);
  lds_sync();
  to_lds<G>(lds, x, tl);
  lds_sync();
  if (tl == 0) store_canonical<G>(lds, pk.n2, c + e * L2, live, ok, err);
}

// One CRT half (prime s = p for half 0, q for half 1) of the decryption of
// the group gi of 64/Tp elements, one element per Tp-lane tile.  The half is
// uniform over the wavefront, so the prime's constants and exponent are
// wave-uniform and zero windows of s-1 are skipped.  Lane 0 of tile t writes
// m_s (Ls limbs) and a validity word to stage[(2 t + half) (Ls + 1) ..].
template <class Gp>
__device__ __forceinline__ void dec_half_group(const SkConst& sk, int half,
                                               const uint32_t* __restrict__ c, size_t count,
                                               size_t gi, uint32_t* lds_all, uint32_t* slots,
                                               size_t slot_words, int w,
                                               uint32_t* __restrict__ stage) {
  constexpr int EPW = 64 / Gp::T;
  const int tl = threadIdx.x & (Gp::T - 1);
  const int tile = threadIdx.x / Gp::T;
  uint32_t* lds = lds_all + tile * Gp::SP;
  uint32_t* slot = slots + tile * slot_words;
  const HalfConst& H = sk.h[half];
  uint32_t N[Gp::K];
  load_chunk<Gp>(N, H.s2.N, tl);
  const uint32_t np = H.s2.nprime;
  const int L2 = 2 * sk.pk.L, Ls = H.Ls;
  size_t e = gi * EPW + tile;
  const bool live = e < count;
  if (!live) e = count - 1;
  const uint32_t* ce = c + e * L2;
  uint32_t cv = 1;
  if (tl == 0) cv = sc_cmp(ce, L2, sk.pk.n2.Nl, L2) < 0;
  Program P = decrypt_program<Gp>(H, sk.ebits, ce, L2, slot, tl, w, true);
  uint32_t x[Gp::K];
  run_program<Gp, true>(P, x, lds, slot, w, N, np, tl);
  lds_sync();
  to_lds<Gp>(lds, x, tl);
  lds_sync();
  if (tl == 0) {
    decrypt_half_finish<Gp>(H, lds, slot, cv);
    if (live) {
      uint32_t* dst = stage + (size_t)(2 * tile + half) * (Ls + 1);
      for (int i = 0; i < Ls; ++i) dst[i] = slot[4 * Ls + 2 + i];
      dst[Ls] = slot[5 * Ls + 2];
    }
  }
}

// Key-holder encryption (the CRT route of Sec. IV applied to f_en): one
// prime s per wavefront, c_s = (1 + m n mod s^2) r^(n mod s (s-1)) mod s^2
// for the group gi of 64/Tp elements.  m, r < n < 2 s^2 (balanced primes),
// so both enter the Montgomery products directly:
//   pre0:  MM(m, n R)        = m n mod s^2, + 1 -> slot entry 0
//   pre1:  MM(R^2, r)        = r R
//   pow:   (r R)^e           (sliding windows of e = n mod s (s-1))
//   post0: MM(g^m, r^e R)    = c_s
// Lane 0 of tile t writes c_s (nl2 limbs) and an input-validity word to
// stage[(2 t + half) (nl2 + 1) ..].
template <class Gp>
__device__ __forceinline__ void enc_half_group(const SkConst& sk, int half,
                                               const uint32_t* __restrict__ m, int m_limbs,
                                               const uint32_t* __restrict__ r, size_t count,
                                               size_t gi, uint32_t* lds_all, uint32_t* slots,
                                               size_t slot_words, int w,
                                               uint32_t* __restrict__ stage) {
  constexpr int EPW = 64 / Gp::T;
  const int tl = threadIdx.x & (Gp::T - 1);
  const int tile = threadIdx.x / Gp::T;
  uint32_t* lds = lds_all + tile * Gp::SP;
  uint32_t* slot = slots + tile * slot_words;
  const HalfConst& H = sk.h[half];
  uint32_t N[Gp::K];
  load_chunk<Gp>(N, H.s2.N, tl);
  const uint32_t np = H.s2.nprime;
  const int L = sk.pk.L, nl2 = H.s2.nl;
  size_t e = gi * EPW + tile;
  const bool live = e < count;
  if (!live) e = count - 1;
  const uint32_t* me = m + e * m_limbs;
  const uint32_t* re = r + e * L;
  uint32_t ok = 1;
  if (tl == 0) ok = encrypt_inputs_ok(sk.pk, me, m_limbs, re);
  chunk_from_limbs<Gp>(slot, me, m_limbs, 0, tl);
  chunk_from_limbs<Gp>(slot + Gp::CH, re, L, 0, tl);
  Program P = empty_program();
  P.npre = 2;
  P.pre0_a = op_chunk(slot);
  P.pre0_b = op_chunk(H.nRs);
  P.pre0_to_slot = true;
  P.pre0_add1 = 1;
  P.pre1_a = op_chunk(H.s2.R2);
  P.pre1_b = op_chunk(slot + Gp::CH);
  P.ebits = sk.pk.nbits;
  P.uniform_e = true;
  use_schedule(P, H.nsch, w);
  P.one = H.s2.R1;
  P.npost = 1;
  P.post0_a = op_chunk(slot);
  P.post0_b = op_x();
  uint32_t x[Gp::K];
  run_program<Gp, true>(P, x, lds, slot, w, N, np, tl);
  lds_sync();
  to_lds<Gp>(lds, x, tl);
  lds_sync();
  if (tl == 0) {
    lds_canonical<Gp>(lds, H.s2);
    if (live) {
      uint32_t* dst = stage + (size_t)(2 * tile + half) * (nl2 + 1);
      for (int i = 0; i < nl2; ++i) dst[i] = lds[i];
      dst[nl2] = ok;
    }
  }
}

// c = c_q + q^2 ((c_p - c_q) (q^2)^-1 mod p^2), the CRT recombination
// modulo n^2 = p^2 q^2 (Lemma 1 for the moduli p^2, q^2), one lane per
// element; writes 2L limbs.  work: 5 nl2 + 2 words.
__device__ __forceinline__ void garner_crt_elem(const SkConst& sk, const uint32_t* __restrict__ cp,
                                                const uint32_t* __restrict__ cq, uint32_t* dst,
                                                int* err, uint32_t* work) {
  const int n2 = sk.h[0].s2.nl, L2 = 2 * sk.pk.L;
  const bool good = cp[n2] && cq[n2];
  const uint32_t* P2 = sk.h[0].s2.Nl;
  const uint32_t* Q2 = sk.h[1].s2.Nl;
  uint32_t* d = work;                  // n2
  uint32_t* h = work + n2;             // n2
  uint32_t* tmp = work + 2 * n2;       // n2 + 2
  uint32_t* prod = work + 3 * n2 + 2;  // 2 n2
  for (int i = 0; i < n2; ++i) d[i] = cp[i];
  // c_q < q^2 < p^2: one conditional addition of p^2 reduces the difference
  if (sc_sub(d, n2, cq, n2)) sc_add(d, n2, P2, n2);
  sc_montmul(h, d, sk.Q2I, P2, sk.p2_n0, n2, tmp);
  sc_mul(prod, Q2, n2, h, n2);
  sc_add(prod, 2 * n2, cq, n2);
  for (int i = 0; i < L2; ++i) dst[i] = (good && i < 2 * n2) ? prod[i] : 0u;
  if (!good) atomicOr(err, pc2k::ERR_RANGE);
}

// CRT recombination of one element from its two halves (one lane per element):
// m = m_q + q ((m_p - m_q) q^-1 mod p), Lemma 1 for the moduli p, q in
// Garner's form.  work: 5 Ls + 2 words.
__device__ __forceinline__ void garner_elem(const SkConst& sk, const uint32_t* __restrict__ hp,
                                            const uint32_t* __restrict__ hq, uint32_t* dst,
                                            int* err, uint32_t* work) {
  const int Ls = sk.h[0].Ls, L = sk.pk.L;
  const bool good = hp[Ls] && hq[Ls];
  uint32_t* d = work;                  // Ls
  uint32_t* h = work + Ls;             // Ls
  uint32_t* tmp = work + 2 * Ls;       // Ls + 2
  uint32_t* prod = work + 3 * Ls + 2;  // 2 Ls
  for (int i = 0; i < Ls; ++i) d[i] = hp[i];
  if (sc_sub(d, Ls, hq, Ls)) sc_add(d, Ls, sk.h[0].s, Ls);
  sc_montmul(h, d, sk.QI, sk.h[0].s, sk.h[0].s_n0, Ls, tmp);
  sc_mul(prod, sk.h[1].s, Ls, h, Ls);
  sc_add(prod, 2 * Ls, hq, Ls);
  for (int i = 0; i < L; ++i) dst[i] = (good && i < 2 * Ls) ? prod[i] : 0u;
  if (!good) atomicOr(err, pc2k::ERR_RANGE);
}

// out[j] = prod_k c_k[j] mod n^2 over the inputs with j < len_k (all inputs
// when lens is null).  acc = MM(c_k, acc) keeps a factor R^-(K-1), removed by
// one product with R^K; an input that does not reach element j contributes
// the integer 1, whose product MM(acc, 1) = acc R^-1 keeps that bookkeeping.
template <class G>
__device__ __forceinline__ void sum_group(const PkConst& pk, const uint32_t* const* cs,
                                          const size_t* lens, int K, uint32_t* __restrict__ out,
                                          size_t count, size_t gi, uint32_t* lds_all, int* err) {
  constexpr int EPW = 64 / G::T;
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const int L2 = 2 * pk.L;
  size_t e = gi * EPW + tile;
  const bool live = e < count;
  if (!live) e = count - 1;
  auto present = [&](int k) { return lens == nullptr || e < lens[k]; };
  uint32_t ok = 1;
  if (tl == 0)
    for (int k = 0; k < K; ++k)
      if (present(k)) ok &= sc_cmp(cs[k] + e * L2, L2, pk.n2.Nl, L2) < 0;
  uint32_t acc[G::K];
  lds_sync();
  if (present(0))
    lds_digits_from_limbs<G>(lds, cs[0] + e * L2, L2, 0, tl);
  else
    lds_from_chunk<G>(lds, pk.n2.ONE, tl);
  lds_sync();
  from_lds<G>(acc, lds, tl);
  for (int k = 1; k <= K; ++k) {
    lds_sync();
    if (k == K)
      lds_from_chunk<G>(lds, pk.Rk + (size_t)K * G::CH, tl);
    else if (present(k))
      lds_digits_from_limbs<G>(lds, cs[k] + e * L2, L2, 0, tl);
    else
      lds_from_chunk<G>(lds, pk.n2.ONE, tl);
    lds_sync();
    // b = the incoming factor (in LDS), a = the running product (registers)
    mont_mul<G>(acc, acc, lds, N, np, tl);
  }
  lds_sync();
  to_lds<G>(lds, acc, tl);
  lds_sync();
  if (tl == 0) store_canonical<G>(lds, pk.n2, out + e * L2, live, ok, err);
}

}  // namespace pc2ops

namespace pc2k {

// Digit geometry of each geometry id: Gn for n^2, Gp for p^2 and q^2
// (mirrors CLASS_GEO in pc2_types.hpp; ids 9 and 10 are the alternative
// encryption tiles of classes 5 and 6).
template <int CLS>
struct Geos;
#define PC2_CLASS(I, nD, nK, nT, pD, pK, pT)   \
  template <>                                   \
  struct Geos<I> {                              \
    using Gn = pc2d::Geo<nD, nK, nT>;           \
    using Gp = pc2d::Geo<pD, pK, pT>;           \
  };
PC2_CLASS(0, 28, 2, 2, 28, 2, 1)
PC2_CLASS(1, 28, 3, 2, 28, 3, 1)
PC2_CLASS(2, 28, 5, 2, 28, 5, 1)
PC2_CLASS(3, 28, 10, 2, 28, 10, 1)
PC2_CLASS(4, 28, 19, 2, 28, 19, 1)
PC2_CLASS(5, 28, 37, 2, 28, 37, 1)
PC2_CLASS(6, 28, 37, 4, 28, 37, 2)
PC2_CLASS(7, 28, 28, 8, 28, 28, 4)
PC2_CLASS(8, 28, 37, 8, 28, 37, 4)
PC2_CLASS(9, 28, 19, 4, 28, 37, 1)
PC2_CLASS(10, 27, 19, 8, 28, 37, 2)
#undef PC2_CLASS

}  // namespace pc2k
