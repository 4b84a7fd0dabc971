// Device-visible key constants and launch plumbing shared by the host code
// and the kernels.  All pointers are device addresses inside one allocation
// owned by the key object.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace pc2k {

// Error bits latched in the context's device word.
enum : int { ERR_RANGE = 1 };

constexpr int RK_MAX = 128;  // largest K of a K-way aggregation in one call

// One odd modulus N in D-digit "chunked" layout: a number is CH words, lane t
// of a tile owns words [t*K4, t*K4 + K).  Nl is N as 32-bit limbs, zero
// padded to nl limbs.
struct ModConst {
  const uint32_t* N;
  const uint32_t* R1;  // R mod N
  const uint32_t* R2;  // R^2 mod N
  const uint32_t* R3;  // R^3 mod N
  const uint32_t* ONE; // the integer 1 (chunked)
  const uint32_t* Nl;
  uint32_t nprime;     // -N^-1 mod 2^D
  int nl;
};

// Sliding-window schedules of an exponent for window widths 2..6 (entry
// (nsq << 16) | d: square nsq times, then multiply by x^d, d odd or 0; the
// first entry's d is the starting power).
constexpr int SCHED_WMIN = 2, SCHED_WMAX = 6;
struct Sched {
  const uint32_t* p[SCHED_WMAX - SCHED_WMIN + 1];
  int n[SCHED_WMAX - SCHED_WMIN + 1];
};

// Constants of n^2 for the i8-MFMA Montgomery product (mfma_mont.hpp):
// R = 2^(28 S); forward arrays of 7-bit digits, one per byte, after 64 zero
// bytes and with a zero tail (64 + D8 + 16 bytes, D8 = 4 S rounded up to 16).
struct MfmaConst {
  const uint8_t* N;      // n^2
  const uint8_t* Np;     // -(n^2)^-1 mod R
  const uint8_t* R2;     // R^2 mod n^2
  const uint8_t* nR;     // n R mod n^2
  const uint8_t* Rk;     // R^k mod n^2 for k = 0..RK_MAX, entry k at k (64 + D8 + 16)
  const uint32_t* N28;   // n^2 as S limbs of 28 bits
  int S;
};

struct PkConst {
  ModConst n2;           // modulus n^2; Nl has 2L limbs
  const uint32_t* nR;    // n R mod n^2 (chunked)
  const uint32_t* Rk;    // R^k mod n^2 for k = 0..RK_MAX, entry k at k*CH
  const uint32_t* n;     // n, L limbs
  int L;                 // limbs of n (ABI: plaintexts L, ciphertexts 2L)
  int nbits;             // bit length of n (the exponent of r^n)
  MfmaConst mf;          // the same modulus for the matrix-core product
  Sched nsch;            // sliding-window schedules of n
};

// One prime s of the CRT decryption (s = p or q, p > q).
struct HalfConst {
  ModConst s2;           // modulus s^2; Nl has Ls2 = s2.nl limbs
  const uint32_t* s;     // s, Ls limbs
  const uint32_t* e;     // s - 1, Ls limbs
  const uint32_t* sinv;  // s^-1 mod 2^(32 Ls)
  const uint32_t* H;     // h_s 2^(32 Ls) mod s, h_s = L_s(g^(s-1) mod s^2)^-1 mod s
  uint32_t s_n0;         // -s^-1 mod 2^32
  int Ls;
  Sched esch;            // sliding-window schedules of s - 1
  // key-holder encryption modulo s^2
  const uint32_t* nRs;   // n R mod s^2 (chunked)
  Sched nsch;            // sliding-window schedules of n mod s (s - 1)
};

struct SkConst {
  PkConst pk;
  HalfConst h[2];        // [0] = p, [1] = q
  const uint32_t* QI;    // q^-1 2^(32 Ls) mod p
  const uint32_t* Q2I;   // (q^2)^-1 2^(32 nl2) mod p^2 (nl2 = limbs of p^2)
  uint32_t p2_n0;        // -(p^2)^-1 mod 2^32
  int ebits;             // max bit length of p-1, q-1
};

struct PtrList {
  const uint32_t* p[RK_MAX];
};

// One job of a persistent batch launch (device copy).  All jobs of a launch
// run the same operation; their key classes (or tiles) may differ.
struct BatchJob {
  int geo, op, m_limbs, K;        // geo: geometry id of the job's key (CLASS_GEO)
  int group;                      // elements per work item
  PkConst pk;                     // encrypt, hom_sum
  SkConst sk;                     // decrypt
  const uint32_t* in0;            // encrypt: m; decrypt: c
  const uint32_t* in1;            // encrypt: r
  uint32_t* out;
  size_t count;                   // output elements
  const uint32_t* const* inputs;  // hom_sum: K device pointers
  const size_t* lengths;          // hom_sum: K input lengths (may be null)
  uint32_t* stage;                // decrypt: the CRT halves of groups stage_g0.. (2 (Ls + 1)
  size_t stage_g0;                //   words per element, element-major)
};
// Largest prime, in 32-bit limbs, that a secret key may hold (the 4096-bit
// class admits primes of up to 2093 bits).
constexpr int LS_MAX = 66;

// A work item: one wavefront's group of elements of one job (decryption:
// one prime, `half`, of the group).
struct BatchItem {
  int job;
  int half;
  size_t group;
};

// Limbs (28-bit) of R for the matrix-core product per key class:
// 28 S >= 2 * (class limit) + 12, so R >= 2^12 n^2 (the margin the signed
// redundant limbs' bounds need; mfma_mont.hpp).
constexpr int MFMA_S[9] = {3, 5, 10, 19, 37, 74, 147, 220, 293};
constexpr int CLASS_LIMIT_BITS[9] = {32, 64, 128, 256, 512, 1024, 2048, 3072, 4096};
constexpr bool mfma_margins_ok() {
  for (int c = 0; c < 9; ++c)
    if (28 * MFMA_S[c] < 2 * CLASS_LIMIT_BITS[c] + 12) return false;
  return true;
}
static_assert(mfma_margins_ok(), "R >= 2^12 n^2 in every key class");

// Key size classes: index by ceil(log2) of the key.  n^2 and s^2 use
// separate digit geometries (see mont_tile.hpp).
constexpr int NUM_CLASSES = 9;
inline int class_for_bits(int nbits) {
  for (int i = 0; i < NUM_CLASSES; ++i)
    if (nbits <= CLASS_LIMIT_BITS[i]) return i;
  return -1;
}

// Digit geometries ("geometry ids").  Ids 0-7 are the key classes' own
// tiles; the others are alternative tiles for the n^2 products of
// encryption, with twice the lanes per ciphertext and half the digits per
// lane (fewer registers, more waves per SIMD, more lane exchanges per digit).
// The s^2 geometry of an alternative is its class's own.
struct ClassGeo {
  int nD, nK, nT;  // n^2
  int pD, pK, pT;  // s^2
};
constexpr int NUM_GEOS = 11;
constexpr ClassGeo CLASS_GEO[NUM_GEOS] = {
    {28, 2, 2, 28, 2, 1},   {28, 3, 2, 28, 3, 1},   {28, 5, 2, 28, 5, 1},
    {28, 10, 2, 28, 10, 1}, {28, 19, 2, 28, 19, 1}, {28, 37, 2, 28, 37, 1},
    {28, 37, 4, 28, 37, 2}, {28, 28, 8, 28, 28, 4}, {28, 37, 8, 28, 37, 4},
    {28, 19, 4, 28, 37, 1},  // class 5 (1024-bit keys), 4 lanes per ciphertext
    {27, 19, 8, 28, 37, 2},  // class 6 (2048-bit keys), 8 lanes per ciphertext
};
constexpr int GEO_CLASS[NUM_GEOS] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 5, 6};  // key class of a geometry
constexpr int ALT_GEO[NUM_CLASSES] = {-1, -1, -1, -1, -1, 9, 10, -1, -1};  // alternative tile, or -1

// Launch configuration chosen by the host for a data call.
struct Launch {
  int grid;              // workgroups (one wavefront each)
  int window;            // window width for the exponentiations
  uint32_t* scratch;     // per-tile tables
  size_t slot_words;     // words of one tile's table slot
  int* err;              // latched error word
  void* stream;
  uint32_t* aux;         // per-element staging after the tables (decryption halves)
};

}  // namespace pc2k
