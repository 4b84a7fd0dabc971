// Montgomery multiplication on the i8 matrix cores (MFMA) of gfx950.
//
// A residue x mod N (R = 2^(28 S) >= 2^12 N at every key size) is held as S
// limbs of 28 bits or, for the matrix products, as D = 4S digits, one signed
// byte each (below).  One wavefront works on one element.  The three limb-product matrices of a separated Montgomery
// product
//
//     T = x y,    q = (T mod R) N' mod R  (N' = -N^-1 mod R),    U = (T + q N) / R
//
// are each computed exactly by v_mfma_i32_16x16x64_i8 with int32
// accumulation.  Output column p = 256 Q + 4 j + alpha(i), with
// alpha(i) = 64 (i / 4) + i % 4, takes row i of tile Q from a Toeplitz band
// of x (digits alpha(i) + 64 t - k, k < 64) and column j from a block of y
// (digits 256 Q + 4 j - 64 t + k); summing over t covers every digit pair
// once.  With that column order, lane l of tile Q ends up holding the four
// columns of limb 64 Q + l in its four accumulators, so the digits fold into
// 28-bit limbs in registers.
//
// Limbs are signed and redundant: a value is sum l_i 2^(28 i) with
// -2^27 - 2^20 <= l_i < 2^28, written as digits l & 127, (l >> 7) & 127,
// (l >> 14) & 127 and l >> 21 (the top digit of a limb signed, so every digit
// fits a signed byte).  A column sum then stays within D 127^2 < 2^31.  The
// carries of a product are never resolved: one balanced split per column
// (keep the low 28 bits less 2^27, hand the rest to the next limb) bounds
// every limb again, and every output stays below 0.52 N in magnitude, since
// |U| <= |x y| / R + |q| N / R with |q| < 0.51 R and N/R <= 2^-12.  The carry
// out of the top limb of U is zero by the same bound; the caller makes the
// final result canonical once.
//
// Only what U needs is formed.  T's limbs below S are split for q (the carry
// out of them moves to limb S); its columns from S up stay in the matrix
// accumulators, and q N is accumulated onto them.  Since T + q N = 0 mod R,
// its part below limb S is c R for an integer c that the two column values
// just below S fix (every lower column adds less than 2^-36 to c), so q N is
// formed only from the tile holding limb S - 2 up.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pc2_types.hpp"

namespace pc2m {

typedef int v4i __attribute__((ext_vector_type(4)));

template <int S_>
struct MGeo {
  static constexpr int S = S_;                       // 28-bit limbs of R
  static constexpr int D = 4 * S;                    // 7-bit digits
  static constexpr int D8 = (D + 15) & ~15;
  static constexpr int PF = 64;                      // zero bytes before a forward array
  static constexpr int FB = PF + D8 + 16;            // bytes of a forward digit array
  static constexpr int NT = (2 * S + 1 + 63) / 64;   // 64-limb tiles of a double-length value
  static constexpr int NTLO = (S + 63) / 64;         // tiles of a product taken mod R
  static constexpr int QLO = (S - 2) / 64;           // lowest tile of q N that is formed
  static constexpr int QH = S / 64;                  // tile holding limb S
  static constexpr int TMIN = -3;                    // Toeplitz bands t = TMIN..TMAX
  static constexpr int TMAX = (D + 62) / 64;
  static constexpr int UMIN = -1;                    // forward chunks u that can reach [0, D)
  static constexpr int UMAX = (D - 1) / 64;
  static constexpr int NU = UMAX - UMIN + 1;
  static constexpr int X0 = 64 * TMAX + 195;         // reversed array: byte X0 - i = digit i
  // A reversed array is kept as four copies, copy c at byte c PR holding it
  // shifted down by c bytes (see mma_tiles).  Every read of copy c lies in
  // [c PR, c PR + X0 + 253) and its digits in [c PR + X0 - D + 1 - c,
  // c PR + X0 - c], so neighbouring copies share their zero pads when
  // PR >= D + 256 and PR > X0.
  static constexpr int PR = ((D + 256 > X0 + 1 ? D + 256 : X0 + 1) + 15) & ~15;
  static constexpr int RBT = (3 * PR + X0 + 253 + 15) & ~15;  // bytes of the four copies
  static_assert(NTLO <= NT, "low product within the full one");
  static_assert(S % 64 != 0 && S >= 3, "limb S lies in the last tile of the low half");
  static_assert(QLO == QH && S - 64 * QH >= 2, "limbs S - 2 .. S in one tile");
  static_assert(D * 127 * 127 * 2 < (1ll << 31), "two products' column sums fit int32");
  static_assert((X0 & 3) == 3, "reversed limbs are dword aligned");
  static_assert(4 * S <= D8, "S limbs fit the digit region of a forward array");
};

// Per-wavefront LDS workspace.
template <class G>
struct MWork {
  uint8_t xr[G::RBT];    // x, reversed, four rotated copies (A operand)
  uint8_t tr[G::RBT];    // T mod R, the same
  uint8_t qr[G::RBT];    // q, the same
  uint8_t xf[G::FB];     // x, forward (B operand of a squaring)
};

using MConst = pc2k::MfmaConst;

constexpr uint32_t M28 = (1u << 28) - 1u;

// value of lane (l - 1) mod 64
__device__ __forceinline__ uint32_t rotate_up(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x13C /* wave_ror:1 */, 0xF, 0xF, false);
}

// limb (signed, -2^27 - 2^20 <= v < 2^28) -> its four digits as bytes, least
// significant first: three of 7 bits and the signed top digit v >> 21
__device__ __forceinline__ uint32_t limb_digits(uint32_t v) {
  return (v & 0x7Fu) | ((v << 1) & 0x7F00u) | ((v << 2) & 0x7F0000u) | ((v << 3) & 0xFF000000u);
}

// The B operand chunks of y, a forward digit array (LDS or global; digit i
// at byte PF + i): lane (j, g) takes digits [64 u + 4 j + 16 g, +16) of
// chunk u = UMIN + k into B[k], read as four dword-aligned words.  Chunks
// that no matrix product of the caller uses are dropped by the compiler.
template <class G>
__device__ __forceinline__ void load_b(v4i (&B)[G::NU], const uint8_t* y, int lane) {
  const int base = 4 * (lane & 15) + 16 * (lane >> 4);
#pragma unroll
  for (int k = 0; k < G::NU; ++k) {
    // chunks past the end of the digits (only in the last chunk, for some
    // lanes) are read from the zero front pad instead
    const int u = G::UMIN + k;
    int off = 64 * u + base;  // >= -64
    if (64 * u + 108 >= G::D8 && off >= G::D8) off = -G::PF;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(y + G::PF + off);
    B[k] = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  }
}

// Digit sums of x y for tiles Q0 .. NTQ - 1, y's B chunks in B (load_b).
// x: its reversed array in LDS; lane (i, g) takes the Toeplitz band of
// digits alpha(i) + 64 t - 16 g - s, s < 16, i.e. bytes
// X0 - alpha(i) - 64 t + 16 g .. +16, which start 3 - i % 4 bytes past a
// 16-byte boundary; in the copy rotated by that many bytes they start at the
// boundary, so every lane makes one aligned 16-byte read (unaligned LDS
// reads stall the LDS pipeline).  Tile Q, lane l: limb 64 Q + l, digit c in
// accumulator c.
// ACC: add to C instead of starting from zero.
template <class G, int NTQ, int Q0 = 0, bool ACC = false>
__device__ __forceinline__ void mma_tiles(v4i (&C)[NTQ], const uint8_t* xr, const v4i (&B)[G::NU],
                                          int lane) {
  const int i = lane & 15;
  const int sb = 3 - (i & 3);
  const uint8_t* bp = xr + sb * G::PR + G::X0 - 3 - 64 * (i >> 2) + 16 * (lane >> 4);
  if constexpr (!ACC) {
#pragma unroll
    for (int q = Q0; q < NTQ; ++q) C[q] = v4i{0, 0, 0, 0};
  }
  // a wavefront issuing matrix products goes first, so that the others'
  // vector instructions fill the matrix cores' busy cycles (measured: 4 %
  // faster at 2048 bits)
  __builtin_amdgcn_s_setprio(1);
#pragma unroll
  for (int t = G::TMIN; t <= G::TMAX; ++t) {
    bool any = false;
#pragma unroll
    for (int q = Q0; q < NTQ; ++q) {
      const int u = 4 * q - t;
      any |= (u >= G::UMIN && u <= G::UMAX);
    }
    if (!any) continue;
    const v4i a = *reinterpret_cast<const v4i*>(__builtin_assume_aligned(bp - 64 * t, 16));
#pragma unroll
    for (int q = Q0; q < NTQ; ++q) {
      const int u = 4 * q - t;
      if (u >= G::UMIN && u <= G::UMAX)
        C[q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, B[u - G::UMIN], C[q], 0, 0, 0);
    }
  }
  __builtin_amdgcn_s_setprio(0);
}

// the value of lane l (a constant) of a 64-bit register pair, wave-uniform
__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int32_t BIAS = 1 << 27;

// The column value of limb 64 q + lane from its four digit-column sums,
// plus 2^27, exactly (|value| < 2^47).  The weights sit in scalar registers
// the compiler cannot see through, so each term is one v_mad_i64_i32.
__device__ __forceinline__ int64_t fold_biased(const v4i& c, int32_t k7, int32_t k14,
                                               int32_t k21) {
  int64_t v = (int64_t)(c[0] + BIAS);
  v = (int64_t)c[1] * k7 + v;
  v = (int64_t)c[2] * k14 + v;
  v = (int64_t)c[3] * k21 + v;
  return v;
}

struct FoldK {
  int32_t k7 = 1 << 7, k14 = 1 << 14, k21 = 1 << 21;
  __device__ FoldK() { asm volatile("" : "+s"(k7), "+s"(k14), "+s"(k21)); }
};

// One balanced split of biased column values vb = v + 2^27: each limb keeps
// v - 2^28 carry (in [-2^27, 2^27)) and takes the carry of the limb below
// (lane - 1 of its tile, lane 63 of the tile below for lane 0, nothing for
// limb 0); cin[q] returns the carry each lane took.  |carry| < 2^20.
template <int NTQ>
__device__ __forceinline__ void split(int32_t (&l)[NTQ], int32_t (&cin)[NTQ],
                                      const int64_t (&vb)[NTQ], int lane) {
  int32_t c[NTQ];
#pragma unroll
  for (int q = 0; q < NTQ; ++q) {
    c[q] = (int32_t)__builtin_amdgcn_alignbit((uint32_t)((uint64_t)vb[q] >> 32), (uint32_t)vb[q],
                                              28);
    l[q] = (int32_t)((uint32_t)vb[q] & M28);
  }
  int32_t r[NTQ];
#pragma unroll
  for (int q = 0; q < NTQ; ++q) r[q] = (int32_t)rotate_up((uint32_t)c[q]);
#pragma unroll
  for (int q = 0; q < NTQ; ++q) {
    cin[q] = lane ? r[q] : (q ? r[q - 1] : 0);
    l[q] = l[q] + cin[q] - BIAS;
  }
}

// reversed dwords of limbs i and i - 1 (zero outside 0 .. S - 1) -> the four
// copies of a reversed array (i = -1 addresses the zero pad above digit 0)
template <class G>
__device__ __forceinline__ void put_rev(uint8_t* xr, int i, uint32_t w, uint32_t wp) {
  uint8_t* at = xr + G::X0 - 4 * i - 3;
  *reinterpret_cast<uint32_t*>(at) = w;
  *reinterpret_cast<uint32_t*>(at + G::PR) = __builtin_amdgcn_alignbyte(wp, w, 1);
  *reinterpret_cast<uint32_t*>(at + 2 * G::PR) = __builtin_amdgcn_alignbyte(wp, w, 2);
  *reinterpret_cast<uint32_t*>(at + 3 * G::PR) = __builtin_amdgcn_alignbyte(wp, w, 3);
}

// Write limbs lo .. lo + S - 1 (as limbs 0 .. S - 1) as digits.  Tiles with
// no such limb are skipped (lo is a constant at every call); in the others a
// lane outside the range writes zero into the zero pad above digit 0, so no
// lane branches.  Reversed arrays: the dword of limb g in copy c is made of
// the dwords of limbs g and g - 1 (the lane below), and the lane of limb S
// writes the copies' dwords that reach into limb S - 1.
template <class G, int NTQ>
__device__ __forceinline__ void write_rev(uint8_t* xr, const int32_t (&o)[NTQ], int lane,
                                          int lo) {
  uint32_t w[NTQ], r[NTQ];
#pragma unroll
  for (int q = 0; q < NTQ; ++q) {
    const int gi = 64 * q + lane - lo;
    const bool skip = 64 * q + 63 < lo || 64 * q - lo > G::S;
    w[q] = !skip && gi >= 0 && gi < G::S ? __builtin_bswap32(limb_digits((uint32_t)o[q])) : 0u;
  }
#pragma unroll
  for (int q = 0; q < NTQ; ++q) r[q] = rotate_up(w[q]);
#pragma unroll
  for (int q = 0; q < NTQ; ++q) {
    if (64 * q + 63 < lo || 64 * q - lo > G::S) continue;
    const int gi = 64 * q + lane - lo;
    const bool in = gi >= 0 && gi <= G::S;
    const uint32_t wp = lane ? r[q] : (q ? r[q - 1] : 0u);  // limb gi - 1
    // (outside 0 .. S both dwords are zero, and so is what the lane writes)
    put_rev<G>(xr, in ? gi : -1, w[q], wp);
  }
}
// (forward arrays also get their zero tail [D, D8 + 16) written, since the
// products read whole 16-byte chunks and global table entries start out
// uninitialised; the front pad is written once, with the table's slot)
template <class G, int NTQ>
__device__ __forceinline__ void write_fwd(uint8_t* y, const int32_t (&o)[NTQ], int lane,
                                          int lo) {
#pragma unroll
  for (int q = 0; q < NTQ; ++q) {
    if (64 * q + 63 < lo || 64 * q - lo >= G::S) continue;
    const int gi = 64 * q + lane - lo;
    const bool in = gi >= 0 && gi < G::S;
    const int at = in ? G::PF + 4 * gi : 0;  // out of range: zero into the front pad
    *reinterpret_cast<uint32_t*>(y + at) = in ? limb_digits((uint32_t)o[q]) : 0u;
  }
  if (lane < (G::D8 + 16) / 4 - G::S)
    *reinterpret_cast<uint32_t*>(y + G::PF + 4 * (G::S + lane)) = 0u;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// x <- x y R^-1 (mod N; |inputs| < N, |output| < 0.52 N), x in ws.xr; y a
// forward digit array (LDS or global); N and N' (K) are read from global
// memory, through the vector L1 cache, which leaves the LDS bandwidth to the
// per-element operands.  The result also goes, as forward
// digits, to ws.xf (fwd) and to out (if not null); plus_one adds 1 to it.
// U: the result's limbs (limb 64 q + lane - S in U[q] for q >= QH; the
// entries below are zero).
template <class G>
__device__ __forceinline__ void mont_mul(MWork<G>& ws, const MConst& K, const uint8_t* y,
                                         int lane, bool fwd, uint8_t* out, bool plus_one,
                                         int32_t (&U)[G::NT]) {
  constexpr int NT = G::NT, NL = G::NTLO, QH = G::QH, NH = NT - QH;
  const FoldK k;
  const int ls = G::S - 64 * QH;  // lane of limb S in tile QH
  v4i C[NT];                      // digit columns of T, then of T + q N
  v4i B[G::NU];                   // B operand chunks: y, then N', then N
  load_b<G>(B, y, lane);
  mma_tiles<G, NT>(C, ws.xr, B, lane);
  // the constants' chunks are loaded before the fold that precedes their
  // products, so that their latency hides behind it (measured: 2-3 % faster)
  load_b<G>(B, K.Np, lane);
  int32_t Lq[NL];                 // T mod R (limbs below S)
  {
    int64_t vb[NL];
    int32_t cin[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) vb[q] = fold_biased(C[q], k.k7, k.k14, k.k21);
    split<NL>(Lq, cin, vb, lane);
    // the carry out of limb S - 1 joins column S
    if (lane == ls) C[QH][0] += cin[QH];
    write_rev<G, NL>(ws.tr, Lq, lane, 0);
  }
  wave_sync();
  {
    v4i Cq[NL];
    int64_t vb[NL];
    int32_t Q[NL], cin[NL];
    mma_tiles<G, NL>(Cq, ws.tr, B, lane);
    load_b<G>(B, K.N, lane);
#pragma unroll
    for (int q = 0; q < NL; ++q) vb[q] = fold_biased(Cq[q], k.k7, k.k14, k.k21);
    split<NL>(Q, cin, vb, lane);  // limbs from S up are not written: q mod R
    write_rev<G, NL>(ws.qr, Q, lane, 0);
  }
  // below limb S, tile QH carries T mod R as limb values into q N
  if (lane < ls) C[QH] = v4i{Lq[QH], 0, 0, 0};
  wave_sync();
  mma_tiles<G, NT, QH, true>(C, ws.qr, B, lane);
  int64_t vb[NH];
#pragma unroll
  for (int q = 0; q < NH; ++q) vb[q] = fold_biased(C[QH + q], k.k7, k.k14, k.k21);
  // c = (the part of T + q N below limb S) / R, rounded from columns S - 1
  // and S - 2
  {
    const int64_t a = (int64_t)read_lane64((uint64_t)vb[0], ls - 1) - BIAS;
    const int64_t b = (int64_t)read_lane64((uint64_t)vb[0], ls - 2) - BIAS;
    const int64_t c = (a + (b >> 28) + BIAS) >> 28;
    if (lane == ls) vb[0] += c + (plus_one ? 1 : 0);
  }
  {
    int32_t Uh[NH], cin[NH];
    split<NH>(Uh, cin, vb, lane);
    // limb S takes no carry from below (the low part is c R)
    if (lane == ls) Uh[0] -= cin[0];
#pragma unroll
    for (int q = 0; q < NT; ++q) U[q] = q < QH ? 0 : Uh[q - QH];
  }
  write_rev<G, NT>(ws.xr, U, lane, G::S);
  if (fwd) write_fwd<G, NT>(ws.xf, U, lane, G::S);
  if (out) write_fwd<G, NT>(out, U, lane, G::S);
  wave_sync();
}

// bits [28 i, 28 i + 28) of a little-endian uint32 array of n words
__device__ __forceinline__ uint32_t limb28_of(const uint32_t* a, int n, int i) {
  const int b = 28 * i, w = b >> 5, s = b & 31;
  const uint64_t lo = w < n ? a[w] : 0u, hi = w + 1 < n ? a[w + 1] : 0u;
  return (uint32_t)(((hi << 32) | lo) >> s) & M28;
}

// x (n 32-bit words, x < R) -> ws.xr
template <class G>
__device__ __forceinline__ void load_x(MWork<G>& ws, const uint32_t* x, int n, int lane) {
  for (int i = lane; i <= G::S; i += 64) {
    const uint32_t w = i < G::S ? __builtin_bswap32(limb_digits(limb28_of(x, n, i))) : 0u;
    const uint32_t wp = i > 0 ? __builtin_bswap32(limb_digits(limb28_of(x, n, i - 1))) : 0u;
    put_rev<G>(ws.xr, i, w, wp);
  }
  wave_sync();
}

// forward digit array (LDS or global) -> ws.xr and ws.xf
template <class G>
__device__ __forceinline__ void load_fwd(MWork<G>& ws, const uint8_t* y, int lane) {
  for (int i = lane; i <= G::S; i += 64) {
    const uint32_t d = i < G::S ? *reinterpret_cast<const uint32_t*>(y + G::PF + 4 * i) : 0u;
    const uint32_t dp = i > 0 ? *reinterpret_cast<const uint32_t*>(y + G::PF + 4 * i - 4) : 0u;
    put_rev<G>(ws.xr, i, __builtin_bswap32(d), __builtin_bswap32(dp));
    if (i < G::S) *reinterpret_cast<uint32_t*>(ws.xf + G::PF + 4 * i) = d;
  }
  wave_sync();
}

// zero the workspace's digit arrays
template <class G>
__device__ __forceinline__ void init_work(MWork<G>& ws, int lane) {
  uint32_t* z = reinterpret_cast<uint32_t*>(ws.xr);
  constexpr int ZW = (3 * G::RBT + G::FB) / 4;
  static_assert(sizeof(MWork<G>) == 3 * G::RBT + G::FB, "no padding between the arrays");
  for (int i = lane; i < ZW; i += 64) z[i] = 0u;
  wave_sync();
}

// zero the front pads of a workgroup's table entries (global)
template <class G>
__device__ __forceinline__ void init_table(uint8_t* table, int entries, int lane) {
  for (int k = 0; k < entries; ++k)
    for (int i = lane; i < G::PF / 4; i += 64)
      reinterpret_cast<uint32_t*>(table + (size_t)k * G::FB)[i] = 0u;
  wave_sync();
}

}  // namespace pc2m
