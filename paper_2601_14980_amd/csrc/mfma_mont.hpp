// Montgomery multiplication on the i8 matrix cores (MFMA) of gfx950.
//
// A residue x mod N (R = 2^(28 S) > 4N) is held as S limbs of 28 bits or,
// for the matrix products, as D = 4S digits of 7 bits (one byte each, so
// the signed i8 operands are never negative).  One wavefront works on one
// element.  The three limb-product matrices of a separated Montgomery
// product
//
//     T = x y,    q = (T mod R) N' mod R  (N' = -N^-1 mod R),    U = (T + q N) / R
//
// are each computed exactly by v_mfma_i32_16x16x64_i8 with int32
// accumulation: one instruction adds, for a 16 x 16 tile of output columns
// p = 256 Q + 16 j + r, the 64 digit products a_i b_(p-i) with
// i = 64 t + r - k (k < 64) -- a Toeplitz band of a times a block of b.
// Column sums stay below D 127^2 < 2^24.  The carry propagation is explicit:
// four columns fold into one 28-bit limb position of a 64-bit value, a
// lane-local pass and one lane shift leave carries of 0 or 1, and a
// wave-wide carry-lookahead (two ballots and one 64-bit add) resolves them.
//
// Work per product: D^2 digit products (7-bit digits), against 2 S^2 limb
// products (28-bit) for the VALU form in mont_tile.hpp.
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
  static constexpr int D8 = (D + 15) & ~15;          // bytes of a forward digit array
  static constexpr int LPL = (2 * S + 1 + 63) / 64;  // limbs per lane of a double-length value
  static constexpr int NT = LPL;                     // 256-column tiles of a full product
  static constexpr int NTLO = (D + 255) / 256;       // tiles of a product taken mod R
  static constexpr int TMAX = (D + 62) / 64;         // Toeplitz bands t = 0..TMAX
  static constexpr int UMIN = -4;                    // forward chunks u that can reach [0, D)
  static constexpr int UMAX = (D - 1) / 64;
  static constexpr int NU = UMAX - UMIN + 1;
  static constexpr int X0 = 64 * TMAX + 15;          // reversed array: byte X0 - i = digit i
  static constexpr int RB = (X0 + 64 + 15) & ~15;    // bytes of a reversed digit array
  static constexpr int COLS = 256 * NT;              // int32 column sums
  static_assert(NTLO <= NT, "low product within the full one");
  static_assert((X0 & 3) == 3, "reversed limbs are dword aligned");
};

// Per-wavefront LDS workspace.
template <class G>
struct MWork {
  int cols[G::COLS];     // column sums of the last product
  uint8_t xr[G::RB];     // x, reversed (A operand)
  uint8_t tr[G::RB];     // T mod R, reversed
  uint8_t qr[G::RB];     // q, reversed
  uint8_t xf[G::D8];     // x, forward (B operand of a squaring)
  uint8_t gm[G::D8];     // a per-element multiplier, forward
  uint8_t nf[G::D8];     // N, forward
  uint8_t npf[G::D8];    // N', forward
};

using MConst = pc2k::MfmaConst;

constexpr uint32_t M28 = (1u << 28) - 1u;

// value of lane l - 1, 0 in lane 0
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xF, 0xF,
                                               false);
}

// 28-bit limb -> its four 7-bit digits as bytes, least significant first
__device__ __forceinline__ uint32_t limb_digits(uint32_t v) {
  return (v & 0x7Fu) | ((v << 1) & 0x7F00u) | ((v << 2) & 0x7F0000u) | ((v << 3) & 0x7F000000u);
}

// B operand chunks of a forward digit array (LDS or global, 16-byte aligned):
// lane (j, g) takes bytes [64 u + 16 j + 16 g, +16) for u = UMIN..UMAX.
template <class G>
__device__ __forceinline__ void load_b(v4i (&B)[G::NU], const uint8_t* y, int lane) {
  const int base = 16 * (lane & 15) + 16 * (lane >> 4);
#pragma unroll
  for (int u = 0; u < G::NU; ++u) {
    const int off = 64 * (u + G::UMIN) + base;
    B[u] = (off >= 0 && off < G::D8) ? *reinterpret_cast<const v4i*>(y + off) : v4i{0, 0, 0, 0};
  }
}

// Column sums of x y for the NTQ lowest tiles: x from its reversed array in
// LDS (lane (r, g) reads bytes X0 - 64 t - r + 16 g .. +16, i.e. digits
// 64 t + r - 16 g - s), y as preloaded B chunks.
template <class G, int NTQ>
__device__ __forceinline__ void product(v4i (&C)[NTQ], const uint8_t* xr, const v4i (&B)[G::NU],
                                        int lane) {
  const uint8_t* ap = xr + G::X0 - (lane & 15) + 16 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < NTQ; ++q) C[q] = v4i{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t <= G::TMAX; ++t) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < NTQ; ++q) {
      const int u = 4 * q - t - G::UMIN;
      any |= (u >= 0 && u < G::NU);
    }
    if (!any) continue;
    // 16 unaligned bytes as two 8-byte LDS reads
    uint64_t lo, hi;
    __builtin_memcpy(&lo, ap - 64 * t, 8);
    __builtin_memcpy(&hi, ap - 64 * t + 8, 8);
    const v4i a = v4i{(int)(uint32_t)lo, (int)(uint32_t)(lo >> 32), (int)(uint32_t)hi,
                      (int)(uint32_t)(hi >> 32)};
#pragma unroll
    for (int q = 0; q < NTQ; ++q) {
      const int u = 4 * q - t - G::UMIN;
      if (u >= 0 && u < G::NU)
        C[q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, B[u], C[q], 0, 0, 0);
    }
  }
}

// C tile q, lane (j, g) holds columns 256 q + 16 j + 4 g + 0..3
template <int NTQ>
__device__ __forceinline__ void store_cols(int* cols, const v4i (&C)[NTQ], int lane) {
  int* p = cols + 16 * (lane & 15) + 4 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < NTQ; ++q) *reinterpret_cast<v4i*>(p + 256 * q) = C[q];
}

// Lane l owns limbs l LPL .. l LPL + LPL - 1: four columns per limb.
template <class G>
__device__ __forceinline__ void fold(uint64_t (&v)[G::LPL], const int* cols, int lane) {
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const v4i c = *reinterpret_cast<const v4i*>(cols + 4 * (lane * G::LPL + i));
    v[i] = (uint64_t)(uint32_t)c[0] + ((uint64_t)(uint32_t)c[1] << 7) +
           ((uint64_t)(uint32_t)c[2] << 14) + ((uint64_t)(uint32_t)c[3] << 21);
  }
}

// 64-bit limb values (< 2^47) -> 28-bit limbs with all carries resolved
// across the wavefront; the carry out of the top limb is dropped.
template <class G>
__device__ __forceinline__ void normalize(uint32_t (&o)[G::LPL], const uint64_t (&v)[G::LPL],
                                          int lane) {
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const uint64_t s = v[i] + c;
    o[i] = (uint32_t)s & M28;
    c = s >> 28;
  }
  // c < 2^20 for the values of a product (v < 2^47), so nothing wraps below
  uint32_t k = from_prev_lane((uint32_t)c);
  bool all = true;
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const uint32_t s = o[i] + k;
    o[i] = s & M28;
    k = s >> 28;
    all &= (o[i] == M28);
  }
  // carry-lookahead over lanes: lane l generates (k = 1) or propagates
  // (all limbs 2^28 - 1); the carry into lane l is bit l of
  // ((G | P) + G) ^ (G | P) ^ G
  const uint64_t gen = __ballot(k != 0);
  const uint64_t prop = __ballot(all && k == 0);
  const uint64_t a = gen | prop;
  uint32_t cin = (uint32_t)((((a + gen) ^ a ^ gen) >> lane) & 1ull);
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const uint32_t s = o[i] + cin;
    o[i] = s & M28;
    cin = s >> 28;
  }
}

// Write limbs with index lo .. lo + S - 1 (as limbs 0 .. S - 1) as digits.
template <class G>
__device__ __forceinline__ void write_rev(uint8_t* xr, const uint32_t (&o)[G::LPL], int lane,
                                          int lo) {
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const int gi = lane * G::LPL + i - lo;
    if (gi >= 0 && gi < G::S)
      *reinterpret_cast<uint32_t*>(xr + G::X0 - 4 * gi - 3) = __builtin_bswap32(limb_digits(o[i]));
  }
}
// (forward arrays also get their zero padding [D, D8) written, since the
// products read whole 8-byte chunks and global table entries start out
// uninitialised)
template <class G>
__device__ __forceinline__ void write_fwd(uint8_t* y, const uint32_t (&o)[G::LPL], int lane,
                                          int lo) {
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    const int gi = lane * G::LPL + i - lo;
    if (gi >= 0 && gi < G::S) *reinterpret_cast<uint32_t*>(y + 4 * gi) = limb_digits(o[i]);
  }
  if (lane < G::D8 / 4 - G::S) *reinterpret_cast<uint32_t*>(y + 4 * (G::S + lane)) = 0u;
}

__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// x <- x y R^-1 mod N (inputs < 2N, output < 2N), x in ws.xr; y a forward
// digit array (LDS or global).  The result also goes, as forward digits, to
// ws.xf (fwd) and to out (if not null); plus_one adds 1 to the result
// before its carries are resolved.  U holds the result's limbs on return
// (lane l: limbs l LPL + i - S).
template <class G>
__device__ __forceinline__ void mont_mul(MWork<G>& ws, const uint8_t* y, int lane, bool fwd,
                                         uint8_t* out, bool plus_one, uint32_t (&U)[G::LPL]) {
  v4i B[G::NU];
  uint64_t v[G::LPL];
  uint32_t T[G::LPL];
  {
    v4i C[G::NT];
    load_b<G>(B, y, lane);
    product<G, G::NT>(C, ws.xr, B, lane);
    store_cols<G::NT>(ws.cols, C, lane);
  }
  wave_sync();
  fold<G>(v, ws.cols, lane);
  normalize<G>(T, v, lane);
  write_rev<G>(ws.tr, T, lane, 0);
  wave_sync();
  {
    v4i C[G::NTLO];
    load_b<G>(B, ws.npf, lane);
    product<G, G::NTLO>(C, ws.tr, B, lane);
    store_cols<G::NTLO>(ws.cols, C, lane);
  }
  wave_sync();
  fold<G>(v, ws.cols, lane);
#pragma unroll
  for (int i = 0; i < G::LPL; ++i)
    if (lane * G::LPL + i >= G::S) v[i] = 0;
  normalize<G>(U, v, lane);
  write_rev<G>(ws.qr, U, lane, 0);
  wave_sync();
  {
    v4i C[G::NT];
    load_b<G>(B, ws.nf, lane);
    product<G, G::NT>(C, ws.qr, B, lane);
    store_cols<G::NT>(ws.cols, C, lane);
  }
  wave_sync();
  fold<G>(v, ws.cols, lane);
#pragma unroll
  for (int i = 0; i < G::LPL; ++i) {
    v[i] += T[i];
    if (plus_one && lane * G::LPL + i == G::S) v[i] += 1;
  }
  normalize<G>(U, v, lane);
  write_rev<G>(ws.xr, U, lane, G::S);
  if (fwd) write_fwd<G>(ws.xf, U, lane, G::S);
  if (out) write_fwd<G>(out, U, lane, G::S);
  wave_sync();
}

// bits [28 i, 28 i + 28) of a little-endian uint32 array of n words
__device__ __forceinline__ uint32_t limb28_of(const uint32_t* a, int n, int i) {
  const int b = 28 * i, w = b >> 5, s = b & 31;
  const uint64_t lo = w < n ? a[w] : 0u, hi = w + 1 < n ? a[w + 1] : 0u;
  return (uint32_t)(((hi << 32) | lo) >> s) & M28;
}

// x (n 32-bit words, x < R) -> ws.xr (and ws.xf if fwd)
template <class G>
__device__ __forceinline__ void load_x(MWork<G>& ws, const uint32_t* x, int n, int lane,
                                       bool fwd) {
  for (int i = lane; i < G::S; i += 64) {
    const uint32_t d = limb_digits(limb28_of(x, n, i));
    *reinterpret_cast<uint32_t*>(ws.xr + G::X0 - 4 * i - 3) = __builtin_bswap32(d);
    if (fwd) *reinterpret_cast<uint32_t*>(ws.xf + 4 * i) = d;
  }
  wave_sync();
}

// forward digit array (LDS or global) -> ws.xr and ws.xf
template <class G>
__device__ __forceinline__ void load_fwd(MWork<G>& ws, const uint8_t* y, int lane) {
  for (int i = lane; i < G::S; i += 64) {
    const uint32_t d = *reinterpret_cast<const uint32_t*>(y + 4 * i);
    *reinterpret_cast<uint32_t*>(ws.xr + G::X0 - 4 * i - 3) = __builtin_bswap32(d);
    *reinterpret_cast<uint32_t*>(ws.xf + 4 * i) = d;
  }
  wave_sync();
}

// zero the workspace's digit arrays and copy N, N' into it
template <class G>
__device__ __forceinline__ void init_work(MWork<G>& ws, const MConst& K, int lane) {
  uint32_t* z = reinterpret_cast<uint32_t*>(ws.xr);
  constexpr int ZW = (3 * G::RB + 2 * G::D8) / 4;
  for (int i = lane; i < ZW; i += 64) z[i] = 0u;
  for (int i = lane; i < G::D8 / 4; i += 64) {
    reinterpret_cast<uint32_t*>(ws.nf)[i] = reinterpret_cast<const uint32_t*>(K.N)[i];
    reinterpret_cast<uint32_t*>(ws.npf)[i] = reinterpret_cast<const uint32_t*>(K.Np)[i];
  }
  wave_sync();
}

}  // namespace pc2m
