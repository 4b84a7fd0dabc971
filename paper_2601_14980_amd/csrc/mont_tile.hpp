// Lazy-carry Montgomery arithmetic for CDNA4 (gfx950), one number per "tile"
// of T adjacent lanes.
//
// Representation.  A residue modulo an odd N is held as S = K*T digits of D
// bits (D = 27 or 28); lane t of a tile owns digits [t*K, t*K + K).  Digits
// are "semi-normalised": each is < 2^D + 2^11, so a value is not unique but
// products of two digits stay below 2^(2D+1).
//
// Product.  mont_mul computes a*b*R^-1 mod N (R = 2^(D*S)) by operand
// scanning: for every digit b_i (read from LDS, broadcast to the tile) each
// lane adds a_j*b_i + m*N_j into 64-bit column accumulators with one
// v_mad_u64_u32 each -- no carry chain -- and the division by 2^D is a
// register shift folded into the destination index.  An accumulator gains
// two products per step; when S steps could overflow 64 bits (28-bit digits
// beyond 127 steps) the product pauses every Geo::SEG steps to renormalise:
// each accumulator keeps its low D bits and hands the rest to the next digit
// position, which leaves the represented value unchanged.
// Only digit 0 of the tile needs its carry resolved each step; the other
// lanes pass their lowest accumulator one lane down (DPP).  With 4N < R the
// result of inputs < 2N stays < 2N, so no conditional subtraction is needed
// until the very end of an exponentiation.
//
// This is the MI355X-native replacement of the FFT product + Barrett
// reduction of the paper's Algorithm 2: on gfx950 v_mad_u64_u32 issues at
// full rate, so a schoolbook product with one instruction per limb product
// beats a floating-point FFT at these operand sizes and is exact by
// construction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc2d {

template <int D_, int K_, int T_>
struct Geo {
  static constexpr int D = D_;
  static constexpr int K = K_;
  static constexpr int T = T_;
  static constexpr int S = K_ * T_;
  static constexpr int K4 = (K_ + 3) & ~3;       // per-lane chunk, padded to 16 B
  static constexpr int SP = ((S + 3) & ~3);      // LDS words of one number
  static constexpr int CH = T_ * K4;             // words of one number in chunked layout
  static constexpr uint32_t MASK = (1u << D_) - 1u;
  // steps an accumulator can take from a renormalised start (< 2^40) with two
  // products below (2^D + 2^11)^2 each per step and one carry (< 2^40)
  static constexpr int NSTEP =
      (int)((~0ull - (1ull << 41)) /
            (2 * ((1ull << (2 * D_)) + (1ull << (D_ + 12)) + (1ull << 22))));
  static constexpr int NSEG = (S + NSTEP - 1) / NSTEP;      // segments of a product
  static constexpr int SEG = ((S + NSEG - 1) / NSEG + 1) & ~1;  // steps per segment, even
  static_assert(SEG <= NSTEP, "a segment stays within the accumulators' headroom");
  static_assert(K_ >= 2, "at least two digits per lane");
  static_assert(T_ == 1 || T_ == 2 || T_ == 4 || T_ == 8, "tile of 1, 2, 4 or 8 lanes");
};

// ---------------------------------------------------------------- DPP moves
// Tiles are aligned groups of T lanes inside a DPP row of 16.  quad_perm
// controls select a source lane inside each quad; row_shl:1 / row_shr:1 move
// values one lane down / up inside the row (the tile-boundary lanes receive a
// neighbour tile's value and are masked by the callers).  A lane whose source
// is outside the row reads zero (bound control), which also lets the
// compiler fold a move into the instruction that consumes it.
enum : int {
  DPP_QUAD_0000 = 0x00,
  DPP_ROW_SHL1 = 0x101,
  DPP_ROW_SHR1 = 0x111,
  DPP_ROW_SHR4 = 0x114,
};
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  uint32_t lo = dpp32<CTRL>((uint32_t)v), hi = dpp32<CTRL>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// value of tile lane 0, in every lane of the tile
template <int T>
__device__ __forceinline__ uint32_t tile_bcast0(uint32_t v) {
  if constexpr (T == 1) {
    return v;
  } else if constexpr (T == 2) {
    return dpp32<0xA0>(v);  // quad_perm [0,0,2,2]
  } else if constexpr (T == 4) {
    return dpp32<DPP_QUAD_0000>(v);
  } else {
    // lane 0 of each quad, then lanes 4-7 of the octet take it from lanes 0-3
    uint32_t q = dpp32<DPP_QUAD_0000>(v);
    return (uint32_t)__builtin_amdgcn_update_dpp((int)q, (int)q, DPP_ROW_SHR4, 0xF, 0xA, false);
  }
}
// tile_bcast0(v) & mask, written so that the mask fuses with the first lane
// move (the bitwise and commutes with moving lanes)
template <int T>
__device__ __forceinline__ uint32_t tile_bcast0_masked(uint32_t v, uint32_t mask) {
  if constexpr (T == 8) {
    uint32_t q = dpp32<DPP_QUAD_0000>(v) & mask;
    return (uint32_t)__builtin_amdgcn_update_dpp((int)q, (int)q, DPP_ROW_SHR4, 0xF, 0xA, false);
  } else {
    return tile_bcast0<T>(v) & mask;
  }
}
// value of tile lane t+1 (meaningless in the top lane of the tile)
template <int T>
__device__ __forceinline__ uint32_t tile_from_next32(uint32_t v) {
  if constexpr (T == 1) return 0;
  else return dpp32<DPP_ROW_SHL1>(v);
}
// value of tile lane t-1 (meaningless in lane 0 of the tile)
template <int T>
__device__ __forceinline__ uint64_t tile_from_prev(uint64_t v) {
  if constexpr (T == 1) return 0;
  else return dpp64<DPP_ROW_SHR1>(v);
}

__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * b + c;
}

// ------------------------------------------------------------ normalisation
// Turn lazy 64-bit column accumulators into semi-normalised digits.
// The represented value must be < R (true for every Montgomery output here).
template <class G>
__device__ __forceinline__ void semi_normalise(uint32_t (&out)[G::K], const uint64_t (&acc)[G::K],
                                               int tl) {
  uint64_t carry = 0;
#pragma unroll
  for (int j = 0; j < G::K; ++j) {
    uint64_t v = acc[j] + carry;
    out[j] = (uint32_t)v & G::MASK;
    carry = v >> G::D;
  }
  if constexpr (G::T > 1) {
    uint64_t cin = tile_from_prev<G::T>(carry);
    if (tl == 0) cin = 0;
    uint64_t v = (uint64_t)out[0] + cin;
    out[0] = (uint32_t)v & G::MASK;
    out[1] += (uint32_t)(v >> G::D);
  }
}

// Between two steps of a product: every accumulator keeps its low D bits and
// adds the high part of the one below; a lane's top carry goes to the next
// lane's digit 0, and the top lane of the tile keeps its top accumulator
// whole (it is zero between steps).  The value represented is unchanged.
template <class G>
__device__ __forceinline__ void renormalise(uint64_t (&acc)[G::K], int tl) {
  constexpr int K = G::K, D = G::D;
  const bool low = (tl == 0), top = (tl == G::T - 1);
  const uint64_t cin = tile_from_prev<G::T>(acc[K - 1] >> D);
  const uint64_t topmask = top ? ~0ull : (uint64_t)G::MASK;
#pragma unroll
  for (int j = K - 1; j >= 1; --j)
    acc[j] = (acc[j] & (j == K - 1 ? topmask : (uint64_t)G::MASK)) + (acc[j - 1] >> D);
  acc[0] = (acc[0] & G::MASK) + (low ? 0ull : cin);
}

// --------------------------------------------------------- Montgomery product
// Digits of b consumed per LDS read (1, 2 or 4).
#ifndef MM_BSTEP
#define MM_BSTEP 2
#endif
// out = a * b * R^-1 mod N (lazy: out < 2N if a, b < 2N; also if a < 4N, b < N).
// a, N: this lane's K digits; b: the tile's S digits in LDS (16-B aligned).
template <class G>
__device__ __forceinline__ void mont_mul(uint32_t (&out)[G::K], const uint32_t (&a)[G::K],
                                         const uint32_t* __restrict__ b,
                                         const uint32_t (&N)[G::K], uint32_t nprime, int tl) {
  constexpr int K = G::K, T = G::T, D = G::D;
  uint64_t acc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = 0;
  // One step: the columns shift down one digit.  Digit 0's low D bits move to
  // the previous lane's top digit and its high part stays in this lane's
  // digit 0, so only 32 bits cross lanes.  In lane 0 of every tile those low
  // bits are zero by the choice of m (they leave the number), and that zero
  // is what the top lane of the tile below reads, so the top digit needs no
  // masking (every tile of a wavefront runs the same step on its own
  // operands; the last lane of a row reads zero by bound control).
  // The digit mask sits in a register so that each lane move below fuses
  // with its masking into one DPP-form v_and_b32 (a DPP operand pair takes
  // no literal); the moves fill with zero where a source lane is absent.
  uint32_t vmask = G::MASK;
  asm volatile("" : "+v"(vmask));
  auto step = [&](uint32_t bi) {
    uint64_t x0 = mad64(a[0], bi, acc[0]);
    uint32_t m = tile_bcast0_masked<T>((uint32_t)x0 * nprime, vmask);
    x0 = mad64(m, N[0], x0);
#pragma unroll
    for (int j = 1; j < K; ++j) acc[j - 1] = mad64(m, N[j], mad64(a[j], bi, acc[j]));
    acc[K - 1] = (uint64_t)(tile_from_next32<T>((uint32_t)x0) & vmask);
    acc[0] += x0 >> D;
  };
  int i = 0;
  for (int seg = 0; seg < G::NSEG; ++seg) {
    const int end = (seg + 1) * G::SEG < G::S ? (seg + 1) * G::SEG : G::S;
    if constexpr (MM_BSTEP == 4) {
      for (; i + 4 <= end; i += 4) {
        uint4 v = *reinterpret_cast<const uint4*>(b + i);
        step(v.x);
        step(v.y);
        step(v.z);
        step(v.w);
      }
    } else if constexpr (MM_BSTEP == 2) {
      for (; i + 2 <= end; i += 2) {
        uint2 v = *reinterpret_cast<const uint2*>(b + i);
        step(v.x);
        step(v.y);
      }
    } else {
#pragma unroll 1
      for (; i + 1 <= end; i += 1) step(b[i]);
    }
    if (seg + 1 < G::NSEG) renormalise<G>(acc, tl);
  }
#pragma unroll
  for (int r = 0; r < (G::S % MM_BSTEP); ++r) step(b[i + r]);
  semi_normalise<G>(out, acc, tl);
}

// out = W * R^-1 mod N for a wide W = lo + hi * R with lo, hi < R
// (Montgomery reduction of a double-length number).  lo: this lane's K
// digits; hi: the tile's S digits in LDS.  Requires W < N*R; out < W/R + N.
template <class G>
__device__ __forceinline__ void mont_redc_wide(uint32_t (&out)[G::K], const uint32_t (&lo)[G::K],
                                               const uint32_t* __restrict__ hi,
                                               const uint32_t (&N)[G::K], uint32_t nprime, int tl) {
  constexpr int K = G::K, T = G::T, D = G::D;
  uint64_t acc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = lo[j];
  const bool top = (tl == T - 1);
  for (int i = 0; i < G::S; ++i) {  // the step of mont_mul without the a*b products
    uint32_t hin = hi[i];
    uint64_t x0 = acc[0];
    uint32_t m = tile_bcast0<T>(((uint32_t)x0 * nprime) & G::MASK);
    x0 = mad64(m, N[0], x0);
#pragma unroll
    for (int j = 1; j < K; ++j) acc[j - 1] = mad64(m, N[j], acc[j]);
    const uint32_t lo = tile_from_next32<T>((uint32_t)x0 & G::MASK);
    acc[K - 1] = top ? (uint64_t)hin : (uint64_t)lo;
    acc[0] += x0 >> D;
  }
  semi_normalise<G>(out, acc, tl);
}

// ------------------------------------------------------------ data movement
// chunked layout in global memory: lane t's digits at [t*K4, t*K4 + K)
template <class G>
__device__ __forceinline__ void load_chunk(uint32_t (&x)[G::K], const uint32_t* __restrict__ base,
                                           int tl) {
  const uint32_t* p = base + tl * G::K4;
#pragma unroll
  for (int j4 = 0; j4 < G::K4; j4 += 4) {
    uint4 v = *reinterpret_cast<const uint4*>(p + j4);
    if (j4 + 0 < G::K) x[j4 + 0] = v.x;
    if (j4 + 1 < G::K) x[j4 + 1] = v.y;
    if (j4 + 2 < G::K) x[j4 + 2] = v.z;
    if (j4 + 3 < G::K) x[j4 + 3] = v.w;
  }
}
template <class G>
__device__ __forceinline__ void store_chunk(uint32_t* __restrict__ base, const uint32_t (&x)[G::K],
                                            int tl) {
  uint32_t* p = base + tl * G::K4;
#pragma unroll
  for (int j4 = 0; j4 < G::K4; j4 += 4) {
    uint4 v;
    v.x = (j4 + 0 < G::K) ? x[j4 + 0] : 0u;
    v.y = (j4 + 1 < G::K) ? x[j4 + 1] : 0u;
    v.z = (j4 + 2 < G::K) ? x[j4 + 2] : 0u;
    v.w = (j4 + 3 < G::K) ? x[j4 + 3] : 0u;
    *reinterpret_cast<uint4*>(p + j4) = v;
  }
}
// tile's LDS number: lane t writes digits [t*K, t*K + K)
template <class G>
__device__ __forceinline__ void to_lds(uint32_t* __restrict__ lds, const uint32_t (&x)[G::K], int tl) {
#pragma unroll
  for (int j = 0; j < G::K; ++j) lds[tl * G::K + j] = x[j];
}

// Extract digit g (D bits at bit g*D) of a little-endian 32-bit limb array.
// Branch-free: out-of-range limbs are read at a clamped index and replaced
// by zero.
__device__ __forceinline__ uint32_t limb_at(const uint32_t* __restrict__ v, int nlimbs, int w) {
  uint32_t x = v[w < nlimbs ? w : nlimbs - 1];
  return w < nlimbs ? x : 0u;
}
template <int D>
__device__ __forceinline__ uint32_t limb_digit(const uint32_t* __restrict__ v, int nlimbs, int g) {
  int bit = g * D;
  int w = bit >> 5, s = bit & 31;
  uint64_t lo = limb_at(v, nlimbs, w);
  uint64_t hi = limb_at(v, nlimbs, w + 1);
  return (uint32_t)(((hi << 32) | lo) >> s) & ((1u << D) - 1u);
}
// The tile's S digits of the integer v (nlimbs limbs), starting at digit g0,
// written to the tile's LDS number.  Digits are spread over the lanes of the
// tile in a runtime loop so that the limb loads are not all hoisted at once.
template <class G>
__device__ __forceinline__ void lds_digits_from_limbs(uint32_t* __restrict__ lds,
                                                      const uint32_t* __restrict__ v, int nlimbs,
                                                      int g0, int tl) {
#pragma unroll 2
  for (int g = tl; g < G::S; g += G::T) lds[g] = limb_digit<G::D>(v, nlimbs, g0 + g);
}
// the tile's LDS number <- a chunked number in global memory (no register array)
template <class G>
__device__ __forceinline__ void lds_from_chunk(uint32_t* __restrict__ lds, const uint32_t* __restrict__ p,
                                               int tl) {
  const uint32_t* src = p + tl * G::K4;
#pragma unroll 2
  for (int j = 0; j < G::K; ++j) lds[tl * G::K + j] = src[j];
}
// chunked number (global) <- digits g0.. of the integer v (nlimbs limbs)
template <class G>
__device__ __forceinline__ void chunk_from_limbs(uint32_t* __restrict__ dst, const uint32_t* __restrict__ v,
                                                 int nlimbs, int g0, int tl) {
  uint32_t* d = dst + tl * G::K4;
#pragma unroll 2
  for (int j = 0; j < G::K; ++j) d[j] = limb_digit<G::D>(v, nlimbs, g0 + tl * G::K + j);
}
// this lane's K digits of the tile's LDS number
template <class G>
__device__ __forceinline__ void from_lds(uint32_t (&x)[G::K], const uint32_t* __restrict__ lds, int tl) {
#pragma unroll
  for (int j = 0; j < G::K; ++j) x[j] = lds[tl * G::K + j];
}

// Wave-level ordering of LDS traffic between the lanes of a tile.  Kernels
// that use it run one wavefront per workgroup, so this is a fence, not a
// rendezvous of several waves.
__device__ __forceinline__ void lds_sync() { __syncthreads(); }

}  // namespace pc2d
