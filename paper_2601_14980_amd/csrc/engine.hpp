// A small sequencer that runs one "Montgomery program" per tile with a single
// inlined copy of the Montgomery product:
//
//   [pre0] [pre1]  table  powering  [post0] [post1]
//
// The powering is either left-to-right fixed windows (table x^1..x^(2^w-1);
// per-tile exponents) or, when the exponent is shared by the wavefront and a
// schedule was precomputed for it, left-to-right sliding windows (table of
// the odd powers x^1, x^3, ..., x^(2^w-1); about w/(w+1) as many window
// products).  A schedule entry (nsq << 16) | d means "square nsq times, then
// multiply by x^d" (d odd, or 0 for no product); the first entry's d is the
// starting power.
//
// Every step is one product MM(a, b) = a b R^-1 mod N whose operands come
// from the running value x, a chunked constant/table entry in global memory,
// an input integer given as 32-bit limbs, or the integer 1.  Keeping one call
// site keeps the kernel at the register budget of a single product (two
// wavefronts per SIMD), where inlining each step separately would not fit.
//
// Control flow is uniform over the wavefront: all tiles run the same
// program; only data (pointers, exponent digits) may differ per tile.
#pragma once
#include "mont_tile.hpp"

namespace pc2d {

enum : int { SRC_X = 0, SRC_CHUNK = 1, SRC_KEEP = 2 };

// Operand of one product: the running value x, or a number in chunked layout
// in global memory (constants, table entries, inputs converted beforehand).
struct Operand {
  int src;
  const uint32_t* p;
};

__device__ __forceinline__ Operand op_x() { return Operand{SRC_X, nullptr}; }
__device__ __forceinline__ Operand op_keep() { return Operand{SRC_KEEP, nullptr}; }
__device__ __forceinline__ Operand op_chunk(const uint32_t* p) { return Operand{SRC_CHUNK, p}; }

struct Program {
  // pre-steps; with redc, pre0 is replaced by x = W R^-1 mod N for the wide
  // W = lo + hi R: lo in chunked layout, hi as limbs (digits S.. of the limb
  // integer redc_hi of redc_hi_n limbs)
  int npre;
  bool redc;
  const uint32_t* redc_lo;
  const uint32_t* redc_hi;
  int redc_hi_n;
  Operand pre0_a, pre0_b, pre1_a, pre1_b;
  bool pre0_to_slot;      // store the result of pre0 (plus add1 in digit 0) to slot entry 0
  uint32_t pre0_add1;
  // powering: skipped when ebits < 0
  const uint32_t* e;
  int elimbs, ebits;
  bool uniform_e;
  const uint32_t* sched;  // sliding-window schedule of e (null: fixed windows)
  int nsched;
  const uint32_t* one;    // R mod N (chunked)
  // post-steps
  int npost;
  Operand post0_a, post0_b, post1_a, post1_b;
};

__device__ __forceinline__ Program empty_program() {
  Program P;
  P.npre = 0;
  P.redc = false;
  P.redc_lo = nullptr;
  P.redc_hi = nullptr;
  P.redc_hi_n = 0;
  P.pre0_a = P.pre0_b = P.pre1_a = P.pre1_b = op_keep();
  P.pre0_to_slot = false;
  P.pre0_add1 = 0;
  P.e = nullptr;
  P.elimbs = 0;
  P.ebits = -1;
  P.uniform_e = true;
  P.sched = nullptr;
  P.nsched = 0;
  P.one = nullptr;
  P.npost = 0;
  P.post0_a = P.post0_b = P.post1_a = P.post1_b = op_keep();
  return P;
}

__device__ __forceinline__ uint32_t exp_window(const uint32_t* __restrict__ e, int elimbs, int pos,
                                               int w) {
  int wd = pos >> 5, s = pos & 31;
  uint64_t lo = limb_at(e, elimbs, wd);
  uint64_t hi = limb_at(e, elimbs, wd + 1);
  return (uint32_t)(((hi << 32) | lo) >> s) & ((1u << w) - 1u);
}

// Runs program P; x holds the result (semi-normalised digits, < 2N).
// lds: the tile's LDS number; slot: the tile's scratch slot (>= 2^w entries
// of G::CH words; entry 0 is free for the program, entries 1.. hold the table).
// SLIDING selects the powering at compile time (a run-time choice would keep
// both forms live in one kernel and push it far past the register budget);
// with SLIDING, P.sched must be set.
template <class G, bool SLIDING = false>
__device__ __forceinline__ void run_program(const Program& P, uint32_t (&x)[G::K],
                                            uint32_t* __restrict__ lds,
                                            uint32_t* __restrict__ slot, int w,
                                            const uint32_t (&N)[G::K], uint32_t np, int tl) {
  enum { PRE0, PRE1, TSQ, TAB1, TAB, SQ, MUL, POST0, POST1, DONE };
  constexpr bool sliding = SLIDING;
  // table entries written: 1..2^w-1 (fixed) or 1..2^(w-1) (odd powers)
  const int tlast = sliding ? (1 << (w - 1)) : (1 << w) - 1;
  int d = 2, win = 0, sq = 0, sqn = w, si = 0;
  uint32_t dig = 0;
  int ph;
  const int post = P.npost > 0 ? POST0 : DONE;

  // sliding schedule: the next entry's squarings and product
  auto next_entry = [&]() -> int {
    if (si >= P.nsched) return post;
    const uint32_t en = P.sched[si++];
    sqn = (int)(en >> 16);
    dig = en & 0xFFFFu;
    sq = 0;
    return sqn > 0 ? SQ : (dig ? MUL : post);
  };
  auto after_pre = [&]() -> int {
    if (P.ebits < 0) return post;
    // table entry 1 is the base; the base stays in LDS while the table grows
    store_chunk<G>(slot + 1 * G::CH, x, tl);
    lds_sync();
    to_lds<G>(lds, x, tl);
    lds_sync();
    d = 2;
    if (sliding) return tlast > 1 ? TSQ : -1;  // x^2 first, then x^3, x^5, ...
    return tlast > 1 ? TAB : -1;
  };
  auto after_table = [&]() -> int {
    if (P.ebits == 0) {
      load_chunk<G>(x, P.one, tl);
      return post;
    }
    if (sliding) {
      si = 0;
      const uint32_t first = P.sched[si++] & 0xFFFFu;
      load_chunk<G>(x, slot + ((first + 1) >> 1) * G::CH, tl);
      return next_entry();
    }
    const int nw = (P.ebits + w - 1) / w;
    uint32_t top = exp_window(P.e, P.elimbs, (nw - 1) * w, w);
    load_chunk<G>(x, top ? slot + top * G::CH : P.one, tl);
    win = nw - 2;
    sq = 0;
    if (win < 0) return post;
    return SQ;
  };

  if (P.redc) {
    // x = W R^-1 mod N: low digits in registers, high digits streamed from LDS
    lds_sync();
    lds_digits_from_limbs<G>(lds, P.redc_hi, P.redc_hi_n, G::S, tl);
    lds_sync();
    load_chunk<G>(x, P.redc_lo, tl);
    mont_redc_wide<G>(x, x, lds, N, np, tl);
    ph = P.npre > 1 ? PRE1 : -2;
  } else {
    ph = P.npre > 0 ? PRE0 : -2;
  }
  if (ph == -2) {
    ph = after_pre();
    if (ph == -1) ph = after_table();
  }

  while (ph != DONE) {
    Operand oa, ob;
    switch (ph) {
      case PRE0: oa = P.pre0_a; ob = P.pre0_b; break;
      case PRE1: oa = P.pre1_a; ob = P.pre1_b; break;
      case TSQ:
      case TAB: oa = op_x(); ob = op_keep(); break;
      case TAB1:  // x^1 x^2
        if constexpr (sliding) {
          oa = op_chunk(slot + 1 * G::CH);
          ob = op_x();
        }
        break;
      case SQ: oa = op_x(); ob = op_x(); break;
      case MUL:
        if constexpr (sliding)
          oa = op_chunk(slot + ((dig + 1) >> 1) * G::CH);
        else
          oa = op_chunk(dig ? slot + dig * G::CH : P.one);
        ob = op_x();
        break;
      case POST0: oa = P.post0_a; ob = P.post0_b; break;
      default: oa = P.post1_a; ob = P.post1_b; break;
    }
    if (ob.src != SRC_KEEP) {
      lds_sync();
      if (ob.src == SRC_X)
        to_lds<G>(lds, x, tl);
      else
        lds_from_chunk<G>(lds, ob.p, tl);
      lds_sync();
    }
    // the multiplicand goes into x itself: x is dead once b is in LDS, and the
    // product reads all of a before it writes its output
    if (oa.src != SRC_X) load_chunk<G>(x, oa.p, tl);
    mont_mul<G>(x, x, lds, N, np, tl);

    switch (ph) {
      case PRE0:
        if (P.pre0_to_slot) {
          if (tl == 0) x[0] += P.pre0_add1;
          store_chunk<G>(slot, x, tl);
        }
        ph = P.npre > 1 ? PRE1 : -2;
        break;
      case PRE1: ph = -2; break;
      case TSQ: ph = TAB1; break;  // x^2 goes to LDS and stays there for TAB
      case TAB1:
        if constexpr (!sliding) break;
        [[fallthrough]];
      case TAB:
        store_chunk<G>(slot + d * G::CH, x, tl);
        ++d;
        ph = d <= tlast ? TAB : -1;
        break;
      case SQ:
        if (++sq < sqn) break;
        sq = 0;
        if (sliding) {
          ph = dig ? MUL : next_entry();
          break;
        }
        dig = exp_window(P.e, P.elimbs, win * w, w);
        if (P.uniform_e && dig == 0) {
          --win;
          if (win < 0) ph = post;
        } else {
          ph = MUL;
        }
        break;
      case MUL:
        if (sliding) {
          ph = next_entry();
          break;
        }
        --win;
        ph = win < 0 ? post : SQ;
        break;
      case POST0: ph = P.npost > 1 ? POST1 : DONE; break;
      default: ph = DONE; break;
    }
    if (ph == -2) ph = after_pre();
    if (ph == -1) ph = after_table();
  }
}

}  // namespace pc2d
