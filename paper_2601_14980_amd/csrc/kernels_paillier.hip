// Paillier kernels for gfx950: encryption, CRT decryption, K-way
// homomorphic aggregation, multiply-by-constant and the fused
// encrypt -> aggregate -> decrypt path.
//
// Work mapping.  One workgroup is one wavefront (64 lanes).  A ciphertext
// (modulus n^2) is owned by a tile of Tn lanes; a decryption splits an
// element into two half-tiles of Tp = Tn/2 lanes, one per prime (p, q), that
// run concurrently in the same wavefront (the Z_{p^2} x Z_{q^2} split of
// Sec. IV, Lemmas 1-2).  Workgroups stride over groups of 64/Tn elements, so
// the grid is sized to the resident capacity of the device and each tile
// reuses one slot of the global scratch for its window table.
//
// Every element's data errors are handled in-band: the element's output is
// zeroed and the context's error word gets ERR_RANGE.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "paillier_ops.hpp"

#include <algorithm>

using namespace pc2ops;

// ------------------------------------------------------------------ kernels
template <class G>
__global__ __launch_bounds__(64, 2) void k_encrypt(PkConst pk, const uint32_t* __restrict__ m,
                                                   int m_limbs, const uint32_t* __restrict__ r,
                                                   uint32_t* __restrict__ c, size_t count,
                                                   uint32_t* __restrict__ scratch,
                                                   size_t slot_words, int w, int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  uint32_t* slots = scratch + (size_t)blockIdx.x * EPW * slot_words;
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x)
    enc_group<G>(pk, m, m_limbs, r, c, count, gi, lds_all, slots, slot_words, w, err);
}

// Decryption, phase 1: work item w covers element group w / 2 for prime
// w % 2, so every wavefront works on one prime.
template <class Gp>
__global__ __launch_bounds__(64, 2) void k_decrypt_half(SkConst sk, const uint32_t* __restrict__ c,
                                                        size_t count,
                                                        uint32_t* __restrict__ scratch,
                                                        size_t slot_words, int w,
                                                        uint32_t* __restrict__ halves) {
  constexpr int EPW = 64 / Gp::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * Gp::SP];
  uint32_t* slots = scratch + (size_t)blockIdx.x * EPW * slot_words;
  const size_t nitems = 2 * ((count + EPW - 1) / EPW);
  const size_t stride = (size_t)EPW * 2 * (sk.h[0].Ls + 1);
  for (size_t it = blockIdx.x; it < nitems; it += gridDim.x)
    dec_half_group<Gp>(sk, (int)(it & 1), c, count, it >> 1, lds_all, slots, slot_words, w,
                       halves + (it >> 1) * stride);
}

// Decryption, phase 2: CRT recombination, one lane per element.
__global__ __launch_bounds__(64) void k_garner(SkConst sk, const uint32_t* __restrict__ halves,
                                               uint32_t* __restrict__ m, size_t count, int* err) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int Ls = sk.h[0].Ls;
  uint32_t work[5 * pc2k::LS_MAX + 2];
  const uint32_t* hp = halves + e * 2 * (size_t)(Ls + 1);
  garner_elem(sk, hp, hp + Ls + 1, m + e * sk.pk.L, err, work);
}

// Key-holder encryption, phase 1: work item w covers element group w / 2
// modulo the square of prime w % 2.
template <class Gp>
__global__ __launch_bounds__(64, 2) void k_encrypt_crt_half(SkConst sk,
                                                            const uint32_t* __restrict__ m,
                                                            int m_limbs,
                                                            const uint32_t* __restrict__ r,
                                                            size_t count,
                                                            uint32_t* __restrict__ scratch,
                                                            size_t slot_words, int w,
                                                            uint32_t* __restrict__ stage) {
  constexpr int EPW = 64 / Gp::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * Gp::SP];
  uint32_t* slots = scratch + (size_t)blockIdx.x * EPW * slot_words;
  const size_t nitems = 2 * ((count + EPW - 1) / EPW);
  const size_t stride = (size_t)EPW * 2 * (sk.h[0].s2.nl + 1);
  for (size_t it = blockIdx.x; it < nitems; it += gridDim.x)
    enc_half_group<Gp>(sk, (int)(it & 1), m, m_limbs, r, count, it >> 1, lds_all, slots,
                       slot_words, w, stage + (it >> 1) * stride);
}

// Key-holder encryption, phase 2: recombination modulo n^2, one lane per element.
constexpr int NL2_MAX = 2 * pc2k::LS_MAX;
__global__ __launch_bounds__(64) void k_garner_crt(SkConst sk, const uint32_t* __restrict__ stage,
                                                   uint32_t* __restrict__ c, size_t count,
                                                   int* err) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int n2 = sk.h[0].s2.nl;
  uint32_t work[5 * NL2_MAX + 2];
  const uint32_t* cp = stage + e * 2 * (size_t)(n2 + 1);
  garner_crt_elem(sk, cp, cp + n2 + 1, c + e * 2 * (size_t)sk.pk.L, err, work);
}

template <class G>
__global__ __launch_bounds__(64, 2) void k_hom_sum(PkConst pk, PtrList cs, int K,
                                                   uint32_t* __restrict__ out, size_t count,
                                                   int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x)
    sum_group<G>(pk, cs.p, nullptr, K, out, count, gi, lds_all, err);
}

// out = c^k mod n^2 with a per-element 64-bit k (Definition 2):
//   pre0: MM(R^2, c) = c R;  pow: (c R)^k = c^k R;  post0: MM(., 1) = c^k
template <class G>
__global__ __launch_bounds__(64, 2) void k_scalar_mul(PkConst pk, const uint32_t* __restrict__ c,
                                                   const uint32_t* __restrict__ kv,
                                                   uint32_t* __restrict__ out, size_t count,
                                                   uint32_t* __restrict__ scratch,
                                                   size_t slot_words, int w, int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t* slot = scratch + ((size_t)blockIdx.x * EPW + tile) * slot_words;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const int L2 = 2 * pk.L;
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    size_t e = gi * EPW + tile;
    const bool live = e < count;
    if (!live) e = count - 1;
    const uint32_t* ce = c + e * L2;
    uint32_t ok = 1;
    if (tl == 0) ok = sc_cmp(ce, L2, pk.n2.Nl, L2) < 0;
    chunk_from_limbs<G>(slot, ce, L2, 0, tl);
    Program P = empty_program();
    P.npre = 1;
    P.pre0_a = op_chunk(pk.n2.R2);
    P.pre0_b = op_chunk(slot);
    P.e = kv + 2 * e;
    P.elimbs = 2;
    P.ebits = 64;
    P.uniform_e = false;
    P.one = pk.n2.R1;
    P.npost = 1;
    P.post0_a = op_x();
    P.post0_b = op_chunk(pk.n2.ONE);
    uint32_t x[G::K];
    run_program<G>(P, x, lds, slot, w, N, np, tl);
    lds_sync();
    to_lds<G>(lds, x, tl);
    lds_sync();
    if (tl == 0) store_canonical<G>(lds, pk.n2, out + e * L2, live, ok, err);
  }
}

// One step of the fused encrypt -> aggregate -> decrypt path, the first
// phase of which is prod[j] = prod_k Enc(m_k[j], r_k[j]) mod n^2: step k
// encrypts (m_k, r_k) and multiplies it into the element's running product
// acc_j (chunked layout, CH words per element), x = MM(c_k, acc_j).  acc
// starts as R^K (a key constant, read by step 0), so after k steps it holds
// c_0 .. c_(k-1) R^(K-k) and the last step leaves the plain product, which
// it writes canonical to prod (2L limbs); the ciphertexts never reach the
// caller's memory.  ok: one word per element, the AND of every step's input
// checks.  Every step runs the encryption kernel's program and then one
// product, so it keeps close to that kernel's register budget (one launch
// that looped over k spilled tens of registers).
template <class G>
__global__ __launch_bounds__(64, 2) void k_enc_acc(PkConst pk, const uint32_t* __restrict__ m,
                                                   int m_limbs, const uint32_t* __restrict__ r,
                                                   int K, int step, uint32_t* __restrict__ acc,
                                                   uint32_t* __restrict__ ok_all,
                                                   uint32_t* __restrict__ prod, size_t count,
                                                   uint32_t* __restrict__ scratch,
                                                   size_t slot_words, int w, int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t* slot = scratch + ((size_t)blockIdx.x * EPW + tile) * slot_words;
  const int L = pk.L, L2 = 2 * L;
  const bool last = step + 1 == K;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    size_t e = gi * EPW + tile;
    const bool live = e < count;
    if (!live) e = count - 1;
    const uint32_t* me = m + e * m_limbs;
    const uint32_t* re = r + e * L;
    uint32_t ok = 1;
    if (tl == 0) ok = encrypt_inputs_ok(pk, me, m_limbs, re) & (step ? ok_all[e] : 1u);
    Program P = encrypt_program<G>(pk, me, m_limbs, re, slot, tl, w);
    uint32_t x[G::K];
    run_program<G, true>(P, x, lds, slot, w, N, np, tl);
    // x = MM(acc, c_k): a program of its own (as a second post-step of the
    // encryption program it pushed the kernel into tens of spilled registers)
    uint32_t* acc_e = acc + e * G::CH;  // formed here: nothing more is live in the powering
    Program Q = empty_program();
    Q.npre = 1;
    Q.pre0_a = op_chunk(step ? acc_e : pk.Rk + (size_t)K * G::CH);
    Q.pre0_b = op_x();
    run_program<G, true>(Q, x, lds, slot, w, N, np, tl);
    if (!last) {
      if (live) {
        store_chunk<G>(acc_e, x, tl);
        if (tl == 0) ok_all[e] = ok;
      }
    } else {
      lds_sync();
      to_lds<G>(lds, x, tl);
      lds_sync();
      if (tl == 0) store_canonical<G>(lds, pk.n2, prod + e * L2, live, ok, err);
    }
  }
}

// ------------------------------------------------------------ host launchers
namespace pc2k {


#define PC2_DISPATCH(cls, EXPR)            \
  switch (cls) {                           \
    case 0: { constexpr int C = 0; EXPR; } \
    case 1: { constexpr int C = 1; EXPR; } \
    case 2: { constexpr int C = 2; EXPR; } \
    case 3: { constexpr int C = 3; EXPR; } \
    case 4: { constexpr int C = 4; EXPR; } \
    case 5: { constexpr int C = 5; EXPR; } \
    case 6: { constexpr int C = 6; EXPR; } \
    case 7: { constexpr int C = 7; EXPR; } \
    case 8: { constexpr int C = 8; EXPR; } \
  }
// the same over every geometry id, alternative encryption tiles included
#define PC2_DISPATCH_GEO(geo, EXPR)        \
  switch (geo) {                           \
    case 0: { constexpr int C = 0; EXPR; } \
    case 1: { constexpr int C = 1; EXPR; } \
    case 2: { constexpr int C = 2; EXPR; } \
    case 3: { constexpr int C = 3; EXPR; } \
    case 4: { constexpr int C = 4; EXPR; } \
    case 5: { constexpr int C = 5; EXPR; } \
    case 6: { constexpr int C = 6; EXPR; } \
    case 7: { constexpr int C = 7; EXPR; } \
    case 8: { constexpr int C = 8; EXPR; } \
    case 9: { constexpr int C = 9; EXPR; } \
    case 10: { constexpr int C = 10; EXPR; } \
  }

template <int C>
static const void* kernel_ptr(int op) {
  using Gn = typename Geos<C>::Gn;
  using Gp = typename Geos<C>::Gp;
  if constexpr (C >= NUM_CLASSES) {  // an alternative tile serves encryption only
    return op == OP_ENC ? (const void*)&k_encrypt<Gn> : nullptr;
  } else {
    switch (op) {
      case OP_ENC: return (const void*)&k_encrypt<Gn>;
      case OP_DEC: return (const void*)&k_decrypt_half<Gp>;
      case OP_SUM: return (const void*)&k_hom_sum<Gn>;
      case OP_SMUL: return (const void*)&k_scalar_mul<Gn>;
      case OP_FUSED: return (const void*)&k_enc_acc<Gn>;
      case OP_ENC_CRT: return (const void*)&k_encrypt_crt_half<Gp>;
    }
    return nullptr;
  }
}

const void* kernel_for(int geo, int op) {
  PC2_DISPATCH_GEO(geo, return kernel_ptr<C>(op));
  return nullptr;
}

// Tiles (scratch slots) per workgroup and words per slot.  A slot holds
// entry 0 plus the window table: 2^w - 1 entries for fixed windows, 2^(w-1)
// odd powers for the sliding windows of a wave-uniform exponent.
inline size_t table_entries(int w, bool sliding) {
  return sliding ? ((size_t)1 << (w - 1)) + 1 : (size_t)1 << w;
}
template <int C>
static void slot_shape_t(int op, int w, int Ls, int L, int* tiles, size_t* words) {
  using Gn = typename Geos<C>::Gn;
  using Gp = typename Geos<C>::Gp;
  const int epw = 64 / Gn::T;
  const size_t scal = (size_t)12 * Ls + 16;
  switch (op) {
    case OP_ENC:
      *tiles = epw;
      *words = (size_t)Gn::CH * table_entries(w, true);
      break;
    case OP_SMUL:
      *tiles = epw;
      *words = (size_t)Gn::CH << w;
      break;
    case OP_DEC:
      *tiles = 64 / Gp::T;
      *words = std::max((size_t)Gp::CH * table_entries(w, true), scal);
      break;
    case OP_FUSED:
      *tiles = epw;
      *words = (size_t)Gn::CH * table_entries(w, true);
      break;
    case OP_ENC_CRT:
      *tiles = 64 / Gp::T;
      *words = (size_t)Gp::CH * table_entries(w, true);
      break;
    default:
      *tiles = 0;
      *words = 0;
  }
}

void slot_shape(int geo, int op, int w, int Ls, int L, int* tiles, size_t* words) {
  *tiles = 0;
  *words = 0;
  PC2_DISPATCH_GEO(geo, slot_shape_t<C>(op, w, Ls, L, tiles, words); return);
}

int elems_per_block(int geo) {
  PC2_DISPATCH_GEO(geo, return 64 / Geos<C>::Gn::T);
  return 0;
}

template <int C>
static hipError_t enc_t(const Launch& l, const PkConst& pk, const uint32_t* m, int m_limbs,
                        const uint32_t* r, uint32_t* c, size_t count, size_t slot) {
  hipLaunchKernelGGL((k_encrypt<typename Geos<C>::Gn>), dim3(l.grid), dim3(64), 0,
                     (hipStream_t)l.stream, pk, m, m_limbs, r, c, count, l.scratch, slot,
                     l.window, l.err);
  return hipGetLastError();
}
hipError_t launch_encrypt(int geo, const Launch& l, const PkConst& pk, const uint32_t* m,
                          int m_limbs, const uint32_t* r, uint32_t* c, size_t count) {
  PC2_DISPATCH_GEO(geo, return enc_t<C>(l, pk, m, m_limbs, r, c, count, l.slot_words));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t dec_t(const Launch& l, const SkConst& sk, const uint32_t* c, uint32_t* m,
                        size_t count, uint32_t* halves) {
  if (sk.h[0].Ls > LS_MAX || halves == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_decrypt_half<typename Geos<C>::Gp>), dim3(l.grid), dim3(64), 0,
                     (hipStream_t)l.stream, sk, c, count, l.scratch, l.slot_words, l.window,
                     halves);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_garner, dim3((unsigned)((count + 63) / 64)), dim3(64), 0,
                     (hipStream_t)l.stream, sk, halves, m, count, l.err);
  return hipGetLastError();
}
hipError_t launch_decrypt(int cls, const Launch& l, const SkConst& sk, const uint32_t* c,
                          uint32_t* m, size_t count, uint32_t* halves) {
  PC2_DISPATCH(cls, return dec_t<C>(l, sk, c, m, count, halves));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t sum_t(const Launch& l, const PkConst& pk, const PtrList& cs, int K,
                        uint32_t* out, size_t count) {
  hipLaunchKernelGGL((k_hom_sum<typename Geos<C>::Gn>), dim3(l.grid), dim3(64), 0,
                     (hipStream_t)l.stream, pk, cs, K, out, count, l.err);
  return hipGetLastError();
}
hipError_t launch_hom_sum(int cls, const Launch& l, const PkConst& pk, const PtrList& cs, int K,
                          uint32_t* out, size_t count) {
  PC2_DISPATCH(cls, return sum_t<C>(l, pk, cs, K, out, count));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t smul_t(const Launch& l, const PkConst& pk, const uint32_t* c,
                         const uint32_t* k, uint32_t* out, size_t count) {
  hipLaunchKernelGGL((k_scalar_mul<typename Geos<C>::Gn>), dim3(l.grid), dim3(64), 0,
                     (hipStream_t)l.stream, pk, c, k, out, count, l.scratch, l.slot_words,
                     l.window, l.err);
  return hipGetLastError();
}
hipError_t launch_scalar_mul(int cls, const Launch& l, const PkConst& pk, const uint32_t* c,
                             const uint32_t* k, uint32_t* out, size_t count) {
  PC2_DISPATCH(cls, return smul_t<C>(l, pk, c, k, out, count));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t enc_crt_t(const Launch& l, const SkConst& sk, const uint32_t* m, int m_limbs,
                            const uint32_t* r, uint32_t* c, size_t count, uint32_t* stage) {
  if (sk.h[0].s2.nl > NL2_MAX || stage == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_encrypt_crt_half<typename Geos<C>::Gp>), dim3(l.grid), dim3(64), 0,
                     (hipStream_t)l.stream, sk, m, m_limbs, r, count, l.scratch, l.slot_words,
                     l.window, stage);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_garner_crt, dim3((unsigned)((count + 63) / 64)), dim3(64), 0,
                     (hipStream_t)l.stream, sk, stage, c, count, l.err);
  return hipGetLastError();
}
hipError_t launch_encrypt_crt(int cls, const Launch& l, const SkConst& sk, const uint32_t* m,
                              int m_limbs, const uint32_t* r, uint32_t* c, size_t count,
                              uint32_t* stage) {
  PC2_DISPATCH(cls, return enc_crt_t<C>(l, sk, m, m_limbs, r, c, count, stage));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t fused_t(const Launch& l, const PkConst& pk, const PtrList& ms,
                          const PtrList& rs, int K, int m_limbs, uint32_t* prod, size_t count,
                          uint32_t* acc, uint32_t* ok) {
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL((k_enc_acc<typename Geos<C>::Gn>), dim3(l.grid), dim3(64), 0,
                       (hipStream_t)l.stream, pk, ms.p[k], m_limbs, rs.p[k], K, k, acc, ok, prod,
                       count, l.scratch, l.slot_words, l.window, l.err);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t launch_enc_prod(int cls, const Launch& l, const PkConst& pk, const PtrList& ms,
                           const PtrList& rs, int K, int m_limbs, uint32_t* prod, size_t count,
                           uint32_t* acc, uint32_t* ok) {
  PC2_DISPATCH(cls, return fused_t<C>(l, pk, ms, rs, K, m_limbs, prod, count, acc, ok));
  return hipErrorInvalidValue;
}
size_t chunk_words(int geo) {
  PC2_DISPATCH_GEO(geo, return (size_t)Geos<C>::Gn::CH);
  return 0;
}

}  // namespace pc2k
