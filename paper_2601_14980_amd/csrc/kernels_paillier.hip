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

template <class Gn, class Gp>
__global__ __launch_bounds__(64, 2) void k_decrypt(SkConst sk, const uint32_t* __restrict__ c,
                                                   uint32_t* __restrict__ m, size_t count,
                                                   uint32_t* __restrict__ scratch,
                                                   size_t slot_words, int w, int* err) {
  constexpr int EPW = 64 / (2 * Gp::T);
  __shared__ __align__(16) uint32_t lds_all[2 * EPW * Gp::SP];
  uint32_t* slots = scratch + (size_t)blockIdx.x * 2 * EPW * slot_words;
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x)
    dec_group<Gn, Gp>(sk, c, m, count, gi, lds_all, slots, slot_words, w, err);
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

// m_out[j] = Dec(prod_k Enc(m_k[j], r_k[j])): the K ciphertexts and their
// product never reach the output; the running product lives in the element's
// scratch slot.
template <class Gn, class Gp>
__global__ __launch_bounds__(64, 2) void k_enc_sum_dec(SkConst sk, PtrList ms, PtrList rs, int K,
                                                    int m_limbs, uint32_t* __restrict__ mout,
                                                    size_t count, uint32_t* __restrict__ scratch,
                                                    size_t slot_words, int w, int* err) {
  static_assert(Gn::T == 2 * Gp::T, "element tile = two half tiles");
  constexpr int EPW = 64 / Gn::T;
  constexpr int LDSW = (Gn::SP > 2 * Gp::SP) ? Gn::SP : 2 * Gp::SP;
  __shared__ __align__(16) uint32_t lds_all[EPW * LDSW];
  const int tn = threadIdx.x & (Gn::T - 1);
  const int tile = threadIdx.x / Gn::T;
  const int tp = threadIdx.x & (Gp::T - 1);
  const int half = (threadIdx.x / Gp::T) & 1;
  uint32_t* lds_n = lds_all + tile * LDSW;
  uint32_t* lds_h = lds_n + half * Gp::SP;
  // per element: the n^2 slot (table, then ciphertext limbs), the running
  // product, then the two half-tile slots
  uint32_t* slot_n = scratch + ((size_t)blockIdx.x * EPW + tile) * 4 * slot_words;
  uint32_t* slot_acc = slot_n + slot_words;
  uint32_t* slot_h = slot_n + (2 + half) * slot_words;
  const PkConst& pk = sk.pk;
  const int L = pk.L, L2 = 2 * L;
  const HalfConst H = half ? sk.h[1] : sk.h[0];
  const size_t ngroups = (count + EPW - 1) / EPW;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    size_t e = gi * EPW + tile;
    const bool live = e < count;
    if (!live) e = count - 1;
    uint32_t okall = 1;
    {
      uint32_t N[Gn::K];
      load_chunk<Gn>(N, pk.n2.N, tn);
      const uint32_t np = pk.n2.nprime;
      uint32_t x[Gn::K];
      // k = 0..K-1: encrypt and fold into the running product; k = K: remove R^-(K-1)
      for (int k = 0; k <= K; ++k) {
        Program P;
        if (k < K) {
          const uint32_t* me = ms.p[k] + e * m_limbs;
          const uint32_t* re = rs.p[k] + e * L;
          if (tn == 0) okall &= encrypt_inputs_ok(pk, me, m_limbs, re);
          P = encrypt_program<Gn>(pk, me, m_limbs, re, slot_n, tn);
          if (k > 0) {
            P.npost = 2;
            P.post1_a = op_x();
            P.post1_b = op_chunk(slot_acc);
          }
        } else {
          P = empty_program();
          P.npre = 1;
          P.pre0_a = op_chunk(pk.Rk + (size_t)K * Gn::CH);
          P.pre0_b = op_chunk(slot_acc);
        }
        run_program<Gn>(P, x, lds_n, slot_n, w, N, np, tn);
        if (k < K) store_chunk<Gn>(slot_acc, x, tn);
      }
      lds_sync();
      to_lds<Gn>(lds_n, x, tn);
      lds_sync();
      if (tn == 0) {
        lds_canonical<Gn>(lds_n, pk.n2);
        for (int i = 0; i < L2; ++i) slot_acc[i] = lds_n[i];
      }
    }
    okall = tile_bcast0<Gn::T>(okall);
    lds_sync();
    uint32_t N[Gp::K];
    load_chunk<Gp>(N, H.s2.N, tp);
    const uint32_t np = H.s2.nprime;
    Program P = decrypt_program<Gp>(H, sk.ebits, slot_acc, L2, slot_h, tp);
    uint32_t x[Gp::K];
    run_program<Gp>(P, x, lds_h, slot_h, w, N, np, tp);
    lds_sync();
    to_lds<Gp>(lds_h, x, tp);
    lds_sync();
    if (tp == 0) decrypt_half_finish<Gp>(H, lds_h, slot_h, okall);
    lds_sync();
    if (tp == 0 && half == 0)
      garner_store(sk, slot_h, slot_h + slot_words, mout + e * L, live, err, slot_n);
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
  }

template <int C>
static const void* kernel_ptr(int op) {
  using Gn = typename Geos<C>::Gn;
  using Gp = typename Geos<C>::Gp;
  switch (op) {
    case OP_ENC: return (const void*)&k_encrypt<Gn>;
    case OP_DEC: return (const void*)&k_decrypt<Gn, Gp>;
    case OP_SUM: return (const void*)&k_hom_sum<Gn>;
    case OP_SMUL: return (const void*)&k_scalar_mul<Gn>;
    case OP_FUSED: return (const void*)&k_enc_sum_dec<Gn, Gp>;
  }
  return nullptr;
}

const void* kernel_for(int cls, int op) {
  PC2_DISPATCH(cls, return kernel_ptr<C>(op));
  return nullptr;
}

// Tiles (scratch slots) per workgroup and words per slot.
template <int C>
static void slot_shape_t(int op, int w, int Ls, int L, int* tiles, size_t* words) {
  using Gn = typename Geos<C>::Gn;
  using Gp = typename Geos<C>::Gp;
  const int epw = 64 / Gn::T;
  const size_t scal = (size_t)12 * Ls + 16;
  switch (op) {
    case OP_ENC:
    case OP_SMUL:
      *tiles = epw;
      *words = (size_t)Gn::CH << w;
      break;
    case OP_DEC:
      *tiles = 2 * epw;
      *words = std::max((size_t)Gp::CH << w, scal);
      break;
    case OP_FUSED:
      *tiles = 4 * epw;
      *words = std::max(std::max((size_t)Gn::CH << w, (size_t)Gp::CH << w),
                        std::max(scal, (size_t)2 * L + 4 + 5 * Ls + 8));
      break;
    default:
      *tiles = 0;
      *words = 0;
  }
}

void slot_shape(int cls, int op, int w, int Ls, int L, int* tiles, size_t* words) {
  *tiles = 0;
  *words = 0;
  PC2_DISPATCH(cls, slot_shape_t<C>(op, w, Ls, L, tiles, words); return);
}

int elems_per_block(int cls) {
  PC2_DISPATCH(cls, return 64 / Geos<C>::Gn::T);
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
hipError_t launch_encrypt(int cls, const Launch& l, const PkConst& pk, const uint32_t* m,
                          int m_limbs, const uint32_t* r, uint32_t* c, size_t count) {
  PC2_DISPATCH(cls, return enc_t<C>(l, pk, m, m_limbs, r, c, count, l.slot_words));
  return hipErrorInvalidValue;
}

template <int C>
static hipError_t dec_t(const Launch& l, const SkConst& sk, const uint32_t* c, uint32_t* m,
                        size_t count) {
  hipLaunchKernelGGL((k_decrypt<typename Geos<C>::Gn, typename Geos<C>::Gp>), dim3(l.grid),
                     dim3(64), 0, (hipStream_t)l.stream, sk, c, m, count, l.scratch,
                     l.slot_words, l.window, l.err);
  return hipGetLastError();
}
hipError_t launch_decrypt(int cls, const Launch& l, const SkConst& sk, const uint32_t* c,
                          uint32_t* m, size_t count) {
  PC2_DISPATCH(cls, return dec_t<C>(l, sk, c, m, count));
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
static hipError_t fused_t(const Launch& l, const SkConst& sk, const PtrList& ms,
                          const PtrList& rs, int K, int m_limbs, uint32_t* mout, size_t count) {
  hipLaunchKernelGGL((k_enc_sum_dec<typename Geos<C>::Gn, typename Geos<C>::Gp>), dim3(l.grid),
                     dim3(64), 0, (hipStream_t)l.stream, sk, ms, rs, K, m_limbs, mout, count,
                     l.scratch, l.slot_words, l.window, l.err);
  return hipGetLastError();
}
hipError_t launch_fused(int cls, const Launch& l, const SkConst& sk, const PtrList& ms,
                        const PtrList& rs, int K, int m_limbs, uint32_t* mout, size_t count) {
  PC2_DISPATCH(cls, return fused_t<C>(l, sk, ms, rs, K, m_limbs, mout, count));
  return hipErrorInvalidValue;
}

}  // namespace pc2k
