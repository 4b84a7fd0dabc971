// Paillier encryption (Sec. III-B, f_en with g = n + 1) with the modular
// products on the i8 matrix cores: c = (1 + m n) r^n mod n^2.
//
// One wavefront per element (mfma_mont.hpp); workgroups stride over the
// elements.  Per element: g^m = MM(m, n R) + 1 = 1 + m n (mod n^2); r R =
// MM(r, R^2); the odd powers (r R)^(2j+1) R^-2j, j < 2^(w-1), in the
// workgroup's scratch slot (after (r R)^2 R^-1, the slot's last entry);
// left-to-right sliding windows over n from the key's precomputed schedule
// (the VALU kernels' schedule: square nsq times, then multiply by an odd
// power); one product with g^m leaves normal form; resolving the signed
// limbs' carries (and adding n^2 to a negative result) makes it canonical.  Data errors (m >= n, r = 0,
// r >= n) zero the element and set ERR_RANGE.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "launch.hpp"
#include "mfma_mont.hpp"
#include "paillier_ops.hpp"

namespace {

using pc2k::PkConst;

// One element's c = r^n g^m (mod n^2) as the limbs U of the last product
// (also in ws.xr).  The workgroup's table (2^w digit arrays, of which the
// powering uses 2^(w-1) + 1) holds the odd powers, after them the square
// sq, and after that g^m (read once, at the end, so global memory serves;
// it leaves the LDS to the operands read at every product).  Returns the
// input checks (m < n, 0 < r < n).
template <class G>
__device__ __forceinline__ uint32_t encrypt_element(pc2m::MWork<G>& ws, const PkConst& pk,
                                                    const uint32_t* me, int m_limbs,
                                                    const uint32_t* re, uint8_t* table, int w,
                                                    int lane, int32_t (&U)[G::NT]) {
  __shared__ uint32_t s_ok;
  const pc2m::MConst& K = pk.mf;
  const int half = 1 << (w - 1);                  // odd powers in the table
  uint8_t* sq = table + (size_t)half * G::FB;     // (r R)^2 R^-1
  uint8_t* gm = sq + G::FB;                        // g^m
  const uint32_t* sched = pk.nsch.p[w - pc2k::SCHED_WMIN];
  const int nsched = pk.nsch.n[w - pc2k::SCHED_WMIN];
  if (lane == 0) s_ok = pc2ops::encrypt_inputs_ok(pk, me, m_limbs, re);
  // g^m = MM(m, n R) + 1 = 1 + m n (mod n^2)
  pc2m::load_x<G>(ws, me, m_limbs, lane);
  pc2m::mont_mul<G>(ws, K, K.nR, lane, false, gm, true, U);
  // table entry j = (r R)^(2j+1) R^-2j: entry 0 = r R, the square, then
  // one product by the square per entry
  pc2m::load_x<G>(ws, re, pk.L, lane);
  pc2m::mont_mul<G>(ws, K, K.R2, lane, true, table, false, U);
  pc2m::mont_mul<G>(ws, K, ws.xf, lane, false, sq, false, U);
  pc2m::load_fwd<G>(ws, table, lane);
  for (int j = 1; j < half; ++j)
    pc2m::mont_mul<G>(ws, K, sq, lane, false, table + (size_t)j * G::FB, false, U);
  // (r R)^n by the sliding-window schedule of n, most significant first
  pc2m::load_fwd<G>(ws, table + (size_t)((sched[0] & 0xFFFFu) >> 1) * G::FB, lane);
  for (int si = 1; si < nsched; ++si) {
    const uint32_t en = sched[si];
    for (uint32_t k = en >> 16; k; --k)
      pc2m::mont_mul<G>(ws, K, ws.xf, lane, true, nullptr, false, U);
    const uint32_t dig = en & 0xFFFFu;
    if (dig)
      pc2m::mont_mul<G>(ws, K, table + (size_t)(dig >> 1) * G::FB, lane, true, nullptr, false,
                        U);
  }
  // r^n g^m = MM(r^n R, g^m), |.| < 0.52 n^2
  pc2m::mont_mul<G>(ws, K, gm, lane, false, nullptr, false, U);
  return s_ok;
}

// Limbs U (|value| < 0.52 n^2) -> the canonical residue as 2L words at out
// (zeros if !ok).  The carries of the signed limbs are resolved in one pass
// and a negative value (a borrow out of the top limb) takes n^2 once.  The
// limbs go to the digit region of ws.xf, which is written before every
// read (its zero pads stay zero for the next element).
template <class G>
__device__ __forceinline__ void store_canonical(pc2m::MWork<G>& ws, const pc2m::MConst& K,
                                                const int32_t (&U)[G::NT], int lane,
                                                uint32_t* out, int L2, bool ok) {
  uint32_t* u = reinterpret_cast<uint32_t*>(ws.xf + G::PF);
#pragma unroll
  for (int q = 0; q < G::NT; ++q) {
    const int gi = 64 * q + lane - G::S;
    if (gi >= 0 && gi < G::S) u[gi] = (uint32_t)U[q];
  }
  pc2m::wave_sync();
  if (lane == 0) {
    int32_t cy = 0;
    for (int i = 0; i < G::S; ++i) {
      const int32_t t = (int32_t)u[i] + cy;
      u[i] = (uint32_t)t & pc2m::M28;
      cy = t >> 28;
    }
    if (cy < 0) {
      uint32_t cr = 0;
      for (int i = 0; i < G::S; ++i) {
        const uint32_t t = u[i] + K.N28[i] + cr;
        u[i] = t & pc2m::M28;
        cr = t >> 28;
      }
    }
  }
  pc2m::wave_sync();
  for (int j = lane; j < L2; j += 64) {
    const int b = 32 * j, i = b / 28, s = b % 28;
    const uint64_t acc = (uint64_t)(i < G::S ? u[i] : 0u) |
                         ((uint64_t)(i + 1 < G::S ? u[i + 1] : 0u) << 28) |
                         ((uint64_t)(i + 2 < G::S ? u[i + 2] : 0u) << 56);
    out[j] = ok ? (uint32_t)(acc >> s) : 0u;
  }
  pc2m::wave_sync();
}

// Wavefronts per SIMD, as measured on the MI355X: three up to 2048-bit keys,
// where the workspace (12 KB of LDS) and 168 registers still allow it, two
// from 3072 bits on, where three spill more than they gain
template <int S>
__global__ __launch_bounds__(64, S <= 160 ? 3 : 2) void k_encrypt_mfma(
    PkConst pk, const uint32_t* __restrict__ m, int m_limbs, const uint32_t* __restrict__ r,
    uint32_t* __restrict__ c, size_t count, uint8_t* __restrict__ scratch, int w, int* err) {
  using G = pc2m::MGeo<S>;
  __shared__ __align__(16) pc2m::MWork<G> ws;
  const int lane = threadIdx.x;
  uint8_t* table = scratch + (size_t)blockIdx.x * ((size_t)G::FB << w);
  const int L = pk.L;
  pc2m::init_work<G>(ws, lane);
  pc2m::init_table<G>(table, (1 << (w - 1)) + 2, lane);
  int32_t U[G::NT];
  for (size_t e = blockIdx.x; e < count; e += gridDim.x) {
    const uint32_t ok =
        encrypt_element<G>(ws, pk, m + e * m_limbs, m_limbs, r + e * L, table, w, lane, U);
    store_canonical<G>(ws, pk.mf, U, lane, c + e * 2 * (size_t)L, 2 * L, ok);
    if (lane == 0 && !ok) atomicOr(err, pc2k::ERR_RANGE);
  }
}

// Step `step` of the fused encrypt -> K-way product (Def. 1 applied K - 1
// times) over the matrix cores: element e's encryption c_k, then one more
// product acc_e <- MM(c_k, y) with y = R^K for the first step and the
// running product acc_e after it, so that the last step leaves
// R^K prod_k c_k R^-K = prod_k c_k, canonical, in prod.  acc: one forward
// digit array per element (mfma_digit_bytes), in the caller's staging; ok:
// one word per element, the AND of every step's input checks.
template <int S>
__global__ __launch_bounds__(64, S <= 160 ? 3 : 2) void k_enc_acc_mfma(
    PkConst pk, const uint32_t* __restrict__ m, int m_limbs, const uint32_t* __restrict__ r,
    int Kn, int step, uint8_t* __restrict__ acc, uint32_t* __restrict__ ok_all,
    uint32_t* __restrict__ prod, size_t count, uint8_t* __restrict__ scratch, int w, int* err) {
  using G = pc2m::MGeo<S>;
  __shared__ __align__(16) pc2m::MWork<G> ws;
  const int lane = threadIdx.x;
  uint8_t* table = scratch + (size_t)blockIdx.x * ((size_t)G::FB << w);
  const int L = pk.L;
  const bool last = step + 1 == Kn;
  pc2m::init_work<G>(ws, lane);
  pc2m::init_table<G>(table, (1 << (w - 1)) + 2, lane);
  int32_t U[G::NT];
  for (size_t e = blockIdx.x; e < count; e += gridDim.x) {
    uint8_t* acc_e = acc + e * (size_t)G::FB;
    uint32_t ok =
        encrypt_element<G>(ws, pk, m + e * m_limbs, m_limbs, r + e * L, table, w, lane, U);
    if (step) ok &= ok_all[e];
    // the running product's front pad is read as zero by the next step
    if (step == 0 && lane < G::PF / 4) reinterpret_cast<uint32_t*>(acc_e)[lane] = 0u;
    const uint8_t* y = step ? acc_e : pk.mf.Rk + (size_t)Kn * G::FB;
    pc2m::mont_mul<G>(ws, pk.mf, y, lane, false, last ? nullptr : acc_e, false, U);
    if (!last) {
      if (lane == 0) ok_all[e] = ok;
    } else {
      store_canonical<G>(ws, pk.mf, U, lane, prod + e * 2 * (size_t)L, 2 * L, ok);
      if (lane == 0 && !ok) atomicOr(err, pc2k::ERR_RANGE);
    }
  }
}

__global__ void k_mfma_queue_reset(int* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

// Persistent batch encryption (the matrix-core form of the batch kernel's
// encryption phase): each workgroup pulls one element at a time from the
// queue (one atomic each: queue position q is element q % sub of item
// q / sub, sub >= every job's group), so that the launch ends within one
// element's time of its last wavefront; it exits when the queue is drained,
// so every wavefront reaches the exit.
template <int S>
__global__ __launch_bounds__(64, S <= 160 ? 3 : 2) void k_batch_mfma(
    const pc2k::BatchJob* __restrict__ jobs, const pc2k::BatchItem* __restrict__ items,
    int nitems, int sub, int* queue, uint8_t* __restrict__ scratch, int w, int* err) {
  using G = pc2m::MGeo<S>;
  __shared__ __align__(16) pc2m::MWork<G> ws;
  __shared__ int s_q;
  const int lane = threadIdx.x;
  uint8_t* table = scratch + (size_t)blockIdx.x * ((size_t)G::FB << w);
  pc2m::init_work<G>(ws, lane);
  pc2m::init_table<G>(table, (1 << (w - 1)) + 2, lane);
  int32_t U[G::NT];
  const long long total = (long long)nitems * sub;
  for (;;) {
    if (lane == 0) s_q = atomicAdd(queue, 1);
    pc2m::wave_sync();
    const long long q = s_q;
    pc2m::wave_sync();
    if (q >= total) break;
    const pc2k::BatchItem item = items[q / sub];
    const pc2k::BatchJob& job = jobs[item.job];
    const int k = (int)(q % sub);
    const size_t e = item.group * (size_t)job.group + k;
    if (k >= job.group || e >= job.count) continue;
    const int L = job.pk.L;
    const uint32_t ok = encrypt_element<G>(ws, job.pk, job.in0 + e * job.m_limbs, job.m_limbs,
                                           job.in1 + e * L, table, w, lane, U);
    store_canonical<G>(ws, job.pk.mf, U, lane, job.out + e * 2 * (size_t)L, 2 * L, ok);
    if (lane == 0 && !ok) atomicOr(err, pc2k::ERR_RANGE);
  }
}

template <int C>
const void* mfma_kernel(bool fused) {
  return fused ? (const void*)&k_enc_acc_mfma<pc2k::MFMA_S[C]>
               : (const void*)&k_encrypt_mfma<pc2k::MFMA_S[C]>;
}

}  // namespace

namespace pc2k {

const void* kernel_encrypt_mfma(int cls, bool fused) {
  switch (cls) {
    case 0: return mfma_kernel<0>(fused);
    case 1: return mfma_kernel<1>(fused);
    case 2: return mfma_kernel<2>(fused);
    case 3: return mfma_kernel<3>(fused);
    case 4: return mfma_kernel<4>(fused);
    case 5: return mfma_kernel<5>(fused);
    case 6: return mfma_kernel<6>(fused);
    case 7: return mfma_kernel<7>(fused);
    case 8: return mfma_kernel<8>(fused);
  }
  return nullptr;
}

const void* batch_mfma_kernel(int cls) {
  switch (cls) {
    case 0: return (const void*)&k_batch_mfma<MFMA_S[0]>;
    case 1: return (const void*)&k_batch_mfma<MFMA_S[1]>;
    case 2: return (const void*)&k_batch_mfma<MFMA_S[2]>;
    case 3: return (const void*)&k_batch_mfma<MFMA_S[3]>;
    case 4: return (const void*)&k_batch_mfma<MFMA_S[4]>;
    case 5: return (const void*)&k_batch_mfma<MFMA_S[5]>;
    case 6: return (const void*)&k_batch_mfma<MFMA_S[6]>;
    case 7: return (const void*)&k_batch_mfma<MFMA_S[7]>;
    case 8: return (const void*)&k_batch_mfma<MFMA_S[8]>;
  }
  return nullptr;
}

hipError_t launch_batch_mfma(int cls, int grid, const BatchJob* jobs, const BatchItem* items,
                             int nitems, int sub, int* queue, uint8_t* scratch, int w, int* err,
                             void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mfma_queue_reset, dim3(1), dim3(64), 0, st, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* k = batch_mfma_kernel(cls);
  if (!k) return hipErrorInvalidValue;
  void* args[] = {(void*)&jobs,    (void*)&items, (void*)&nitems, (void*)&sub,
                  (void*)&queue,   (void*)&scratch, (void*)&w, (void*)&err};
  return hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, st);
}

size_t mfma_digit_bytes(int cls) {  // a forward digit array, with its zero pads
  const int D = 4 * MFMA_S[cls];
  return (size_t)(64 + ((D + 15) & ~15) + 16);
}

hipError_t launch_encrypt_mfma(int cls, const Launch& l, const PkConst& pk, const uint32_t* m,
                               int m_limbs, const uint32_t* r, uint32_t* c, size_t count) {
  const void* k = kernel_encrypt_mfma(cls);
  if (!k) return hipErrorInvalidValue;
  uint8_t* scratch = reinterpret_cast<uint8_t*>(l.scratch);
  int w = l.window;
  void* args[] = {(void*)&pk, (void*)&m, (void*)&m_limbs, (void*)&r, (void*)&c,
                  (void*)&count, (void*)&scratch, (void*)&w, (void*)&l.err};
  return hipLaunchKernel(k, dim3(l.grid), dim3(64), args, 0, (hipStream_t)l.stream);
}

hipError_t launch_enc_prod_mfma(int cls, const Launch& l, const PkConst& pk, const PtrList& ms,
                                const PtrList& rs, int K, int m_limbs, uint32_t* prod,
                                size_t count, uint8_t* acc, uint32_t* ok) {
  const void* k = kernel_encrypt_mfma(cls, true);
  if (!k) return hipErrorInvalidValue;
  uint8_t* scratch = reinterpret_cast<uint8_t*>(l.scratch);
  int w = l.window;
  for (int step = 0; step < K; ++step) {
    const uint32_t* m = ms.p[step];
    const uint32_t* r = rs.p[step];
    void* args[] = {(void*)&pk,   (void*)&m,    (void*)&m_limbs, (void*)&r,
                    (void*)&K,    (void*)&step, (void*)&acc,     (void*)&ok,
                    (void*)&prod, (void*)&count, (void*)&scratch, (void*)&w,
                    (void*)&l.err};
    const hipError_t e =
        hipLaunchKernel(k, dim3(l.grid), dim3(64), args, 0, (hipStream_t)l.stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pc2k
