// Persistent batch kernels: one launch runs every job of a phase (all
// encryptions, all aggregations or all decryptions of many edge nodes'
// vectors of uneven lengths, under keys of up to two size classes).
//
// The grid is the device's resident capacity.  Each workgroup (one
// wavefront) pulls work items -- one element group of one job -- from a
// device queue with a single global atomic per item, runs the job's
// per-group body for the job's key class, and exits when the queue is
// drained, so every wavefront reaches the exit.  The host orders items from
// the most to the least expensive so that the tail of the launch is made of
// short items.  The queue counter is reset by a one-lane kernel launched
// just before, so the pair can be captured in a HIP graph and replayed.
// Decryption runs in two launches with no dependency between wavefronts:
// the first takes one prime of one group per item (the per-prime form of the
// one-call path, its staging in the batch's own memory), the second
// recombines every group's two halves (one lane per element).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.hpp"
#include "paillier_ops.hpp"

using namespace pc2ops;

namespace {

template <int OP, int C>
struct OpShape {
  using Gn = typename pc2k::Geos<C>::Gn;
  using Gp = typename pc2k::Geos<C>::Gp;
  // elements per item: a tile of the n^2 geometry, or (decryption) of the s^2 one
  static constexpr int EPW = (OP == pc2k::OP_DEC) ? 64 / Gp::T : 64 / Gn::T;
  static constexpr int LDSW = (OP == pc2k::OP_DEC) ? EPW * Gp::SP : EPW * Gn::SP;
  static constexpr int TILES = (OP == pc2k::OP_SUM) ? 0 : EPW;
};

template <int OP, int C>
__device__ __forceinline__ void run_item(const pc2k::BatchJob& job, const pc2k::BatchItem& item,
                                         uint32_t* lds_all, uint32_t* slots, size_t slot_words,
                                         int w, int* err) {
  using S = OpShape<OP, C>;
  const size_t group = item.group;
  if constexpr (OP == pc2k::OP_ENC) {
    enc_group<typename S::Gn>(job.pk, job.in0, job.m_limbs, job.in1, job.out, job.count, group,
                              lds_all, slots, slot_words, w, err);
  } else if constexpr (OP == pc2k::OP_DEC) {
    const size_t per = (size_t)S::EPW * 2 * (job.sk.h[0].Ls + 1);  // staging words per group
    dec_half_group<typename S::Gp>(job.sk, item.half, job.in0, job.count, group, lds_all, slots,
                                   slot_words, w, job.stage + (group - job.stage_g0) * per);
  } else {
    sum_group<typename S::Gn>(job.pk, job.inputs, job.lengths, job.K, job.out, job.count,
                              group, lds_all, err);
  }
}

__global__ void k_queue_reset(int* queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

template <int OP, int CA, int CB>
__global__ __launch_bounds__(64, 2) void k_batch(const pc2k::BatchJob* __restrict__ jobs,
                                                 const pc2k::BatchItem* __restrict__ items,
                                                 int nitems, int* queue,
                                                 uint32_t* __restrict__ scratch,
                                                 size_t slot_words, int w_a, int w_b, int* err) {
  using A = OpShape<OP, CA>;
  using B = OpShape<OP, CB>;
  constexpr int LDSW = A::LDSW > B::LDSW ? A::LDSW : B::LDSW;
  constexpr int TILES = A::TILES > B::TILES ? A::TILES : B::TILES;
  __shared__ __align__(16) uint32_t lds_all[LDSW];
  __shared__ int s_item;
  uint32_t* slots = scratch + (size_t)blockIdx.x * TILES * slot_words;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= nitems) break;
    const pc2k::BatchItem item = items[it];
    const pc2k::BatchJob& job = jobs[item.job];
    if constexpr (CA == CB) {
      run_item<OP, CA>(job, item, lds_all, slots, slot_words, w_a, err);
    } else {
      if (job.geo == CA)
        run_item<OP, CA>(job, item, lds_all, slots, slot_words, w_a, err);
      else
        run_item<OP, CB>(job, item, lds_all, slots, slot_words, w_b, err);
    }
  }
}

// Second launch of a batch decryption: for every item of prime 0, lane t
// recombines element t of the item's group from the two staged halves.
template <int CA, int CB>
__global__ __launch_bounds__(64) void k_batch_garner(const pc2k::BatchJob* __restrict__ jobs,
                                                     const pc2k::BatchItem* __restrict__ items,
                                                     int nitems, int* err) {
  uint32_t work[5 * pc2k::LS_MAX + 2];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const pc2k::BatchItem item = items[it];
    if (item.half != 0) continue;
    const pc2k::BatchJob& job = jobs[item.job];
    const int epw = job.geo == CA ? OpShape<pc2k::OP_DEC, CA>::EPW : OpShape<pc2k::OP_DEC, CB>::EPW;
    const size_t e = item.group * epw + threadIdx.x;
    if ((int)threadIdx.x >= epw || e >= job.count) continue;
    const int Ls = job.sk.h[0].Ls;
    const uint32_t* hp = job.stage + (e - job.stage_g0 * epw) * 2 * (size_t)(Ls + 1);
    garner_elem(job.sk, hp, hp + Ls + 1, job.out + e * job.sk.pk.L, err, work);
  }
}

// (CA, CB) pairs of geometry ids with a compiled batch kernel: single
// classes and the 1024 + 2048-bit mix, each also with the alternative
// encryption tiles (ids 9 and 10) of those two classes.
constexpr int PAIRS[][2] = {{3, 3}, {5, 5}, {6, 6}, {7, 7}, {8, 8}, {5, 6},
                            {9, 9}, {10, 10}, {5, 10}, {6, 9}, {9, 10}};
constexpr int NPAIRS = sizeof(PAIRS) / sizeof(PAIRS[0]);

template <int OP, int P>
const void* batch_ptr() {
  constexpr bool alt = PAIRS[P][0] >= pc2k::NUM_CLASSES || PAIRS[P][1] >= pc2k::NUM_CLASSES;
  if constexpr (alt && OP != pc2k::OP_ENC)
    return nullptr;
  else
    return (const void*)&k_batch<OP, PAIRS[P][0], PAIRS[P][1]>;
}

template <int P>
const void* garner_ptr() {
  constexpr bool alt = PAIRS[P][0] >= pc2k::NUM_CLASSES || PAIRS[P][1] >= pc2k::NUM_CLASSES;
  if constexpr (alt)
    return nullptr;
  else
    return (const void*)&k_batch_garner<PAIRS[P][0], PAIRS[P][1]>;
}

const void* garner_kernel(int pair) {
  switch (pair) {
    case 0: return garner_ptr<0>();
    case 1: return garner_ptr<1>();
    case 2: return garner_ptr<2>();
    case 3: return garner_ptr<3>();
    case 4: return garner_ptr<4>();
    case 5: return garner_ptr<5>();
  }
  return nullptr;
}

template <int OP>
const void* batch_kernel_op(int pair) {
  switch (pair) {
    case 0: return batch_ptr<OP, 0>();
    case 1: return batch_ptr<OP, 1>();
    case 2: return batch_ptr<OP, 2>();
    case 3: return batch_ptr<OP, 3>();
    case 4: return batch_ptr<OP, 4>();
    case 5: return batch_ptr<OP, 5>();
    case 6: return batch_ptr<OP, 6>();
    case 7: return batch_ptr<OP, 7>();
    case 8: return batch_ptr<OP, 8>();
    case 9: return batch_ptr<OP, 9>();
    case 10: return batch_ptr<OP, 10>();
  }
  return nullptr;
}
static_assert(NPAIRS == 11, "one case per pair above");

template <int OP, int C>
void shape_of(int w, int Ls, int* tiles, size_t* words, int* epw) {
  using S = OpShape<OP, C>;
  *tiles = S::TILES;
  *epw = S::EPW;
  const size_t scal = (size_t)12 * Ls + 16;
  if constexpr (OP == pc2k::OP_ENC)
    *words = (size_t)S::Gn::CH << w;
  else if constexpr (OP == pc2k::OP_DEC)
    *words = std::max((size_t)S::Gp::CH << w, scal);
  else
    *words = 0;
}

template <int OP>
void shape_geo(int geo, int w, int Ls, int* tiles, size_t* words, int* epw) {
  switch (geo) {
    case 3: shape_of<OP, 3>(w, Ls, tiles, words, epw); return;
    case 5: shape_of<OP, 5>(w, Ls, tiles, words, epw); return;
    case 6: shape_of<OP, 6>(w, Ls, tiles, words, epw); return;
    case 7: shape_of<OP, 7>(w, Ls, tiles, words, epw); return;
    case 8: shape_of<OP, 8>(w, Ls, tiles, words, epw); return;
    case 9: if constexpr (OP == pc2k::OP_ENC) { shape_of<OP, 9>(w, Ls, tiles, words, epw); return; } break;
    case 10: if constexpr (OP == pc2k::OP_ENC) { shape_of<OP, 10>(w, Ls, tiles, words, epw); return; } break;
  }
  *tiles = 0;
  *words = 0;
  *epw = 0;
}

}  // namespace

namespace pc2k {

int batch_pair(int ga, int gb) {
  if (ga > gb) std::swap(ga, gb);
  for (int i = 0; i < NPAIRS; ++i)
    if (PAIRS[i][0] == ga && PAIRS[i][1] == gb) return i;
  return -1;
}

int batch_pair_geo(int pair, int which) { return PAIRS[pair][which]; }

int batch_npairs() { return NPAIRS; }

const void* batch_kernel(int op, int pair) {
  switch (op) {
    case OP_ENC: return batch_kernel_op<OP_ENC>(pair);
    case OP_DEC: return batch_kernel_op<OP_DEC>(pair);
    case OP_SUM: return batch_kernel_op<OP_SUM>(pair);
  }
  return nullptr;
}

void batch_slot_shape(int op, int geo, int w, int Ls, int* tiles, size_t* words) {
  int epw = 0;
  switch (op) {
    case OP_ENC: shape_geo<OP_ENC>(geo, w, Ls, tiles, words, &epw); return;
    case OP_DEC: shape_geo<OP_DEC>(geo, w, Ls, tiles, words, &epw); return;
    case OP_SUM: shape_geo<OP_SUM>(geo, w, Ls, tiles, words, &epw); return;
  }
  *tiles = 0;
  *words = 0;
}

int batch_group_elems(int op, int geo) {
  int tiles = 0, epw = 0;
  size_t words = 0;
  switch (op) {
    case OP_ENC: shape_geo<OP_ENC>(geo, 4, 1, &tiles, &words, &epw); break;
    case OP_DEC: shape_geo<OP_DEC>(geo, 4, 1, &tiles, &words, &epw); break;
    case OP_SUM: shape_geo<OP_SUM>(geo, 4, 1, &tiles, &words, &epw); break;
  }
  return epw;
}

hipError_t launch_batch(int op, int pair, int grid, const BatchJob* jobs, const BatchItem* items,
                        int nitems, int* queue, uint32_t* scratch, size_t slot_words, int w_a,
                        int w_b, int* err, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* k = batch_kernel(op, pair);
  if (!k) return hipErrorInvalidValue;
  void* args[] = {(void*)&jobs, (void*)&items, (void*)&nitems, (void*)&queue,
                  (void*)&scratch, (void*)&slot_words, (void*)&w_a, (void*)&w_b, (void*)&err};
  e = hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, st);
  if (e != hipSuccess || op != OP_DEC) return e;
  const void* g = garner_kernel(pair);
  if (!g) return hipErrorInvalidValue;
  void* gargs[] = {(void*)&jobs, (void*)&items, (void*)&nitems, (void*)&err};
  return hipLaunchKernel(g, dim3(grid), dim3(64), gargs, 0, st);
}

}  // namespace pc2k
