// Host-side entry points into the kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "pc2_types.hpp"

namespace pc2k {

enum Op { OP_ENC = 0, OP_DEC = 1, OP_SUM = 2, OP_SMUL = 3, OP_FUSED = 4, OP_COUNT = 5 };

const void* kernel_for(int cls, int op);
void slot_shape(int cls, int op, int w, int Ls, int L, int* tiles, size_t* words);
int elems_per_block(int cls);

hipError_t launch_encrypt(int cls, const Launch& l, const PkConst& pk, const uint32_t* m,
                          int m_limbs, const uint32_t* r, uint32_t* c, size_t count);
hipError_t launch_decrypt(int cls, const Launch& l, const SkConst& sk, const uint32_t* c,
                          uint32_t* m, size_t count);
hipError_t launch_hom_sum(int cls, const Launch& l, const PkConst& pk, const PtrList& cs, int K,
                          uint32_t* out, size_t count);
hipError_t launch_scalar_mul(int cls, const Launch& l, const PkConst& pk, const uint32_t* c,
                             const uint32_t* k, uint32_t* out, size_t count);
hipError_t launch_fused(int cls, const Launch& l, const SkConst& sk, const PtrList& ms,
                        const PtrList& rs, int K, int m_limbs, uint32_t* mout, size_t count);

// persistent batch kernels (kernels_batch.hip)
int batch_pair(int ca, int cb);
int batch_pair_class(int pair, int which);
const void* batch_kernel(int op, int pair);
void batch_slot_shape(int op, int cls, int w, int Ls, int* tiles, size_t* words);
hipError_t launch_batch(int op, int pair, int grid, const BatchJob* jobs, const BatchItem* items,
                        int nitems, int* queue, uint32_t* scratch, size_t slot_words, int w_a,
                        int w_b, int* err, void* stream);

hipError_t launch_quantize(const Launch& l, int log2_scale, uint64_t offset, const double* x,
                           uint64_t* m, size_t count);
hipError_t launch_dequantize(const Launch& l, int log2_scale, uint64_t offset, const uint32_t* m,
                             int m_limbs, uint64_t weight, double* x, size_t count);

}  // namespace pc2k
