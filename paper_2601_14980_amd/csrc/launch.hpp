// Host-side entry points into the kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "pc2_types.hpp"

namespace pc2k {

enum Op {
  OP_ENC = 0, OP_DEC = 1, OP_SUM = 2, OP_SMUL = 3, OP_FUSED = 4,
  OP_ENC_MFMA = 5,  // encryption with the matrix-core product (kernels_mfma.hip)
  OP_ENC_CRT = 6,   // key-holder encryption through p^2 and q^2
  OP_FUSED_MFMA = 7,  // OP_FUSED with the matrix-core product
  OP_COUNT = 8
};

// kernel_for, slot_shape, elems_per_block and launch_encrypt take a geometry
// id (CLASS_GEO: a key class, or an alternative encryption tile); the other
// launches take the key class.
const void* kernel_for(int geo, int op);
void slot_shape(int geo, int op, int w, int Ls, int L, int* tiles, size_t* words);
int elems_per_block(int geo);          // elements per workgroup pass (modulus n^2)

hipError_t launch_encrypt(int geo, const Launch& l, const PkConst& pk, const uint32_t* m,
                          int m_limbs, const uint32_t* r, uint32_t* c, size_t count);
// halves: 2 (Ls + 1) words per element of staging between the two phases;
// count <= DEC_CHUNK per launch pair
constexpr size_t DEC_CHUNK = (size_t)1 << 18;
hipError_t launch_decrypt(int cls, const Launch& l, const SkConst& sk, const uint32_t* c,
                          uint32_t* m, size_t count, uint32_t* halves);
hipError_t launch_hom_sum(int cls, const Launch& l, const PkConst& pk, const PtrList& cs, int K,
                          uint32_t* out, size_t count);
hipError_t launch_scalar_mul(int cls, const Launch& l, const PkConst& pk, const uint32_t* c,
                             const uint32_t* k, uint32_t* out, size_t count);
// key-holder encryption: the two prime halves, then the recombination mod
// n^2; stage: 2 (nl2 + 1) words per element, count <= DEC_CHUNK per call
hipError_t launch_encrypt_crt(int cls, const Launch& l, const SkConst& sk, const uint32_t* m,
                              int m_limbs, const uint32_t* r, uint32_t* c, size_t count,
                              uint32_t* stage);
// first phase of the fused path: prod = prod_k Enc(m_k, r_k), 2L limbs per
// element, as K launches; acc: chunk_words(cls) words per element of running
// products, ok: one word per element
hipError_t launch_enc_prod(int cls, const Launch& l, const PkConst& pk, const PtrList& ms,
                           const PtrList& rs, int K, int m_limbs, uint32_t* prod, size_t count,
                           uint32_t* acc, uint32_t* ok);
size_t chunk_words(int geo);  // words of one n^2 residue in the geometry's chunked layout

// encryption with the i8-MFMA Montgomery product (kernels_mfma.hip); the
// scratch holds 2^window forward digit arrays per workgroup; fused: the
// kernel of one step of the fused path
const void* kernel_encrypt_mfma(int cls, bool fused = false);
size_t mfma_digit_bytes(int cls);
hipError_t launch_encrypt_mfma(int cls, const Launch& l, const PkConst& pk, const uint32_t* m,
                               int m_limbs, const uint32_t* r, uint32_t* c, size_t count);
// persistent batch encryption over the matrix cores for jobs of key class
// cls: queue reset, then grid workgroups (one wavefront each) pulling single
// elements of the items (job.group elements of one job; sub >= every
// job.group); scratch: grid tables of 2^w forward digit arrays
const void* batch_mfma_kernel(int cls);
hipError_t launch_batch_mfma(int cls, int grid, const BatchJob* jobs, const BatchItem* items,
                             int nitems, int sub, int* queue, uint8_t* scratch, int w, int* err,
                             void* stream);
// launch_enc_prod over the matrix cores; acc: mfma_digit_bytes(cls) bytes
// (16-byte aligned) per element
hipError_t launch_enc_prod_mfma(int cls, const Launch& l, const PkConst& pk, const PtrList& ms,
                                const PtrList& rs, int K, int m_limbs, uint32_t* prod,
                                size_t count, uint8_t* acc, uint32_t* ok);

// ciphertext matrix-vector product (kernels_matvec.hip), by key class:
// which = 0 the table kernel, 1 the row kernel
const void* kernel_matvec(int cls, int which);
size_t matvec_entry_words(int cls);  // words of one table entry (chunked n^2 digits)
hipError_t launch_mv_table(int cls, int grid, const PkConst& pk, const uint32_t* c, size_t cols,
                           int nw, int w, uint32_t* tab, int* err, void* stream);
hipError_t launch_mv_apply(int cls, int grid, const PkConst& pk, const uint64_t* B, size_t rows,
                           size_t cols, int ebits, int nw, int w, const uint32_t* tab,
                           const uint32_t* alpha, size_t nchunks, size_t chunk_cols,
                           uint32_t* out, size_t chunk_stride, int* err, void* stream);

// column-split ADMM (kernels_colsplit.hip): float64 setup of one node's
// constants (alpha_k, rho B_k), their quantization at scale 2^k (G, R and
// Gamma_1(alpha_k) as 4 limbs in g1), and the float64 / integer steps of an
// iteration around the encrypted node step.  T: Nk x 2Nk doubles; rp: 2Nk;
// f, aty: Nk doubles of workspace.
hipError_t cs_setup_node(const double* A, const double* y, int M, int N, int k0, int Nk,
                         double rho, double* T, double* rp, double* f, double* aty,
                         double* alpha, double* rhoB, void* stream);
hipError_t cs_quantize_node(const double* rhoB, const double* alpha, int Nk, int k, uint64_t* G,
                            uint64_t* R, uint32_t* g1, int* err, void* stream);
// every node at once over N = K Nk elements (S: K sums, R: [K][Nk])
hipError_t cs_quant_zv(const double* z, const double* v, int N, int K, int k, uint64_t* wz,
                       uint64_t* wv, uint64_t* S, int* err, void* stream);
hipError_t cs_dequant(const uint32_t* P, int L, int N, int K, const uint64_t* R,
                      const uint64_t* S, int k, double* x, int* err, void* stream);
hipError_t cs_plain_node(const double* rhoB, int Nk, const double* z, const double* v,
                         const double* alpha, double* x, void* stream);
hipError_t cs_update(const double* x, double* z, double* v, int N, double kappa, void* stream);

// persistent batch kernels (kernels_batch.hip)
// pairs of geometry ids with a compiled kernel; alternative tiles are
// compiled for encryption only (batch_kernel returns null otherwise)
int batch_pair(int ga, int gb);
int batch_pair_geo(int pair, int which);
int batch_npairs();
const void* batch_kernel(int op, int pair);
void batch_slot_shape(int op, int geo, int w, int Ls, int* tiles, size_t* words);
// elements per work item of a batch (decryption: per prime-half group)
int batch_group_elems(int op, int geo);
hipError_t launch_batch(int op, int pair, int grid, const BatchJob* jobs, const BatchItem* items,
                        int nitems, int* queue, uint32_t* scratch, size_t slot_words, int w_a,
                        int w_b, int* err, void* stream);

// FP64 ADMM kernels (kernels_admm.hip)
hipError_t admm_setup(const double* A, const double* y, int N, int B, int K, double rho,
                      double* W, double* aty, void* stream);
hipError_t admm_local(const double* A, const double* Lchol, const double* aty, const double* z,
                      const double* u, int N, int B, int K, double rho, double* w, double* t,
                      double* s, double* x, double* xu, void* stream);
hipError_t admm_consensus(const double* sum, const double* x, int N, int K, double kappa,
                          double* z, double* u, void* stream);

hipError_t launch_quantize(const Launch& l, int log2_scale, uint64_t offset, uint64_t delta,
                           const double* x, uint64_t* m, size_t count);
hipError_t launch_dequantize(const Launch& l, int log2_scale, uint64_t offset, const uint32_t* m,
                             int m_limbs, uint64_t weight, double* x, size_t count);

// the static device scratch of the allocation-free calls (static_scratch.hip):
// setup takes its address on `device`, which must be current (0, or -1 on
// failure); static_scratch returns that address (null before setup)
int static_scratch_setup(int device);
uint32_t* static_scratch(int device);

}  // namespace pc2k
