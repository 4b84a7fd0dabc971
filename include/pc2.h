/*
 * pc2.h -- C ABI of libpc2: batched Paillier encryption, decryption and
 * homomorphic aggregation of quantized vectors on one AMD Instinct MI355X
 * (gfx950), for the privacy-preserving distributed ADMM of
 * "Parallel Collaborative ADMM Privacy Computing and Adaptive GPU
 * Acceleration for Distributed Edge Networks" (Xia et al.).
 *
 * Conventions shared by every call
 * --------------------------------
 * Status.     Every function returns an int status: PC2_OK (0) or a negative
 *             PC2_E_* code.  Nothing aborts, throws or prints.
 * Integers.   Multi-precision values are little-endian arrays of uint32
 *             limbs.  For a key with nbits-bit n, L = ceil(nbits / 32);
 *             plaintexts and randomness have L limbs, ciphertexts 2L limbs.
 *             Inputs and outputs are canonical residues (in [0, modulus)),
 *             in normal (not Montgomery) form.
 * Arrays.     Data calls take DEVICE pointers to element-major arrays
 *             ([count][limbs]), owned and freed by the caller.  They are
 *             enqueued on the given HIP stream (NULL = the null stream) and
 *             return before the work finishes.  Outputs may alias an input
 *             of identical size exactly (same address, same bytes); any
 *             other overlap of an output with an input is PC2_E_INVAL.
 * Keys.       Key material is passed once, as HOST arrays, to the key
 *             constructors; the library derives and uploads every constant.
 *             g = n + 1 is implied (the paper admits any g in Z*_{n^2}).
 * Errors.     Argument errors (NULL pointer with count > 0, unsupported
 *             size, bad key) are reported synchronously and nothing is
 *             enqueued.  count == 0 is a no-op returning PC2_OK.  Data errors
 *             found on the device (a plaintext >= n, r = 0 or r >= n, a
 *             ciphertext >= n^2, a value outside the quantizer's range, a
 *             ciphertext that does not decrypt) make that element's output
 *             all-zero bits (NaN for dequantize) and latch PC2_E_RANGE in the
 *             context; pc2_ctx_sync returns and clears the latch.
 * Threads.    A context and its keys are used from one host thread at a
 *             time.  Calls on one stream run in order.  The data calls that
 *             use the context's scratch memory (encryptions, decryptions,
 *             scalar powers, the fused path) also run one after another
 *             across streams: a call on a stream other than the previous
 *             such call's makes its stream wait (on the device) for that
 *             call's completion event.  Under HIP graph capture no event is
 *             waited for or recorded; the caller orders a graph's replays
 *             against other calls on the context.
 * Memory.     Data calls never allocate.  The key constructors (and
 *             pc2_ctx_reserve) size the context's scratch for every data
 *             call of the key's size class at any element count, window
 *             and tile; a call that would still not fit returns
 *             PC2_E_NOMEM and enqueues nothing.
 */
#ifndef PC2_H
#define PC2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PC2_OK = 0,
  PC2_E_INVAL = -1,       /* bad argument (NULL, size, mismatched key/context) */
  PC2_E_RANGE = -2,       /* latched device data error (see Errors above) */
  PC2_E_NOMEM = -3,       /* device or host allocation failed */
  PC2_E_DEVICE = -4,      /* HIP runtime error or no usable device */
  PC2_E_UNSUPPORTED = -5, /* key size or option the library does not support */
  PC2_E_BUSY = -6         /* resource limit reached (serving admission) */
};

typedef struct pc2_ctx pc2_ctx;
typedef struct pc2_pk pc2_pk;
typedef struct pc2_sk pc2_sk;

/* Affine quantizer (Sec. III-A, Gamma_2 with a common interval and a
 * power-of-two scale): m = rint(x * 2^log2_scale) + offset on the common
 * interval [z_min, z_max) = [-offset, delta - offset) / 2^log2_scale (the
 * interval Theorem 1 assumes every quantized value lies in), onto
 * {0, ..., delta}; 0 <= offset <= delta.  Only pc2_quantize reads delta. */
typedef struct {
  int32_t log2_scale;
  uint64_t offset;
  uint64_t delta;
} pc2_qparams;

/* ------------------------------------------------------------- context */

/* Create a context bound to HIP device `hip_device`.  *out receives the
 * handle.  PC2_E_DEVICE if the device does not exist or is not gfx950. */
int pc2_ctx_create(int hip_device, pc2_ctx **out);
int pc2_ctx_destroy(pc2_ctx *ctx);

/* Wait for all work the library enqueued on `hip_stream`, then return and
 * clear the latched device data error (PC2_OK or PC2_E_RANGE). */
int pc2_ctx_sync(pc2_ctx *ctx, void *hip_stream);

/* Return and clear the latched data error without synchronising.  The value
 * reflects kernels that have completed. */
int pc2_ctx_take_error(pc2_ctx *ctx);

/* Size the scratch memory for every data call under keys of up to
 * `max_nbits` bits (the key constructors do this for their own size).  It
 * waits for the device when the scratch grows; data calls never do. */
int pc2_ctx_reserve(pc2_ctx *ctx, uint32_t max_nbits);

/* Options.  PC2_OPT_WINDOW: window width w in {0 (auto), 2..6} of the
 * modular exponentiations (sliding windows over the key's exponents n,
 * p - 1, q - 1; fixed windows over per-element exponents).
 * PC2_OPT_MODMUL: limb-product engine for the Montgomery products of
 * public-key encryption (pc2_encrypt, pc2_enc_sum_dec, and the encryption
 * jobs of batches and runners): PC2_MODMUL_VALU (27/28-bit digits, one
 * v_mad_u64_u32 per limb product), PC2_MODMUL_MFMA (7-bit digits in signed
 * redundant 28-bit limbs, the three limb-product matrices of each product on
 * the i8 matrix cores with int32 accumulation, one carry split per column on
 * the vector ALUs) or PC2_MODMUL_AUTO (the default: the MFMA engine for
 * keys of 2048 bits and more, where it is the faster one on the MI355X, the
 * VALU engine otherwise).  All give identical results; the other operations
 * always use the VALU engine.  A batch or runner launch holds encryption
 * jobs of at most two key classes per engine.
 * PC2_OPT_TILE: the limb tile of the VALU encryption kernels (pc2_encrypt,
 * batches and runners of encryptions), i.e. how many lanes of a wavefront
 * share one ciphertext.  1024-bit keys run with 2 (own) or 4 lanes,
 * 2048-bit keys with 4 (own) or 8; other sizes have their own tile only.
 * Values: 0 = automatic (pc2_encrypt of at most one wavefront per SIMD of
 * the wider tile, i.e. count <= 4 * CUs * 64 / lanes, takes the wider tile,
 * which has the shorter latency; larger calls, batches and runners take the
 * tile pc2_autotune chose for the key's class, else the class's own);
 * 2, 4 or 8 = that many lanes where the class has
 * such a tile, else its own; PC2_TILE_WIDE = the alternative tile of every
 * class that has one.  Fewer lanes mean more 27/28-bit digits per lane and
 * fewer lane exchanges per digit; more lanes mean fewer registers and more
 * resident wavefronts.  Results are identical in every tile.
 * Options apply to calls made after they are set. */
enum { PC2_OPT_WINDOW = 1, PC2_OPT_MODMUL = 2, PC2_OPT_TILE = 3 };
enum { PC2_TILE_AUTO = 0, PC2_TILE_WIDE = 1 };
enum { PC2_MODMUL_VALU = 0, PC2_MODMUL_MFMA = 1, PC2_MODMUL_AUTO = 2 };
int pc2_ctx_set_option(pc2_ctx *ctx, int option, int64_t value);
int pc2_ctx_get_option(pc2_ctx *ctx, int option, int64_t *value);

const char *pc2_strerror(int status);

/* ------------------------------------------------------------------ keys */

/* Public key (Sec. III-B key generation: public key (n, g), g = n + 1).
 * n: host array of ceil(nbits/32) limbs, odd, 15 <= n < 2^nbits, with
 * 2 <= nbits <= 4096. */
int pc2_pk_create(pc2_ctx *ctx, uint32_t nbits, const uint32_t *n, pc2_pk **out);

/* Private key from the primes p and q (Sec. III-B: n = pq,
 * eps = lcm(p-1, q-1)).  p, q: host arrays of ceil(nbits/32) limbs, distinct
 * odd primes with pq < 2^nbits.  Primality is the caller's contract.  The
 * key also serves as a public key for the data calls below through
 * pc2_sk_public. */
int pc2_sk_create(pc2_ctx *ctx, uint32_t nbits, const uint32_t *p, const uint32_t *q,
                  pc2_sk **out);
const pc2_pk *pc2_sk_public(const pc2_sk *sk);
int pc2_pk_destroy(pc2_pk *pk);
int pc2_sk_destroy(pc2_sk *sk);
/* Bit size and limb count L of a key. */
int pc2_pk_info(const pc2_pk *pk, uint32_t *nbits, uint32_t *limbs);
/* The context a key was created in, and that context's HIP device (either
 * output may be NULL). */
int pc2_pk_context(const pc2_pk *pk, pc2_ctx **ctx, int *hip_device);

/* ------------------------------------------------------------ data calls */

/* Quantize (Sec. III-A, Gamma_2 in affine form): m[i] = rint(x[i] * 2^k) + o,
 * rint = round half to even.  x: double[count]; m: uint64[count] (equal to
 * two uint32 limbs per element).  Non-finite x or x outside the common
 * interval [-o, delta - o) / 2^k (compared exactly) -> m = 0 and PC2_E_RANGE
 * latched; there is no clamping.  offset > delta is PC2_E_INVAL. */
int pc2_quantize(pc2_ctx *ctx, const pc2_qparams *q, const double *x, uint64_t *m,
                 size_t count, void *stream);

/* Inverse quantization of an aggregate of `weight` quantized addends
 * (Sec. III-C inverse quantization, generalised to weight W):
 * x[i] = double(M_i - W * o) / 2^k with round-to-nearest-even conversion.
 * m: uint32[count][m_limbs]; limbs above the first two must be zero and
 * |M_i - W*o| < 2^63, else x = NaN and PC2_E_RANGE latched. */
int pc2_dequantize(pc2_ctx *ctx, const pc2_qparams *q, const uint32_t *m,
                   uint32_t m_limbs, uint64_t weight, double *x, size_t count,
                   void *stream);

/* Encryption (Sec. III-B, f_en): c = g^m r^n mod n^2 with g = n + 1, i.e.
 * c = (1 + m n) r^n mod n^2.  m: [count][m_limbs] with 1 <= m_limbs <= L,
 * m < n; r: [count][L], 0 < r < n, one r per element (gcd(r, n) = 1 is the
 * caller's contract); c: [count][2L]. */
int pc2_encrypt(const pc2_pk *pk, const uint32_t *m, uint32_t m_limbs, const uint32_t *r,
                uint32_t *c, size_t count, void *stream);

/* Encryption by the key holder (Sec. III-B f_en evaluated through the split
 * of Z_{n^2} into Z_{p^2} x Z_{q^2} of Sec. IV, the paper's "EP"): the same
 * c = (1 + m n) r^n mod n^2 as pc2_encrypt, bit for bit, computed as
 * c_s = (1 + m n) r^(n mod s(s-1)) mod s^2 for s = p, q and recombined
 * modulo n^2 (Lemma 1 for the moduli p^2, q^2).  Arguments, layouts and data
 * errors as pc2_encrypt.  Requires balanced primes (p < 2q for p > q;
 * otherwise PC2_E_UNSUPPORTED), which every key of equal-length primes is. */
int pc2_encrypt_sk(const pc2_sk *sk, const uint32_t *m, uint32_t m_limbs, const uint32_t *r,
                   uint32_t *c, size_t count, void *stream);

/* Decryption (Sec. III-C, f_de = L(c^eps mod n^2) mu mod n), evaluated through
 * the split into Z_{p^2} x Z_{q^2} (Sec. IV, Lemmas 1-2).  c: [count][2L],
 * c < n^2; m: [count][L]. */
int pc2_decrypt(const pc2_sk *sk, const uint32_t *c, uint32_t *m, size_t count,
                void *stream);

/* Decryption for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * pc2_decrypt's arguments, layouts, data errors and results, bit for bit,
 * with its staging and window tables in a static device array of
 * PC2_STATIC_SCRATCH_BYTES per device (placed when the library's code is
 * loaded on the device, held until the process ends; its address is taken
 * by pc2_ctx_create) instead of the context's scratch.  The call allocates
 * nothing and waits for nothing.  Any count is accepted: it runs in chunks
 * whose staging fits an eighth of the array, with the widest window (up to
 * pc2_decrypt's) whose device-filling grid's tables fit the rest (w = 3 at
 * 2048-4096 bits), else a narrower grid; a key whose single workgroup does not fit is PC2_E_NOMEM
 * (no supported key size reaches it).  Every call on one device shares that
 * device's array: calls that overlap on one device (other streams, other
 * contexts or threads) race and give wrong results; calls on one stream run
 * in order.  The array's contents are overwritten before they are read, so
 * nothing needs clearing between calls.  PC2_E_DEVICE if the array's
 * address could not be taken on the key's device. */
#define PC2_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int pc2_decrypt_static(const pc2_sk *sk, const uint32_t *c, uint32_t *m, size_t count,
                       void *stream);

/* Homomorphic addition (Definition 1): out = c1 c2 mod n^2.  [count][2L]. */
int pc2_hom_add(const pc2_pk *pk, const uint32_t *c1, const uint32_t *c2, uint32_t *out,
                size_t count, void *stream);

/* Multiply by a constant (Definition 2): out = c^k mod n^2, k a uint64 per
 * element (k = 0 gives 1). */
int pc2_hom_scalar_mul(const pc2_pk *pk, const uint32_t *c, const uint64_t *k,
                       uint32_t *out, size_t count, void *stream);

/* K-way aggregation (Definition 1 applied K-1 times): out = prod_k c_k mod n^2.
 * c_k: HOST array of K device pointers, each [count][2L]; 1 <= K <= 128. */
int pc2_hom_sum(const pc2_pk *pk, const uint32_t *const *c_k, uint32_t K, uint32_t *out,
                size_t count, void *stream);

/* Fused encrypt -> aggregate -> decrypt: m_out[j] = Dec(prod_k Enc(m_k[j], r_k[j])).
 * m_k, r_k: HOST arrays of K device pointers ([count][m_limbs], [count][L]);
 * m_out: [count][L].  The ciphertexts never reach the caller's memory.
 * 1 <= K <= 128. */
int pc2_enc_sum_dec(const pc2_sk *sk, const uint32_t *const *m_k, const uint32_t *const *r_k,
                    uint32_t K, uint32_t m_limbs, uint32_t *m_out, size_t count,
                    void *stream);

/* ------------------------------------------- ciphertext matrix-vector */

/* The edge node's update in the paper's column form (Sec. III-C, eq. (itq2)):
 *     out_i = alpha_i * prod_j c_j^(B_ij) mod n^2,   i < rows, j < cols,
 * i.e. Definition 2 with a matrix of non-negative integer constants B applied
 * to the ciphertext vector c (eq. (hemul)), then Definition 1 with the
 * ciphertexts alpha.  It decrypts to Dec(alpha_i) + sum_j B_ij Dec(c_j) mod n.
 *
 * A plan holds fixed-base tables of the bases: for column j and window t,
 * (c_j^(2^(w t)))^d for d = 1 .. 2^w - 1 in Montgomery form, so that a row
 * costs one modular product per nonzero w-bit digit of its constants and no
 * squarings; the tables take cols * ceil(ebits / w) * (2^w - 1) entries of
 * the n^2 digit layout (640 B at 2048 bits).
 *
 * pc2_matvec_create: cols >= 1; ebits in 1..64 bounds the constants
 * (B_ij < 2^ebits); window w in 1..12, or 0 = automatic: the w minimising
 * ceil(ebits / w) (rows_hint + 2^w) (rows_hint = 0: w = 8) among those whose
 * tables fit in a quarter of the free device memory.  Allocates the tables
 * (PC2_E_NOMEM if they do not fit).
 * pc2_matvec_info: the window and the table bytes of a plan (either may be NULL).
 * pc2_matvec_load: builds the tables of c ([cols][2L], device) on the stream.
 *   c_j >= n^2 latches PC2_E_RANGE and zeroes that column's tables.
 * pc2_matvec_apply: B: device uint64 [rows][cols] row-major; alpha: device
 *   [rows][2L] or NULL (then alpha_i = 1, the encryption of 0 with r = 1);
 *   out: device [rows][2L], may be alpha itself (no partial overlap).  Needs a
 *   completed load on the same stream order.  rows = 0 is a no-op.  A row with
 *   B_ij >= 2^ebits or alpha_i >= n^2 is written as zero with PC2_E_RANGE
 *   latched; rows that use a zeroed column come out zero.  Staging for
 *   partial products (rows split over column chunks to fill the device) is
 *   allocated on the first call that needs more than the plan holds.
 * The plan's device memory is owned by the plan; the caller owns c, B, alpha,
 * out.  A plan is used from one host thread at a time. */
typedef struct pc2_matvec pc2_matvec;
int pc2_matvec_create(const pc2_pk *pk, size_t cols, uint32_t ebits, uint32_t window,
                      size_t rows_hint, pc2_matvec **out);
int pc2_matvec_info(const pc2_matvec *mv, uint32_t *window, size_t *table_bytes);
int pc2_matvec_load(pc2_matvec *mv, const uint32_t *c, void *hip_stream);
int pc2_matvec_apply(pc2_matvec *mv, const uint64_t *B, const uint32_t *alpha, uint32_t *out,
                     size_t rows, void *hip_stream);
int pc2_matvec_destroy(pc2_matvec *mv);

/* --------------------------------------- column-split 3P-ADMM-PC2 loop */

/* Algorithm 1 with A split by COLUMNS over K nodes (Sec. II, eqs. (sldi231),
 * (sldo34), (iu43)): node k keeps B_k = (A_k^T A_k + rho I)^-1 and
 * G_k = Gamma_2(rho B_k); the master sends Enc(Gamma_1(B_k A_k^T y)) once and
 * Enc(Gamma_2(z_k)), Enc(Gamma_2(-v_k)) every iteration; the node returns
 * alpha_k (+) G_k (x) (z_k (+) -v_k) (eq. (itq2)); the master decrypts,
 * inverts the quantization and updates z = S_{lambda/rho}(v + x),
 * v = v + x - z.  Quantizers with scale s = 2^log2_scale on [-8, 8):
 * Gamma_2(u) = rint(u s) + 8 s, Gamma_1(u) = rint(u s^2) + 8 s^2; the inverse
 * quantization of a row of Nk terms is
 *   x_i = float64(P_i - 8 s^2 - 16 s R_i - 8 s S + 128 Nk s^2) / s^2
 * with R_i = sum_j (G_k)_ij and S = sum_j (Gamma_2(z_k) + Gamma_2(-v_k))_j (the
 * form of Theorem 1's cross terms for Nk > 1).  All work runs on the device:
 * the setup computes A_k^T A_k + rho I and its Gauss-Jordan inverse in
 * float64 in a fixed summation order.
 *
 * pc2_colsplit_create: A: device double [M][N] row-major, y: device double [M];
 *   N a multiple of K; rho > 0; 1 <= log2_scale with 2 log2_scale + 9 +
 *   ceil(log2(N / K)) bits below both 127 and the key's size
 *   (PC2_E_UNSUPPORTED otherwise); r_pool: device [r_count][L] randomness
 *   (0 < r < n), r_count >= 3 N: rows 0 .. N-1 encrypt alpha, and each
 *   iteration takes the next 2 N rows of the rest, cyclically.
 *   Synchronises the stream (the setup's workspace is released); A, y and
 *   r_pool must stay valid while the object lives (r_pool is read every
 *   iteration).
 * pc2_colsplit_set_scale: quantize again at scale 2^log2_scale (same bounds as
 *   at creation): G_k, its row sums, Enc(Gamma_1(alpha_k)) (pool rows 0 .. N-1
 *   again) and the mat-vec plans over (log2_scale + 4)-bit constants; the
 *   float64 setup (B_k, alpha_k) is kept.  Synchronises the stream.  After
 *   an error the object only runs unquantized iterations (quantized ones
 *   return PC2_E_INVAL) until a change of scale succeeds.
 * pc2_colsplit_iterate: one iteration on device double [N] arrays x (out),
 *   z and v (in and out).  quantized != 0 runs the encrypted node step;
 *   quantized = 0 the same iteration in float64 without quantization
 *   (x_k = alpha_k + (rho B_k)(z_k - v_k)), the reference of the
 *   quantization error.  Values that leave [-8, 8) latch PC2_E_RANGE.  Asynchronous. */
typedef struct pc2_colsplit pc2_colsplit;
int pc2_colsplit_create(const pc2_sk *sk, const double *A, const double *y, uint32_t M,
                        uint32_t N, uint32_t K, double rho, uint32_t log2_scale,
                        const uint32_t *r_pool, size_t r_count, void *hip_stream,
                        pc2_colsplit **out);
int pc2_colsplit_set_scale(pc2_colsplit *cs, uint32_t log2_scale, void *hip_stream);
int pc2_colsplit_iterate(pc2_colsplit *cs, double lambda, int quantized, double *x, double *z,
                         double *v, void *hip_stream);
int pc2_colsplit_destroy(pc2_colsplit *cs);

/* ------------------------------------------------------ batched launches */

/* One job of a batch.  (Its output may be one of its inputs exactly, as for
 * the data calls; any other overlap is PC2_E_INVAL.)  A batch runs one phase
 * of many edge nodes' work --
 * all their encryptions, all their aggregations or all their decryptions --
 * in ONE persistent launch per Montgomery engine, whatever the vector
 * lengths, under keys of up to two size classes per engine (supported mixes
 * for the VALU engine: one class of 256, 1024, 2048, 3072 or 4096 bits, or
 * 1024 with 2048 bits; encryption jobs whose class runs on the matrix cores
 * (PC2_OPT_MODMUL) go to a launch of their own per class, after the VALU
 * launch, with single elements as work items).  Results are identical to
 * the one-call-per-job entry points above. */
enum { PC2_OP_ENCRYPT = 1, PC2_OP_HOM_SUM = 2, PC2_OP_DECRYPT = 3 };
typedef struct {
  int op;                        /* PC2_OP_*; every job of a batch has the same op */
  const pc2_pk *pk;              /* encrypt, hom_sum */
  const pc2_sk *sk;              /* decrypt */
  const uint32_t *in0;           /* encrypt: m [count][m_limbs]; decrypt: c [count][2L] */
  const uint32_t *in1;           /* encrypt: r [count][L] */
  uint32_t m_limbs;              /* encrypt */
  uint32_t *out;                 /* encrypt: c [count][2L]; decrypt: m [count][L];
                                    hom_sum: product [count][2L] */
  size_t count;                  /* output elements (0: the job is skipped) */
  uint32_t K;                    /* hom_sum: number of inputs, 1..128 */
  const uint32_t *const *inputs; /* hom_sum: HOST array of K device pointers */
  const size_t *lengths;         /* hom_sum: HOST array of K input lengths or NULL; element j
                                    multiplies the inputs k with j < lengths[k] (ragged
                                    aggregation), or all K inputs when NULL */
} pc2_job;
typedef struct pc2_batch pc2_batch;

/* Plan a batch: validates the jobs, uploads job descriptors and a work
 * queue, and allocates the batch's own scratch (so that later calls never
 * allocate).  The device arrays named by the jobs must stay valid for the
 * life of the batch; their contents may change between runs. */
int pc2_batch_create(pc2_ctx *ctx, const pc2_job *jobs, size_t njobs, pc2_batch **out);

/* Run a planned batch on a stream.  On a non-null stream the first run
 * captures the launch in a HIP graph and later runs replay it. */
int pc2_batch_run(pc2_batch *batch, void *hip_stream);
int pc2_batch_destroy(pc2_batch *batch);

/* A reusable persistent launcher for schedulers that form a new batch at
 * every launch (continuous batching, see the serving loop): descriptor and
 * work-queue buffers (device and pinned host) and scratch are allocated once,
 * for up to max_jobs jobs and max_groups element groups per launch, with keys
 * of at most max_nbits bits. */
typedef struct pc2_runner pc2_runner;
int pc2_runner_create(pc2_ctx *ctx, int op, uint32_t max_nbits, size_t max_jobs,
                      size_t max_groups, pc2_runner **out);
/* Elements per group (one wavefront's share) for a key and op. */
int pc2_runner_group_size(const pc2_pk *pk, int op, uint32_t *elems);
/* One persistent launch over element groups [first[i], first[i] + ngroups[i])
 * of each job i (jobs as for pc2_batch_create; the key classes of one launch
 * must form a supported mix).  Asynchronous on the stream; the launcher's
 * staging buffers are reused by the next launch once this one's copies are
 * done. */
int pc2_runner_launch(pc2_runner *runner, const pc2_job *jobs, const size_t *first,
                      const size_t *ngroups, size_t njobs, void *hip_stream);
int pc2_runner_destroy(pc2_runner *runner);

/* --------------------------------------------------------------- serving
 *
 * A request server (continuous batching) for one private key: clients submit
 * encryptions, aggregations and decryptions of vectors of any length as they
 * arrive and poll for completion by request id.  A request is admitted when
 * the bytes of its inputs and output (encrypt: count * (4 m_limbs + 12 L);
 * hom_sum: count * 8 L (K + 1); decrypt: count * 12 L) fit in the server's
 * HBM budget beside those already admitted (in arrival order; see the launch
 * policy for what happens to requests behind one that does not fit).  Each
 * operation has its own persistent launcher and stream; whenever a stream is
 * idle, the next scheduling pass launches up to tick_groups element groups
 * (pc2_runner_group_size elements each) drawn from the admitted requests of
 * that operation in the order of the launch policy (pc2_server_set_policy),
 * so requests that arrive while others run join the next launch and the
 * three operations overlap on the device.  (They overlap when HIP gives the
 * three streams hardware queues of their own; in a process that has created
 * many streams before -- torch's stream pool holds dozens -- they can share
 * queues, and launches of different operations then run one after the
 * other.)  Results are identical to the one-call entry points.
 *
 * Every pc2_serve_* call makes one scheduling pass (retire finished
 * launches, admit, launch on idle streams); nothing advances between calls,
 * so a client waiting for results keeps calling pc2_serve_poll,
 * pc2_serve_progress or pc2_serve_completed.  A server is used from one host
 * thread at a time; data errors latch in the context as for every data call.
 * Changing the key's encryption tile (PC2_OPT_TILE, pc2_autotune) while
 * requests of an operation are admitted makes the next pass return
 * PC2_E_UNSUPPORTED (their element groups were cut for the old tile) until
 * the tile is restored; with none admitted the new tile is used.
 * PC2_E_DEVICE from a pass leaves the server unusable: destroy it. */
typedef struct pc2_server pc2_server;

/* sk: the key every request uses (created in ctx).  hbm_budget: bytes of
 * admitted requests at once (0 = half the device memory free now).
 * tick_groups: element groups per launch.  max_requests: requests tracked at
 * once (submitted and not yet reported done).  Allocates the three
 * launchers, streams and events. */
int pc2_server_create(pc2_ctx *ctx, const pc2_sk *sk, size_t hbm_budget, size_t tick_groups,
                      size_t max_requests, pc2_server **out);

/* Queue one request: a pc2_job (as for pc2_batch_create) with op, the
 * server's key (pk = pc2_sk_public(sk) for encrypt and hom_sum, sk for
 * decrypt), device inputs and a device output of count elements, all owned
 * by the caller and valid until the request is reported done.  The HOST
 * arrays of a hom_sum job are copied.  *req_id receives the request's id.
 * PC2_E_INVAL for a bad job or another key; PC2_E_NOMEM if the request could
 * never fit the budget; PC2_E_BUSY if max_requests are tracked.  count == 0
 * completes at once. */
int pc2_serve_submit(pc2_server *srv, const pc2_job *job, uint64_t *req_id);

/* One pass, then *done = 1 if request req_id has finished (its output is
 * complete on the device); the id is then forgotten.  PC2_E_INVAL for an id
 * the server does not track. */
int pc2_serve_poll(pc2_server *srv, uint64_t req_id, int *done);

/* One pass; *pending (may be NULL) = requests waiting or admitted and not
 * finished. */
int pc2_serve_progress(pc2_server *srv, size_t *pending);

/* Drain up to cap ids of finished requests, in the order they finished
 * (requests already reported by pc2_serve_poll are skipped); *n = how many.
 * The ids are then forgotten.  Makes no pass. */
int pc2_serve_completed(pc2_server *srv, uint64_t *ids, size_t cap, size_t *n);

/* Launch and admission policy.  PC2_SERVE_SHORTEST (the default, with
 * max_age_s = 1): requests take the launch in increasing order of the groups
 * they have left (shortest remaining first, the order that minimises mean
 * latency), except that requests admitted more than max_age_s seconds ago go
 * first, oldest first, which bounds how long a long request can be passed
 * over; every waiting request that fits the budget is admitted, except that
 * one submitted more than max_age_s ago which does not fit holds back those
 * behind it.  PC2_SERVE_FAIR: every admitted request of the operation gets an
 * equal slice of the launch, what is left goes to the oldest; admission is
 * first come, first served (a request that does not fit holds back those
 * behind it).  Applies from the next scheduling pass. */
enum { PC2_SERVE_FAIR = 0, PC2_SERVE_SHORTEST = 1 };
int pc2_server_set_policy(pc2_server *srv, int policy, double max_age_s);

/* Launches so far, the largest and the current admitted bytes (any output
 * may be NULL). */
int pc2_server_stats(const pc2_server *srv, uint64_t *launches, size_t *max_bytes,
                     size_t *used_bytes);

/* Waits for the server's launches, then frees it.  Requests not finished are
 * dropped. */
int pc2_server_destroy(pc2_server *srv);

/* ------------------------------------------------ ADMM update (FP64 kernels)
 *
 * The consensus-lasso iteration around the encrypted aggregation: A (M x N,
 * row-major doubles) is split by rows over K nodes of B = M/K rows; node k
 * holds A_k, y_k and u_k (Sec. II's x/z/v updates with v = u/rho, in the
 * global-consensus form of this row split).
 *   pc2_admm_local:     w_k = A_k^T y_k + rho (z - u_k),
 *                       x_k = (w_k - A_k^T W_k^-1 A_k w_k) / rho,  W_k = rho I + A_k A_k^T,
 *                       xu_k = x_k + u_k (the vector each node quantizes and encrypts)
 *   pc2_admm_consensus: z = S_{lambda/(rho K)}(sum / K) with S the soft threshold and
 *                       sum = sum_k xu_k (the decrypted, dequantized aggregate);
 *                       u_k += x_k - z
 * A and y are device pointers owned by the caller (valid for the handle's
 * life); z [N], u, x, xu [K][N] and sum [N] are device doubles. */
typedef struct pc2_admm pc2_admm;
int pc2_admm_create(pc2_ctx *ctx, const double *A, const double *y, uint32_t M, uint32_t N,
                    uint32_t K, double rho, void *hip_stream, pc2_admm **out);
int pc2_admm_local(pc2_admm *admm, const double *z, const double *u, double *x, double *xu,
                   void *hip_stream);
int pc2_admm_consensus(pc2_admm *admm, const double *sum, const double *x, double lambda,
                       double *z, double *u, void *hip_stream);
int pc2_admm_destroy(pc2_admm *admm);

/* Autotuner: times encryption under this key's size class in every limb
 * tile the class has (see PC2_OPT_TILE) with exponentiation windows w in
 * {4, 5, 6}, and decryption with w in {4, 5, 6}, on the same synthetic
 * sample of a few device-filling waves (VALU engine).  Keeps the fastest
 * tile and windows in the context (used by later calls, batches and runners
 * of that class while PC2_OPT_TILE and PC2_OPT_WINDOW are 0) and reports
 * them: w_enc, w_dec, and tile_enc = lanes per ciphertext (any output may be
 * NULL).  Synchronises the stream; allocates temporary buffers. */
int pc2_autotune(const pc2_sk *sk, void *hip_stream, int *w_enc, int *w_dec, int *tile_enc);

#ifdef __cplusplus
}
#endif
#endif /* PC2_H */
