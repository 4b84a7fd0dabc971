// C ABI of libpc2 (declared in include/pc2.h): contexts, keys, argument
// validation, scratch sizing and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pc2.h"
#include "host_bn.hpp"
#include "launch.hpp"
#include "pc2_types.hpp"

using pc2h::Limbs;

struct pc2_ctx {
  int device = 0;
  int cus = 0;
  int* err = nullptr;          // device word, latched error bits
  uint32_t* scratch = nullptr; // per-tile tables
  size_t scratch_bytes = 0;
  int window = 0;              // 0 = automatic
  int modmul = PC2_MODMUL_VALU;
  int occ[pc2k::NUM_CLASSES][pc2k::OP_COUNT] = {};  // workgroups per CU (0 = not queried)
};

struct pc2_pk {
  pc2_ctx* ctx = nullptr;
  uint32_t nbits = 0;
  int L = 0;
  int cls = 0;
  void* dev = nullptr;  // one allocation holding every constant
  pc2k::PkConst c{};
};

struct pc2_sk {
  pc2_ctx* ctx = nullptr;
  pc2_pk pk;            // the public part (owns nothing; dev below owns all)
  void* dev = nullptr;
  pc2k::SkConst c{};
};

namespace {

// ------------------------------------------------------------ helpers
struct DevBuf {
  std::vector<uint32_t> words;
  // append words, 16-byte aligned; returns the word offset
  size_t add(const std::vector<uint32_t>& w) {
    size_t off = words.size();
    words.insert(words.end(), w.begin(), w.end());
    while (words.size() % 4) words.push_back(0);
    return off;
  }
};

// value -> chunked D-digit layout for geometry (D, K, T)
std::vector<uint32_t> to_chunk(const Limbs& v, int D, int K, int T) {
  const int K4 = (K + 3) & ~3;
  std::vector<uint32_t> out((size_t)T * K4, 0);
  const int S = K * T;
  for (int g = 0; g < S; ++g) {
    long bit = (long)g * D;
    size_t w = bit / 32;
    int s = bit % 32;
    uint64_t lo = w < v.size() ? v[w] : 0, hi = w + 1 < v.size() ? v[w + 1] : 0;
    uint32_t d = (uint32_t)(((hi << 32) | lo) >> s) & ((1u << D) - 1u);
    out[(size_t)(g / K) * K4 + (g % K)] = d;
  }
  return out;
}

bool fits_digits(const Limbs& v, int D, int S) { return pc2h::bitlen(v) <= D * S; }

// Montgomery constants of odd N in geometry (D, K, T), appended to buf.
struct ModOffsets {
  size_t N, R1, R2, R3, ONE, Nl;
  uint32_t nprime;
  int nl;
};
ModOffsets add_modulus(DevBuf& buf, const Limbs& N0, int D, int K, int T, int nl) {
  Limbs N = N0;
  pc2h::trim(N);
  const int S = K * T;
  const uint64_t RB = (uint64_t)D * S;  // R = 2^RB
  ModOffsets o{};
  Limbs r1 = pc2h::pow2_mod(RB, N);
  Limbs r2 = pc2h::shl_mod(r1, RB, N);
  Limbs r3 = pc2h::shl_mod(r2, RB, N);
  o.N = buf.add(to_chunk(N, D, K, T));
  o.R1 = buf.add(to_chunk(r1, D, K, T));
  o.R2 = buf.add(to_chunk(r2, D, K, T));
  o.R3 = buf.add(to_chunk(r3, D, K, T));
  o.ONE = buf.add(to_chunk(Limbs{1}, D, K, T));
  o.Nl = buf.add(pc2h::resized(N, nl));
  uint32_t inv = pc2h::inv32(N[0]);
  o.nprime = (0u - inv) & ((1u << D) - 1u);
  o.nl = nl;
  return o;
}
pc2k::ModConst mod_const(const uint32_t* base, const ModOffsets& o) {
  pc2k::ModConst m{};
  m.N = base + o.N;
  m.R1 = base + o.R1;
  m.R2 = base + o.R2;
  m.R3 = base + o.R3;
  m.ONE = base + o.ONE;
  m.Nl = base + o.Nl;
  m.nprime = o.nprime;
  m.nl = o.nl;
  return m;
}

struct PkOffsets {
  ModOffsets n2;
  size_t nR, Rk, n;
};

PkOffsets add_public(DevBuf& buf, const Limbs& n, int cls, int L) {
  const pc2k::ClassGeo g = pc2k::CLASS_GEO[cls];
  Limbs n2 = pc2h::mul(n, n);
  PkOffsets o{};
  o.n2 = add_modulus(buf, n2, g.nD, g.nK, g.nT, 2 * L);
  const uint64_t RB = (uint64_t)g.nD * g.nK * g.nT;
  Limbs nR = pc2h::shl_mod(n, RB, n2);
  o.nR = buf.add(to_chunk(nR, g.nD, g.nK, g.nT));
  // R^k mod n^2, k = 0..RK_MAX, by Montgomery products with 32-bit limbs
  pc2h::Mont32 M(n2);
  Limbs r1m = M.to(pc2h::pow2_mod(RB, n2));
  Limbs rkm = M.to(Limbs{1});
  std::vector<uint32_t> tab;
  for (int k = 0; k <= pc2k::RK_MAX; ++k) {
    std::vector<uint32_t> ch = to_chunk(M.from(rkm), g.nD, g.nK, g.nT);
    tab.insert(tab.end(), ch.begin(), ch.end());
    rkm = M.mm(rkm, r1m);
  }
  o.Rk = buf.add(tab);
  o.n = buf.add(pc2h::resized(n, L));
  return o;
}

pc2k::PkConst pk_const(const uint32_t* base, const PkOffsets& o, int L, int nbits) {
  pc2k::PkConst c{};
  c.n2 = mod_const(base, o.n2);
  c.nR = base + o.nR;
  c.Rk = base + o.Rk;
  c.n = base + o.n;
  c.L = L;
  c.nbits = nbits;
  return c;
}

struct HalfOffsets {
  ModOffsets s2;
  size_t s, e, sinv, H;
  uint32_t s_n0;
  int Ls;
};

// constants for the prime s (other prime t, n = s t) of the CRT decryption
HalfOffsets add_half(DevBuf& buf, const Limbs& s, const Limbs& t, const Limbs& n, int cls, int Ls,
                     int nl2) {
  const pc2k::ClassGeo g = pc2k::CLASS_GEO[cls];
  HalfOffsets o{};
  Limbs s2 = pc2h::mul(s, s);
  o.s2 = add_modulus(buf, s2, g.pD, g.pK, g.pT, nl2);
  o.s = buf.add(pc2h::resized(s, Ls));
  o.e = buf.add(pc2h::resized(pc2h::sub(pc2h::resized(s, Ls), Limbs{1}), Ls));
  Limbs sinv = pc2h::inv_pow2(s, Ls);
  o.sinv = buf.add(sinv);
  // h_s = L_s(g^(s-1) mod s^2)^-1 mod s with g = n + 1
  pc2h::Mont32 M2(s2);
  Limbs gm = pc2h::mod(pc2h::add(n, Limbs{1}), s2);
  Limbs y = M2.pow(gm, pc2h::sub(pc2h::resized(s, Ls), Limbs{1}));
  Limbs ym1 = pc2h::sub(pc2h::resized(y, (size_t)2 * Ls + 1), Limbs{1});
  Limbs u = pc2h::resized(pc2h::mul(pc2h::resized(ym1, Ls), sinv), Ls);  // exact (y-1)/s
  Limbs hs = pc2h::inv_mod_prime(pc2h::mod(u, s), s);
  Limbs H = pc2h::shl_mod(hs, (uint64_t)32 * Ls, s);
  o.H = buf.add(pc2h::resized(H, Ls));
  o.s_n0 = 0u - pc2h::inv32(s[0]);
  o.Ls = Ls;
  (void)t;
  return o;
}

pc2k::HalfConst half_const(const uint32_t* base, const HalfOffsets& o) {
  pc2k::HalfConst h{};
  h.s2 = mod_const(base, o.s2);
  h.s = base + o.s;
  h.e = base + o.e;
  h.sinv = base + o.sinv;
  h.H = base + o.H;
  h.s_n0 = o.s_n0;
  h.Ls = o.Ls;
  return h;
}

Limbs limbs_from(const uint32_t* p, size_t n) {
  Limbs v(p, p + n);
  pc2h::trim(v);
  return v;
}

int upload(pc2_ctx* ctx, const DevBuf& buf, void** dev) {
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  if (hipMalloc(dev, buf.words.size() * 4) != hipSuccess) return PC2_E_NOMEM;
  if (hipMemcpy(*dev, buf.words.data(), buf.words.size() * 4, hipMemcpyHostToDevice) !=
      hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
    return PC2_E_DEVICE;
  }
  return PC2_OK;
}

int auto_window(int cls, int op) {
  // window width minimising products for the exponent lengths of each class
  if (op == pc2k::OP_SMUL) return 4;
  return cls >= 5 ? 5 : (cls >= 3 ? 4 : 3);
}

int occupancy(pc2_ctx* ctx, int cls, int op) {
  int& o = ctx->occ[cls][op];
  if (o == 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, pc2k::kernel_for(cls, op), 64, 0) !=
            hipSuccess ||
        v <= 0)
      v = 1;
    o = v;
  }
  return o;
}

// grid + scratch for a Paillier launch over `count` elements
int prepare(pc2_ctx* ctx, int cls, int op, size_t count, int Ls, int L, pc2k::Launch* l,
            void* stream) {
  const int w = ctx->window ? ctx->window : auto_window(cls, op);
  const size_t epb = (size_t)pc2k::elems_per_block(cls);
  const size_t groups = (count + epb - 1) / epb;
  const size_t cap = (size_t)ctx->cus * occupancy(ctx, cls, op);
  l->grid = (int)std::max<size_t>(1, std::min(groups, cap));
  l->window = w;
  l->err = ctx->err;
  l->stream = stream;
  int tiles = 0;
  size_t words = 0;
  pc2k::slot_shape(cls, op, w, Ls, L, &tiles, &words);
  words = (words + 3) & ~(size_t)3;
  l->slot_words = words;
  const size_t need = (size_t)l->grid * tiles * words * 4;
  if (need > ctx->scratch_bytes) {
    // growing the scratch: wait for in-flight work that may use the old one
    if (hipDeviceSynchronize() != hipSuccess) return PC2_E_DEVICE;
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    if (hipMalloc(&ctx->scratch, need) != hipSuccess) return PC2_E_NOMEM;
    ctx->scratch_bytes = need;
  }
  l->scratch = ctx->scratch;
  return PC2_OK;
}

int status_of(hipError_t e) { return e == hipSuccess ? PC2_OK : PC2_E_DEVICE; }

}  // namespace

// ================================================================ ABI
extern "C" {

const char* pc2_strerror(int status) {
  switch (status) {
    case PC2_OK: return "ok";
    case PC2_E_INVAL: return "invalid argument";
    case PC2_E_RANGE: return "input value out of range";
    case PC2_E_NOMEM: return "out of memory";
    case PC2_E_DEVICE: return "HIP device error";
    case PC2_E_UNSUPPORTED: return "unsupported size or option";
    case PC2_E_BUSY: return "resource busy";
  }
  return "unknown status";
}

int pc2_ctx_create(int hip_device, pc2_ctx** out) {
  if (!out) return PC2_E_INVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return PC2_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return PC2_E_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PC2_E_DEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return PC2_E_DEVICE;
  pc2_ctx* c = new (std::nothrow) pc2_ctx();
  if (!c) return PC2_E_NOMEM;
  c->device = hip_device;
  c->cus = prop.multiProcessorCount;
  if (hipMalloc(&c->err, sizeof(int)) != hipSuccess) {
    delete c;
    return PC2_E_NOMEM;
  }
  if (hipMemset(c->err, 0, sizeof(int)) != hipSuccess) {
    (void)hipFree(c->err);
    delete c;
    return PC2_E_DEVICE;
  }
  *out = c;
  return PC2_OK;
}

int pc2_ctx_destroy(pc2_ctx* ctx) {
  if (!ctx) return PC2_E_INVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->err) (void)hipFree(ctx->err);
  delete ctx;
  return PC2_OK;
}

int pc2_ctx_take_error(pc2_ctx* ctx) {
  if (!ctx) return PC2_E_INVAL;
  int v = 0;
  if (hipMemcpy(&v, ctx->err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return PC2_E_DEVICE;
  if (v && hipMemset(ctx->err, 0, sizeof(int)) != hipSuccess) return PC2_E_DEVICE;
  return (v & pc2k::ERR_RANGE) ? PC2_E_RANGE : PC2_OK;
}

int pc2_ctx_sync(pc2_ctx* ctx, void* hip_stream) {
  if (!ctx) return PC2_E_INVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return PC2_E_DEVICE;
  return pc2_ctx_take_error(ctx);
}

int pc2_ctx_reserve(pc2_ctx* ctx, uint32_t max_nbits) {
  if (!ctx) return PC2_E_INVAL;
  const int cls = pc2k::class_for_bits((int)max_nbits);
  if (cls < 0) return PC2_E_UNSUPPORTED;
  const int L = (int)((max_nbits + 31) / 32);
  const int Ls = (L + 1) / 2 + 1;
  pc2k::Launch l{};
  const size_t big = (size_t)1 << 40;  // enough elements to fill the device
  for (int op : {pc2k::OP_ENC, pc2k::OP_DEC, pc2k::OP_SMUL, pc2k::OP_FUSED}) {
    int rc = prepare(ctx, cls, op, big, Ls, L, &l, nullptr);
    if (rc) return rc;
  }
  return PC2_OK;
}

int pc2_ctx_set_option(pc2_ctx* ctx, int option, int64_t value) {
  if (!ctx) return PC2_E_INVAL;
  if (option == PC2_OPT_WINDOW) {
    if (value != 0 && (value < 2 || value > 6)) return PC2_E_INVAL;
    ctx->window = (int)value;
    return PC2_OK;
  }
  if (option == PC2_OPT_MODMUL) {
    if (value == PC2_MODMUL_VALU) {
      ctx->modmul = (int)value;
      return PC2_OK;
    }
    return PC2_E_UNSUPPORTED;
  }
  return PC2_E_INVAL;
}

int pc2_ctx_get_option(pc2_ctx* ctx, int option, int64_t* value) {
  if (!ctx || !value) return PC2_E_INVAL;
  if (option == PC2_OPT_WINDOW) *value = ctx->window;
  else if (option == PC2_OPT_MODMUL) *value = ctx->modmul;
  else return PC2_E_INVAL;
  return PC2_OK;
}

// ---------------------------------------------------------------- keys
int pc2_pk_create(pc2_ctx* ctx, uint32_t nbits, const uint32_t* n_limbs, pc2_pk** out) {
  if (!ctx || !n_limbs || !out) return PC2_E_INVAL;
  *out = nullptr;
  const int cls = pc2k::class_for_bits((int)nbits);
  if (nbits < 2 || cls < 0) return PC2_E_UNSUPPORTED;
  const int L = (int)((nbits + 31) / 32);
  Limbs n = limbs_from(n_limbs, L);
  const int nb = pc2h::bitlen(n);
  if (nb > (int)nbits || (n[0] & 1u) == 0 || pc2h::cmp(n, Limbs{15}) < 0) return PC2_E_INVAL;
  DevBuf buf;
  PkOffsets o = add_public(buf, n, cls, L);
  pc2_pk* pk = new (std::nothrow) pc2_pk();
  if (!pk) return PC2_E_NOMEM;
  int rc = upload(ctx, buf, &pk->dev);
  if (rc) {
    delete pk;
    return rc;
  }
  pk->ctx = ctx;
  pk->nbits = nbits;
  pk->L = L;
  pk->cls = cls;
  pk->c = pk_const((const uint32_t*)pk->dev, o, L, nb);
  *out = pk;
  return PC2_OK;
}

int pc2_sk_create(pc2_ctx* ctx, uint32_t nbits, const uint32_t* p_limbs, const uint32_t* q_limbs,
                  pc2_sk** out) {
  if (!ctx || !p_limbs || !q_limbs || !out) return PC2_E_INVAL;
  *out = nullptr;
  const int cls = pc2k::class_for_bits((int)nbits);
  if (nbits < 2 || cls < 0) return PC2_E_UNSUPPORTED;
  const int L = (int)((nbits + 31) / 32);
  Limbs p = limbs_from(p_limbs, L), q = limbs_from(q_limbs, L);
  if ((p[0] & 1u) == 0 || (q[0] & 1u) == 0 || pc2h::cmp(p, Limbs{3}) < 0 ||
      pc2h::cmp(q, Limbs{3}) < 0 || pc2h::cmp(p, q) == 0)
    return PC2_E_INVAL;
  if (pc2h::cmp(p, q) < 0) std::swap(p, q);  // p > q: m_q < q < p in the recombination
  Limbs n = pc2h::mul(p, q);
  pc2h::trim(n);
  const int nb = pc2h::bitlen(n);
  if (nb > (int)nbits) return PC2_E_INVAL;
  const pc2k::ClassGeo g = pc2k::CLASS_GEO[cls];
  Limbs p2 = pc2h::mul(p, p);
  // the s^2 moduli must satisfy 4 s^2 < R for their digit geometry
  if (pc2h::bitlen(p2) + 2 > g.pD * g.pK * g.pT) return PC2_E_UNSUPPORTED;
  const int Ls = (int)pc2h::resized(p, p.size()).size();
  const int nl2 = (pc2h::bitlen(p2) + 31) / 32;
  DevBuf buf;
  PkOffsets po = add_public(buf, n, cls, L);
  HalfOffsets hp = add_half(buf, p, q, n, cls, Ls, nl2);
  HalfOffsets hq = add_half(buf, q, p, n, cls, Ls, nl2);
  // q^-1 2^(32 Ls) mod p
  Limbs qinv = pc2h::inv_mod_prime(pc2h::mod(q, p), p);
  size_t qi = buf.add(pc2h::resized(pc2h::shl_mod(qinv, (uint64_t)32 * Ls, p), Ls));
  pc2_sk* sk = new (std::nothrow) pc2_sk();
  if (!sk) return PC2_E_NOMEM;
  int rc = upload(ctx, buf, &sk->dev);
  if (rc) {
    delete sk;
    return rc;
  }
  const uint32_t* base = (const uint32_t*)sk->dev;
  sk->ctx = ctx;
  sk->pk.ctx = ctx;
  sk->pk.nbits = nbits;
  sk->pk.L = L;
  sk->pk.cls = cls;
  sk->pk.dev = nullptr;
  sk->pk.c = pk_const(base, po, L, nb);
  sk->c.pk = sk->pk.c;
  sk->c.h[0] = half_const(base, hp);
  sk->c.h[1] = half_const(base, hq);
  sk->c.QI = base + qi;
  Limbs pm1 = pc2h::sub(p, Limbs{1}), qm1 = pc2h::sub(q, Limbs{1});
  sk->c.ebits = std::max(pc2h::bitlen(pm1), pc2h::bitlen(qm1));
  *out = sk;
  return PC2_OK;
}

const pc2_pk* pc2_sk_public(const pc2_sk* sk) { return sk ? &sk->pk : nullptr; }

int pc2_pk_destroy(pc2_pk* pk) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (!pk->dev) return PC2_E_INVAL;  // the public part of a private key
  (void)hipSetDevice(pk->ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(pk->dev);
  delete pk;
  return PC2_OK;
}

int pc2_sk_destroy(pc2_sk* sk) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(sk->ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(sk->dev);
  delete sk;
  return PC2_OK;
}

int pc2_pk_info(const pc2_pk* pk, uint32_t* nbits, uint32_t* limbs) {
  if (!pk) return PC2_E_INVAL;
  if (nbits) *nbits = pk->nbits;
  if (limbs) *limbs = (uint32_t)pk->L;
  return PC2_OK;
}

// ---------------------------------------------------------------- data
int pc2_quantize(pc2_ctx* ctx, const pc2_qparams* q, const double* x, uint64_t* m, size_t count,
                 void* stream) {
  if (!ctx || !q) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!x || !m) return PC2_E_INVAL;
  if (q->log2_scale < -1074 || q->log2_scale > 1023) return PC2_E_INVAL;
  pc2k::Launch l{};
  l.grid = (int)std::min<size_t>((count + 255) / 256, (size_t)ctx->cus * 8);
  l.err = ctx->err;
  l.stream = stream;
  return status_of(pc2k::launch_quantize(l, q->log2_scale, q->offset, x, m, count));
}

int pc2_dequantize(pc2_ctx* ctx, const pc2_qparams* q, const uint32_t* m, uint32_t m_limbs,
                   uint64_t weight, double* x, size_t count, void* stream) {
  if (!ctx || !q) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!x || !m || m_limbs < 1 || m_limbs > 4096) return PC2_E_INVAL;
  if (q->log2_scale < -1074 || q->log2_scale > 1023) return PC2_E_INVAL;
  pc2k::Launch l{};
  l.grid = (int)std::min<size_t>((count + 255) / 256, (size_t)ctx->cus * 8);
  l.err = ctx->err;
  l.stream = stream;
  return status_of(pc2k::launch_dequantize(l, q->log2_scale, q->offset, m, (int)m_limbs, weight,
                                           x, count));
}

int pc2_encrypt(const pc2_pk* pk, const uint32_t* m, uint32_t m_limbs, const uint32_t* r,
                uint32_t* c, size_t count, void* stream) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!m || !r || !c || m_limbs < 1 || (int)m_limbs > pk->L) return PC2_E_INVAL;
  pc2k::Launch l{};
  int rc = prepare(pk->ctx, pk->cls, pc2k::OP_ENC, count, 0, pk->L, &l, stream);
  if (rc) return rc;
  return status_of(pc2k::launch_encrypt(pk->cls, l, pk->c, m, (int)m_limbs, r, c, count));
}

int pc2_decrypt(const pc2_sk* sk, const uint32_t* c, uint32_t* m, size_t count, void* stream) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c || !m) return PC2_E_INVAL;
  pc2k::Launch l{};
  int rc = prepare(sk->ctx, sk->pk.cls, pc2k::OP_DEC, count, sk->c.h[0].Ls, sk->pk.L, &l, stream);
  if (rc) return rc;
  return status_of(pc2k::launch_decrypt(sk->pk.cls, l, sk->c, c, m, count));
}

int pc2_hom_sum(const pc2_pk* pk, const uint32_t* const* c_k, uint32_t K, uint32_t* out,
                size_t count, void* stream) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c_k || !out || K < 1 || K > (uint32_t)pc2k::RK_MAX) return PC2_E_INVAL;
  pc2k::PtrList lst{};
  for (uint32_t k = 0; k < K; ++k) {
    if (!c_k[k]) return PC2_E_INVAL;
    lst.p[k] = c_k[k];
  }
  pc2_ctx* ctx = pk->ctx;
  pc2k::Launch l{};
  const size_t epb = (size_t)pc2k::elems_per_block(pk->cls);
  const size_t groups = (count + epb - 1) / epb;
  l.grid = (int)std::max<size_t>(
      1, std::min(groups, (size_t)ctx->cus * occupancy(ctx, pk->cls, pc2k::OP_SUM)));
  l.err = ctx->err;
  l.stream = stream;
  return status_of(pc2k::launch_hom_sum(pk->cls, l, pk->c, lst, (int)K, out, count));
}

int pc2_hom_add(const pc2_pk* pk, const uint32_t* c1, const uint32_t* c2, uint32_t* out,
                size_t count, void* stream) {
  if (!pk) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c1 || !c2) return PC2_E_INVAL;
  const uint32_t* lst[2] = {c1, c2};
  return pc2_hom_sum(pk, lst, 2, out, count, stream);
}

int pc2_hom_scalar_mul(const pc2_pk* pk, const uint32_t* c, const uint64_t* k, uint32_t* out,
                       size_t count, void* stream) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c || !k || !out) return PC2_E_INVAL;
  pc2k::Launch l{};
  int rc = prepare(pk->ctx, pk->cls, pc2k::OP_SMUL, count, 0, pk->L, &l, stream);
  if (rc) return rc;
  return status_of(
      pc2k::launch_scalar_mul(pk->cls, l, pk->c, c, (const uint32_t*)k, out, count));
}

int pc2_enc_sum_dec(const pc2_sk* sk, const uint32_t* const* m_k, const uint32_t* const* r_k,
                    uint32_t K, uint32_t m_limbs, uint32_t* m_out, size_t count, void* stream) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!m_k || !r_k || !m_out || K < 1 || K > (uint32_t)pc2k::RK_MAX || m_limbs < 1 ||
      (int)m_limbs > sk->pk.L)
    return PC2_E_INVAL;
  pc2k::PtrList ms{}, rs{};
  for (uint32_t k = 0; k < K; ++k) {
    if (!m_k[k] || !r_k[k]) return PC2_E_INVAL;
    ms.p[k] = m_k[k];
    rs.p[k] = r_k[k];
  }
  pc2k::Launch l{};
  int rc = prepare(sk->ctx, sk->pk.cls, pc2k::OP_FUSED, count, sk->c.h[0].Ls, sk->pk.L, &l,
                   stream);
  if (rc) return rc;
  return status_of(
      pc2k::launch_fused(sk->pk.cls, l, sk->c, ms, rs, (int)K, (int)m_limbs, m_out, count));
}

}  // extern "C"
