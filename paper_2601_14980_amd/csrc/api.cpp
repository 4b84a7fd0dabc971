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
  uint32_t* scratch = nullptr; // per-tile tables and per-call staging
  size_t scratch_bytes = 0;    // sized by the key constructors and pc2_ctx_reserve
  hipEvent_t done = nullptr;   // recorded after the last call that used the scratch
  void* done_stream = nullptr; // ... on this stream
  bool done_valid = false;
  int window = 0;              // 0 = automatic
  int modmul = PC2_MODMUL_AUTO;
  int tile = 0;                // PC2_OPT_TILE: 0 automatic, 1 wide, else lanes per ciphertext
  int occ[pc2k::NUM_GEOS][pc2k::OP_COUNT] = {};    // workgroups per CU (0 = not queried)
  int tuned[pc2k::NUM_GEOS][pc2k::OP_COUNT] = {};  // autotuned windows (0 = none)
  int tuned_geo[pc2k::NUM_CLASSES] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};  // encryption tile
};

struct pc2_runner {
  pc2_ctx* ctx = nullptr;
  int op = 0, max_cls = 0;
  size_t max_jobs = 0, max_groups = 0, max_ptrs = 0;
  size_t slot_words = 0;
  int grid_cap = 0;
  int ls = 0;            // largest prime (limbs) the decryption staging holds
  void* dev = nullptr;   // jobs | items | pointers | queue
  void* host = nullptr;  // pinned staging, same layout
  size_t jobs_b = 0, items_b = 0, ptr_b = 0;
  uint32_t* scratch = nullptr;
  uint32_t* stage = nullptr;  // decryption: CRT halves of one launch's groups
  uint8_t* mscratch = nullptr;  // encryption on the matrix cores: tables of the widest grid
  size_t mscratch_bytes = 0;
  int mocc[pc2k::NUM_CLASSES] = {};  // resident workgroups per CU of k_batch_mfma per class
  hipEvent_t copied = nullptr;
  bool pending = false;
};

struct pc2_admm {
  pc2_ctx* ctx = nullptr;
  const double* A = nullptr;
  int N = 0, B = 0, K = 0;
  double rho = 1.0;
  double* buf = nullptr;  // W (K B B) | aty (K N) | w (K N) | t (K B) | s (K B)
  double *W = nullptr, *aty = nullptr, *w = nullptr, *t = nullptr, *s = nullptr;
};

struct pc2_batch {
  pc2_ctx* ctx = nullptr;
  int op = 0, pair = 0, grid = 0, nitems = 0;
  int w_a = 5, w_b = 5;
  size_t slot_words = 0;
  void* dev = nullptr;  // jobs, items, pointer/length arrays, queue
  pc2k::BatchJob* jobs = nullptr;
  pc2k::BatchItem* items = nullptr;
  int* queue = nullptr;
  uint32_t* scratch = nullptr;
  uint32_t* stage = nullptr;  // decryption: CRT halves of every job's elements
  // encryption jobs of up to two key classes that run on the matrix cores:
  // per class its own items (after the others), queue, grid and window; one
  // table scratch for both (the launches run in order on one stream)
  struct MPart {
    int cls = -1, grid = 0, nitems = 0, w = 6, sub = 1;  // sub: largest group of its jobs
    pc2k::BatchItem* items = nullptr;
    int* queue = nullptr;
  } mp[2];
  uint8_t* mscratch = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_stream = nullptr;
};

struct pc2_matvec {
  pc2_ctx* ctx = nullptr;
  const pc2_pk* pk = nullptr;
  int w = 0, nw = 0, ebits = 0;
  size_t cols = 0, table_bytes = 0;
  uint32_t* tab = nullptr;    // fixed-base tables [cols][nw][2^w - 1] entries
  uint32_t* parts = nullptr;  // partial products of row chunks [chunks][rows][2L]
  size_t parts_bytes = 0;
  int cap_table = 1, cap_apply = 1;  // resident workgroups of the two kernels
  bool loaded = false;
};

struct pc2_colsplit {
  pc2_ctx* ctx = nullptr;
  const pc2_sk* sk = nullptr;
  int M = 0, N = 0, K = 0, Nk = 0, k = 0;
  double rho = 1.0;
  const uint32_t* r_pool = nullptr;
  size_t r_count = 0, iter = 0;
  std::vector<pc2_matvec*> mv;  // one plan per node over Gamma_2(rho B_k)
  void* dev = nullptr;          // per-node constants, then per-iteration staging
  double *alpha = nullptr, *rhoB = nullptr;       // [K][Nk], [K][Nk][Nk]
  uint64_t *G = nullptr, *R = nullptr;            // [K][Nk][Nk], [K][Nk]
  uint32_t* ahat = nullptr;                       // [K][Nk][2L] Enc(Gamma_1(alpha_k))
  uint64_t *w = nullptr, *S = nullptr;            // [2][N] Gamma_2(z), Gamma_2(-v); [K]
  uint32_t *cw = nullptr, *c = nullptr, *xhat = nullptr, *P = nullptr;  // [2N][2L], [N][2L] x2, [N][L]
  uint32_t* g1 = nullptr;                         // [K][Nk][4] Gamma_1(alpha_k)
};

struct pc2_pk {
  pc2_ctx* ctx = nullptr;
  int device = 0;
  uint32_t nbits = 0;
  int L = 0;
  int cls = 0;
  void* dev = nullptr;  // one allocation holding every constant
  pc2k::PkConst c{};
  pc2k::PkConst alt{};  // n^2 constants in the alternative tile (ALT_GEO[cls] >= 0)
};

struct pc2_sk {
  pc2_ctx* ctx = nullptr;
  pc2_pk pk;            // the public part (owns nothing; dev below owns all)
  void* dev = nullptr;
  pc2k::SkConst c{};
  bool crt_ok = false;  // p < 2 q: the key-holder encryption's inputs fit mod q^2
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


// Left-to-right sliding-window schedule of e > 0 (see pc2k::Sched)
std::vector<uint32_t> sliding_schedule(const Limbs& e0, int w) {
  Limbs e = e0;
  pc2h::trim(e);
  auto bit = [&](int i) -> uint32_t { return (e[i / 32] >> (i % 32)) & 1u; };
  std::vector<uint32_t> out;
  int i = pc2h::bitlen(e) - 1;
  uint32_t sq = 0;
  bool first = true;
  while (i >= 0) {
    if (!bit(i)) {
      ++sq;
      --i;
      continue;
    }
    int j = std::max(i - w + 1, 0);
    while (!bit(j)) ++j;
    uint32_t d = 0;
    for (int k = i; k >= j; --k) d = (d << 1) | bit(k);
    if (!first) sq += (uint32_t)(i - j + 1);
    out.push_back((sq << 16) | d);
    first = false;
    sq = 0;
    i = j - 1;
  }
  if (sq) out.push_back(sq << 16);
  return out;
}

struct SchedOffsets {
  size_t off[pc2k::SCHED_WMAX - pc2k::SCHED_WMIN + 1];
  int n[pc2k::SCHED_WMAX - pc2k::SCHED_WMIN + 1];
};
SchedOffsets add_schedules(DevBuf& buf, const Limbs& e) {
  SchedOffsets o{};
  for (int w = pc2k::SCHED_WMIN; w <= pc2k::SCHED_WMAX; ++w) {
    std::vector<uint32_t> sc = sliding_schedule(e, w);
    o.off[w - pc2k::SCHED_WMIN] = buf.add(sc);
    o.n[w - pc2k::SCHED_WMIN] = (int)sc.size();
  }
  return o;
}
pc2k::Sched sched_const(const uint32_t* base, const SchedOffsets& o) {
  pc2k::Sched c{};
  for (int i = 0; i <= pc2k::SCHED_WMAX - pc2k::SCHED_WMIN; ++i) {
    c.p[i] = base + o.off[i];
    c.n[i] = o.n[i];
  }
  return c;
}

struct GeoOffsets {  // the n^2 constants that depend on the digit geometry
  ModOffsets n2;
  size_t nR, Rk;
};
struct PkOffsets {
  GeoOffsets g, alt;  // alt: only for classes with an alternative tile
  size_t n;
  size_t mN, mNp, mR2, mnR, mRk, mN28;  // matrix-core product constants
  int mS;
  SchedOffsets nsch;
};

// v -> D = 4 S forward 7-bit digits, one per byte after 64 zero bytes, with
// a zero tail to 64 + D8 + 16 bytes (D8 = D rounded up to 16)
std::vector<uint32_t> to_digits7(const Limbs& v, int S) {
  const int D = 4 * S, FB = 64 + ((D + 15) & ~15) + 16;
  std::vector<uint32_t> out(FB / 4, 0);
  for (int i = 0; i < D; ++i) {
    const long bit = (long)i * 7;
    const size_t w = bit / 32;
    const int sh = bit % 32;
    const uint64_t lo = w < v.size() ? v[w] : 0, hi = w + 1 < v.size() ? v[w + 1] : 0;
    const uint32_t d = (uint32_t)(((hi << 32) | lo) >> sh) & 0x7Fu;
    out[(64 + i) / 4] |= d << (8 * (i % 4));
  }
  return out;
}

// v -> S limbs of 28 bits
std::vector<uint32_t> to_limbs28(const Limbs& v, int S) {
  std::vector<uint32_t> out(S, 0);
  for (int i = 0; i < S; ++i) {
    const long bit = (long)i * 28;
    const size_t w = bit / 32;
    const int sh = bit % 32;
    const uint64_t lo = w < v.size() ? v[w] : 0, hi = w + 1 < v.size() ? v[w + 1] : 0;
    out[i] = (uint32_t)(((hi << 32) | lo) >> sh) & ((1u << 28) - 1u);
  }
  return out;
}

// n^2, n R and the powers R^k mod n^2 in the digit geometry `geo`
GeoOffsets add_geo(DevBuf& buf, const Limbs& n, const Limbs& n2, int geo, int L) {
  const pc2k::ClassGeo g = pc2k::CLASS_GEO[geo];
  GeoOffsets o{};
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
  return o;
}

PkOffsets add_public(DevBuf& buf, const Limbs& n, int cls, int L) {
  Limbs n2 = pc2h::mul(n, n);
  PkOffsets o{};
  o.g = add_geo(buf, n, n2, cls, L);
  if (pc2k::ALT_GEO[cls] >= 0) o.alt = add_geo(buf, n, n2, pc2k::ALT_GEO[cls], L);
  o.n = buf.add(pc2h::resized(n, L));
  // matrix-core form: R = 2^(28 S), N' = -N^-1 mod R
  const int S = pc2k::MFMA_S[cls];
  const uint64_t RBm = 28ull * S;
  Limbs N = n2;
  pc2h::trim(N);
  const size_t nw = (RBm + 31) / 32;
  Limbs inv = pc2h::inv_pow2(N, nw);
  Limbs Rm = pc2h::resized(Limbs{}, nw + 1);
  Rm[RBm / 32] |= 1u << (RBm % 32);  // 2^RBm (RBm < 32 nw + 32)
  Limbs invR = pc2h::resized(inv, nw);
  if (RBm % 32) invR[nw - 1] &= (1u << (RBm % 32)) - 1u;  // inv mod 2^RBm
  pc2h::trim(invR);
  Limbs np = pc2h::sub(Rm, invR);  // 2^RBm - inv (inv != 0 for odd N)
  pc2h::trim(np);
  o.mS = S;
  o.mN = buf.add(to_digits7(N, S));
  o.mNp = buf.add(to_digits7(np, S));
  o.mR2 = buf.add(to_digits7(pc2h::pow2_mod(2 * RBm, N), S));
  o.mnR = buf.add(to_digits7(pc2h::shl_mod(n, RBm, N), S));
  {  // R^k mod n^2, k = 0..RK_MAX (R = 2^RBm), by Montgomery products with 32-bit limbs
    pc2h::Mont32 M(N);
    const Limbs r1m = M.to(pc2h::pow2_mod(RBm, N));
    Limbs rkm = M.to(Limbs{1});
    std::vector<uint32_t> tab;
    for (int k = 0; k <= pc2k::RK_MAX; ++k) {
      const std::vector<uint32_t> d = to_digits7(M.from(rkm), S);
      tab.insert(tab.end(), d.begin(), d.end());
      rkm = M.mm(rkm, r1m);
    }
    o.mRk = buf.add(tab);
  }
  o.mN28 = buf.add(to_limbs28(N, S));
  o.nsch = add_schedules(buf, n);
  return o;
}

pc2k::PkConst pk_const(const uint32_t* base, const PkOffsets& o, int L, int nbits) {
  pc2k::PkConst c{};
  c.n2 = mod_const(base, o.g.n2);
  c.nR = base + o.g.nR;
  c.Rk = base + o.g.Rk;
  c.n = base + o.n;
  c.L = L;
  c.nbits = nbits;
  c.mf.N = (const uint8_t*)(base + o.mN);
  c.mf.Np = (const uint8_t*)(base + o.mNp);
  c.mf.R2 = (const uint8_t*)(base + o.mR2);
  c.mf.nR = (const uint8_t*)(base + o.mnR);
  c.mf.Rk = (const uint8_t*)(base + o.mRk);
  c.mf.N28 = base + o.mN28;
  c.mf.S = o.mS;
  c.nsch = sched_const(base, o.nsch);
  return c;
}

// the same key with the n^2 constants of the alternative tile
pc2k::PkConst pk_const_alt(const uint32_t* base, const PkOffsets& o, const pc2k::PkConst& c) {
  pc2k::PkConst a = c;
  a.n2 = mod_const(base, o.alt.n2);
  a.nR = base + o.alt.nR;
  a.Rk = base + o.alt.Rk;
  return a;
}

struct HalfOffsets {
  ModOffsets s2;
  size_t s, e, sinv, H;
  uint32_t s_n0;
  int Ls;
  SchedOffsets esch;
  size_t nRs;
  SchedOffsets nsch;
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
  o.esch = add_schedules(buf, pc2h::sub(s, Limbs{1}));
  // key-holder encryption mod s^2: n R mod s^2 and n mod s (s - 1)
  const uint64_t RBs = (uint64_t)g.pD * g.pK * g.pT;
  o.nRs = buf.add(to_chunk(pc2h::shl_mod(n, RBs, s2), g.pD, g.pK, g.pT));
  Limbs order = pc2h::mul(s, pc2h::sub(s, Limbs{1}));
  pc2h::trim(order);
  Limbs ne = pc2h::mod(n, order);
  pc2h::trim(ne);
  if (ne.empty()) ne = order;  // n = 0 mod s (s-1) cannot happen for n = p q, s | n
  o.nsch = add_schedules(buf, ne);
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
  h.esch = sched_const(base, o.esch);
  h.nRs = base + o.nRs;
  h.nsch = sched_const(base, o.nsch);
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

int auto_window(int geo, int op) {
  // window width minimising products for the exponent lengths of each class
  // (sliding windows for the wave-uniform exponents of encryption and
  // decryption)
  const int cls = pc2k::GEO_CLASS[geo];
  if (op == pc2k::OP_SMUL) return 4;
  return cls >= 6 ? 6 : (cls >= 5 ? 5 : (cls >= 3 ? 4 : 3));
}

int window_for(const pc2_ctx* ctx, int geo, int op) {
  if (ctx->window) return ctx->window;
  if (op == pc2k::OP_FUSED_MFMA) op = pc2k::OP_ENC_MFMA;
  const int t = ctx->tuned[geo][op == pc2k::OP_FUSED ? pc2k::OP_ENC : op];
  // (matrix-core engine, 2048-bit keys: w = 6 measured 1 % faster than 5)
  if (op == pc2k::OP_ENC_MFMA) return t ? t : (geo >= 6 ? 6 : (geo >= 5 ? 5 : 4));
  return t ? t : auto_window(geo, op);
}

// The Montgomery engine of an encryption (pc2_encrypt, pc2_enc_sum_dec)
// under a key of class cls: the matrix cores when asked for, or
// automatically from 2048-bit keys (class 6) on, where they measured faster
// than the VALU engine on the MI355X.
constexpr int MFMA_AUTO_CLASS = 6;
bool use_mfma(const pc2_ctx* ctx, int cls) {
  return ctx->modmul == PC2_MODMUL_MFMA ||
         (ctx->modmul == PC2_MODMUL_AUTO && cls >= MFMA_AUTO_CLASS);
}

// Geometry of an encryption of `count` elements under the key class cls:
// the alternative tile if PC2_OPT_TILE asks for wide tiles or names its lane
// count, the class's own tile for any other lane count.  Automatic: a launch
// that gives every SIMD at most one wavefront of the (wider) alternative tile
// is latency-bound, and the wider tile finishes it sooner, so it takes that;
// a larger one takes the autotuned tile, else the class's own.  Batches and
// runners pass no count (their geometry is fixed per key when groups are cut).
int enc_geo(const pc2_ctx* ctx, int cls, size_t count = SIZE_MAX) {
  const int alt = pc2k::ALT_GEO[cls];
  if (alt < 0) return cls;
  if (ctx->tile == PC2_TILE_WIDE) return alt;
  if (ctx->tile) return pc2k::CLASS_GEO[alt].nT == ctx->tile ? alt : cls;
  if (count <= (size_t)ctx->cus * 4 * (size_t)pc2k::elems_per_block(alt)) return alt;
  return ctx->tuned_geo[cls] >= 0 ? ctx->tuned_geo[cls] : cls;
}
// the key's constants in geometry geo (its own class or its alternative tile)
const pc2k::PkConst& geo_const(const pc2_pk* pk, int geo) {
  return geo == pk->cls ? pk->c : pk->alt;
}
// the geometry a batched or queued job of operation op runs in
int job_geo(const pc2_ctx* ctx, const pc2_pk* pk, int op) {
  return op == pc2k::OP_ENC ? enc_geo(ctx, pk->cls) : pk->cls;
}

int occupancy(pc2_ctx* ctx, int geo, int op) {
  int& o = ctx->occ[geo][op];
  if (o == 0) {
    int v = 0;
    const void* k = op == pc2k::OP_ENC_MFMA     ? pc2k::kernel_encrypt_mfma(geo)
                    : op == pc2k::OP_FUSED_MFMA ? pc2k::kernel_encrypt_mfma(geo, true)
                                                : pc2k::kernel_for(geo, op);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k, 64, 0) != hipSuccess ||
        v <= 0)
      v = 1;
    o = v;
  }
  return o;
}

// Grid and table slot of a Paillier launch over `count` elements in geometry
// geo (the key class, except for an encryption in an alternative tile) with
// window w; returns the bytes of scratch the launch needs.  The scratch holds
// aux_words of per-call staging first (Launch::aux, at the same place for
// every launch that asks for the same amount), then the tables.
size_t plan_launch(pc2_ctx* ctx, int geo, int op, size_t count, int Ls, int L, int w,
                   pc2k::Launch* l, void* stream, size_t aux_words) {
  const bool mf = op == pc2k::OP_ENC_MFMA || op == pc2k::OP_FUSED_MFMA;
  const size_t epb = mf ? 1 : (size_t)pc2k::elems_per_block(geo);
  const size_t groups = (count + epb - 1) / epb;
  const size_t cap = (size_t)ctx->cus * occupancy(ctx, geo, op);
  l->grid = (int)std::max<size_t>(1, std::min(groups, cap));
  l->window = w;
  l->err = ctx->err;
  l->stream = stream;
  int tiles = 0;
  size_t words = 0;
  if (mf) {  // one table of 2^w digit arrays per workgroup
    tiles = 1;
    words = (pc2k::mfma_digit_bytes(geo) << w) / 4;
  } else {
    pc2k::slot_shape(geo, op, w, Ls, L, &tiles, &words);
  }
  words = (words + 3) & ~(size_t)3;
  l->slot_words = words;
  const size_t aux = (aux_words + 63) & ~(size_t)63;
  return (aux + (size_t)l->grid * tiles * words) * 4;
}

// A data call's launch in the context's scratch.  Data calls never allocate:
// the key constructors sized the scratch for every call of their key class
// (class_scratch_need), so a launch that does not fit is PC2_E_NOMEM.
int prepare(pc2_ctx* ctx, int geo, int op, size_t count, int Ls, int L, pc2k::Launch* l,
            void* stream, size_t aux_words = 0) {
  const size_t need = plan_launch(ctx, geo, op, count, Ls, L, window_for(ctx, geo, op), l,
                                  stream, aux_words);
  if (need > ctx->scratch_bytes || !ctx->scratch) return PC2_E_NOMEM;
  const size_t aux = (aux_words + 63) & ~(size_t)63;
  l->aux = aux_words ? ctx->scratch : nullptr;
  l->scratch = ctx->scratch + aux;
  return PC2_OK;
}

// Largest scratch any data call under a key of class cls can need: every
// operation and encryption tile, the widest window an option can select,
// a device-filling grid and the largest per-call staging (DEC_CHUNK
// elements).  L: limbs of n; Ls, nl2: limbs of the larger prime and of its
// square.  Also caches every occupancy the calls will look up, so that no
// data call queries the runtime for it (e.g. under graph capture).
size_t class_scratch_need(pc2_ctx* ctx, int cls, int L, int Ls, int nl2) {
  const size_t big = (size_t)1 << 40;  // enough elements to fill the device
  const size_t ch = pc2k::DEC_CHUNK;
  const int w = pc2k::SCHED_WMAX;
  pc2k::Launch l{};
  size_t need = 0;
  auto take = [&](int geo, int op, size_t aux) {
    need = std::max(need, plan_launch(ctx, geo, op, big, Ls, L, w, &l, nullptr, aux));
  };
  take(cls, pc2k::OP_ENC, 0);
  if (pc2k::ALT_GEO[cls] >= 0) take(pc2k::ALT_GEO[cls], pc2k::OP_ENC, 0);
  take(cls, pc2k::OP_SMUL, 0);
  take(cls, pc2k::OP_ENC_MFMA, 0);
  take(cls, pc2k::OP_DEC, ch * 2 * (size_t)(Ls + 1));
  const size_t acc_words =
      std::max(pc2k::chunk_words(cls), pc2k::mfma_digit_bytes(cls) / 4);  // either engine
  const size_t fused_aux =
      ch * 2 * (size_t)L + ch * 2 * (size_t)(Ls + 1) + 128 + ch * (acc_words + 1);
  take(cls, pc2k::OP_DEC, fused_aux);
  take(cls, pc2k::OP_FUSED, fused_aux);
  take(cls, pc2k::OP_FUSED_MFMA, fused_aux);
  take(cls, pc2k::OP_ENC_CRT, ch * 2 * (size_t)(nl2 + 1));
  (void)occupancy(ctx, cls, pc2k::OP_SUM);
  return need;
}

// Grow the context's scratch to `need` bytes.  Only the key constructors and
// pc2_ctx_reserve call this (never a data call): it waits for the device,
// since work in flight may still use the old buffer.
int grow_scratch(pc2_ctx* ctx, size_t need) {
  if (need <= ctx->scratch_bytes && ctx->scratch) return PC2_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return PC2_E_DEVICE;
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  ctx->done_valid = false;
  if (hipMalloc(&ctx->scratch, need) != hipSuccess) return PC2_E_NOMEM;
  ctx->scratch_bytes = need;
  return PC2_OK;
}

// Bounds on a private key's prime sizes in class cls: a prime s must satisfy
// 4 s^2 < R of the class's s^2 digit geometry.
void class_prime_limbs(int cls, int* Ls, int* nl2) {
  const pc2k::ClassGeo g = pc2k::CLASS_GEO[cls];
  const int p2bits = g.pD * g.pK * g.pT - 2;
  *nl2 = (p2bits + 31) / 32;
  *Ls = (p2bits / 2 + 31) / 32;
}

bool capturing(void* stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing((hipStream_t)stream, &st) == hipSuccess &&
         st != hipStreamCaptureStatusNone;
}

// Calls that use the context's scratch run one after another whatever their
// streams: a call on a stream other than the previous call's first makes its
// stream wait for that call's completion event (on the device; the host does
// not block), and records the event after its own launches.  Under graph
// capture neither happens: the caller orders a graph's replays against other
// calls on the context.
int scratch_begin(pc2_ctx* ctx, void* stream) {
  if (!ctx->done_valid || ctx->done_stream == stream || capturing(stream)) return PC2_OK;
  return hipStreamWaitEvent((hipStream_t)stream, ctx->done, 0) == hipSuccess ? PC2_OK
                                                                            : PC2_E_DEVICE;
}
int scratch_end(pc2_ctx* ctx, void* stream, int rc) {
  if (rc || capturing(stream)) return rc;
  if (hipEventRecord(ctx->done, (hipStream_t)stream) != hipSuccess) return PC2_E_DEVICE;
  ctx->done_stream = stream;
  ctx->done_valid = true;
  return PC2_OK;
}

int status_of(hipError_t e) { return e == hipSuccess ? PC2_OK : PC2_E_DEVICE; }



// Two device arrays [a, a + na) and [b, b + nb) overlap without being the
// same array of the same size (the only aliasing the data calls accept).
bool partial_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  if (x + na <= y || y + nb <= x) return false;
  return !(x == y && na == nb);
}

// A job's output against its inputs under the same rule (L: limbs of n).
bool job_overlaps(const pc2_job& j, int L) {
  const size_t n = j.count;
  if (j.op == PC2_OP_ENCRYPT) {
    const size_t cb = 8 * (size_t)L * n;
    return partial_overlap(j.out, cb, j.in0, 4 * (size_t)j.m_limbs * n) ||
           partial_overlap(j.out, cb, j.in1, 4 * (size_t)L * n);
  }
  if (j.op == PC2_OP_DECRYPT) return partial_overlap(j.out, 4 * (size_t)L * n, j.in0, 8 * (size_t)L * n);
  for (uint32_t k = 0; k < j.K; ++k) {  // input k holds lengths[k] rows (ragged) or count
    const size_t rows = j.lengths ? j.lengths[k] : n;
    if (partial_overlap(j.out, 8 * (size_t)L * n, j.inputs[k], 8 * (size_t)L * rows)) return true;
  }
  return false;
}
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
  // the device address of the allocation-free calls' static scratch
  if (pc2k::static_scratch_setup(hip_device) != 0) return PC2_E_DEVICE;
  pc2_ctx* c = new (std::nothrow) pc2_ctx();
  if (!c) return PC2_E_NOMEM;
  c->device = hip_device;
  c->cus = prop.multiProcessorCount;
  if (hipMalloc(&c->err, sizeof(int)) != hipSuccess) {
    delete c;
    return PC2_E_NOMEM;
  }
  if (hipMemset(c->err, 0, sizeof(int)) != hipSuccess ||
      hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
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
  if (ctx->done) (void)hipEventDestroy(ctx->done);
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
  if (max_nbits < 2 || cls < 0) return PC2_E_UNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  int Ls = 0, nl2 = 0;
  class_prime_limbs(cls, &Ls, &nl2);
  return grow_scratch(ctx, class_scratch_need(ctx, cls, (int)((max_nbits + 31) / 32), Ls, nl2));
}

int pc2_ctx_set_option(pc2_ctx* ctx, int option, int64_t value) {
  if (!ctx) return PC2_E_INVAL;
  if (option == PC2_OPT_WINDOW) {
    if (value != 0 && (value < 2 || value > 6)) return PC2_E_INVAL;
    ctx->window = (int)value;
    return PC2_OK;
  }
  if (option == PC2_OPT_MODMUL) {
    if (value == PC2_MODMUL_VALU || value == PC2_MODMUL_MFMA || value == PC2_MODMUL_AUTO) {
      ctx->modmul = (int)value;
      return PC2_OK;
    }
    return PC2_E_UNSUPPORTED;
  }
  if (option == PC2_OPT_TILE) {
    if (value != 0 && value != PC2_TILE_WIDE && value != 2 && value != 4 && value != 8)
      return PC2_E_INVAL;
    ctx->tile = (int)value;
    return PC2_OK;
  }
  return PC2_E_INVAL;
}

int pc2_ctx_get_option(pc2_ctx* ctx, int option, int64_t* value) {
  if (!ctx || !value) return PC2_E_INVAL;
  if (option == PC2_OPT_WINDOW) *value = ctx->window;
  else if (option == PC2_OPT_MODMUL) *value = ctx->modmul;
  else if (option == PC2_OPT_TILE) *value = ctx->tile;
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
  pk->device = ctx->device;
  pk->nbits = nbits;
  pk->L = L;
  pk->cls = cls;
  pk->c = pk_const((const uint32_t*)pk->dev, o, L, nb);
  if (pc2k::ALT_GEO[cls] >= 0) pk->alt = pk_const_alt((const uint32_t*)pk->dev, o, pk->c);
  rc = pc2_ctx_reserve(ctx, nbits);  // every later data call under this key fits
  if (rc) {
    (void)hipFree(pk->dev);
    delete pk;
    return rc;
  }
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
  if (Ls > pc2k::LS_MAX) return PC2_E_UNSUPPORTED;
  const int nl2 = (pc2h::bitlen(p2) + 31) / 32;
  DevBuf buf;
  PkOffsets po = add_public(buf, n, cls, L);
  HalfOffsets hp = add_half(buf, p, q, n, cls, Ls, nl2);
  HalfOffsets hq = add_half(buf, q, p, n, cls, Ls, nl2);
  // q^-1 2^(32 Ls) mod p
  Limbs qinv = pc2h::inv_mod_prime(pc2h::mod(q, p), p);
  size_t qi = buf.add(pc2h::resized(pc2h::shl_mod(qinv, (uint64_t)32 * Ls, p), Ls));
  // (q^2)^-1 2^(32 nl2) mod p^2: q^-2 mod p^2 by Euler (phi(p^2) = p (p - 1))
  Limbs q2 = pc2h::mul(q, q);
  pc2h::trim(q2);
  pc2h::Mont32 MP2(p2);
  Limbs phi = pc2h::mul(p, pc2h::sub(p, Limbs{1}));
  pc2h::trim(phi);
  Limbs q2inv = MP2.pow(pc2h::mod(q2, p2), pc2h::sub(phi, Limbs{1}));
  size_t q2i = buf.add(pc2h::resized(pc2h::shl_mod(q2inv, (uint64_t)32 * nl2, p2), nl2));
  // the key-holder encryption needs r, m < n < 2 q^2, i.e. p < 2 q
  const bool crt_ok = pc2h::cmp(p, pc2h::add(q, q)) < 0;
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
  sk->pk.device = ctx->device;
  sk->pk.nbits = nbits;
  sk->pk.L = L;
  sk->pk.cls = cls;
  sk->pk.dev = nullptr;
  sk->pk.c = pk_const(base, po, L, nb);
  if (pc2k::ALT_GEO[cls] >= 0) sk->pk.alt = pk_const_alt(base, po, sk->pk.c);
  sk->c.pk = sk->pk.c;
  sk->c.h[0] = half_const(base, hp);
  sk->c.h[1] = half_const(base, hq);
  sk->c.QI = base + qi;
  sk->c.Q2I = base + q2i;
  sk->c.p2_n0 = 0u - pc2h::inv32(p2[0]);
  sk->crt_ok = crt_ok;
  Limbs pm1 = pc2h::sub(p, Limbs{1}), qm1 = pc2h::sub(q, Limbs{1});
  sk->c.ebits = std::max(pc2h::bitlen(pm1), pc2h::bitlen(qm1));
  rc = pc2_ctx_reserve(ctx, nbits);  // every later data call under this key fits
  if (rc) {
    (void)hipFree(sk->dev);
    delete sk;
    return rc;
  }
  *out = sk;
  return PC2_OK;
}

const pc2_pk* pc2_sk_public(const pc2_sk* sk) { return sk ? &sk->pk : nullptr; }

int pc2_pk_destroy(pc2_pk* pk) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (!pk->dev) return PC2_E_INVAL;  // the public part of a private key
  (void)hipSetDevice(pk->device);  // the context may already be gone
  (void)hipDeviceSynchronize();
  (void)hipFree(pk->dev);
  delete pk;
  return PC2_OK;
}

int pc2_sk_destroy(pc2_sk* sk) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(sk->pk.device);  // the context may already be gone
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

int pc2_pk_context(const pc2_pk* pk, pc2_ctx** ctx, int* hip_device) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (ctx) *ctx = pk->ctx;
  if (hip_device) *hip_device = pk->ctx->device;
  return PC2_OK;
}

// ---------------------------------------------------------------- data
int pc2_quantize(pc2_ctx* ctx, const pc2_qparams* q, const double* x, uint64_t* m, size_t count,
                 void* stream) {
  if (!ctx || !q) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!x || !m) return PC2_E_INVAL;
  if (partial_overlap(x, 8 * count, m, 8 * count)) return PC2_E_INVAL;
  if (q->log2_scale < -1074 || q->log2_scale > 1023 || q->offset > q->delta) return PC2_E_INVAL;
  pc2k::Launch l{};
  l.grid = (int)std::min<size_t>((count + 255) / 256, (size_t)ctx->cus * 8);
  l.err = ctx->err;
  l.stream = stream;
  return status_of(pc2k::launch_quantize(l, q->log2_scale, q->offset, q->delta, x, m, count));
}

int pc2_dequantize(pc2_ctx* ctx, const pc2_qparams* q, const uint32_t* m, uint32_t m_limbs,
                   uint64_t weight, double* x, size_t count, void* stream) {
  if (!ctx || !q) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!x || !m || m_limbs < 1 || m_limbs > 4096) return PC2_E_INVAL;
  if (partial_overlap(m, 4 * (size_t)m_limbs * count, x, 8 * count)) return PC2_E_INVAL;
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
  const size_t cb = 8 * (size_t)pk->L * count;
  if (partial_overlap(c, cb, m, 4 * (size_t)m_limbs * count) ||
      partial_overlap(c, cb, r, 4 * (size_t)pk->L * count))
    return PC2_E_INVAL;
  pc2_ctx* ctx = pk->ctx;
  pc2k::Launch l{};
  if (use_mfma(ctx, pk->cls)) {
    int rc = prepare(ctx, pk->cls, pc2k::OP_ENC_MFMA, count, 0, pk->L, &l, stream);
    if (!rc) rc = scratch_begin(ctx, stream);
    if (rc) return rc;
    return scratch_end(ctx, stream, status_of(pc2k::launch_encrypt_mfma(
                                        pk->cls, l, pk->c, m, (int)m_limbs, r, c, count)));
  }
  const int geo = enc_geo(ctx, pk->cls, count);
  int rc = prepare(ctx, geo, pc2k::OP_ENC, count, 0, pk->L, &l, stream);
  if (!rc) rc = scratch_begin(ctx, stream);
  if (rc) return rc;
  return scratch_end(ctx, stream, status_of(pc2k::launch_encrypt(
                                      geo, l, geo_const(pk, geo), m, (int)m_limbs, r, c, count)));
}

int pc2_decrypt(const pc2_sk* sk, const uint32_t* c, uint32_t* m, size_t count, void* stream) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c || !m) return PC2_E_INVAL;
  if (partial_overlap(c, 8 * (size_t)sk->pk.L * count, m, 4 * (size_t)sk->pk.L * count))
    return PC2_E_INVAL;
  // the two CRT halves of up to DEC_CHUNK elements are staged between the
  // per-prime phase and the recombination
  const int Ls = sk->c.h[0].Ls;
  const size_t chunk = std::min(count, pc2k::DEC_CHUNK);
  pc2k::Launch l{};
  int rc = prepare(sk->ctx, sk->pk.cls, pc2k::OP_DEC, chunk, Ls, sk->pk.L, &l, stream,
                   chunk * 2 * (size_t)(Ls + 1));
  if (!rc) rc = scratch_begin(sk->ctx, stream);
  if (rc) return rc;
  const size_t L2 = 2 * (size_t)sk->pk.L;
  for (size_t b = 0; b < count && !rc; b += chunk) {
    const size_t n = std::min(chunk, count - b);
    rc = status_of(pc2k::launch_decrypt(sk->pk.cls, l, sk->c, c + b * L2, m + b * sk->pk.L, n,
                                        l.aux));
  }
  return scratch_end(sk->ctx, stream, rc);
}

// pc2_decrypt with its staging and tables in the static device scratch
// (static_scratch.hip) instead of the context's: nothing is allocated and no
// event is waited for or recorded.
int pc2_decrypt_static(const pc2_sk* sk, const uint32_t* c, uint32_t* m, size_t count,
                       void* stream) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c || !m) return PC2_E_INVAL;
  if (partial_overlap(c, 8 * (size_t)sk->pk.L * count, m, 4 * (size_t)sk->pk.L * count))
    return PC2_E_INVAL;
  uint32_t* base = pc2k::static_scratch(sk->pk.device);
  if (!base) return PC2_E_DEVICE;
  pc2_ctx* ctx = sk->ctx;
  const int Ls = sk->c.h[0].Ls, L = sk->pk.L, cls = sk->pk.cls;
  const size_t total = PC2_STATIC_SCRATCH_BYTES / 4;
  // staging of one chunk's CRT halves: at most an eighth of the array
  const size_t per = 2 * (size_t)(Ls + 1);
  const size_t chunk = std::min({count, pc2k::DEC_CHUNK, total / 8 / per});
  if (chunk == 0) return PC2_E_NOMEM;
  const size_t aux = (chunk * per + 63) & ~(size_t)63;
  const size_t tab_words = total - aux;
  // the widest window up to pc2_decrypt's whose device-filling grid fits;
  // else the narrowest window on as many workgroups as fit
  pc2k::Launch l{};
  int w = window_for(ctx, cls, pc2k::OP_DEC);
  size_t need = 0;
  for (;; --w) {
    need = plan_launch(ctx, cls, pc2k::OP_DEC, chunk, Ls, L, w, &l, stream, 0) / 4;
    if (need <= tab_words || w == pc2k::SCHED_WMIN) break;
  }
  if (need > tab_words) {
    const size_t per_wg = need / (size_t)l.grid;  // tiles x slot words of one workgroup
    const size_t grid = tab_words / per_wg;
    if (grid == 0) return PC2_E_NOMEM;
    l.grid = (int)grid;
  }
  l.aux = base;
  l.scratch = base + aux;
  const size_t L2 = 2 * (size_t)L;
  int rc = PC2_OK;
  for (size_t b = 0; b < count && !rc; b += chunk) {
    const size_t n = std::min(chunk, count - b);
    rc = status_of(pc2k::launch_decrypt(cls, l, sk->c, c + b * L2, m + b * L, n, l.aux));
  }
  return rc;
}

int pc2_encrypt_sk(const pc2_sk* sk, const uint32_t* m, uint32_t m_limbs, const uint32_t* r,
                   uint32_t* c, size_t count, void* stream) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!m || !r || !c || m_limbs < 1 || (int)m_limbs > sk->pk.L) return PC2_E_INVAL;
  {
    const size_t cb = 8 * (size_t)sk->pk.L * count;
    if (partial_overlap(c, cb, m, 4 * (size_t)m_limbs * count) ||
        partial_overlap(c, cb, r, 4 * (size_t)sk->pk.L * count))
      return PC2_E_INVAL;
  }
  if (!sk->crt_ok) return PC2_E_UNSUPPORTED;
  // the two halves of up to DEC_CHUNK elements are staged before the recombination
  const int nl2 = sk->c.h[0].s2.nl, L = sk->pk.L, cls = sk->pk.cls;
  const size_t chunk = std::min(count, pc2k::DEC_CHUNK);
  pc2k::Launch l{};
  int rc = prepare(sk->ctx, cls, pc2k::OP_ENC_CRT, chunk, sk->c.h[0].Ls, L, &l, stream,
                   chunk * 2 * (size_t)(nl2 + 1));
  if (!rc) rc = scratch_begin(sk->ctx, stream);
  if (rc) return rc;
  for (size_t b = 0; b < count && !rc; b += chunk) {
    const size_t n = std::min(chunk, count - b);
    rc = status_of(pc2k::launch_encrypt_crt(cls, l, sk->c, m + b * m_limbs, (int)m_limbs,
                                            r + b * (size_t)L, c + b * 2 * (size_t)L, n, l.aux));
  }
  return scratch_end(sk->ctx, stream, rc);
}

int pc2_hom_sum(const pc2_pk* pk, const uint32_t* const* c_k, uint32_t K, uint32_t* out,
                size_t count, void* stream) {
  if (!pk || !pk->ctx) return PC2_E_INVAL;
  if (count == 0) return PC2_OK;
  if (!c_k || !out || K < 1 || K > (uint32_t)pc2k::RK_MAX) return PC2_E_INVAL;
  pc2k::PtrList lst{};
  const size_t cb = 8 * (size_t)pk->L * count;
  for (uint32_t k = 0; k < K; ++k) {
    if (!c_k[k] || partial_overlap(out, cb, c_k[k], cb)) return PC2_E_INVAL;
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
  {
    const size_t cb = 8 * (size_t)pk->L * count;
    if (partial_overlap(out, cb, c, cb) || partial_overlap(out, cb, k, 8 * count))
      return PC2_E_INVAL;
  }
  pc2k::Launch l{};
  int rc = prepare(pk->ctx, pk->cls, pc2k::OP_SMUL, count, 0, pk->L, &l, stream);
  if (!rc) rc = scratch_begin(pk->ctx, stream);
  if (rc) return rc;
  return scratch_end(pk->ctx, stream, status_of(pc2k::launch_scalar_mul(
                                          pk->cls, l, pk->c, c, (const uint32_t*)k, out, count)));
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
    if (partial_overlap(m_out, 4 * (size_t)sk->pk.L * count, m_k[k],
                        4 * (size_t)m_limbs * count) ||
        partial_overlap(m_out, 4 * (size_t)sk->pk.L * count, r_k[k],
                        4 * (size_t)sk->pk.L * count))
      return PC2_E_INVAL;
    ms.p[k] = m_k[k];
    rs.p[k] = r_k[k];
  }
  // per chunk: the products (2L limbs per element), the CRT halves, the
  // running products (chunked, 16-byte aligned) and the input checks
  pc2_ctx* ctx = sk->ctx;
  const int Ls = sk->c.h[0].Ls, L = sk->pk.L, cls = sk->pk.cls;
  const bool mf = use_mfma(ctx, cls);
  const size_t chunk = std::min(count, pc2k::DEC_CHUNK);
  const size_t prod_words = (chunk * 2 * (size_t)L + 63) & ~(size_t)63;
  const size_t half_words = (chunk * 2 * (size_t)(Ls + 1) + 63) & ~(size_t)63;
  const size_t acc_words =
      chunk * (mf ? pc2k::mfma_digit_bytes(cls) / 4 : pc2k::chunk_words(cls));
  const size_t aux = prod_words + half_words + acc_words + chunk;
  pc2k::Launch le{}, ld{};
  int rc = prepare(ctx, cls, pc2k::OP_DEC, chunk, Ls, L, &ld, stream, aux);
  if (!rc)
    rc = prepare(ctx, cls, mf ? pc2k::OP_FUSED_MFMA : pc2k::OP_FUSED, chunk, Ls, L, &le, stream,
                 aux);
  if (!rc) rc = scratch_begin(ctx, stream);
  if (rc) return rc;
  uint32_t* prod = le.aux;
  uint32_t* halves = le.aux + prod_words;
  uint32_t* acc = halves + half_words;
  uint32_t* okw = acc + acc_words;
  for (size_t b = 0; b < count && !rc; b += chunk) {
    const size_t n = std::min(chunk, count - b);
    pc2k::PtrList mb{}, rb{};
    for (uint32_t k = 0; k < K; ++k) {
      mb.p[k] = ms.p[k] + b * m_limbs;
      rb.p[k] = rs.p[k] + b * (size_t)L;
    }
    rc = status_of(mf ? pc2k::launch_enc_prod_mfma(cls, le, sk->pk.c, mb, rb, (int)K,
                                                   (int)m_limbs, prod, n,
                                                   reinterpret_cast<uint8_t*>(acc), okw)
                      : pc2k::launch_enc_prod(cls, le, sk->pk.c, mb, rb, (int)K, (int)m_limbs,
                                              prod, n, acc, okw));
    if (!rc)
      rc = status_of(pc2k::launch_decrypt(cls, ld, sk->c, prod, m_out + b * L, n, halves));
  }
  return scratch_end(ctx, stream, rc);
}

// ---------------------------------------------------------------- batches
// Work-queue counters at the end of a batch's or runner's descriptor
// allocation: the VALU launch's, then one per matrix-core class, each on
// its own 128-byte line.
constexpr int QUEUE_STRIDE = 32;                 // ints between two counters
constexpr size_t QUEUE_BYTES = 3 * QUEUE_STRIDE * sizeof(int);
// resident workgroups per CU of a 64-lane kernel (1 if the runtime cannot tell)
int occupancy_of(const void* k) {
  int occ = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 64, 0) != hipSuccess ||
      occ <= 0)
    occ = 1;
  return occ;
}

int pc2_batch_create(pc2_ctx* ctx, const pc2_job* jobs, size_t njobs, pc2_batch** out) {
  if (!ctx || !jobs || !out || njobs == 0) return PC2_E_INVAL;
  *out = nullptr;
  const int op_abi = jobs[0].op;
  int op;
  if (op_abi == PC2_OP_ENCRYPT) op = pc2k::OP_ENC;
  else if (op_abi == PC2_OP_DECRYPT) op = pc2k::OP_DEC;
  else if (op_abi == PC2_OP_HOM_SUM) op = pc2k::OP_SUM;
  else return PC2_E_INVAL;
  // validate and collect classes: the VALU kernel's pair, and the (up to
  // two) classes whose encryptions run on the matrix cores (use_mfma)
  int ca = -1, cb = -1, mca = -1, mcb = -1, Ls = 0;
  for (size_t i = 0; i < njobs; ++i) {
    const pc2_job& j = jobs[i];
    if (j.op != op_abi) return PC2_E_INVAL;
    if (j.count == 0) continue;
    const pc2_pk* pk = (op == pc2k::OP_DEC) ? (j.sk ? &j.sk->pk : nullptr) : j.pk;
    if (!pk || pk->ctx != ctx || !j.out) return PC2_E_INVAL;
    if (op == pc2k::OP_ENC &&
        (!j.in0 || !j.in1 || j.m_limbs < 1 || (int)j.m_limbs > pk->L))
      return PC2_E_INVAL;
    if (op == pc2k::OP_DEC && !j.in0) return PC2_E_INVAL;
    if (op == pc2k::OP_SUM) {
      if (!j.inputs || j.K < 1 || j.K > (uint32_t)pc2k::RK_MAX) return PC2_E_INVAL;
      for (uint32_t k = 0; k < j.K; ++k)
        if (!j.inputs[k] || (j.lengths && j.lengths[k] > j.count)) return PC2_E_INVAL;
    }
    if (job_overlaps(j, pk->L)) return PC2_E_INVAL;
    if (op == pc2k::OP_DEC) Ls = std::max(Ls, j.sk->c.h[0].Ls);
    if (op == pc2k::OP_ENC && use_mfma(ctx, pk->cls)) {
      if (mca < 0 || mca == pk->cls) mca = pk->cls;
      else if (mcb < 0 || mcb == pk->cls) mcb = pk->cls;
      else return PC2_E_UNSUPPORTED;
      continue;
    }
    const int g = job_geo(ctx, pk, op);
    if (ca < 0 || ca == g) ca = g;
    else if (cb < 0 || cb == g) cb = g;
    else return PC2_E_UNSUPPORTED;
  }
  if (ca < 0 && mca < 0) return PC2_E_INVAL;  // every job empty
  if (mca >= 0 && mcb > mca) std::swap(mca, mcb);  // the more expensive class first
  int pair = -1, pa = -1, pb = -1;
  if (ca >= 0) {
    if (cb < 0) cb = ca;
    pair = pc2k::batch_pair(ca, cb);
    if (pair < 0) return PC2_E_UNSUPPORTED;
    pa = pc2k::batch_pair_geo(pair, 0);
    pb = pc2k::batch_pair_geo(pair, 1);
  }
  pc2_batch* b = new (std::nothrow) pc2_batch();
  if (!b) return PC2_E_NOMEM;
  b->ctx = ctx;
  b->op = op;
  b->pair = pair;
  if (pair >= 0) {
    b->w_a = window_for(ctx, pa, op);
    b->w_b = window_for(ctx, pb, op);
  }
  b->mp[0].cls = mca;
  b->mp[1].cls = mcb;
  for (auto& m : b->mp)
    if (m.cls >= 0) m.w = window_for(ctx, m.cls, pc2k::OP_ENC_MFMA);
  // descriptors and items (most expensive class first)
  std::vector<pc2k::BatchJob> dj;
  std::vector<pc2k::BatchItem> items;
  std::vector<size_t> ptrbuf;  // per hom_sum job: K pointers then K lengths
  std::vector<size_t> ptr_off;
  std::vector<bool> mjob;      // runs on the matrix cores
  for (size_t i = 0; i < njobs; ++i) {
    const pc2_job& j = jobs[i];
    if (j.count == 0) continue;
    pc2k::BatchJob d{};
    const pc2_pk* pk = (op == pc2k::OP_DEC) ? &j.sk->pk : j.pk;
    const bool mf = op == pc2k::OP_ENC && (pk->cls == mca || pk->cls == mcb);
    d.geo = mf ? pk->cls : job_geo(ctx, pk, op);
    d.group = pc2k::batch_group_elems(op, job_geo(ctx, pk, op));
    d.op = op;
    d.m_limbs = (int)j.m_limbs;
    d.K = (int)j.K;
    d.pk = mf ? pk->c : geo_const(pk, d.geo);
    mjob.push_back(mf);
    if (op == pc2k::OP_DEC) d.sk = j.sk->c;
    d.in0 = j.in0;
    d.in1 = j.in1;
    d.out = j.out;
    d.count = j.count;
    size_t off = ptrbuf.size();
    if (op == pc2k::OP_SUM) {
      for (uint32_t k = 0; k < j.K; ++k) ptrbuf.push_back((size_t)j.inputs[k]);
      for (uint32_t k = 0; k < j.K; ++k) ptrbuf.push_back(j.lengths ? j.lengths[k] : j.count);
    }
    ptr_off.push_back(off);
    dj.push_back(d);
  }
  for (int pass = 0; pair >= 0 && pass < 2; ++pass) {
    const int first_geo = pc2k::GEO_CLASS[pa] >= pc2k::GEO_CLASS[pb] ? pa : pb;
    const int want = pass == 0 ? first_geo : (first_geo == pa ? pb : pa);
    if (pass == 1 && pa == pb) break;
    for (size_t ji = 0; ji < dj.size(); ++ji) {
      if (mjob[ji] || dj[ji].geo != want) continue;
      const size_t epw = (size_t)pc2k::batch_group_elems(op, dj[ji].geo);
      const size_t groups = (dj[ji].count + epw - 1) / epw;
      for (size_t g = 0; g < groups; ++g) {
        items.push_back(pc2k::BatchItem{(int)ji, 0, g});
        if (op == pc2k::OP_DEC) items.push_back(pc2k::BatchItem{(int)ji, 1, g});
      }
    }
  }
  b->nitems = (int)items.size();
  std::vector<size_t> mfirst(2, 0);
  for (int part = 0; part < 2; ++part) {  // matrix-core items after the others, per class
    mfirst[part] = items.size();
    for (size_t ji = 0; ji < dj.size(); ++ji) {
      if (!mjob[ji] || b->mp[part].cls < 0 || dj[ji].geo != b->mp[part].cls) continue;
      b->mp[part].sub = std::max(b->mp[part].sub, dj[ji].group);
      const size_t groups = (dj[ji].count + dj[ji].group - 1) / dj[ji].group;
      for (size_t g = 0; g < groups; ++g) items.push_back(pc2k::BatchItem{(int)ji, 0, g});
    }
    b->mp[part].nitems = (int)(items.size() - mfirst[part]);
  }
  // decryption: staging for the two CRT halves of every element
  std::vector<size_t> stage_off(dj.size(), 0);
  size_t stage_words = 0;
  if (op == pc2k::OP_DEC) {
    for (size_t ji = 0; ji < dj.size(); ++ji) {
      const size_t epw = (size_t)pc2k::batch_group_elems(op, dj[ji].geo);
      stage_off[ji] = stage_words;
      stage_words += (dj[ji].count + epw - 1) / epw * epw * 2 * (size_t)(dj[ji].sk.h[0].Ls + 1);
    }
  }
  // one device allocation: jobs | items | pointer/length arrays | queue
  const size_t jobs_b = (dj.size() * sizeof(pc2k::BatchJob) + 255) & ~(size_t)255;
  const size_t items_b = (items.size() * sizeof(pc2k::BatchItem) + 255) & ~(size_t)255;
  const size_t ptr_b = (ptrbuf.size() * sizeof(size_t) + 255) & ~(size_t)255;
  const size_t total = jobs_b + items_b + ptr_b + QUEUE_BYTES;
  int rc = PC2_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) rc = PC2_E_DEVICE;
  if (!rc && hipMalloc(&b->dev, total) != hipSuccess) rc = PC2_E_NOMEM;
  if (!rc && stage_words && hipMalloc(&b->stage, stage_words * 4) != hipSuccess)
    rc = PC2_E_NOMEM;
  if (!rc && stage_words)
    for (size_t ji = 0; ji < dj.size(); ++ji) {
      dj[ji].stage = b->stage + stage_off[ji];
      dj[ji].stage_g0 = 0;
    }
  if (!rc) {
    char* base = (char*)b->dev;
    b->jobs = (pc2k::BatchJob*)base;
    b->items = (pc2k::BatchItem*)(base + jobs_b);
    size_t* dptr = (size_t*)(base + jobs_b + items_b);
    b->queue = (int*)(base + jobs_b + items_b + ptr_b);
    for (int part = 0; part < 2; ++part) {
      b->mp[part].items = b->items + mfirst[part];
      b->mp[part].queue = b->queue + QUEUE_STRIDE * (part + 1);
    }
    for (size_t ji = 0; ji < dj.size(); ++ji)
      if (op == pc2k::OP_SUM) {
        dj[ji].inputs = (const uint32_t* const*)(dptr + ptr_off[ji]);
        dj[ji].lengths = dptr + ptr_off[ji] + dj[ji].K;
      }
    if (hipMemcpy(b->jobs, dj.data(), dj.size() * sizeof(pc2k::BatchJob),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->items, items.data(), items.size() * sizeof(pc2k::BatchItem),
                  hipMemcpyHostToDevice) != hipSuccess ||
        (!ptrbuf.empty() && hipMemcpy(dptr, ptrbuf.data(), ptrbuf.size() * sizeof(size_t),
                                      hipMemcpyHostToDevice) != hipSuccess))
      rc = PC2_E_DEVICE;
  }
  // grids and the batch's own scratch
  size_t mbytes = 0;
  for (auto& m : b->mp) {
    if (rc || !m.nitems) continue;
    m.grid = std::max<int>(
        1, (int)std::min<size_t>((size_t)ctx->cus * occupancy_of(pc2k::batch_mfma_kernel(m.cls)),
                                 (size_t)m.nitems * m.sub));
    mbytes = std::max(mbytes, (size_t)m.grid * (pc2k::mfma_digit_bytes(m.cls) << m.w));
  }
  if (!rc && mbytes && hipMalloc(&b->mscratch, mbytes) != hipSuccess) rc = PC2_E_NOMEM;
  if (!rc && b->nitems) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pc2k::batch_kernel(op, pair), 64, 0) !=
            hipSuccess ||
        occ <= 0)
      occ = 1;
    b->grid = std::max(1, std::min(ctx->cus * occ, b->nitems));
    int ta = 0, tb = 0;
    size_t wa = 0, wb = 0;
    pc2k::batch_slot_shape(op, pa, b->w_a, Ls, &ta, &wa);
    pc2k::batch_slot_shape(op, pb, b->w_b, Ls, &tb, &wb);
    const int tiles = std::max(ta, tb);
    b->slot_words = (std::max(wa, wb) + 3) & ~(size_t)3;
    const size_t bytes = (size_t)b->grid * tiles * b->slot_words * 4;
    if (bytes && hipMalloc(&b->scratch, bytes) != hipSuccess) rc = PC2_E_NOMEM;
  }
  if (rc) {
    if (b->dev) (void)hipFree(b->dev);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->mscratch) (void)hipFree(b->mscratch);
    if (b->stage) (void)hipFree(b->stage);
    delete b;
    return rc;
  }
  *out = b;
  return PC2_OK;
}

int pc2_batch_run(pc2_batch* b, void* hip_stream) {
  if (!b || !b->ctx) return PC2_E_INVAL;
  if (hipSetDevice(b->ctx->device) != hipSuccess) return PC2_E_DEVICE;
  auto launch = [&](void* st) {
    hipError_t e = hipSuccess;
    if (b->nitems)
      e = pc2k::launch_batch(b->op, b->pair, b->grid, b->jobs, b->items, b->nitems, b->queue,
                             b->scratch, b->slot_words, b->w_a, b->w_b, b->ctx->err, st);
    for (const auto& m : b->mp)
      if (e == hipSuccess && m.nitems)
        e = pc2k::launch_batch_mfma(m.cls, m.grid, b->jobs, m.items, m.nitems, m.sub, m.queue,
                                    b->mscratch, m.w, b->ctx->err, st);
    return e;
  };
  if (!hip_stream) return status_of(launch(nullptr));
  if (!b->exec || b->graph_stream != hip_stream) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return PC2_E_DEVICE;
    hipError_t le = launch(hip_stream);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(st, &g);
    if (le != hipSuccess || ee != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return PC2_E_DEVICE;
    }
    hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      b->exec = nullptr;
      return PC2_E_DEVICE;
    }
    b->graph_stream = hip_stream;
  }
  return status_of(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
}

int pc2_batch_destroy(pc2_batch* b) {
  if (!b || !b->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->dev) (void)hipFree(b->dev);
  if (b->scratch) (void)hipFree(b->scratch);
  if (b->mscratch) (void)hipFree(b->mscratch);
  if (b->stage) (void)hipFree(b->stage);
  delete b;
  return PC2_OK;
}

// -------------------------------------------------------------- autotune
// Times encryption in each tile the key's class has (lanes per ciphertext)
// with windows 4..6, and decryption with windows 4..6, on a few
// device-filling waves of elements; keeps the fastest choices in the context.
int pc2_autotune(const pc2_sk* sk, void* hip_stream, int* w_enc, int* w_dec, int* tile_enc) {
  if (!sk || !sk->ctx) return PC2_E_INVAL;
  pc2_ctx* ctx = sk->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  const int cls = sk->pk.cls, L = sk->pk.L;
  int geos[2] = {cls, pc2k::ALT_GEO[cls]};
  const int ngeo = geos[1] >= 0 ? 2 : 1;
  // the same element count for every candidate: four waves of the widest
  size_t count = 0;
  for (int g = 0; g < ngeo; ++g)
    count = std::max(count, (size_t)ctx->cus * occupancy(ctx, geos[g], pc2k::OP_ENC) *
                                (size_t)pc2k::elems_per_block(geos[g]));
  count *= 4;
  // the work of the exponentiations does not depend on the data: m = 0,
  // r = 1 is valid under every key
  std::vector<uint32_t> hm(count, 0), hr(count * L, 0);
  for (size_t i = 0; i < count; ++i) hr[i * L] = 1;
  uint32_t *m = nullptr, *r = nullptr, *c = nullptr, *d = nullptr;
  int rc = PC2_OK;
  if (hipMalloc(&m, count * 4) != hipSuccess || hipMalloc(&r, count * L * 4) != hipSuccess ||
      hipMalloc(&c, count * 2 * L * 4) != hipSuccess || hipMalloc(&d, count * L * 4) != hipSuccess)
    rc = PC2_E_NOMEM;
  if (!rc && (hipMemcpy(m, hm.data(), count * 4, hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(r, hr.data(), count * L * 4, hipMemcpyHostToDevice) != hipSuccess))
    rc = PC2_E_DEVICE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = PC2_E_DEVICE;
  const int saved_window = ctx->window, saved_tile = ctx->tile, saved_modmul = ctx->modmul;
  ctx->modmul = PC2_MODMUL_VALU;
  int best_w[2] = {0, 0}, best_geo = cls;
  float best_ms[2] = {1e30f, 1e30f};
  // trials: (encryption, geometry) for each tile, then decryption
  for (int trial = 0; trial <= ngeo && !rc; ++trial) {
    const bool dec = trial == ngeo;
    if (!dec) ctx->tile = pc2k::CLASS_GEO[geos[trial]].nT;
    for (int w = 4; w <= 6 && !rc; ++w) {
      ctx->window = w;
      for (int rep = 0; rep < 2 && !rc; ++rep) {  // rep 0 warms up (and sizes scratch)
        if (hipEventRecord(e0, (hipStream_t)hip_stream) != hipSuccess) rc = PC2_E_DEVICE;
        int st = dec ? pc2_decrypt(sk, c, d, count, hip_stream)
                     : pc2_encrypt(&sk->pk, m, 1, r, c, count, hip_stream);
        if (st) rc = st;
        if (!rc && (hipEventRecord(e1, (hipStream_t)hip_stream) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess))
          rc = PC2_E_DEVICE;
        float ms = 0;
        if (!rc && rep == 1 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            ms < best_ms[dec]) {
          best_ms[dec] = ms;
          best_w[dec] = w;
          if (!dec) best_geo = geos[trial];
        }
      }
    }
  }
  ctx->window = saved_window;
  ctx->tile = saved_tile;
  ctx->modmul = saved_modmul;
  if (!rc) {
    ctx->tuned_geo[cls] = best_geo;
    ctx->tuned[best_geo][pc2k::OP_ENC] = best_w[0];
    ctx->tuned[cls][pc2k::OP_DEC] = best_w[1];
    if (w_enc) *w_enc = best_w[0];
    if (w_dec) *w_dec = best_w[1];
    if (tile_enc) *tile_enc = pc2k::CLASS_GEO[best_geo].nT;
    rc = pc2_ctx_take_error(ctx);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (m) (void)hipFree(m);
  if (r) (void)hipFree(r);
  if (c) (void)hipFree(c);
  if (d) (void)hipFree(d);
  return rc;
}

// ---------------------------------------------------------------- runners
namespace {
int op_from_abi(int op_abi) {
  if (op_abi == PC2_OP_ENCRYPT) return pc2k::OP_ENC;
  if (op_abi == PC2_OP_DECRYPT) return pc2k::OP_DEC;
  if (op_abi == PC2_OP_HOM_SUM) return pc2k::OP_SUM;
  return -1;
}
}  // namespace

int pc2_runner_create(pc2_ctx* ctx, int op_abi, uint32_t max_nbits, size_t max_jobs,
                      size_t max_groups, pc2_runner** out) {
  if (!ctx || !out || max_jobs == 0 || max_groups == 0) return PC2_E_INVAL;
  *out = nullptr;
  const int op = op_from_abi(op_abi);
  const int cls = pc2k::class_for_bits((int)max_nbits);
  if (op < 0) return PC2_E_INVAL;
  if (cls < 0) return PC2_E_UNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  pc2_runner* r = new (std::nothrow) pc2_runner();
  if (!r) return PC2_E_NOMEM;
  r->ctx = ctx;
  r->op = op;
  r->max_cls = cls;
  r->max_jobs = max_jobs;
  r->max_groups = max_groups;
  r->max_ptrs = op == pc2k::OP_SUM ? 2 * (size_t)pc2k::RK_MAX * max_jobs : 0;
  r->jobs_b = (max_jobs * sizeof(pc2k::BatchJob) + 255) & ~(size_t)255;
  // a decryption group is two items (one per prime)
  const size_t max_items = (op == pc2k::OP_DEC ? 2 : 1) * max_groups;
  r->items_b = (max_items * sizeof(pc2k::BatchItem) + 255) & ~(size_t)255;
  r->ptr_b = (r->max_ptrs * sizeof(size_t) + 255) & ~(size_t)255;
  const size_t total = r->jobs_b + r->items_b + r->ptr_b + QUEUE_BYTES;
  int rc = PC2_OK;
  if (hipMalloc(&r->dev, total) != hipSuccess || hipHostMalloc(&r->host, total) != hipSuccess ||
      hipEventCreateWithFlags(&r->copied, hipEventDisableTiming) != hipSuccess)
    rc = PC2_E_NOMEM;
  // scratch for the widest pair this runner may launch
  if (!rc) {
    int tiles = 0;
    size_t words = 0;
    int occ_max = 1;
    const int L = (int)((max_nbits + 31) / 32);
    const int Ls = std::min(L / 2 + 2, pc2k::LS_MAX);
    r->ls = Ls;
    for (int g = 0; g < pc2k::NUM_GEOS; ++g) {
      if (pc2k::GEO_CLASS[g] > cls) continue;
      const int pair = pc2k::batch_pair(g, g);
      if (pair < 0 || !pc2k::batch_kernel(op, pair)) continue;
      const int w = std::max(window_for(ctx, g, op), 6);
      int t = 0;
      size_t wd = 0;
      pc2k::batch_slot_shape(op, g, w, Ls, &t, &wd);
      tiles = std::max(tiles, t);
      words = std::max(words, wd);
    }
    for (int pair = 0; pair < pc2k::batch_npairs(); ++pair) {
      const void* k = pc2k::batch_kernel(op, pair);
      if (!k) continue;
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 64, 0) == hipSuccess)
        occ_max = std::max(occ_max, occ);
    }
    r->grid_cap = ctx->cus * occ_max;
    r->slot_words = (words + 3) & ~(size_t)3;
    const size_t bytes = (size_t)r->grid_cap * tiles * r->slot_words * 4;
    if (bytes && hipMalloc(&r->scratch, bytes) != hipSuccess) rc = PC2_E_NOMEM;
    // encryption jobs of a class on the matrix cores (the engine option may
    // change after creation, so every class up to the largest is covered)
    for (int c = 0; !rc && op == pc2k::OP_ENC && c <= cls; ++c) {
      r->mocc[c] = occupancy_of(pc2k::batch_mfma_kernel(c));
      r->mscratch_bytes =
          std::max(r->mscratch_bytes, (size_t)ctx->cus * r->mocc[c] *
                                          (pc2k::mfma_digit_bytes(c) << pc2k::SCHED_WMAX));
    }
    if (!rc && r->mscratch_bytes && hipMalloc(&r->mscratch, r->mscratch_bytes) != hipSuccess)
      rc = PC2_E_NOMEM;
    if (!rc && op == pc2k::OP_DEC) {  // CRT halves of up to max_groups groups
      size_t per = 0;
      for (int g = 0; g < pc2k::NUM_GEOS; ++g)
        if (pc2k::GEO_CLASS[g] <= cls && pc2k::batch_group_elems(op, g) > 0)
          per = std::max(per, (size_t)pc2k::batch_group_elems(op, g) * 2 * (Ls + 1));
      if (hipMalloc(&r->stage, max_groups * per * 4) != hipSuccess) rc = PC2_E_NOMEM;
    }
  }
  if (rc) {
    if (r->dev) (void)hipFree(r->dev);
    if (r->host) (void)hipHostFree(r->host);
    if (r->scratch) (void)hipFree(r->scratch);
    if (r->mscratch) (void)hipFree(r->mscratch);
    if (r->stage) (void)hipFree(r->stage);
    if (r->copied) (void)hipEventDestroy(r->copied);
    delete r;
    return rc;
  }
  *out = r;
  return PC2_OK;
}

int pc2_runner_group_size(const pc2_pk* pk, int op_abi, uint32_t* elems) {
  if (!pk || !pk->ctx || !elems || op_from_abi(op_abi) < 0) return PC2_E_INVAL;
  const int op = op_from_abi(op_abi);
  *elems = (uint32_t)pc2k::batch_group_elems(op, job_geo(pk->ctx, pk, op));
  return PC2_OK;
}

int pc2_runner_launch(pc2_runner* r, const pc2_job* jobs, const size_t* first,
                      const size_t* ngroups, size_t njobs, void* hip_stream) {
  if (!r || !r->ctx || !jobs || !first || !ngroups || njobs == 0) return PC2_E_INVAL;
  if (njobs > r->max_jobs) return PC2_E_BUSY;
  pc2_ctx* ctx = r->ctx;
  const int op = r->op;
  int ca = -1, cb = -1, mca = -1, mcb = -1;
  size_t nitems = 0, nptrs = 0;
  for (size_t i = 0; i < njobs; ++i) {
    const pc2_job& j = jobs[i];
    if (op_from_abi(j.op) != op) return PC2_E_INVAL;
    const pc2_pk* pk = (op == pc2k::OP_DEC) ? (j.sk ? &j.sk->pk : nullptr) : j.pk;
    if (!pk || pk->ctx != ctx || !j.out || pk->cls > r->max_cls) return PC2_E_INVAL;
    const int g = job_geo(ctx, pk, op);
    const size_t epw = (size_t)pc2k::batch_group_elems(op, g);
    if (first[i] + ngroups[i] > (j.count + epw - 1) / epw) return PC2_E_INVAL;
    if (op == pc2k::OP_ENC && (!j.in0 || !j.in1 || j.m_limbs < 1 || (int)j.m_limbs > pk->L))
      return PC2_E_INVAL;
    if (op == pc2k::OP_DEC && (!j.in0 || j.sk->c.h[0].Ls > r->ls)) return PC2_E_INVAL;
    if (op == pc2k::OP_SUM) {
      if (!j.inputs || j.K < 1 || j.K > (uint32_t)pc2k::RK_MAX) return PC2_E_INVAL;
      for (uint32_t k = 0; k < j.K; ++k)
        if (!j.inputs[k] || (j.lengths && j.lengths[k] > j.count)) return PC2_E_INVAL;
      nptrs += 2 * (size_t)j.K;
    }
    if (job_overlaps(j, pk->L)) return PC2_E_INVAL;
    nitems += ngroups[i];
    if (ngroups[i] == 0) continue;
    if (op == pc2k::OP_ENC && use_mfma(ctx, pk->cls)) {
      if (mca < 0 || mca == pk->cls) mca = pk->cls;
      else if (mcb < 0 || mcb == pk->cls) mcb = pk->cls;
      else return PC2_E_UNSUPPORTED;
      continue;
    }
    if (ca < 0 || ca == g) ca = g;
    else if (cb < 0 || cb == g) cb = g;
    else return PC2_E_UNSUPPORTED;
  }
  if (nitems == 0) return PC2_OK;
  if (nitems > r->max_groups || nptrs > r->max_ptrs) return PC2_E_BUSY;
  for (int c : {mca, mcb})  // (the scratch covers every class up to max_cls)
    if (c >= 0 && (!r->mscratch || (pc2k::mfma_digit_bytes(c)
                                    << window_for(ctx, c, pc2k::OP_ENC_MFMA)) > r->mscratch_bytes))
      return PC2_E_NOMEM;
  int pair = -1;
  if (ca >= 0) {
    if (cb < 0) cb = ca;
    pair = pc2k::batch_pair(ca, cb);
    if (pair < 0) return PC2_E_UNSUPPORTED;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  // the previous launch's copies must have read the staging buffers
  if (r->pending && hipEventSynchronize(r->copied) != hipSuccess) return PC2_E_DEVICE;
  char* hb = (char*)r->host;
  char* db = (char*)r->dev;
  auto* hj = (pc2k::BatchJob*)hb;
  auto* hi = (pc2k::BatchItem*)(hb + r->jobs_b);
  auto* hp = (size_t*)(hb + r->jobs_b + r->items_b);
  auto* dp = (size_t*)(db + r->jobs_b + r->items_b);
  size_t pofs = 0, it = 0, sofs = 0;
  const int pa = pair >= 0 ? pc2k::batch_pair_geo(pair, 0) : -1;
  const int pb = pair >= 0 ? pc2k::batch_pair_geo(pair, 1) : -1;
  for (size_t i = 0; i < njobs; ++i) {
    const pc2_job& j = jobs[i];
    const pc2_pk* pk = (op == pc2k::OP_DEC) ? &j.sk->pk : j.pk;
    const bool mf = op == pc2k::OP_ENC && (pk->cls == mca || pk->cls == mcb);
    pc2k::BatchJob d{};
    d.geo = mf ? pk->cls : job_geo(ctx, pk, op);
    d.group = pc2k::batch_group_elems(op, job_geo(ctx, pk, op));
    d.op = op;
    d.m_limbs = (int)j.m_limbs;
    d.K = (int)j.K;
    d.pk = mf ? pk->c : geo_const(pk, d.geo);
    if (op == pc2k::OP_DEC) d.sk = j.sk->c;
    d.in0 = j.in0;
    d.in1 = j.in1;
    d.out = j.out;
    d.count = j.count;
    if (op == pc2k::OP_DEC) {  // this launch's groups of job i, back to back
      const size_t epw = (size_t)pc2k::batch_group_elems(op, d.geo);
      d.stage = r->stage + sofs;
      d.stage_g0 = first[i];
      sofs += ngroups[i] * epw * 2 * (size_t)(d.sk.h[0].Ls + 1);
    }
    if (op == pc2k::OP_SUM) {
      for (uint32_t k = 0; k < j.K; ++k) hp[pofs + k] = (size_t)j.inputs[k];
      for (uint32_t k = 0; k < j.K; ++k) hp[pofs + j.K + k] = j.lengths ? j.lengths[k] : j.count;
      d.inputs = (const uint32_t* const*)(dp + pofs);
      d.lengths = dp + pofs + j.K;
      pofs += 2 * (size_t)j.K;
    }
    hj[i] = d;
  }
  // most expensive class first; the matrix-core items after the others
  auto on_mfma = [&](size_t i) {
    const pc2_pk* pk = (op == pc2k::OP_DEC) ? &jobs[i].sk->pk : jobs[i].pk;
    return op == pc2k::OP_ENC && (pk->cls == mca || pk->cls == mcb);
  };
  for (int pass = 0; pair >= 0 && pass < 2; ++pass) {
    const int first_geo = pc2k::GEO_CLASS[pa] >= pc2k::GEO_CLASS[pb] ? pa : pb;
    const int want = pass == 0 ? first_geo : (first_geo == pa ? pb : pa);
    if (pass == 1 && pa == pb) break;
    for (size_t i = 0; i < njobs; ++i) {
      if (on_mfma(i) || hj[i].geo != want) continue;
      for (size_t g = 0; g < ngroups[i]; ++g) {
        hi[it++] = pc2k::BatchItem{(int)i, 0, first[i] + g};
        if (op == pc2k::OP_DEC) hi[it++] = pc2k::BatchItem{(int)i, 1, first[i] + g};
      }
    }
  }
  const size_t it_valu = it;
  const int mcls[2] = {std::max(mca, mcb), std::min(mca, mcb)};  // the more expensive first
  size_t mfirst[3] = {it, it, it};
  int msub[2] = {1, 1};
  for (int part = 0; part < 2; ++part) {
    mfirst[part] = it;
    for (size_t i = 0; mcls[part] >= 0 && i < njobs; ++i)
      if (on_mfma(i) && hj[i].geo == mcls[part]) {
        msub[part] = std::max(msub[part], hj[i].group);
        for (size_t g = 0; g < ngroups[i]; ++g)
          hi[it++] = pc2k::BatchItem{(int)i, 0, first[i] + g};
      }
    mfirst[part + 1] = it;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipMemcpyAsync(db, hb, njobs * sizeof(pc2k::BatchJob), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(db + r->jobs_b, hb + r->jobs_b, it * sizeof(pc2k::BatchItem),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      (pofs && hipMemcpyAsync(dp, hp, pofs * sizeof(size_t), hipMemcpyHostToDevice, st) !=
                   hipSuccess) ||
      hipEventRecord(r->copied, st) != hipSuccess)
    return PC2_E_DEVICE;
  r->pending = true;
  int* queue = (int*)(db + r->jobs_b + r->items_b + r->ptr_b);
  const auto* ditems = (const pc2k::BatchItem*)(db + r->jobs_b);
  hipError_t e = hipSuccess;
  if (it_valu) {
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(r->grid_cap, it_valu));
    const int w_a = window_for(ctx, pa, op), w_b = window_for(ctx, pb, op);
    e = pc2k::launch_batch(op, pair, grid, (const pc2k::BatchJob*)db, ditems, (int)it_valu,
                           queue, r->scratch, r->slot_words, w_a, w_b, ctx->err, st);
  }
  for (int part = 0; part < 2 && e == hipSuccess; ++part) {
    const size_t n = mfirst[part + 1] - mfirst[part];
    if (!n) continue;
    const int c = mcls[part];
    const int w = window_for(ctx, c, pc2k::OP_ENC_MFMA);
    const size_t per = pc2k::mfma_digit_bytes(c) << w;
    const size_t cap = (size_t)ctx->cus * std::max(1, r->mocc[c]);
    const int grid = (int)std::max<size_t>(
        1, std::min<size_t>({cap, n * msub[part], r->mscratch_bytes / per}));
    e = pc2k::launch_batch_mfma(c, grid, (const pc2k::BatchJob*)db, ditems + mfirst[part],
                                (int)n, msub[part], queue + QUEUE_STRIDE * (part + 1),
                                r->mscratch, w,
                                ctx->err, st);
  }
  return status_of(e);
}

int pc2_runner_destroy(pc2_runner* r) {
  if (!r || !r->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(r->ctx->device);
  (void)hipDeviceSynchronize();
  if (r->dev) (void)hipFree(r->dev);
  if (r->host) (void)hipHostFree(r->host);
  if (r->scratch) (void)hipFree(r->scratch);
  if (r->mscratch) (void)hipFree(r->mscratch);
  if (r->stage) (void)hipFree(r->stage);
  if (r->copied) (void)hipEventDestroy(r->copied);
  delete r;
  return PC2_OK;
}

// ------------------------------------------------------ ciphertext mat-vec
namespace {
size_t matvec_table_bytes(int cls, size_t cols, int ebits, int w) {
  const size_t nw = (size_t)((ebits + w - 1) / w);
  return cols * nw * (((size_t)1 << w) - 1) * pc2k::matvec_entry_words(cls) * 4;
}
int resident_groups(pc2_ctx* ctx, const void* k) {
  int occ = 0;
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 64, 0) != hipSuccess || occ <= 0)
    occ = 1;
  return ctx->cus * occ;
}
// Column chunks of a mat-vec of `rows` rows: the count (up to the aggregation
// limit and max_chunks) whose whole wavefront groups fill the resident
// capacity best; fewer on a near tie.
void pick_chunks(const pc2_matvec* mv, size_t rows, size_t max_chunks, size_t* nch,
                 size_t* chunk_cols) {
  const size_t epw = (size_t)pc2k::elems_per_block(mv->pk->cls);
  const size_t gpc = (rows + epw - 1) / epw;
  const size_t cap = (size_t)mv->cap_apply;
  *nch = 1;
  *chunk_cols = mv->cols;
  double best = -1;
  const size_t top = std::min(std::min(mv->cols, (size_t)pc2k::RK_MAX), std::max<size_t>(1, max_chunks));
  for (size_t c = 1; c <= top; ++c) {
    const size_t cc = (mv->cols + c - 1) / c;
    if ((mv->cols + cc - 1) / cc != c) continue;  // the same split as a smaller count
    const size_t groups = gpc * c;
    const double eff = (double)groups / (double)(((groups + cap - 1) / cap) * cap);
    if (eff > best + 0.02) {
      best = eff;
      *nch = c;
      *chunk_cols = cc;
    }
  }
}
}  // namespace

int pc2_matvec_create(const pc2_pk* pk, size_t cols, uint32_t ebits, uint32_t window,
                      size_t rows_hint, pc2_matvec** out) {
  if (!pk || !pk->ctx || !out || cols == 0 || ebits < 1 || ebits > 64 || window > 12)
    return PC2_E_INVAL;
  *out = nullptr;
  pc2_ctx* ctx = pk->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  int w = (int)window;
  if (w == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return PC2_E_DEVICE;
    double best = 0;
    for (int c = 1; c <= 12; ++c) {
      if (matvec_table_bytes(pk->cls, cols, (int)ebits, c) > free_b / 4) break;
      const double nwc = (double)((ebits + c - 1) / c);
      // products per column: rows x windows (rows), windows x table entries (tables)
      const double cost = rows_hint ? nwc * ((double)rows_hint + (double)((1 << c) - 1))
                                    : (c <= 8 ? 1.0 / c : 1e300);
      if (w == 0 || cost < best) {
        w = c;
        best = cost;
      }
    }
    if (w == 0) return PC2_E_NOMEM;
  }
  pc2_matvec* mv = new (std::nothrow) pc2_matvec();
  if (!mv) return PC2_E_NOMEM;
  mv->ctx = ctx;
  mv->pk = pk;
  mv->w = w;
  mv->nw = ((int)ebits + w - 1) / w;
  mv->ebits = (int)ebits;
  mv->cols = cols;
  mv->table_bytes = matvec_table_bytes(pk->cls, cols, (int)ebits, w);
  if (hipMalloc(&mv->tab, mv->table_bytes) != hipSuccess) {
    delete mv;
    return PC2_E_NOMEM;
  }
  mv->cap_table = resident_groups(ctx, pc2k::kernel_matvec(pk->cls, 0));
  mv->cap_apply = resident_groups(ctx, pc2k::kernel_matvec(pk->cls, 1));
  // staging for the partial products of rows_hint rows split over column
  // chunks (pc2_matvec_apply allocates nothing)
  if (rows_hint) {
    size_t nch = 1, cc = 0;
    pick_chunks(mv, rows_hint, (size_t)pc2k::RK_MAX, &nch, &cc);
    if (nch > 1) {
      mv->parts_bytes = nch * rows_hint * 8 * (size_t)pk->L;
      if (hipMalloc(&mv->parts, mv->parts_bytes) != hipSuccess) {
        (void)hipFree(mv->tab);
        delete mv;
        return PC2_E_NOMEM;
      }
    }
  }
  (void)occupancy(ctx, pk->cls, pc2k::OP_SUM);
  *out = mv;
  return PC2_OK;
}

int pc2_matvec_info(const pc2_matvec* mv, uint32_t* window, size_t* table_bytes) {
  if (!mv) return PC2_E_INVAL;
  if (window) *window = (uint32_t)mv->w;
  if (table_bytes) *table_bytes = mv->table_bytes;
  return PC2_OK;
}

int pc2_matvec_load(pc2_matvec* mv, const uint32_t* c, void* hip_stream) {
  if (!mv || !mv->ctx || !c) return PC2_E_INVAL;
  if (hipSetDevice(mv->ctx->device) != hipSuccess) return PC2_E_DEVICE;
  const int cls = mv->pk->cls;
  const size_t epw = (size_t)pc2k::elems_per_block(cls);
  const size_t groups = (mv->cols + epw - 1) / epw * (size_t)mv->nw;
  const int grid = (int)std::max<size_t>(1, std::min<size_t>(groups, (size_t)mv->cap_table));
  int rc = status_of(pc2k::launch_mv_table(cls, grid, mv->pk->c, c, mv->cols, mv->nw, mv->w,
                                           mv->tab, mv->ctx->err, hip_stream));
  if (!rc) mv->loaded = true;
  return rc;
}

int pc2_matvec_apply(pc2_matvec* mv, const uint64_t* B, const uint32_t* alpha, uint32_t* out,
                     size_t rows, void* hip_stream) {
  if (!mv || !mv->ctx) return PC2_E_INVAL;
  if (rows == 0) return PC2_OK;
  if (!B || !out || !mv->loaded) return PC2_E_INVAL;
  pc2_ctx* ctx = mv->ctx;
  const pc2_pk* pk = mv->pk;
  const int cls = pk->cls;
  const size_t L2 = 2 * (size_t)pk->L, row_bytes = L2 * 4;
  if (alpha && alpha != out) {  // exact aliasing is allowed, partial overlap is not
    const char *a0 = (const char*)alpha, *o0 = (const char*)out;
    if (a0 < o0 + rows * row_bytes && o0 < a0 + rows * row_bytes) return PC2_E_INVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  // column chunks, as many as the plan's staging holds for this many rows
  const size_t epw = (size_t)pc2k::elems_per_block(cls);
  const size_t gpc = (rows + epw - 1) / epw;
  const size_t cap = (size_t)mv->cap_apply;
  size_t nch = 1, chunk_cols = mv->cols;
  pick_chunks(mv, rows, mv->parts_bytes / (rows * row_bytes), &nch, &chunk_cols);
  const size_t groups = gpc * nch;
  const int grid = (int)std::max<size_t>(1, std::min(groups, cap));
  if (nch == 1)
    return status_of(pc2k::launch_mv_apply(cls, grid, pk->c, B, rows, mv->cols, mv->ebits,
                                           mv->nw, mv->w, mv->tab, alpha, 1, chunk_cols, out,
                                           0, ctx->err, hip_stream));
  int rc = status_of(pc2k::launch_mv_apply(cls, grid, pk->c, B, rows, mv->cols, mv->ebits,
                                           mv->nw, mv->w, mv->tab, alpha, nch, chunk_cols,
                                           mv->parts, rows * L2, ctx->err, hip_stream));
  if (rc) return rc;
  pc2k::PtrList lst{};
  for (size_t k = 0; k < nch; ++k) lst.p[k] = mv->parts + k * rows * L2;
  pc2k::Launch l{};
  l.grid = (int)std::max<size_t>(
      1, std::min(gpc, (size_t)ctx->cus * occupancy(ctx, cls, pc2k::OP_SUM)));
  l.err = ctx->err;
  l.stream = hip_stream;
  return status_of(pc2k::launch_hom_sum(cls, l, pk->c, lst, (int)nch, out, rows));
}

int pc2_matvec_destroy(pc2_matvec* mv) {
  if (!mv || !mv->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(mv->ctx->device);
  (void)hipDeviceSynchronize();
  if (mv->tab) (void)hipFree(mv->tab);
  if (mv->parts) (void)hipFree(mv->parts);
  delete mv;
  return PC2_OK;
}

// ------------------------------------------------- column-split ADMM
namespace {
void* carve(char*& at, size_t bytes) {  // 256-byte aligned sub-buffers of one allocation
  void* p = at;
  at += (bytes + 255) & ~(size_t)255;
  return p;
}
int ceil_log2(size_t v) {
  int b = 0;
  while (((size_t)1 << b) < v) ++b;
  return b;
}
}  // namespace

namespace {
// Plaintexts of the node step stay below 2^(2k + 9 + log2 Nk): they must fit
// 127 bits (the inverse quantization's integers) and the key.
bool colsplit_scale_ok(const pc2_sk* sk, int Nk, int k) {
  const int pbits = 2 * k + 9 + ceil_log2((size_t)Nk);
  return k >= 1 && pbits <= 126 && pbits < (int)sk->pk.c.nbits && sk->pk.L >= 4;
}

// Quantization of every node at scale 2^k: G_k = Gamma_2(rho B_k), its row
// sums, Enc(Gamma_1(alpha_k)) (randomness rows kk Nk .. (kk + 1) Nk - 1 of the
// pool) and the nodes' mat-vec plans over (k + 4)-bit constants.  Earlier
// plans are destroyed first (after the stream's work that reads them).
int colsplit_quantize(pc2_colsplit* cs, int k, void* stream) {
  const pc2_sk* sk = cs->sk;
  const size_t nk = (size_t)cs->Nk, L2 = 2 * (size_t)sk->pk.L;
  if (!cs->mv.empty()) {
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PC2_E_DEVICE;
    for (pc2_matvec* mv : cs->mv) pc2_matvec_destroy(mv);
    cs->mv.clear();
  }
  int rc = PC2_OK;
  for (int kk = 0; kk < cs->K && !rc; ++kk) {
    const size_t o1 = kk * nk, o2 = kk * nk * nk;
    rc = status_of(pc2k::cs_quantize_node(cs->rhoB + o2, cs->alpha + o1, cs->Nk, k, cs->G + o2,
                                          cs->R + o1, cs->g1 + o1 * 4, cs->ctx->err, stream));
    if (!rc)
      rc = pc2_encrypt(&sk->pk, cs->g1 + o1 * 4, 4, cs->r_pool + o1 * sk->pk.L,
                       cs->ahat + o1 * L2, nk, stream);
    pc2_matvec* mv = nullptr;
    if (!rc) rc = pc2_matvec_create(&sk->pk, nk, (uint32_t)(k + 4), 0, nk, &mv);
    if (!rc) cs->mv.push_back(mv);
  }
  if (!rc) cs->k = k;
  return rc;
}
}  // namespace

int pc2_colsplit_create(const pc2_sk* sk, const double* A, const double* y, uint32_t M,
                        uint32_t N, uint32_t K, double rho, uint32_t log2_scale,
                        const uint32_t* r_pool, size_t r_count, void* hip_stream,
                        pc2_colsplit** out) {
  if (!sk || !sk->ctx || !A || !y || !r_pool || !out || M == 0 || N == 0 || K == 0 ||
      N % K != 0 || !(rho > 0) || log2_scale < 1)
    return PC2_E_INVAL;
  *out = nullptr;
  const int Nk = (int)(N / K), k = (int)log2_scale, L = sk->pk.L;
  if (!colsplit_scale_ok(sk, Nk, k)) return PC2_E_UNSUPPORTED;
  if (r_count < 3 * (size_t)N) return PC2_E_INVAL;
  pc2_ctx* ctx = sk->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  pc2_colsplit* cs = new (std::nothrow) pc2_colsplit();
  if (!cs) return PC2_E_NOMEM;
  cs->ctx = ctx;
  cs->sk = sk;
  cs->M = (int)M;
  cs->N = (int)N;
  cs->K = (int)K;
  cs->Nk = Nk;
  cs->k = k;
  cs->rho = rho;
  cs->r_pool = r_pool;
  cs->r_count = r_count;
  const size_t nk = (size_t)Nk, L2 = 2 * (size_t)L, n = N;
  const size_t bytes = 256 * 16 + K * nk * 8 * 2 + K * nk * nk * 16 + K * nk * L2 * 4 +
                       n * 8 * 2 + K * 8 + n * L2 * 4 * 4 + n * L * 4 + K * nk * 16;
  void* tmp = nullptr;
  int rc = PC2_OK;
  if (hipMalloc(&cs->dev, bytes) != hipSuccess) rc = PC2_E_NOMEM;
  // setup workspace: T (Nk x 2Nk), rp (2Nk), f (Nk), aty (Nk)
  const size_t tbytes = 256 * 8 + nk * 2 * nk * 8 + nk * 4 * 8;
  if (!rc && hipMalloc(&tmp, tbytes) != hipSuccess) rc = PC2_E_NOMEM;
  if (!rc) {
    char* at = (char*)cs->dev;
    cs->alpha = (double*)carve(at, (K * nk) * sizeof(double));
    cs->rhoB = (double*)carve(at, (K * nk * nk) * sizeof(double));
    cs->G = (uint64_t*)carve(at, (K * nk * nk) * sizeof(uint64_t));
    cs->R = (uint64_t*)carve(at, (K * nk) * sizeof(uint64_t));
    cs->ahat = (uint32_t*)carve(at, (K * nk * L2) * sizeof(uint32_t));
    cs->w = (uint64_t*)carve(at, (2 * n) * sizeof(uint64_t));
    cs->S = (uint64_t*)carve(at, (size_t)K * sizeof(uint64_t));
    cs->cw = (uint32_t*)carve(at, (2 * n * L2) * sizeof(uint32_t));
    cs->c = (uint32_t*)carve(at, (n * L2) * sizeof(uint32_t));
    cs->xhat = (uint32_t*)carve(at, (n * L2) * sizeof(uint32_t));
    cs->P = (uint32_t*)carve(at, (n * L) * sizeof(uint32_t));
    cs->g1 = (uint32_t*)carve(at, (K * nk * 4) * sizeof(uint32_t));
    char* wt = (char*)tmp;
    double* T = (double*)carve(wt, (nk * 2 * nk) * sizeof(double));
    double* rp = (double*)carve(wt, (2 * nk) * sizeof(double));
    double* f = (double*)carve(wt, (nk) * sizeof(double));
    double* aty = (double*)carve(wt, (nk) * sizeof(double));
    for (int kk = 0; kk < (int)K && !rc; ++kk) {
      const size_t o1 = kk * nk, o2 = kk * nk * nk;
      rc = status_of(pc2k::cs_setup_node(A, y, (int)M, (int)N, kk * Nk, Nk, rho, T, rp, f, aty,
                                         cs->alpha + o1, cs->rhoB + o2, hip_stream));
    }
    if (!rc) rc = colsplit_quantize(cs, k, hip_stream);
    // the workspace is released once the setup has run
    if (!rc && hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) rc = PC2_E_DEVICE;
  }
  if (tmp) (void)hipFree(tmp);
  if (rc) {
    (void)hipDeviceSynchronize();
    for (pc2_matvec* mv : cs->mv) pc2_matvec_destroy(mv);
    if (cs->dev) (void)hipFree(cs->dev);
    delete cs;
    return rc;
  }
  *out = cs;
  return PC2_OK;
}

int pc2_colsplit_set_scale(pc2_colsplit* cs, uint32_t log2_scale, void* hip_stream) {
  if (!cs || !cs->ctx) return PC2_E_INVAL;
  if (!colsplit_scale_ok(cs->sk, cs->Nk, (int)log2_scale)) return PC2_E_UNSUPPORTED;
  if (hipSetDevice(cs->ctx->device) != hipSuccess) return PC2_E_DEVICE;
  int rc = colsplit_quantize(cs, (int)log2_scale, hip_stream);
  if (!rc && hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) rc = PC2_E_DEVICE;
  return rc;
}

int pc2_colsplit_iterate(pc2_colsplit* cs, double lambda, int quantized, double* x, double* z,
                         double* v, void* hip_stream) {
  if (!cs || !cs->ctx || !x || !z || !v || !(lambda >= 0)) return PC2_E_INVAL;
  pc2_ctx* ctx = cs->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  const pc2_sk* sk = cs->sk;
  const pc2_pk* pk = &sk->pk;
  const int Nk = cs->Nk, L = pk->L, k = cs->k;
  const size_t nk = (size_t)Nk, L2 = 2 * (size_t)L, n = (size_t)cs->N;
  int rc = PC2_OK;
  if (quantized) {
    if (cs->mv.size() != (size_t)cs->K) return PC2_E_INVAL;  // a failed change of scale
    // master: Gamma_2(z) and Gamma_2(-v) of every node, encrypted in one launch
    // with the next 2N rows of the randomness pool (after the rows of alpha)
    const size_t span = cs->r_count - 3 * n + 1;
    const size_t base = n + (cs->iter * 2 * n) % span;
    rc = status_of(pc2k::cs_quant_zv(z, v, cs->N, cs->K, k, cs->w, cs->w + n, cs->S, ctx->err,
                                     hip_stream));
    if (!rc) rc = pc2_encrypt(pk, (const uint32_t*)cs->w, 2, cs->r_pool + base * L, cs->cw,
                              2 * n, hip_stream);
    // node k: alpha_k (+) G_k (x) (z_k (+) -v_k)  (eq. (itq2))
    if (!rc) rc = pc2_hom_add(pk, cs->cw, cs->cw + n * L2, cs->c, n, hip_stream);
    for (int kk = 0; kk < cs->K && !rc; ++kk) {
      const size_t k0 = kk * nk;
      rc = pc2_matvec_load(cs->mv[kk], cs->c + k0 * L2, hip_stream);
      if (!rc) rc = pc2_matvec_apply(cs->mv[kk], cs->G + kk * nk * nk, cs->ahat + k0 * L2,
                                     cs->xhat + k0 * L2, nk, hip_stream);
    }
    // master: decrypt every node's result and invert the quantization
    if (!rc) rc = pc2_decrypt(sk, cs->xhat, cs->P, n, hip_stream);
    if (!rc) rc = status_of(pc2k::cs_dequant(cs->P, L, cs->N, cs->K, cs->R, cs->S, k, x,
                                             ctx->err, hip_stream));
  } else {
    for (int kk = 0; kk < cs->K && !rc; ++kk) {
      const size_t k0 = kk * nk;
      rc = status_of(pc2k::cs_plain_node(cs->rhoB + kk * nk * nk, Nk, z + k0, v + k0,
                                         cs->alpha + k0, x + k0, hip_stream));
    }
  }
  if (!rc) rc = status_of(pc2k::cs_update(x, z, v, cs->N, lambda / cs->rho, hip_stream));
  if (!rc) ++cs->iter;
  return rc;
}

int pc2_colsplit_destroy(pc2_colsplit* cs) {
  if (!cs || !cs->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(cs->ctx->device);
  (void)hipDeviceSynchronize();
  for (pc2_matvec* mv : cs->mv) pc2_matvec_destroy(mv);
  if (cs->dev) (void)hipFree(cs->dev);
  delete cs;
  return PC2_OK;
}

// ------------------------------------------------------------------ ADMM
int pc2_admm_create(pc2_ctx* ctx, const double* A, const double* y, uint32_t M, uint32_t N,
                    uint32_t K, double rho, void* hip_stream, pc2_admm** out) {
  if (!ctx || !A || !y || !out || M == 0 || N == 0 || K == 0 || M % K != 0 || !(rho > 0.0))
    return PC2_E_INVAL;
  *out = nullptr;
  const size_t B = M / K;
  if (B > 4096) return PC2_E_UNSUPPORTED;  // the per-node solve keeps B doubles in LDS
  if (hipSetDevice(ctx->device) != hipSuccess) return PC2_E_DEVICE;
  pc2_admm* a = new (std::nothrow) pc2_admm();
  if (!a) return PC2_E_NOMEM;
  const size_t words = K * B * B + 2 * (size_t)K * N + 2 * (size_t)K * B;
  if (hipMalloc(&a->buf, words * sizeof(double)) != hipSuccess) {
    delete a;
    return PC2_E_NOMEM;
  }
  a->ctx = ctx;
  a->A = A;
  a->N = (int)N;
  a->B = (int)B;
  a->K = (int)K;
  a->rho = rho;
  a->W = a->buf;
  a->aty = a->W + K * B * B;
  a->w = a->aty + (size_t)K * N;
  a->t = a->w + (size_t)K * N;
  a->s = a->t + (size_t)K * B;
  if (pc2k::admm_setup(A, y, (int)N, (int)B, (int)K, rho, a->W, a->aty, hip_stream) !=
      hipSuccess) {
    (void)hipFree(a->buf);
    delete a;
    return PC2_E_DEVICE;
  }
  *out = a;
  return PC2_OK;
}

int pc2_admm_local(pc2_admm* a, const double* z, const double* u, double* x, double* xu,
                   void* hip_stream) {
  if (!a || !z || !u || !x || !xu) return PC2_E_INVAL;
  if (hipSetDevice(a->ctx->device) != hipSuccess) return PC2_E_DEVICE;
  return status_of(pc2k::admm_local(a->A, a->W, a->aty, z, u, a->N, a->B, a->K, a->rho, a->w,
                                    a->t, a->s, x, xu, hip_stream));
}

int pc2_admm_consensus(pc2_admm* a, const double* sum, const double* x, double lambda, double* z,
                       double* u, void* hip_stream) {
  if (!a || !sum || !x || !z || !u || !(lambda >= 0.0)) return PC2_E_INVAL;
  if (hipSetDevice(a->ctx->device) != hipSuccess) return PC2_E_DEVICE;
  const double kappa = lambda / (a->rho * a->K);
  return status_of(pc2k::admm_consensus(sum, x, a->N, a->K, kappa, z, u, hip_stream));
}

int pc2_admm_destroy(pc2_admm* a) {
  if (!a || !a->ctx) return PC2_E_INVAL;
  (void)hipSetDevice(a->ctx->device);
  (void)hipDeviceSynchronize();
  if (a->buf) (void)hipFree(a->buf);
  delete a;
  return PC2_OK;
}

}  // extern "C"
