// Float64 and integer kernels around the encrypted node step of the
// column-split 3P-ADMM-PC2 iteration (Algorithm 1; Sec. II eqs. (sldi231),
// (sldo34), (iu43); quantization Sec. III-A; node step eq. (itq2); inverse
// quantization Sec. III-C with the N > 1 cross terms).
//
// Setup of node k (columns k0 .. k0 + Nk - 1 of A):
//   k_cs_gram        T = [A_k^T A_k + rho I | I]   (rows of A summed in order)
//   k_cs_gj_pivot/update   Gauss-Jordan on T, pivots in order, no exchanges
//   k_cs_aty, k_cs_matvec  alpha_k = B_k (A_k^T y)  (sums in index order)
//   k_cs_rhob        rho B_k
// Quantization of node k at scale 2^k (at setup, and again on a change of scale):
//   k_cs_quant_g     G = Gamma_2(rho B_k) = rint(rho B 2^k) + 2^(k+3)
//   k_cs_rowsum      R_i = sum_j G_ij
//   k_cs_gamma1      Gamma_1(alpha) = rint(alpha 2^(2k)) + 2^(2k+3), 4 limbs
// Per iteration (all nodes at once; node of element i = i / Nk):
//   k_cs_quant_zv    W_z = Gamma_2(z), W_v = Gamma_2(-v)
//   k_cs_sumw        S_k = sum_{j in node k} (W_z + W_v)_j   (one workgroup per node)
//   k_cs_dequant     x_i = float64(P_i - o1 - 2 o R_i - o S_k + 2 Nk o^2) 2^(-2k)
//   k_cs_plain_node  x_k = alpha_k + (rho B_k)(z_k - v_k)   (unquantized)
//   k_cs_update      z = S_{lambda/rho}(v + x), v = v + x - z
// The file is compiled without floating-point contraction, so every sum and
// product rounds separately in the order written; the sums run over indices
// in ascending order.  Quantities outside [-8, 8) latch ERR_RANGE and
// quantize to zero.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "launch.hpp"

namespace {

constexpr int ZLOG2 = 3;  // common quantization interval [-2^3, 2^3)

__device__ __forceinline__ bool in_range(double u) {
  return u >= -(double)(1 << ZLOG2) && u < (double)(1 << ZLOG2);
}

__global__ void k_cs_gram(const double* __restrict__ A, int M, int N, int k0, int Nk, double rho,
                          double* __restrict__ T) {
  const size_t W = 2 * (size_t)Nk;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)Nk * W) return;
  const int i = (int)(idx / W), j = (int)(idx % W);
  double out;
  if (j < Nk) {
    double acc = 0.0;
    for (int m = 0; m < M; ++m)
      acc = acc + A[(size_t)m * N + k0 + i] * A[(size_t)m * N + k0 + j];
    if (i == j) acc = acc + rho;
    out = acc;
  } else {
    out = (j - Nk == i) ? 1.0 : 0.0;
  }
  T[idx] = out;
}

// rp = row p / T[p][p]; f = column p (before this pivot's update)
__global__ void k_cs_gj_pivot(const double* __restrict__ T, int Nk, int p, double* __restrict__ rp,
                              double* __restrict__ f) {
  const int W = 2 * Nk;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < W) rp[t] = T[(size_t)p * W + t] / T[(size_t)p * W + p];
  if (t < Nk) f[t] = T[(size_t)t * W + p];
}

// every row i != p: T[i][j] -= f[i] rp[j]; row p: rp.  Columns left of p
// hold zero in the pivot row, so they are left as they are.
__global__ void k_cs_gj_update(double* __restrict__ T, int Nk, int p, const double* __restrict__ rp,
                               const double* __restrict__ f) {
  const int W = 2 * Nk, span = W - p;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)Nk * span) return;
  const int i = (int)(idx / span), j = p + (int)(idx % span);
  double* e = T + (size_t)i * W + j;
  *e = (i == p) ? rp[j] : *e - f[i] * rp[j];
}

__global__ void k_cs_aty(const double* __restrict__ A, const double* __restrict__ y, int M, int N,
                         int k0, int Nk, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  double acc = 0.0;
  for (int m = 0; m < M; ++m) acc = acc + A[(size_t)m * N + k0 + i] * y[m];
  out[i] = acc;
}

// out_i = (add ? add_i + s_i : s_i), s_i = sum_j Bm[i][j] x_j (ld: row stride)
__global__ void k_cs_matvec(const double* __restrict__ Bm, size_t ld, int Nk,
                            const double* __restrict__ x, const double* __restrict__ add,
                            double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  double acc = 0.0;
  for (int j = 0; j < Nk; ++j) acc = acc + Bm[(size_t)i * ld + j] * x[j];
  out[i] = add ? add[i] + acc : acc;
}

// rho B (from the right half of T)
__global__ void k_cs_rhob(const double* __restrict__ T, int Nk, double rho,
                          double* __restrict__ rhoB) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)Nk * Nk) return;
  const size_t i = idx / Nk, j = idx % Nk;
  rhoB[idx] = rho * T[i * 2 * Nk + Nk + j];
}

// G = Gamma_2(rho B)
__global__ void k_cs_quant_g(const double* __restrict__ rhoB, size_t count, int k,
                             uint64_t* __restrict__ G, int* err) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const double u = rhoB[idx];
  const bool ok = in_range(u);
  G[idx] = ok ? (uint64_t)((int64_t)rint(ldexp(u, k)) + ((int64_t)1 << (k + ZLOG2))) : 0;
  if (!ok) atomicOr(err, pc2k::ERR_RANGE);
}

__global__ void k_cs_rowsum(const uint64_t* __restrict__ G, int Nk, uint64_t* __restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  uint64_t s = 0;
  for (int j = 0; j < Nk; ++j) s += G[(size_t)i * Nk + j];
  R[i] = s;
}

// Gamma_1(alpha) as 4 little-endian 32-bit limbs.  rint(alpha 2^(2k)) is an
// integer-valued double; its exact value is mantissa x 2^e.
__global__ void k_cs_gamma1(const double* __restrict__ alpha, int Nk, int k,
                            uint32_t* __restrict__ out, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  const double u = alpha[i];
  const bool ok = in_range(u);
  __int128 v = 0;
  if (ok) {
    const double d = rint(ldexp(u, 2 * k));
    int e = 0;
    const double fr = frexp(fabs(d), &e);            // |d| = fr 2^e, fr in [0.5, 1)
    const int64_t mant = (int64_t)ldexp(fr, 53);     // exact: 53 significant bits
    const int sh = e - 53;
    __int128 mag = sh >= 0 ? ((__int128)mant << sh) : (__int128)(mant >> (-sh));
    v = (d < 0 ? -mag : mag) + ((__int128)1 << (2 * k + ZLOG2));
  } else {
    atomicOr(err, pc2k::ERR_RANGE);
  }
  const unsigned __int128 w = (unsigned __int128)v;
  for (int l = 0; l < 4; ++l) out[(size_t)i * 4 + l] = (uint32_t)(w >> (32 * l));
}

__global__ void k_cs_quant_zv(const double* __restrict__ z, const double* __restrict__ v, int N,
                              int k, uint64_t* __restrict__ wz, uint64_t* __restrict__ wv,
                              int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t o = (int64_t)1 << (k + ZLOG2);
  const double a = z[i], b = -v[i];
  const bool ok = in_range(a) && in_range(b);
  wz[i] = ok ? (uint64_t)((int64_t)rint(ldexp(a, k)) + o) : 0;
  wv[i] = ok ? (uint64_t)((int64_t)rint(ldexp(b, k)) + o) : 0;
  if (!ok) atomicOr(err, pc2k::ERR_RANGE);
}

// one workgroup of 256 lanes per node
__global__ void k_cs_sumw(const uint64_t* __restrict__ wz, const uint64_t* __restrict__ wv, int Nk,
                          uint64_t* __restrict__ S) {
  __shared__ uint64_t part[256];
  const size_t k0 = (size_t)blockIdx.x * Nk;
  uint64_t s = 0;
  for (int i = threadIdx.x; i < Nk; i += blockDim.x) s += wz[k0 + i] + wv[k0 + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) S[blockIdx.x] = part[0];
}

// signed 128-bit integer -> double, rounded to nearest, ties to even
__device__ __forceinline__ double i128_to_double(__int128 x) {
  const bool neg = x < 0;
  unsigned __int128 u = neg ? (unsigned __int128)(-x) : (unsigned __int128)x;
  const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
  const int nb = hi ? 128 - __clzll((long long)hi) : (lo ? 64 - __clzll((long long)lo) : 0);
  double r;
  if (nb <= 53) {
    r = (double)lo;  // exact
  } else {
    const int sh = nb - 53;
    uint64_t mant = (uint64_t)(u >> sh);
    const unsigned __int128 rem = u & ((((unsigned __int128)1) << sh) - 1);
    const unsigned __int128 half = ((unsigned __int128)1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) ++mant;  // may reach 2^53: still exact
    r = ldexp((double)mant, sh);
  }
  return neg ? -r : r;
}

// x_i = float64(P_i - o1 - 2 o R_i - o S + 2 Nk o^2) 2^(-2k), o = 2^(k+3),
// o1 = 2^(2k+3); P: decrypted plaintexts, L limbs (values must fit 127 bits)
__global__ void k_cs_dequant(const uint32_t* __restrict__ P, int L, int N, int Nk,
                             const uint64_t* __restrict__ R, const uint64_t* __restrict__ S,
                             int k, double* __restrict__ x, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t* p = P + (size_t)i * L;
  bool ok = (p[3] >> 31) == 0;
  for (int l = 4; l < L; ++l) ok &= p[l] == 0;
  unsigned __int128 pu = 0;
  for (int l = 3; l >= 0; --l) pu = (pu << 32) | p[l];
  const __int128 X = (__int128)pu - ((__int128)1 << (2 * k + ZLOG2)) -
                     ((__int128)R[i] << (k + ZLOG2 + 1)) - ((__int128)S[i / Nk] << (k + ZLOG2)) +
                     ((__int128)Nk << (2 * k + 2 * ZLOG2 + 1));
  x[i] = ok ? ldexp(i128_to_double(X), -2 * k) : __builtin_nan("");
  if (!ok) atomicOr(err, pc2k::ERR_RANGE);
}

__global__ void k_cs_plain_node(const double* __restrict__ rhoB, int Nk,
                                const double* __restrict__ z, const double* __restrict__ v,
                                const double* __restrict__ alpha, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  double acc = 0.0;
  for (int j = 0; j < Nk; ++j) acc = acc + rhoB[(size_t)i * Nk + j] * (z[j] - v[j]);
  x[i] = alpha[i] + acc;
}

__global__ void k_cs_update(const double* __restrict__ x, double* __restrict__ z,
                            double* __restrict__ v, int N, double kappa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double t = v[i] + x[i];
  const double zn = t > kappa ? t - kappa : (t < -kappa ? t + kappa : 0.0);
  z[i] = zn;
  v[i] = t - zn;
}

inline unsigned blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

namespace pc2k {

hipError_t cs_setup_node(const double* A, const double* y, int M, int N, int k0, int Nk,
                         double rho, double* T, double* rp, double* f, double* aty,
                         double* alpha, double* rhoB, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t nt = (size_t)Nk * 2 * Nk;
  hipLaunchKernelGGL(k_cs_gram, dim3(blocks(nt, 256)), dim3(256), 0, s, A, M, N, k0, Nk, rho, T);
  for (int p = 0; p < Nk; ++p) {
    hipLaunchKernelGGL(k_cs_gj_pivot, dim3(blocks(2 * (size_t)Nk, 256)), dim3(256), 0, s, T,
                       Nk, p, rp, f);
    const size_t nu = (size_t)Nk * (2 * Nk - p);
    hipLaunchKernelGGL(k_cs_gj_update, dim3(blocks(nu, 256)), dim3(256), 0, s, T, Nk, p, rp, f);
  }
  hipLaunchKernelGGL(k_cs_aty, dim3(blocks(Nk, 256)), dim3(256), 0, s, A, y, M, N, k0, Nk, aty);
  hipLaunchKernelGGL(k_cs_matvec, dim3(blocks(Nk, 256)), dim3(256), 0, s, T + Nk,
                     2 * (size_t)Nk, Nk, aty, (const double*)nullptr, alpha);
  hipLaunchKernelGGL(k_cs_rhob, dim3(blocks((size_t)Nk * Nk, 256)), dim3(256), 0, s, T, Nk, rho,
                     rhoB);
  return hipGetLastError();
}

hipError_t cs_quantize_node(const double* rhoB, const double* alpha, int Nk, int k, uint64_t* G,
                            uint64_t* R, uint32_t* g1, int* err, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t nn = (size_t)Nk * Nk;
  hipLaunchKernelGGL(k_cs_quant_g, dim3(blocks(nn, 256)), dim3(256), 0, s, rhoB, nn, k, G, err);
  hipLaunchKernelGGL(k_cs_rowsum, dim3(blocks(Nk, 256)), dim3(256), 0, s, G, Nk, R);
  hipLaunchKernelGGL(k_cs_gamma1, dim3(blocks(Nk, 256)), dim3(256), 0, s, alpha, Nk, k, g1, err);
  return hipGetLastError();
}

hipError_t cs_quant_zv(const double* z, const double* v, int N, int K, int k, uint64_t* wz,
                       uint64_t* wv, uint64_t* S, int* err, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_cs_quant_zv, dim3(blocks(N, 256)), dim3(256), 0, s, z, v, N, k, wz, wv,
                     err);
  hipLaunchKernelGGL(k_cs_sumw, dim3(K), dim3(256), 0, s, wz, wv, N / K, S);
  return hipGetLastError();
}

hipError_t cs_dequant(const uint32_t* P, int L, int N, int K, const uint64_t* R,
                      const uint64_t* S, int k, double* x, int* err, void* stream) {
  hipLaunchKernelGGL(k_cs_dequant, dim3(blocks(N, 256)), dim3(256), 0, (hipStream_t)stream, P,
                     L, N, N / K, R, S, k, x, err);
  return hipGetLastError();
}

hipError_t cs_plain_node(const double* rhoB, int Nk, const double* z, const double* v,
                         const double* alpha, double* x, void* stream) {
  hipLaunchKernelGGL(k_cs_plain_node, dim3(blocks(Nk, 256)), dim3(256), 0, (hipStream_t)stream,
                     rhoB, Nk, z, v, alpha, x);
  return hipGetLastError();
}

hipError_t cs_update(const double* x, double* z, double* v, int N, double kappa, void* stream) {
  hipLaunchKernelGGL(k_cs_update, dim3(blocks(N, 256)), dim3(256), 0, (hipStream_t)stream, x, z,
                     v, N, kappa);
  return hipGetLastError();
}

}  // namespace pc2k
