// FP64 kernels of the consensus-lasso ADMM iteration around the encrypted
// aggregation (row-split A over K nodes; Sec. II's x/z/v updates with the
// soft threshold S, in the global-consensus form):
//
//   node k:  w_k = A_k^T y_k + rho (z - u_k)
//            x_k = (1/rho) (w_k - A_k^T W_k^-1 A_k w_k),  W_k = rho I + A_k A_k^T
//            (the Woodbury form of (A_k^T A_k + rho I)^-1 w_k; W_k is B x B)
//   master:  z = S_{lambda/(rho K)}( (1/K) sum_k (x_k + u_k) ),  u_k += x_k - z
//
// All of it is memory-bound on A (M x N doubles, read twice per iteration):
// the GEMVs stream A with coalesced rows (t = A_k w) or columns (v = A_k^T s),
// the B x B Cholesky factors are computed once.  Built with
// -ffp-contract=off; the dot products use explicit fma().
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace {

constexpr int TS = 16;  // Gram tile

// W_k = rho I + A_k A_k^T for the B rows of node k (row-major B x B)
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A, int N, int B,
                                              double rho, double* __restrict__ W) {
  const int k = blockIdx.z;
  const int ti = blockIdx.y * TS, tj = blockIdx.x * TS;
  __shared__ double sa[TS][TS + 1], sb[TS][TS + 1];
  const int ly = threadIdx.x / TS, lx = threadIdx.x % TS;
  const double* Ak = A + (size_t)k * B * N;
  double acc = 0.0;
  for (int c0 = 0; c0 < N; c0 += TS) {
    const int c = c0 + lx;
    sa[ly][lx] = (ti + ly < B && c < N) ? Ak[(size_t)(ti + ly) * N + c] : 0.0;
    sb[ly][lx] = (tj + ly < B && c < N) ? Ak[(size_t)(tj + ly) * N + c] : 0.0;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < TS; ++p) acc = fma(sa[ly][p], sb[lx][p], acc);
    __syncthreads();
  }
  const int i = ti + ly, j = tj + lx;
  if (i < B && j < B) W[((size_t)k * B + i) * B + j] = acc + (i == j ? rho : 0.0);
}

// in-place lower Cholesky of each node's W_k (one workgroup per node)
__global__ __launch_bounds__(256) void k_cholesky(double* __restrict__ W, int B) {
  double* L = W + (size_t)blockIdx.x * B * B;
  __shared__ double diag;
  for (int j = 0; j < B; ++j) {
    if (threadIdx.x == 0) {
      double s = L[(size_t)j * B + j];
      for (int p = 0; p < j; ++p) s = fma(-L[(size_t)j * B + p], L[(size_t)j * B + p], s);
      diag = sqrt(s);
      L[(size_t)j * B + j] = diag;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < B; i += blockDim.x) {
      double s = L[(size_t)i * B + j];
      for (int p = 0; p < j; ++p) s = fma(-L[(size_t)i * B + p], L[(size_t)j * B + p], s);
      L[(size_t)i * B + j] = s / diag;
    }
    __syncthreads();
  }
  // zero the strict upper triangle
  for (int idx = threadIdx.x; idx < B * B; idx += blockDim.x) {
    const int i = idx / B, j = idx % B;
    if (j > i) L[idx] = 0.0;
  }
}

// Aty_k[c] = sum_i A[kB+i][c] y[kB+i]
__global__ __launch_bounds__(256) void k_aty(const double* __restrict__ A,
                                             const double* __restrict__ y, int N, int B, int K,
                                             double* __restrict__ aty) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)K * N) return;
  const int k = (int)(idx / N), c = (int)(idx % N);
  const double* Ak = A + (size_t)k * B * N;
  double s = 0.0;
  for (int i = 0; i < B; ++i) s = fma(Ak[(size_t)i * N + c], y[(size_t)k * B + i], s);
  aty[idx] = s;
}

// w_k = Aty_k + rho (z - u_k)
__global__ __launch_bounds__(256) void k_w(const double* __restrict__ aty,
                                           const double* __restrict__ z,
                                           const double* __restrict__ u, int N, int K, double rho,
                                           double* __restrict__ w) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)K * N) return;
  w[idx] = fma(rho, z[idx % N] - u[idx], aty[idx]);
}

// t_k[i] = sum_c A[kB+i][c] w_k[c]   (one workgroup per (node, row))
__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ A,
                                                const double* __restrict__ w, int N, int B,
                                                double* __restrict__ t) {
  const int row = blockIdx.x;  // global row kB + i
  const int k = row / B;
  const double* a = A + (size_t)row * N;
  const double* wk = w + (size_t)k * N;
  double s = 0.0;
  for (int c = threadIdx.x; c < N; c += blockDim.x) s = fma(a[c], wk[c], s);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) t[row] = red[0];
}

// s_k = W_k^-1 t_k with the Cholesky factor (forward then backward
// substitution, column-oriented, one workgroup per node)
__global__ __launch_bounds__(256) void k_cholsolve(const double* __restrict__ Lall,
                                                   const double* __restrict__ t, int B,
                                                   double* __restrict__ s) {
  const int k = blockIdx.x;
  const double* L = Lall + (size_t)k * B * B;
  extern __shared__ double v[];  // B
  for (int i = threadIdx.x; i < B; i += blockDim.x) v[i] = t[(size_t)k * B + i];
  __syncthreads();
  for (int j = 0; j < B; ++j) {  // L y = t
    const double yj = v[j] / L[(size_t)j * B + j];
    __syncthreads();
    if (threadIdx.x == 0) v[j] = yj;
    for (int i = j + 1 + threadIdx.x; i < B; i += blockDim.x)
      v[i] = fma(-L[(size_t)i * B + j], yj, v[i]);
    __syncthreads();
  }
  for (int j = B - 1; j >= 0; --j) {  // L^T x = y
    const double xj = v[j] / L[(size_t)j * B + j];
    __syncthreads();
    if (threadIdx.x == 0) v[j] = xj;
    for (int i = threadIdx.x; i < j; i += blockDim.x) v[i] = fma(-L[(size_t)j * B + i], xj, v[i]);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < B; i += blockDim.x) s[(size_t)k * B + i] = v[i];
}

// x_k = (w_k - A_k^T s_k)/rho,  xu_k = x_k + u_k
__global__ __launch_bounds__(256) void k_xupdate(const double* __restrict__ A,
                                                 const double* __restrict__ s,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ u, int N, int B,
                                                 int K, double rho, double* __restrict__ x,
                                                 double* __restrict__ xu) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)K * N) return;
  const int k = (int)(idx / N), c = (int)(idx % N);
  const double* Ak = A + (size_t)k * B * N;
  double v = 0.0;
  for (int i = 0; i < B; ++i) v = fma(Ak[(size_t)i * N + c], s[(size_t)k * B + i], v);
  const double xv = (w[idx] - v) / rho;
  x[idx] = xv;
  xu[idx] = xv + u[idx];
}

// z = S_kappa(sum / K), u_k += x_k - z
__global__ __launch_bounds__(256) void k_consensus(const double* __restrict__ sum,
                                                   const double* __restrict__ x, int N, int K,
                                                   double kappa, double* __restrict__ z,
                                                   double* __restrict__ u) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double a = sum[c] / (double)K;
  const double m = fabs(a) - kappa;
  const double zc = m > 0.0 ? copysign(m, a) : 0.0;
  z[c] = zc;
  for (int k = 0; k < K; ++k) {
    const size_t idx = (size_t)k * N + c;
    u[idx] = u[idx] + (x[idx] - zc);
  }
}

inline dim3 blocks_for(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

namespace pc2k {

hipError_t admm_setup(const double* A, const double* y, int N, int B, int K, double rho,
                      double* W, double* aty, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_gram, dim3((B + TS - 1) / TS, (B + TS - 1) / TS, K), dim3(TS * TS), 0, st,
                     A, N, B, rho, W);
  hipLaunchKernelGGL(k_cholesky, dim3(K), dim3(256), 0, st, W, B);
  hipLaunchKernelGGL(k_aty, blocks_for((size_t)K * N), dim3(256), 0, st, A, y, N, B, K, aty);
  return hipGetLastError();
}

hipError_t admm_local(const double* A, const double* Lchol, const double* aty, const double* z,
                      const double* u, int N, int B, int K, double rho, double* w, double* t,
                      double* s, double* x, double* xu, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_w, blocks_for((size_t)K * N), dim3(256), 0, st, aty, z, u, N, K, rho, w);
  hipLaunchKernelGGL(k_rowdot, dim3(K * B), dim3(256), 0, st, A, w, N, B, t);
  hipLaunchKernelGGL(k_cholsolve, dim3(K), dim3(256), B * sizeof(double), st, Lchol, t, B, s);
  hipLaunchKernelGGL(k_xupdate, blocks_for((size_t)K * N), dim3(256), 0, st, A, s, w, u, N, B, K,
                     rho, x, xu);
  return hipGetLastError();
}

hipError_t admm_consensus(const double* sum, const double* x, int N, int K, double kappa,
                          double* z, double* u, void* stream) {
  hipLaunchKernelGGL(k_consensus, blocks_for((size_t)N), dim3(256), 0, (hipStream_t)stream, sum, x,
                     N, K, kappa, z, u);
  return hipGetLastError();
}

}  // namespace pc2k
