// Quantization (Sec. III-A, Gamma_2 in affine form with a power-of-two
// scale) and inverse quantization of an aggregate (Sec. III-C).  Memory-bound
// element-wise kernels: 8 B in + 8 B out per element for quantize.
// Compiled with -ffp-contract=off; with a power-of-two scale both directions
// round exactly once.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "pc2_types.hpp"

namespace {

// x must lie in the common interval [-o, delta - o) / 2^k.  t = x 2^k is
// exact, and for the integer bounds -o <= t < hi (hi = delta - o) holds
// exactly when it holds for floor(t); then rint(t) <= floor(t) + 1 <= hi, so
// m = o + rint(t) lies in {0, ..., delta}.
__global__ __launch_bounds__(256) void k_quantize(int log2_scale, uint64_t offset, uint64_t hi,
                                                  const double* __restrict__ x,
                                                  uint64_t* __restrict__ m, size_t count,
                                                  int* err) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double t = ldexp(x[i], log2_scale);
    const double f = floor(t);
    const double v = rint(t);  // one rounding, half to even
    bool ok = fabs(f) < 18446744073709551616.0;  // false for NaN and infinities
    if (ok) ok = f >= 0.0 ? (uint64_t)f < hi : (uint64_t)(-f) <= offset;
    uint64_t out = 0;
    if (ok) out = v >= 0.0 ? offset + (uint64_t)v : offset - (uint64_t)(-v);
    m[i] = out;
    bad |= !ok;
  }
  if (bad) atomicOr(err, pc2k::ERR_RANGE);
}

__global__ __launch_bounds__(256) void k_dequantize(int log2_scale, uint64_t offset,
                                                    const uint32_t* __restrict__ m, int m_limbs,
                                                    uint64_t weight, double* __restrict__ x,
                                                    size_t count, int* err) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint32_t* mi = m + i * m_limbs;
    uint32_t hi_or = 0;
    for (int j = 2; j < m_limbs; ++j) hi_or |= mi[j];
    uint64_t M = mi[0];
    if (m_limbs > 1) M |= (uint64_t)mi[1] << 32;
    // D = M - W*o as a signed 128-bit integer
    __int128 d = (__int128)(unsigned __int128)M - (__int128)((unsigned __int128)weight * offset);
    const __int128 lim = (__int128)1 << 63;
    bool ok = (hi_or == 0) && (d > -lim) && (d < lim);
    double v = ok ? ldexp((double)(int64_t)d, -log2_scale) : __builtin_nan("");
    x[i] = v;
    bad |= !ok;
  }
  if (bad) atomicOr(err, pc2k::ERR_RANGE);
}

}  // namespace

namespace pc2k {

hipError_t launch_quantize(const Launch& l, int log2_scale, uint64_t offset, uint64_t delta,
                           const double* x, uint64_t* m, size_t count) {
  hipLaunchKernelGGL(k_quantize, dim3(l.grid), dim3(256), 0, (hipStream_t)l.stream, log2_scale,
                     offset, delta - offset, x, m, count, l.err);
  return hipGetLastError();
}

hipError_t launch_dequantize(const Launch& l, int log2_scale, uint64_t offset, const uint32_t* m,
                             int m_limbs, uint64_t weight, double* x, size_t count) {
  hipLaunchKernelGGL(k_dequantize, dim3(l.grid), dim3(256), 0, (hipStream_t)l.stream, log2_scale,
                     offset, m, m_limbs, weight, x, count, l.err);
  return hipGetLastError();
}

}  // namespace pc2k
