// Ciphertext matrix-vector product of the edge-node update (Sec. III-C,
// eq. (itq2)): out_i = alpha_i * prod_j c_j^(B_ij) mod n^2, i.e. Definition 2
// with a matrix of constants followed by Definition 1.
//
// Every row raises the same bases c_j, so the bases get fixed-base tables:
// for column j and window t < nw = ceil(ebits / w),
//     T[j][t][d - 1] = (c_j^(2^(w t)))^d R mod n^2,   d = 1 .. 2^w - 1
// (Montgomery form).  A row then needs one Montgomery product per w-bit digit
// of each of its constants and no squarings: starting from alpha_i in normal
// form, MM(acc, T) = acc * c_j^(d 2^(w t)) stays in normal form.  Digits equal
// to zero multiply by R (the Montgomery one), so the tiles of a wavefront
// never diverge; a wavefront skips a step only when all its tiles have a zero
// digit.
//
// Work mapping (tiles of G::T lanes, as in kernels_paillier.hip):
//   k_mv_table: one tile per (column, window): w t squarings from c_j R, then
//               2^w - 2 products by the window's base, each result stored.
//   k_mv_apply: one tile per (row, column chunk), chunk-major so that the
//               wavefronts in flight read the tables of the same columns;
//               each chunk's partial product goes to staging (or straight
//               to out when there is one chunk), and k_hom_sum multiplies the
//               partials of a row.
// Items are numbered window-major (chunk-major) with the columns (rows)
// padded to whole wavefronts, so every tile of a wavefront runs the same
// sequence of steps (the LDS fences inside the loops are then reached by
// all lanes); padding tiles redo the last real item and store nothing.
// Data errors (c_j >= n^2, alpha_i >= n^2, B_ij >= 2^ebits) latch ERR_RANGE; a
// bad column's tables are zero, so every row that uses it comes out zero, and
// a bad row is written as zero.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "paillier_ops.hpp"

using namespace pc2ops;

namespace {

template <class G>
__global__ __launch_bounds__(64, 2) void k_mv_table(PkConst pk, const uint32_t* __restrict__ c,
                                                    size_t cols, int nw, int w,
                                                    uint32_t* __restrict__ tab, int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const int L2 = 2 * pk.L;
  const int per = (1 << w) - 1;  // table entries per (column, window)
  const size_t gpw = (cols + EPW - 1) / EPW;  // wavefront groups per window
  const size_t ngroups = gpw * (size_t)nw;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    const int t = (int)(gi / gpw);                   // the same in the whole wavefront
    size_t j = (gi % gpw) * EPW + tile;
    const bool live = j < cols;
    if (!live) j = cols - 1;
    const uint32_t* cj = c + j * L2;
    const bool ok = sc_cmp(cj, L2, pk.n2.Nl, L2) < 0;  // the same in every lane of the tile
    uint32_t* dst = tab + (j * nw + t) * (size_t)per * G::CH;
    // step 0: acc = MM(R^2, c_j) = c_j R; steps 1..w t: squarings up to the
    // window's base; then products by the base (kept in LDS): base^2 .. base^per
    const int nsq = w * t;
    uint32_t acc[G::K];
    load_chunk<G>(acc, pk.n2.R2, tl);
    lds_sync();
    lds_digits_from_limbs<G>(lds, cj, L2, 0, tl);
    lds_sync();
    for (int s = 0; s < nsq + per; ++s) {
      if (s >= 1 && s <= nsq + 1) {  // b = the running value: a squaring, or the base from here on
        lds_sync();
        to_lds<G>(lds, acc, tl);
        lds_sync();
      }
      mont_mul<G>(acc, acc, lds, N, np, tl);
      if (s >= nsq && live) {
        uint32_t z[G::K];
#pragma unroll
        for (int k = 0; k < G::K; ++k) z[k] = ok ? acc[k] : 0u;
        store_chunk<G>(dst + (size_t)(s - nsq) * G::CH, z, tl);
      }
    }
    if (live && !ok && tl == 0) atomicOr(err, pc2k::ERR_RANGE);
  }
}

template <class G>
__global__ __launch_bounds__(64, 2) void k_mv_apply(PkConst pk, const uint64_t* __restrict__ B,
                                                    size_t rows, size_t cols, int ebits, int nw,
                                                    int w, const uint32_t* __restrict__ tab,
                                                    const uint32_t* __restrict__ alpha,
                                                    size_t nchunks, size_t chunk_cols,
                                                    uint32_t* __restrict__ out,
                                                    size_t chunk_stride, int* err) {
  constexpr int EPW = 64 / G::T;
  __shared__ __align__(16) uint32_t lds_all[EPW * G::SP];
  const int tl = threadIdx.x & (G::T - 1);
  const int tile = threadIdx.x / G::T;
  uint32_t* lds = lds_all + tile * G::SP;
  uint32_t N[G::K];
  load_chunk<G>(N, pk.n2.N, tl);
  const uint32_t np = pk.n2.nprime;
  const int L2 = 2 * pk.L;
  const size_t per = ((size_t)1 << w) - 1;
  const uint64_t dmask = ((uint64_t)1 << w) - 1;
  const size_t gpc = (rows + EPW - 1) / EPW;  // wavefront groups per chunk
  const size_t ngroups = gpc * nchunks;
  for (size_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    const size_t k = gi / gpc;                         // the same in the whole wavefront
    size_t i = (gi % gpc) * EPW + tile;
    const bool live = i < rows;
    if (!live) i = rows - 1;
    const size_t j0 = k * chunk_cols;
    const size_t j1 = j0 + chunk_cols < cols ? j0 + chunk_cols : cols;
    uint32_t ok = 1;
    uint32_t acc[G::K];
    if (k == 0 && alpha != nullptr) {
      const uint32_t* ai = alpha + i * L2;
      ok = sc_cmp(ai, L2, pk.n2.Nl, L2) < 0;
      lds_sync();
      lds_digits_from_limbs<G>(lds, ai, L2, 0, tl);
      lds_sync();
      from_lds<G>(acc, lds, tl);
    } else {
      load_chunk<G>(acc, pk.n2.ONE, tl);
    }
    const uint64_t* Bi = B + i * cols;
    for (size_t j = j0; j < j1; ++j) {
      const uint64_t e = Bi[j];
      if (ebits < 64 && (e >> ebits) != 0) ok = 0;
      const uint32_t* tj = tab + j * nw * per * G::CH;
      for (int t = 0; t < nw; ++t) {
        const uint32_t d = (uint32_t)((e >> (w * t)) & dmask);
        if (__ballot(d != 0) == 0) continue;  // wave-uniform: no tile has work here
        const uint32_t* b = d ? tj + ((size_t)t * per + d - 1) * G::CH : pk.n2.R1;
        // the running value goes to LDS and the table entry into its
        // registers (one vector load per four digits, all in flight at once)
        lds_sync();
        to_lds<G>(lds, acc, tl);
        lds_sync();
        load_chunk<G>(acc, b, tl);
        mont_mul<G>(acc, acc, lds, N, np, tl);
      }
    }
    lds_sync();
    to_lds<G>(lds, acc, tl);
    lds_sync();
    if (tl == 0) store_canonical<G>(lds, pk.n2, out + k * chunk_stride + i * L2, live, ok, err);
  }
}

#define PC2_MV_DISPATCH(cls, EXPR)         \
  switch (cls) {                           \
    case 0: { constexpr int C = 0; EXPR; } \
    case 1: { constexpr int C = 1; EXPR; } \
    case 2: { constexpr int C = 2; EXPR; } \
    case 3: { constexpr int C = 3; EXPR; } \
    case 4: { constexpr int C = 4; EXPR; } \
    case 5: { constexpr int C = 5; EXPR; } \
    case 6: { constexpr int C = 6; EXPR; } \
    case 7: { constexpr int C = 7; EXPR; } \
    case 8: { constexpr int C = 8; EXPR; } \
  }

}  // namespace

namespace pc2k {

const void* kernel_matvec(int cls, int which) {
  PC2_MV_DISPATCH(cls, {
    using G = typename Geos<C>::Gn;
    return which == 0 ? (const void*)&k_mv_table<G> : (const void*)&k_mv_apply<G>;
  });
  return nullptr;
}

size_t matvec_entry_words(int cls) {
  PC2_MV_DISPATCH(cls, return (size_t)Geos<C>::Gn::CH);
  return 0;
}

hipError_t launch_mv_table(int cls, int grid, const PkConst& pk, const uint32_t* c, size_t cols,
                           int nw, int w, uint32_t* tab, int* err, void* stream) {
  PC2_MV_DISPATCH(cls, {
    hipLaunchKernelGGL((k_mv_table<typename Geos<C>::Gn>), dim3(grid), dim3(64), 0,
                       (hipStream_t)stream, pk, c, cols, nw, w, tab, err);
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}

hipError_t launch_mv_apply(int cls, int grid, const PkConst& pk, const uint64_t* B, size_t rows,
                           size_t cols, int ebits, int nw, int w, const uint32_t* tab,
                           const uint32_t* alpha, size_t nchunks, size_t chunk_cols,
                           uint32_t* out, size_t chunk_stride, int* err, void* stream) {
  PC2_MV_DISPATCH(cls, {
    hipLaunchKernelGGL((k_mv_apply<typename Geos<C>::Gn>), dim3(grid), dim3(64), 0,
                       (hipStream_t)stream, pk, B, rows, cols, ebits, nw, w, tab, alpha,
                       nchunks, chunk_cols, out, chunk_stride, err);
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}

}  // namespace pc2k
