// Types and load helpers of the bfloat16 matrix-core products (gfx950,
// v_mfma_f32_16x16x32_bf16), shared by the streaming product kernels and the
// serving kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace enmf {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

__device__ __forceinline__ bf16x8 as_bf16x8(const uint4& q) { return __builtin_bit_cast(bf16x8, q); }

// Zero the elements of a vector of E elements starting at column col that are >= n.
template <typename ET>
__device__ __forceinline__ uint4 mask_cols(uint4 q, int64_t col, int64_t n) {
  constexpr int E = 16 / sizeof(ET);
  if (col + E <= n) return q;
  unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (col + e >= n) {
      if constexpr (sizeof(ET) == 4) w[e] = 0u;
      else w[e / 2] &= (e & 1) ? 0x0000ffffu : 0xffff0000u;
    }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// 16 bytes of row `row` of X starting at column col (zero outside the matrix).
template <typename ET>
__device__ __forceinline__ uint4 load16(const ET* __restrict__ X, int64_t rows, int64_t n,
                                        int64_t ld, int64_t row, int64_t col, bool vec) {
  constexpr int E = 16 / sizeof(ET);
  if (row >= rows || col >= n) return make_uint4(0u, 0u, 0u, 0u);
  const ET* src = X + row * ld + col;
  if (vec) return mask_cols<ET>(*reinterpret_cast<const uint4*>(src), col, n);
  unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (col + e < n) {
      if constexpr (sizeof(ET) == 4) w[e] = __float_as_uint(src[e]);
      else w[e / 2] |= ((unsigned)src[e]) << (16 * (e & 1));
    }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Unconditional 16-byte load (interior chunks: no data-dependent masking, so
// the loads stay in flight until their first use).
template <typename ET>
__device__ __forceinline__ uint4 ldg16(const ET* p) { return *reinterpret_cast<const uint4*>(p); }

// The same, marked non-temporal, for X^T A's loads of X: each wave's loads
// cover whole cache lines of a row run, X is streamed once per product, and
// the hint leaves the caches to the factor chunks that every block re-reads.
// (X B's operand-layout loads take half lines, whose other halves another
// load reads later, so they keep the plain form.)
template <typename ET>
__device__ __forceinline__ uint4 ldg16_nt(const ET* p) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

}  // namespace enmf
