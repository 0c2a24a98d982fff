// Device helpers shared by the libenmf kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace enmf {

constexpr int kWave = 64;

__device__ __forceinline__ float bf16_bits_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

__device__ __forceinline__ float f16_bits_to_f32(unsigned short h) {
  _Float16 v;
  __builtin_memcpy(&v, &h, 2);
  return (float)v;
}

// Element type of X for storage code XT (0 float32, 1 bfloat16, 2 float16).
template <int XT> struct XElem { using T = unsigned short; };
template <> struct XElem<0> { using T = float; };

template <int XT>
__device__ __forceinline__ float to_f32(typename XElem<XT>::T v) {
  if constexpr (XT == 0) return v;
  else if constexpr (XT == 1) return bf16_bits_to_f32(v);
  else return f16_bits_to_f32(v);
}

// bfloat16 bits of x, rounded to nearest even (NaN stays NaN).
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Eight consecutive factor rows of one column, split into three bfloat16
// terms (hi = rne(v), mid = rne(v - hi), lo = rne(v - hi - mid)), stored as
// one 16-byte run per term at dst, dst + term_stride, dst + 2 term_stride
// (the transposed split-chunk layout of the matrix-core products).
__device__ __forceinline__ void store_split_run8(const float (&v)[8], unsigned short* dst,
                                                 int64_t term_stride) {
  unsigned h[4], md[4], lw[4];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const unsigned short hi = bf16_rne(v[u]);
    const float r1 = v[u] - __uint_as_float((unsigned)hi << 16);
    const unsigned short mid = bf16_rne(r1);
    const unsigned short lo = bf16_rne(r1 - __uint_as_float((unsigned)mid << 16));
    if ((u & 1) == 0) {
      h[u / 2] = hi; md[u / 2] = mid; lw[u / 2] = lo;
    } else {
      h[u / 2] |= (unsigned)hi << 16; md[u / 2] |= (unsigned)mid << 16; lw[u / 2] |= (unsigned)lo << 16;
    }
  }
  *reinterpret_cast<uint4*>(dst) = make_uint4(h[0], h[1], h[2], h[3]);
  *reinterpret_cast<uint4*>(dst + term_stride) = make_uint4(md[0], md[1], md[2], md[3]);
  *reinterpret_cast<uint4*>(dst + 2 * term_stride) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// Butterfly sum over the 64 lanes of a wave; every lane gets the same value
// and the combination order does not depend on scheduling.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// (ti, tj), ti <= tj, of upper-triangle tile `task` of an ntile x ntile
// grid of 4x4 tiles, numbered row by row.
__device__ __forceinline__ void upper_tile(int task, int ntile, int& ti, int& tj) {
  int i = 0, rem = task;
  while (rem >= ntile - i) { rem -= ntile - i; ++i; }
  ti = i;
  tj = i + rem;
}

// v moved across lanes by the data-parallel-primitive pattern CTRL (a
// v_mov_b32_dpp pair); lanes of rows outside ROWMASK keep `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v, double old) {
  const long long vi = __double_as_longlong(v), oi = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)vi, CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(vi >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Reduction (KIND 0 sum, 1 max, 2 min) over the 64 lanes of a wave in a
// fixed order, all in registers: pairs (quad_perm 1,0,3,2), pairs of pairs
// (quad_perm 2,3,0,1), the two quads of each half row (row_half_mirror), the
// two halves of each row (row_mirror), then row 0 into row 1 and row 2 into
// row 3 (row_bcast:15) and rows 0-1 into rows 2-3 (row_bcast:31); rows left
// out of a broadcast take the identity.  The result is valid in lane 63.
// Every lane of the wave must be active.
template <int KIND>
__device__ __forceinline__ double wave_reduce_last(double x) {
  auto op = [](double a, double b) { return KIND == 1 ? fmax(a, b) : (KIND == 2 ? fmin(a, b) : a + b); };
  x = op(x, dpp_move<0xB1, 0xF>(x, x));
  x = op(x, dpp_move<0x4E, 0xF>(x, x));
  x = op(x, dpp_move<0x141, 0xF>(x, x));
  x = op(x, dpp_move<0x140, 0xF>(x, x));
  x = op(x, dpp_move<0x142, 0xA>(x, KIND == 0 ? 0.0 : x));
  x = op(x, dpp_move<0x143, 0xC>(x, KIND == 0 ? 0.0 : x));
  return x;
}

__device__ __forceinline__ double wave_sum_last(double x) { return wave_reduce_last<0>(x); }

// out (kp x kp, symmetric, float64) = sum of nparts partial Grams, each the
// upper 4x4 tiles of one row block (16 doubles per tile, tiles in upper_tile
// order).  One wave per group of 4 consecutive entries (a 32-byte run of
// each part): lane l adds parts l, l + 64, ... in order (4 parts, 8 loads, in
// flight at a time), then the wave combines each entry (wave_sum_last).
// The calling wave takes groups wave, wave + nwaves, ...
__device__ __forceinline__ void gram_combine(const double* __restrict__ gpart, int nparts, int kp,
                                             double* __restrict__ out, int64_t wave,
                                             int64_t nwaves) {
  const int ntile = kp / 4;
  const int ne = 16 * (ntile * (ntile + 1) / 2);
  const int lane = threadIdx.x % kWave;
  for (int64_t q = wave; 4 * q < ne; q += nwaves) {
    const int64_t e0 = 4 * q;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b0 = lane; b0 < nparts; b0 += 4 * kWave) {
      double2 v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u * kWave;
        const double2* src = reinterpret_cast<const double2*>(gpart + (int64_t)(b < nparts ? b : 0) * ne + e0);
        v[u][0] = src[0];
        v[u][1] = src[1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (b0 + u * kWave < nparts) {
          s[0] += v[u][0].x;
          s[1] += v[u][0].y;
          s[2] += v[u][1].x;
          s[3] += v[u][1].y;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = wave_sum_last(s[c]);
    if (lane == kWave - 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t e = e0 + c;
        int ti, tj;
        upper_tile((int)(e / 16), ntile, ti, tj);
        const int ii = 4 * ti + (int)(e % 16) / 4, jj = 4 * tj + (int)(e % 4);
        out[ii * kp + jj] = s[c];
        out[jj * kp + ii] = s[c];
      }
    }
  }
}


// Fixed-order block reductions for blocks of NT threads (NT a multiple of 64,
// every thread active): wave_reduce_last in each wave, then the waves' values
// in wave order.  `sh` must hold NT/64 doubles.  The result is valid in every
// thread.
template <int KIND, int NT>
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  v = wave_reduce_last<KIND>(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x % kWave) == kWave - 1) sh[w] = v;
  __syncthreads();
  double t = sh[0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i)
    t = KIND == 1 ? fmax(t, sh[i]) : (KIND == 2 ? fmin(t, sh[i]) : t + sh[i]);
  return t;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) { return block_reduce<0, NT>(v, sh); }

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) { return block_reduce<1, NT>(v, sh); }

template <int NT>
__device__ __forceinline__ double block_min(double v, double* sh) { return block_reduce<2, NT>(v, sh); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

}  // namespace enmf
