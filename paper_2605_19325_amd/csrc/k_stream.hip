// X-streaming kernels: P = X B, Q = X^T A, the direct residual, ||X||^2 and
// the FP32 -> BF16/FP16 conversion.  These read X (m x n, row-major) once per
// launch; they are the O(mnr) core of every iteration (appendix on
// computational complexity).
//
// Vector-ALU forms, used for every width (matrix-core forms for wide ranks
// live in k_mfma.hip):
//   X B   : one lane per row of X.  A 64-row x 512-byte tile of X is staged
//           through LDS with coalesced 16-byte loads; each lane then reads its
//           own row back and multiplies it with rows of B that are uniform
//           across the wave (scalar loads, one SGPR operand per FMA).
//   X^T A : one lane per column of X; rows of X are read coalesced straight
//           from HBM and the matching row of A is uniform across the wave.
// Both split the contraction over blocks ("split-K") and reduce the float32
// partials in a fixed order, so results do not depend on scheduling.
#include <type_traits>

#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kRows = 64;      // rows of X per X B block (one per lane)
constexpr int kThreads = 256;  // 4 waves
constexpr int kTargetBlocks = 2048;

template <int XT> struct Tile {
  using ET = typename XElem<XT>::T;
  static constexpr int EPV = 16 / sizeof(ET);     // elements per 16-byte vector
  static constexpr int TW = 512 / sizeof(ET);     // tile width in elements (512 bytes per row)
  static constexpr int LDT = TW + EPV;            // padded LDS row (breaks bank aliasing)
  static constexpr int VPR = TW / EPV;            // 32 vectors per tile row
  static constexpr int VPT = kRows * VPR / kThreads;  // 8 vectors per thread per tile
  static constexpr int WCOLS = TW / 4;            // columns per wave per tile
};

template <int XT>
__device__ __forceinline__ void unpack(const uint4& q, float* xs) {
  if constexpr (XT == 0) {
    xs[0] = __uint_as_float(q.x);
    xs[1] = __uint_as_float(q.y);
    xs[2] = __uint_as_float(q.z);
    xs[3] = __uint_as_float(q.w);
  } else {
    const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xs[2 * i] = to_f32<XT>((unsigned short)(w[i] & 0xffffu));
      xs[2 * i + 1] = to_f32<XT>((unsigned short)(w[i] >> 16));
    }
  }
}

// Zero the elements of a 16-byte vector whose column index is >= n.
template <int XT>
__device__ __forceinline__ uint4 mask_tail(uint4 q, int64_t col, int64_t n) {
  using T = Tile<XT>;
  if (col + T::EPV <= n) return q;
  unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int e = 0; e < T::EPV; ++e) {
    if (col + e >= n) {
      if constexpr (XT == 0) w[e] = 0u;
      else w[e / 2] &= (e & 1) ? 0x0000ffffu : 0xffff0000u;
    }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Loads this thread's share of a 64-row x TW-column tile of X.  With
// `vec` (16-byte aligned rows) each share is one 16-byte load; otherwise the
// same vector is assembled from element loads (any leading dimension).
template <int XT>
__device__ __forceinline__ void load_tile(const typename XElem<XT>::T* __restrict__ X, int64_t m,
                                          int64_t n, int64_t ld, int64_t i0, int64_t jt, bool vec,
                                          uint4* vb) {
  using T = Tile<XT>;
  using ET = typename XElem<XT>::T;
#pragma unroll
  for (int u = 0; u < T::VPT; ++u) {
    const int q = threadIdx.x + kThreads * u;
    const int row = q / T::VPR;
    const int vc = q % T::VPR;
    const int64_t col = jt + (int64_t)vc * T::EPV;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i0 + row < m && col < n) {
      const ET* src = X + (i0 + row) * ld + col;
      if (vec) {
        v = mask_tail<XT>(*reinterpret_cast<const uint4*>(src), col, n);
      } else {
        unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < T::EPV; ++e) {
          if (col + e < n) {
            if constexpr (XT == 0) w[e] = __float_as_uint(src[e]);
            else w[e / 2] |= ((unsigned)src[e]) << (16 * (e & 1));
          }
        }
        v = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    vb[u] = v;
  }
}

// Side job of the vector-ALU products: with a Gram job, the grid has one
// more row of workgroups after the split rows, and those combine the previous
// row pass's partial Grams (gram_combine, one wave per group of entries)
// instead of streaming X.  Returns true in those workgroups.
__device__ __forceinline__ bool xv_gram_side(const GramJob& gj) {
  if (gj.src == nullptr || blockIdx.y != gridDim.y - 1) return false;
  gram_combine(gj.src, gj.nparts, gj.kp, gj.dst,
               (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave,
               (int64_t)gridDim.x * (kThreads / kWave));
  return true;
}

// P_part[s] (rows i0..i0+63, k columns) = X[i0.., tiles of split s] * Bp.
// Bp: zero-padded copy of B, KP floats per row, rows up to the tiled width.
template <int XT, int KP>
__global__ __launch_bounds__(kThreads) void k_xv(const void* __restrict__ Xv, int64_t m, int64_t n,
                                                 int64_t ld, const float* __restrict__ Bp, int k,
                                                 int tiles_per_split, int64_t ntiles, int vec,
                                                 float* __restrict__ out, int64_t split_stride,
                                                 GramJob gj) {
  using T = Tile<XT>;
  using ET = typename T::ET;
  constexpr int kTileBytes = kRows * T::LDT * (int)sizeof(ET);
  constexpr int kRedBytes = 2 * kRows * KP * 4;
  constexpr int kSmem = kTileBytes > kRedBytes ? kTileBytes : kRedBytes;
  __shared__ __align__(16) unsigned char smem[kSmem];
  ET* tile = reinterpret_cast<ET*>(smem);
  if (xv_gram_side(gj)) return;

  const ET* __restrict__ X = reinterpret_cast<const ET*>(Xv);
  const int lane = threadIdx.x % kWave;
  const int w = uniform(threadIdx.x / kWave);
  const int64_t i0 = (int64_t)blockIdx.x * kRows;
  const int64_t t0 = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t t1 = t0 + tiles_per_split < ntiles ? t0 + tiles_per_split : ntiles;

  float acc[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) acc[c] = 0.f;

  uint4 vb[T::VPT];
  if (t0 < t1) load_tile<XT>(X, m, n, ld, i0, t0 * T::TW, vec != 0, vb);
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < T::VPT; ++u) {
      const int q = threadIdx.x + kThreads * u;
      *reinterpret_cast<uint4*>(tile + (q / T::VPR) * T::LDT + (q % T::VPR) * T::EPV) = vb[u];
    }
    __syncthreads();
    if (t + 1 < t1) load_tile<XT>(X, m, n, ld, i0, (t + 1) * T::TW, vec != 0, vb);

    const ET* trow = tile + lane * T::LDT + w * T::WCOLS;
    const float* __restrict__ bbase = Bp + (t * T::TW + (int64_t)w * T::WCOLS) * KP;
#pragma unroll
    for (int v = 0; v < T::WCOLS / T::EPV; ++v) {
      const uint4 q = *reinterpret_cast<const uint4*>(trow + v * T::EPV);
      float xs[T::EPV];
      unpack<XT>(q, xs);
#pragma unroll
      for (int e = 0; e < T::EPV; ++e) {
        const float* __restrict__ brow = bbase + (v * T::EPV + e) * KP;
#pragma unroll
        for (int c = 0; c < KP; ++c) acc[c] = fmaf(xs[e], brow[c], acc[c]);
      }
    }
  }

  // Fixed-order reduction of the four waves: (w0 + w2) + (w1 + w3).
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem);   // [2][KP][64]
  if (w >= 2) {
#pragma unroll
    for (int c = 0; c < KP; ++c) red[((w - 2) * KP + c) * kWave + lane] = acc[c];
  }
  __syncthreads();
  if (w < 2) {
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] += red[(w * KP + c) * kWave + lane];
  }
  __syncthreads();
  if (w == 1) {
#pragma unroll
    for (int c = 0; c < KP; ++c) red[c * kWave + lane] = acc[c];
  }
  __syncthreads();
  if (w == 0 && i0 + lane < m) {
    float* o = out + (int64_t)blockIdx.y * split_stride + (i0 + lane) * k;
#pragma unroll
    for (int c = 0; c < KP; ++c)
      if (c < k) o[c] = acc[c] + red[c * kWave + lane];
  }
}

// Q_part[s] (columns j0..j0+255, k values each) = X[rows of split s, j]^T Ap.
template <int XT, int KP>
__global__ __launch_bounds__(kThreads) void k_xtu(const void* __restrict__ Xv, int64_t m, int64_t n,
                                                  int64_t ld, const float* __restrict__ Ap, int k,
                                                  int64_t rows_per_split, float* __restrict__ out,
                                                  int64_t split_stride, GramJob gj) {
  using ET = typename XElem<XT>::T;
  if (xv_gram_side(gj)) return;
  const ET* __restrict__ X = reinterpret_cast<const ET*>(Xv);
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool valid = j < n;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < m ? r0 + rows_per_split : m;
  const int64_t jc = valid ? j : 0;

  float acc[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) acc[c] = 0.f;

  constexpr int U = 8;
  int64_t i = r0;
  for (; i + U <= r1; i += U) {
    float xs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xs[u] = valid ? to_f32<XT>(X[(i + u) * ld + jc]) : 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float* __restrict__ arow = Ap + (i + u) * KP;
#pragma unroll
      for (int c = 0; c < KP; ++c) acc[c] = fmaf(xs[u], arow[c], acc[c]);
    }
  }
  for (; i < r1; ++i) {
    const float x = valid ? to_f32<XT>(X[i * ld + jc]) : 0.f;
    const float* __restrict__ arow = Ap + i * KP;
#pragma unroll
    for (int c = 0; c < KP; ++c) acc[c] = fmaf(x, arow[c], acc[c]);
  }
  if (valid) {
    float* o = out + (int64_t)blockIdx.y * split_stride + j * k;
#pragma unroll
    for (int c = 0; c < KP; ++c)
      if (c < k) o[c] = acc[c];
  }
}

// out[e] = sum_s part[s * stride + e], s in order.
__global__ void k_reduce_splits(const float* __restrict__ part, int splits, int64_t stride,
                                int64_t count, float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = part[e];
    for (int q = 1; q < splits; ++q) s += part[q * stride + e];
    out[e] = s;
  }
}

// out[j][c] = c < k ? in[j][c] : 0, rows j < rows_out (rows >= rows_in are zero).
template <typename TO>
__global__ void k_pad_cols(const float* __restrict__ in, int64_t rows_in, int k, int kp,
                           int64_t rows_out, TO* __restrict__ out) {
  const int64_t count = rows_out * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / kp;
    const int c = (int)(e % kp);
    out[e] = (j < rows_in && c < k) ? (TO)in[j * k + c] : (TO)0;
  }
}

// Direct residual: part[b] = sum over this block's (i, j) of (X_ij - U_i . V_j)^2,
// with the dot products on the float64 matrix cores (v_mfma_f64_16x16x4f64)
// and the squares accumulated in float64.  A wave owns 64 columns (four
// 16 x 16 output tiles) and walks the block's rows 16 at a time: U V^T of a
// 16-row group is KS = ceil(r / 4) steps of 4 for each tile, with the wave's
// V operands held in registers for the whole kernel and the group's U
// operands read from the float64 copy of U (issued once the previous group's
// matrix-core steps are in).  Lane (i, g)
// supplies U[row i][4s + g] and receives the entries in rows g + 4v of each
// tile.  Column i of tile t is column 4i + t of the wave's 64, so a lane's
// four x values of one row are adjacent in memory: one 8-byte (16-bit X) or
// 16-byte (float32 X) load per row, issued one group ahead (vec: rows 16-byte
// aligned).  Groups that reach past the block's rows or the matrix's columns
// load element by element, clamped into the matrix, and add nothing for
// entries outside it.
template <int XT, int KS>
__global__ __launch_bounds__(kThreads) void k_residual_mfma(const void* __restrict__ Xv, int64_t m,
                                                            int64_t n, int64_t ld,
                                                            const double* __restrict__ Ud, int ldu,
                                                            const float* __restrict__ V, int r,
                                                            int64_t rows_per_split, int vec,
                                                            double* __restrict__ part) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ double sh[kThreads / kWave];
  using ET = typename XElem<XT>::T;
  const ET* __restrict__ X = reinterpret_cast<const ET*>(Xv);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  const int64_t col0 = (int64_t)blockIdx.x * kThreads + 64 * w;
  const int64_t jl = col0 + 4 * i;                 // the lane's column in tile 0
  double vb[4][KS];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t j = jl + t;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int c = 4 * q + g;
      vb[t][q] = (j < n && c < r) ? (double)V[j * r + c] : 0.0;
    }
  }
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < m ? r0 + rows_per_split : m;
  const bool cols_in = col0 + 64 <= n;             // wave-uniform
  // x of rows row0 + g + 4v (v = 0..3), columns jl .. jl + 3, kept in storage
  // form until use (float4, or four 16-bit values in a uint2)
  using Raw = typename std::conditional<XT == 0, float4, uint2>::type;
  auto load_x = [&](int64_t row0, Raw (&xs)[4]) {
    if (vec && cols_in && row0 + 16 <= r1) {
      const ET* __restrict__ base = X + (row0 + g) * ld + jl;
#pragma unroll
      for (int v = 0; v < 4; ++v) xs[v] = *reinterpret_cast<const Raw*>(base + 4 * v * ld);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t row = row0 + g + 4 * v;
        row = row < r1 ? row : r1 - 1;
        ET e[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int64_t j = jl + t;
          j = j < n ? j : n - 1;
          e[t] = X[row * ld + j];
        }
        if constexpr (XT == 0) xs[v] = make_float4(e[0], e[1], e[2], e[3]);
        else xs[v] = make_uint2((unsigned)e[0] | ((unsigned)e[1] << 16), (unsigned)e[2] | ((unsigned)e[3] << 16));
      }
    }
  };
  auto elem = [&](const Raw& q, int t) -> double {
    if constexpr (XT == 0) return (double)(t == 0 ? q.x : t == 1 ? q.y : t == 2 ? q.z : q.w);
    else {
      const unsigned h = t < 2 ? q.x : q.y;
      return (double)to_f32<XT>((unsigned short)(t % 2 == 0 ? (h & 0xffffu) : (h >> 16)));
    }
  };
  auto load_u = [&](int64_t row0, double (&u)[KS]) {
    int64_t row = row0 + i;
    row = row < r1 ? row : r1 - 1;
#pragma unroll
    for (int q = 0; q < KS; ++q) u[q] = Ud[row * ldu + 4 * q + g];   // zero past r
  };
  double acc = 0.0;
  Raw xa[4], xb[4];
  double ua[KS];
  if (r0 < r1) {
    load_x(r0, xa);
    load_u(r0, ua);
  }
  for (int64_t row0 = r0; row0 < r1; row0 += 16) {
    const bool more = row0 + 16 < r1;
    if (more) load_x(row0 + 16, xb);
    const bool all_in = cols_in && row0 + 16 <= r1;   // wave-uniform
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      d4 d = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KS; ++q) d = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[q], vb[t][q], d, 0, 0, 0);
      if (all_in) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double e = elem(xa[v], t) - d[v];
          acc = fma(e, e, acc);
        }
      } else {
        const bool colok = jl + t < n;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double e = elem(xa[v], t) - d[v];
          const bool ok = colok && row0 + g + 4 * v < r1;
          acc = ok ? fma(e, e, acc) : acc;
        }
      }
    }
    if (more) {
#pragma unroll
      for (int v = 0; v < 4; ++v) xa[v] = xb[v];
      load_u(row0 + 16, ua);     // after this group's matrix-core steps
    }
  }
  const double tot = block_sum<kThreads>(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// part[b] = sum of x^2 over the rows of block b, accumulated in float64.  The
// block's rows are walked as one row-major range of 16-byte vectors (vec: rows
// 16-byte aligned) or of elements, thread t taking every kThreads-th one with
// four loads in flight; its (row, position) advances without a division.  A
// row whose length is not a whole number of vectors adds its last elements
// separately.
template <int XT>
__global__ __launch_bounds__(kThreads) void k_sumsq(const void* __restrict__ Xv, int64_t m,
                                                    int64_t n, int64_t ld, int64_t rows_per_block,
                                                    int vec, double* __restrict__ part) {
  __shared__ double sh[kThreads / kWave];
  using ET = typename XElem<XT>::T;
  constexpr int EPV = 16 / sizeof(ET);
  const ET* __restrict__ X = reinterpret_cast<const ET*>(Xv);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < m ? r0 + rows_per_block : m;
  // units per row: whole vectors, or elements
  const int64_t nu = vec ? n / EPV : n;
  double acc = 0.0;
  if (nu > 0) {
    int64_t i = r0 + threadIdx.x / nu, p = threadIdx.x % nu;
    while (i < r1) {
      uint4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i < r1) {
          if (vec) {
            q[u] = *reinterpret_cast<const uint4*>(X + i * ld + p * EPV);
          } else {
            const float x = to_f32<XT>(X[i * ld + p]);
            q[u] = make_uint4(__float_as_uint(x), 0u, 0u, 0u);
          }
          p += kThreads;
          while (p >= nu) { p -= nu; ++i; }
        } else {
          q[u] = make_uint4(0u, 0u, 0u, 0u);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (vec) {
          float xs[8];
          unpack<XT>(q[u], xs);
#pragma unroll
          for (int e = 0; e < EPV; ++e) acc = fma((double)xs[e], (double)xs[e], acc);
        } else {
          const double x = (double)__uint_as_float(q[u].x);
          acc = fma(x, x, acc);
        }
      }
    }
  }
  if (vec) {
    const int64_t tail = n - (n / EPV) * EPV;
    if (threadIdx.x < tail)
      for (int64_t i = r0; i < r1; ++i) {
        const double x = (double)to_f32<XT>(X[i * ld + (n / EPV) * EPV + threadIdx.x]);
        acc = fma(x, x, acc);
      }
  }
  const double t = block_sum<kThreads>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[f] = sum_b part[b * stride + f] for f < nfields.  One wave per field:
// lane l adds parts l, l + 64, ... in order (8 loads in flight), then the
// wave sums its lanes (wave_sum_last), so the result does not depend on
// scheduling.
__global__ void k_sum_parts(const double* __restrict__ part, int nparts, int stride, int nfields,
                            double* __restrict__ out) {
  const int f = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x % kWave;
  if (f >= nfields) return;   // whole waves
  double s = 0.0;
  for (int b0 = lane; b0 < nparts; b0 += 8 * kWave) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * kWave;
      v[u] = part[(int64_t)(b < nparts ? b : 0) * stride + f];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u * kWave < nparts) s += v[u];
  }
  s = wave_sum_last(s);
  if (lane == kWave - 1) out[f] = s;
}

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x0040u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__global__ void k_convert(const float* __restrict__ x, int64_t m, int64_t n, int64_t ldi, int to,
                          unsigned short* __restrict__ out, int64_t ldo) {
  const int64_t count = m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    const float v = x[i * ldi + j];
    unsigned short h;
    if (to == ENMF_BF16) {
      h = f32_to_bf16_rne(v);
    } else {
      const _Float16 hv = (_Float16)v;
      __builtin_memcpy(&h, &hv, 2);
    }
    out[i * ldo + j] = h;
  }
}

// XT (n x m, ld ldt) = X^T for X (m x n, ld ld), element type ET (2 or 4
// bytes).  One block moves a 64 x 64 tile through LDS: thread t reads 16
// consecutive elements of input row t / 4 and writes 16 consecutive elements
// of output row t / 4, with 16-byte accesses where the rows allow them.
template <typename ET>
__global__ __launch_bounds__(256) void k_transpose(const ET* __restrict__ X, int64_t m, int64_t n,
                                                   int64_t ld, ET* __restrict__ XT, int64_t ldt,
                                                   int vin, int vout) {
  constexpr int EPV = 16 / sizeof(ET);
  __shared__ ET tile[64][64 + EPV];
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  const int rr = threadIdx.x / 4, seg = 16 * (threadIdx.x % 4);
  {
    const int64_t i = i0 + rr, j = j0 + seg;
    ET v[16];
    if (vin && i < m && j + 16 <= n) {
#pragma unroll
      for (int q = 0; q < 16 / EPV; ++q) {
        const uint4 w = *reinterpret_cast<const uint4*>(X + i * ld + j + q * EPV);
        __builtin_memcpy(&v[q * EPV], &w, 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = (i < m && j + e < n) ? X[i * ld + j + e] : ET(0);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) tile[rr][seg + e] = v[e];
  }
  __syncthreads();
  {
    const int64_t jo = j0 + rr, io = i0 + seg;   // output row jo, columns io ..
    if (jo < n) {
      ET v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = tile[seg + e][rr];
      if (vout && io + 16 <= m) {
#pragma unroll
        for (int q = 0; q < 16 / EPV; ++q) {
          uint4 w;
          __builtin_memcpy(&w, &v[q * EPV], 16);
          *reinterpret_cast<uint4*>(XT + jo * ldt + io + q * EPV) = w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (io + e < m) XT[jo * ldt + io + e] = v[e];
      }
    }
  }
}

int grid_for(int64_t count, int threads = 256, int cap = 8192) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

template <int XT, int KP>
void xv_launch(dim3 grid, const void* X, int64_t m, int64_t n, int64_t ld, const float* Bp, int k,
               int tps, int64_t ntiles, float* out, int64_t stride, hipStream_t s, GramJob gj) {
  const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0) &&
                  ((ld * (int64_t)sizeof(typename XElem<XT>::T)) % 16 == 0);
  hipLaunchKernelGGL((k_xv<XT, KP>), grid, dim3(kThreads), 0, s, X, m, n, ld, Bp, k, tps, ntiles,
                     vec, out, stride, gj);
}

template <int XT, int KP>
void xtu_launch(dim3 grid, const void* X, int64_t m, int64_t n, int64_t ld, const float* Ap, int k,
                int64_t rps, float* out, int64_t stride, hipStream_t s, GramJob gj) {
  hipLaunchKernelGGL((k_xtu<XT, KP>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ap, k, rps, out,
                     stride, gj);
}

template <int XT>
void xv_dispatch_kp(int kp, dim3 grid, const void* X, int64_t m, int64_t n, int64_t ld,
                    const float* Bp, int k, int tps, int64_t ntiles, float* out, int64_t stride,
                    hipStream_t s, GramJob gj) {
  switch (kp) {
    case 8: xv_launch<XT, 8>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
    case 16: xv_launch<XT, 16>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
    case 32: xv_launch<XT, 32>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
    case 48: xv_launch<XT, 48>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
    case 64: xv_launch<XT, 64>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
    default: xv_launch<XT, 80>(grid, X, m, n, ld, Bp, k, tps, ntiles, out, stride, s, gj); break;
  }
}

template <int XT>
void xtu_dispatch_kp(int kp, dim3 grid, const void* X, int64_t m, int64_t n, int64_t ld,
                     const float* Ap, int k, int64_t rps, float* out, int64_t stride,
                     hipStream_t s, GramJob gj) {
  switch (kp) {
    case 8: xtu_launch<XT, 8>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
    case 16: xtu_launch<XT, 16>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
    case 32: xtu_launch<XT, 32>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
    case 48: xtu_launch<XT, 48>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
    case 64: xtu_launch<XT, 64>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
    default: xtu_launch<XT, 80>(grid, X, m, n, ld, Ap, k, rps, out, stride, s, gj); break;
  }
}

template <int XT>
void residual_dispatch(dim3 grid, const void* X, int64_t m, int64_t n, int64_t ld, const double* Ud,
                       int ldu, const float* V, int r, int64_t rps, int vec, double* part, hipStream_t s) {
  switch ((r + 3) / 4) {
    case 1: hipLaunchKernelGGL((k_residual_mfma<XT, 1>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 2: hipLaunchKernelGGL((k_residual_mfma<XT, 2>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 3: hipLaunchKernelGGL((k_residual_mfma<XT, 3>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 4: hipLaunchKernelGGL((k_residual_mfma<XT, 4>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 5: hipLaunchKernelGGL((k_residual_mfma<XT, 5>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 6: hipLaunchKernelGGL((k_residual_mfma<XT, 6>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 7: hipLaunchKernelGGL((k_residual_mfma<XT, 7>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 8: hipLaunchKernelGGL((k_residual_mfma<XT, 8>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    case 9: case 10: case 11: case 12:
      hipLaunchKernelGGL((k_residual_mfma<XT, 12>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
    default:
      hipLaunchKernelGGL((k_residual_mfma<XT, 16>), grid, dim3(kThreads), 0, s, X, m, n, ld, Ud, ldu, V, r, rps, vec, part); return;
  }
}

}  // namespace

int64_t xv_tile_width(int xt) { return xt == ENMF_F32 ? 128 : 256; }

int xv_splits(int64_t m, int64_t n, int xt) {
  const int64_t rb = (m + kRows - 1) / kRows;
  const int64_t nt = (n + xv_tile_width(xt) - 1) / xv_tile_width(xt);
  int64_t s = (kTargetBlocks + rb - 1) / rb;
  if (s > nt) s = nt;
  if (s < 1) s = 1;
  return (int)s;
}

int xtu_splits(int64_t m, int64_t n) {
  const int64_t cb = (n + kThreads - 1) / kThreads;
  int64_t s = (kTargetBlocks + cb - 1) / cb;
  const int64_t smax = (m + 31) / 32;
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t launch_pad_cols(const float* in, int64_t rows, int k, int kp, float* out, hipStream_t s) {
  hipLaunchKernelGGL((k_pad_cols<float>), dim3(grid_for(rows * kp)), dim3(256), 0, s, in, rows, k,
                     kp, rows, out);
  return hipGetLastError();
}

hipError_t launch_pad_rows_cols(const float* in, int64_t rows_in, int k, int kp, int64_t rows_out,
                                float* out, hipStream_t s) {
  hipLaunchKernelGGL((k_pad_cols<float>), dim3(grid_for(rows_out * kp)), dim3(256), 0, s, in,
                     rows_in, k, kp, rows_out, out);
  return hipGetLastError();
}

hipError_t launch_pad_cols_f64(const float* in, int64_t rows, int k, int kp, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL((k_pad_cols<double>), dim3(grid_for(rows * kp)), dim3(256), 0, s, in, rows, k,
                     kp, rows, out);
  return hipGetLastError();
}

// P = X B.  Bp is B zero padded to kp columns and to ntiles*TW rows;
// part must hold splits*m*k floats when splits > 1.
hipError_t launch_xv(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* Bp, int k,
                     int kp, int splits, float* part, float* out, hipStream_t s, int reduce,
                     int* nsplit, const GramJob* gj) {
  const GramJob g = gj != nullptr ? *gj : GramJob();
  const int64_t tw = xv_tile_width(xt);
  const int64_t ntiles = (n + tw - 1) / tw;
  const int tps = (int)((ntiles + splits - 1) / splits);
  const int eff = (int)((ntiles + tps - 1) / tps);
  const int64_t rb = (m + kRows - 1) / kRows;
  float* dst = eff > 1 ? part : out;
  const int64_t stride = m * k;
  dim3 grid((unsigned)rb, (unsigned)(eff + (g.src != nullptr ? 1 : 0)));
  switch (xt) {
    case ENMF_F32: xv_dispatch_kp<0>(kp, grid, X, m, n, ld, Bp, k, tps, ntiles, dst, stride, s, g); break;
    case ENMF_BF16: xv_dispatch_kp<1>(kp, grid, X, m, n, ld, Bp, k, tps, ntiles, dst, stride, s, g); break;
    default: xv_dispatch_kp<2>(kp, grid, X, m, n, ld, Bp, k, tps, ntiles, dst, stride, s, g); break;
  }
  hipError_t e = hipGetLastError();
  if (nsplit) *nsplit = (e == hipSuccess && !reduce) ? (int)eff : 1;
  if (e != hipSuccess || eff <= 1 || !reduce) return e;
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid_for(stride)), dim3(256), 0, s, part, eff, stride,
                     stride, out);
  return hipGetLastError();
}

hipError_t launch_xtu(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* Ap, int k,
                      int kp, int splits, float* part, float* out, hipStream_t s, int reduce,
                     int* nsplit, const GramJob* gj) {
  const GramJob g = gj != nullptr ? *gj : GramJob();
  const int64_t rps = (m + splits - 1) / splits;
  const int eff = (int)((m + rps - 1) / rps);
  const int64_t cb = (n + kThreads - 1) / kThreads;
  float* dst = eff > 1 ? part : out;
  const int64_t stride = n * k;
  dim3 grid((unsigned)cb, (unsigned)(eff + (g.src != nullptr ? 1 : 0)));
  switch (xt) {
    case ENMF_F32: xtu_dispatch_kp<0>(kp, grid, X, m, n, ld, Ap, k, rps, dst, stride, s, g); break;
    case ENMF_BF16: xtu_dispatch_kp<1>(kp, grid, X, m, n, ld, Ap, k, rps, dst, stride, s, g); break;
    default: xtu_dispatch_kp<2>(kp, grid, X, m, n, ld, Ap, k, rps, dst, stride, s, g); break;
  }
  hipError_t e = hipGetLastError();
  if (nsplit) *nsplit = (e == hipSuccess && !reduce) ? (int)eff : 1;
  if (e != hipSuccess || eff <= 1 || !reduce) return e;
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid_for(stride)), dim3(256), 0, s, part, eff, stride,
                     stride, out);
  return hipGetLastError();
}

// Residual partials: Ud is U padded to kp float64 columns (m rows).
hipError_t launch_residual(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const double* Ud,
                           const float* V, int r, double* part, int* nparts, hipStream_t s) {
  // Ud has pad_width(r) columns, zero past r; the kernel reads the first
  // 4 KS of them (4 KS <= pad_width(r) for every r <= 64)
  const int ldu = pad_width(r);
  const int64_t cb = (n + kThreads - 1) / kThreads;
  int64_t sp = (kTargetBlocks + cb - 1) / cb;
  if (sp > m) sp = m;
  if (sp < 1) sp = 1;
  const int64_t rps = (m + sp - 1) / sp;
  sp = (m + rps - 1) / rps;
  dim3 grid((unsigned)cb, (unsigned)sp);
  const int esz = xt == ENMF_F32 ? 4 : 2;
  const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && (ld * esz) % 16 == 0) ? 1 : 0;
  switch (xt) {
    case ENMF_F32: residual_dispatch<0>(grid, X, m, n, ld, Ud, ldu, V, r, rps, vec, part, s); break;
    case ENMF_BF16: residual_dispatch<1>(grid, X, m, n, ld, Ud, ldu, V, r, rps, vec, part, s); break;
    default: residual_dispatch<2>(grid, X, m, n, ld, Ud, ldu, V, r, rps, vec, part, s); break;
  }
  *nparts = (int)(cb * sp);
  return hipGetLastError();
}

hipError_t launch_sumsq_x(const void* X, int xt, int64_t m, int64_t n, int64_t ld, double* part,
                          int* nparts, hipStream_t s) {
  int64_t nb = m < 1024 ? m : 1024;
  if (nb < 1) nb = 1;
  const int64_t rpb = (m + nb - 1) / nb;
  nb = (m + rpb - 1) / rpb;
  const int esz = xt == ENMF_F32 ? 4 : 2;
  const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && (ld * esz) % 16 == 0) ? 1 : 0;
  switch (xt) {
    case ENMF_F32: hipLaunchKernelGGL((k_sumsq<0>), dim3((unsigned)nb), dim3(kThreads), 0, s, X, m, n, ld, rpb, vec, part); break;
    case ENMF_BF16: hipLaunchKernelGGL((k_sumsq<1>), dim3((unsigned)nb), dim3(kThreads), 0, s, X, m, n, ld, rpb, vec, part); break;
    default: hipLaunchKernelGGL((k_sumsq<2>), dim3((unsigned)nb), dim3(kThreads), 0, s, X, m, n, ld, rpb, vec, part); break;
  }
  *nparts = (int)nb;
  return hipGetLastError();
}

hipError_t launch_sum_parts(const double* part, int nparts, int stride, int nfields, double* out,
                            hipStream_t s) {
  if (nfields < 1) return hipSuccess;
  hipLaunchKernelGGL(k_sum_parts, dim3((nfields + 3) / 4), dim3(256), 0, s, part, nparts, stride,
                     nfields, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const void* X, int xt, int64_t m, int64_t n, int64_t ld, void* XT,
                            int64_t ldt, hipStream_t s) {
  const int esz = xt == ENMF_F32 ? 4 : 2;
  const int vin = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && (ld * esz) % 16 == 0) ? 1 : 0;
  const int vout = (reinterpret_cast<uintptr_t>(XT) % 16 == 0 && (ldt * esz) % 16 == 0) ? 1 : 0;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
  if (grid.y > 65535u) return hipErrorInvalidValue;
  if (xt == ENMF_F32)
    hipLaunchKernelGGL((k_transpose<float>), grid, dim3(256), 0, s, reinterpret_cast<const float*>(X),
                       m, n, ld, reinterpret_cast<float*>(XT), ldt, vin, vout);
  else
    hipLaunchKernelGGL((k_transpose<unsigned short>), grid, dim3(256), 0, s,
                       reinterpret_cast<const unsigned short*>(X), m, n, ld,
                       reinterpret_cast<unsigned short*>(XT), ldt, vin, vout);
  return hipGetLastError();
}

hipError_t launch_convert(const float* x, int64_t m, int64_t n, int64_t ldi, int to, void* out,
                          int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(m * n)), dim3(256), 0, s, x, m, n, ldi, to,
                     reinterpret_cast<unsigned short*>(out), ldo);
  return hipGetLastError();
}

}  // namespace enmf
