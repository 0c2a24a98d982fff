// Exterior nonnegative matrix completion (the appendix "Exterior NMC
// algorithm"): the masked products of fhat = 1/2 ||M o (X - U V^T)||_F^2 on a
// bit mask of the observed entries, the masked PBCD row step, the
// softImpute-ALS step and the check of the masked problem.
//
// X is float32, row-major (ld >= n).  The mask is one bit per entry, row
// major: bit (j % 32) of word bits[i * ldm + j / 32] is set when X[i][j] is
// observed.  The factors U (m x r) and V (n x r) are float32 row-major.
//
// The masked residual products stream X in 64 x 64 tiles with both factor
// tiles in LDS: S = U V^T of the tile (each thread a 4 x 4 block, r
// multiply-adds per entry), E = M o (X - S), then E V (rows) or E^T U
// (columns) accumulated over the tiles of the block's contraction range, in
// tile order, float32 accumulate.  Contraction ranges are split over blocks;
// the consumer sums the partials in split order.
#include "dev_common.h"
#include "enmf_internal.h"
#include "row_team.h"

namespace enmf {

namespace {

constexpr int kEt = 256;    // threads per block
constexpr int kTile = 64;   // rows and columns of an X tile
constexpr int kTp = kTile + 4;

// Observed bits of X[row][col .. col + 3] (col a multiple of 4, col < n).
__device__ __forceinline__ unsigned mask4(const uint32_t* __restrict__ bits, int64_t ldm,
                                          int64_t row, int64_t col) {
  return (bits[row * ldm + (col >> 5)] >> (col & 31)) & 0xFu;
}

// Rows [t0, t0 + 64) of a rows x r factor into sT[k][row] (and sR[row][k]),
// zero outside.
template <int KP>
__device__ __forceinline__ void stage_factor(const float* __restrict__ F, int64_t nrows, int r,
                                             int64_t t0, float (*sT)[kTp], float (*sR)[KP + 4]) {
  for (int e = threadIdx.x; e < kTile * KP; e += kEt) {
    const int row = e / KP, k = e % KP;
    const int64_t gr = t0 + row;
    const float v = (gr < nrows && k < r) ? F[gr * r + k] : 0.f;
    sT[k][row] = v;
    if (sR != nullptr) sR[row][k] = v;
  }
}

// g = M_A+ o grad for rows [t0, t0 + 64): grad = -(sum of the nsplit
// partials of R, in split order) and M_A+ = (A >= 0); into sT[k][row].
template <int KP>
__device__ __forceinline__ void stage_grad(const float* __restrict__ A, const float* __restrict__ Rp,
                                           int nsplit, int64_t pstride, int64_t nrows, int r,
                                           int64_t t0, float (*sT)[kTp]) {
  for (int e = threadIdx.x; e < kTile * KP; e += kEt) {
    const int row = e / KP, k = e % KP;
    const int64_t gr = t0 + row;
    float g = 0.f;
    if (gr < nrows && k < r) {
      const int64_t o = gr * r + k;
      float R = Rp[o];
      for (int s = 1; s < nsplit; ++s) R += Rp[s * pstride + o];
      g = A[o] >= 0.f ? -R : 0.f;
    }
    sT[k][row] = g;
  }
}

// X[row][col .. col + 3] and its observed bits (zero and unobserved outside X).
__device__ __forceinline__ void load_block_row(const float* __restrict__ X, int64_t m, int64_t n,
                                               int64_t ld, bool vec,
                                               const uint32_t* __restrict__ bits, int64_t ldm,
                                               int64_t row, int64_t col, float* x, unsigned& mb) {
  x[0] = x[1] = x[2] = x[3] = 0.f;
  mb = 0u;
  if (row >= m || col >= n) return;
  const float* p = X + row * ld + col;
  if (vec && col + 4 <= n) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (col + b < n) x[b] = p[b];
  }
  const int64_t left = n - col;
  mb = mask4(bits, ldm, row, col) & (left >= 4 ? 0xFu : ((1u << left) - 1u));
}

// Masked residual products.  COLS = 0: out (m x r) = (M o (X - U V^T)) V, one
// block per 64-row tile and range of column tiles.  COLS = 1: out (n x r) =
// (M o (X - U V^T))^T U, one block per 64-column tile and range of row tiles.
// rss (optional): per block, sum of the squared masked residuals.
template <int KP, int COLS>
__global__ __launch_bounds__(kEt) void k_mres(const float* __restrict__ X, int64_t m, int64_t n,
                                              int64_t ld, int vec, const uint32_t* __restrict__ bits,
                                              int64_t ldm, const float* __restrict__ U,
                                              const float* __restrict__ V, int r,
                                              int tiles_per_split, float* __restrict__ out,
                                              int64_t out_stride, double* __restrict__ rss) {
  constexpr int KPT = KP / 16;
  __shared__ __align__(16) float sUt[KP][kTp];
  __shared__ __align__(16) float sVt[KP][kTp];
  __shared__ __align__(16) float sF[kTile][KP + 4];
  __shared__ __align__(16) float sE[kTile][kTp];
  __shared__ double sh[kEt / kWave];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int64_t ntile_r = (m + kTile - 1) / kTile, ntile_c = (n + kTile - 1) / kTile;
  const int64_t ot = blockIdx.x;
  const int64_t cb = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t ctiles = COLS ? ntile_r : ntile_c;
  const int64_t ce = cb + tiles_per_split < ctiles ? cb + tiles_per_split : ctiles;
  if (COLS) stage_factor<KP>(V, n, r, ot * kTile, sVt, nullptr);
  else stage_factor<KP>(U, m, r, ot * kTile, sUt, nullptr);
  float acc[4][KPT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < KPT; ++q) acc[a][q] = 0.f;
  double ss = 0.0;
  const int kc = tx * KPT;
  for (int64_t ct = cb; ct < ce; ++ct) {
    const int64_t row0 = COLS ? ct * kTile : ot * kTile;
    const int64_t col0 = COLS ? ot * kTile : ct * kTile;
    __syncthreads();   // the previous tile's readers are done
    if (COLS) stage_factor<KP>(U, m, r, row0, sUt, sF);
    else stage_factor<KP>(V, n, r, col0, sVt, sF);
    float x[4][4];
    unsigned mb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      load_block_row(X, m, n, ld, vec != 0, bits, ldm, row0 + 4 * ty + a, col0 + 4 * tx, x[a], mb[a]);
    __syncthreads();
    float s[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) s[a][b] = 0.f;
#pragma unroll 4
    for (int k = 0; k < KP; ++k) {
      const float4 uu = *reinterpret_cast<const float4*>(&sUt[k][4 * ty]);
      const float4 vv = *reinterpret_cast<const float4*>(&sVt[k][4 * tx]);
      const float ua[4] = {uu.x, uu.y, uu.z, uu.w};
      const float vb[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) s[a][b] = fmaf(ua[a], vb[b], s[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float e[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        e[b] = ((mb[a] >> b) & 1u) ? x[a][b] - s[a][b] : 0.f;
        ss = fma((double)e[b], (double)e[b], ss);
      }
      *reinterpret_cast<float4*>(&sE[4 * ty + a][4 * tx]) = make_float4(e[0], e[1], e[2], e[3]);
    }
    __syncthreads();
    if (!COLS) {
      // rows 4ty..4ty+3 of E V: columns of the tile in order
#pragma unroll 2
      for (int c = 0; c < kTile; c += 4) {
        float ev[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float4 q = *reinterpret_cast<const float4*>(&sE[4 * ty + a][c]);
          ev[a][0] = q.x; ev[a][1] = q.y; ev[a][2] = q.z; ev[a][3] = q.w;
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          float f[KPT];
#pragma unroll
          for (int q = 0; q < KPT; ++q) f[q] = sF[c + cc][kc + q];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < KPT; ++q) acc[a][q] = fmaf(ev[a][cc], f[q], acc[a][q]);
        }
      }
    } else {
      // columns 4ty..4ty+3 of E^T U: rows of the tile in order
#pragma unroll 4
      for (int row = 0; row < kTile; ++row) {
        const float4 q4 = *reinterpret_cast<const float4*>(&sE[row][4 * ty]);
        const float ev[4] = {q4.x, q4.y, q4.z, q4.w};
        float f[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) f[q] = sF[row][kc + q];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int q = 0; q < KPT; ++q) acc[a][q] = fmaf(ev[a], f[q], acc[a][q]);
      }
    }
  }
  const int64_t nout = COLS ? n : m;
  float* o = out + (int64_t)blockIdx.y * out_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t row = ot * kTile + 4 * ty + a;
    if (row < nout) {
#pragma unroll
      for (int q = 0; q < KPT; ++q)
        if (kc + q < r) o[row * r + kc + q] = acc[a][q];
    }
  }
  if (rss != nullptr) {
    ss = block_sum<kEt>(ss, sh);
    if (threadIdx.x == 0) rss[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ss;
  }
}

// Masked row energies of the PBCD step.  COLS = 0: e_i = sum over observed j
// of (g_i . v_j)^2 with g the masked gradient rows of U (from U and the
// partials of R_U); COLS = 1: e_j = sum over observed i of (u_i . g_j)^2 with
// g from V and R_V.  Float32 products, float64 sums; per block partials
// (split y) of the energies of its 64-row (column) tile.
template <int KP, int COLS>
__global__ __launch_bounds__(kEt) void k_menergy(int64_t m, int64_t n,
                                                 const uint32_t* __restrict__ bits, int64_t ldm,
                                                 const float* __restrict__ U,
                                                 const float* __restrict__ V, int r,
                                                 const float* __restrict__ Rp, int nsplit,
                                                 int64_t pstride, int tiles_per_split,
                                                 double* __restrict__ out, int64_t out_stride) {
  __shared__ __align__(16) float sUt[KP][kTp];
  __shared__ __align__(16) float sVt[KP][kTp];
  __shared__ double sred[16][kTile + 1];
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  const int64_t ntile_r = (m + kTile - 1) / kTile, ntile_c = (n + kTile - 1) / kTile;
  const int64_t ot = blockIdx.x;
  const int64_t cb = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t ctiles = COLS ? ntile_r : ntile_c;
  const int64_t ce = cb + tiles_per_split < ctiles ? cb + tiles_per_split : ctiles;
  if (COLS) stage_grad<KP>(V, Rp, nsplit, pstride, n, r, ot * kTile, sVt);
  else stage_grad<KP>(U, Rp, nsplit, pstride, m, r, ot * kTile, sUt);
  double es[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t ct = cb; ct < ce; ++ct) {
    const int64_t row0 = COLS ? ct * kTile : ot * kTile;
    const int64_t col0 = COLS ? ot * kTile : ct * kTile;
    __syncthreads();
    if (COLS) stage_factor<KP>(U, m, r, row0, sUt, nullptr);
    else stage_factor<KP>(V, n, r, col0, sVt, nullptr);
    unsigned mb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t row = row0 + 4 * ty + a, col = col0 + 4 * tx;
      mb[a] = 0u;
      if (row < m && col < n) {
        const int64_t left = n - col;
        mb[a] = mask4(bits, ldm, row, col) & (left >= 4 ? 0xFu : ((1u << left) - 1u));
      }
    }
    __syncthreads();
    float s[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) s[a][b] = 0.f;
#pragma unroll 4
    for (int k = 0; k < KP; ++k) {
      const float4 uu = *reinterpret_cast<const float4*>(&sUt[k][4 * ty]);
      const float4 vv = *reinterpret_cast<const float4*>(&sVt[k][4 * tx]);
      const float ua[4] = {uu.x, uu.y, uu.z, uu.w};
      const float vb[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) s[a][b] = fmaf(ua[a], vb[b], s[a][b]);
    }
    // rows: es[a] over the thread's columns; columns: es[b] over its rows
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double v = ((mb[a] >> b) & 1u) ? (double)s[a][b] * (double)s[a][b] : 0.0;
        if (COLS) es[b] += v;
        else es[a] += v;
      }
  }
  double* o = out + (int64_t)blockIdx.y * out_stride;
  if (!COLS) {
    // combine the 16 column groups of a row (lanes tx of one wave) by butterfly
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double v = es[a];
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off);
      const int64_t row = ot * kTile + 4 * ty + a;
      if (tx == 0 && row < m) o[row] = v;
    }
  } else {
    // combine the 16 row groups of a column (ty, across waves) in order
#pragma unroll
    for (int b = 0; b < 4; ++b) sred[ty][4 * tx + b] = es[b];
    __syncthreads();
    if (threadIdx.x < kTile) {
      double v = 0.0;
      for (int q = 0; q < 16; ++q) v += sred[q][threadIdx.x];
      const int64_t col = ot * kTile + threadIdx.x;
      if (col < n) o[col] = v;
    }
  }
}

// Push of eq. negup: every negative entry moves up by `step`.  Counts the
// negative entries before the push (per block).
__global__ __launch_bounds__(kEt) void k_enmc_push(float* __restrict__ A, int64_t count, double step,
                                                   double* __restrict__ negs) {
  __shared__ double sh[kEt / kWave];
  double c = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kEt + threadIdx.x; e < count; e += (int64_t)gridDim.x * kEt) {
    const float a = A[e];
    if (a < 0.f) {
      A[e] = (float)((double)a + step);
      c += 1.0;
    }
  }
  c = block_sum<kEt>(c, sh);
  if (threadIdx.x == 0 && negs != nullptr) negs[blockIdx.x] = c;
}

// Masked PBCD step of the rows of A (one thread per row): g = M_A+ o grad
// with grad = -(sum of the partials of R) as k_menergy stages it,
// d = |g|^2 / e (0 when e is not positive; dfix >= 0 replaces d), and
// a <- (a - d g)_+ on the mask, unmasked entries unchanged.
template <int KP>
__global__ __launch_bounds__(kEt) void k_enmc_step(float* __restrict__ A, int64_t rows, int r,
                                                   const float* __restrict__ Rp, int nsplit,
                                                   int64_t pstride, const double* __restrict__ Ep,
                                                   int esplit, int64_t estride, double dfix) {
  const int64_t i = (int64_t)blockIdx.x * kEt + threadIdx.x;
  if (i >= rows) return;
  double e = Ep[i];
  for (int s = 1; s < esplit; ++s) e += Ep[s * estride + i];
  float g[KP], a[KP];
  double num = 0.0;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    g[k] = 0.f;
    a[k] = 0.f;
    if (k < r) {
      const int64_t o = i * r + k;
      float R = Rp[o];
      for (int s = 1; s < nsplit; ++s) R += Rp[s * pstride + o];
      a[k] = A[o];
      g[k] = a[k] >= 0.f ? -R : 0.f;
      num = fma((double)g[k], (double)g[k], num);
    }
  }
  const double d = dfix >= 0.0 ? dfix : (e > 0.0 ? num / e : 0.0);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    if (k < r && a[k] >= 0.f) {
      const double v = (double)a[k] - d * (double)g[k];
      A[i * r + k] = (float)(v > 0.0 ? v : 0.0);
    }
  }
}

// softImpute-ALS step of the rows of A: a <- a + R Ginv, R = sum of the
// partials (the masked residual product), Ginv (kp x kp float64) the inverse
// Gram of the other factor.
template <int KP>
__global__ __launch_bounds__(kEt) void k_als_step(float* __restrict__ A, int64_t rows, int r,
                                                  const float* __restrict__ Rp, int nsplit,
                                                  int64_t pstride, const double* __restrict__ Ginv,
                                                  int kp) {
  __shared__ double sG[KP * KP];
  for (int e = threadIdx.x; e < KP * KP; e += kEt) {
    const int l = e / KP, k = e % KP;
    sG[e] = (l < r && k < r) ? Ginv[l * kp + k] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kEt + threadIdx.x;
  if (i >= rows) return;
  float R[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    R[k] = 0.f;
    if (k < r) {
      const int64_t o = i * r + k;
      float v = Rp[o];
      for (int s = 1; s < nsplit; ++s) v += Rp[s * pstride + o];
      R[k] = v;
    }
  }
  for (int k = 0; k < r; ++k) {
    double v = (double)A[i * r + k];
#pragma unroll
    for (int l = 0; l < KP; ++l) v = fma((double)R[l], sG[l * KP + k], v);
    A[i * r + k] = (float)v;
  }
}

// Inverse of a symmetric positive definite r x r matrix (leading block of a
// kp x kp array) by Gauss-Jordan elimination in float64, one block.
__global__ __launch_bounds__(kEt) void k_spd_inverse(const double* __restrict__ G, int r, int kp,
                                                     double* __restrict__ Ginv, int* __restrict__ bad) {
  __shared__ double a[ENMF_MAX_RANK][2 * ENMF_MAX_RANK + 1];
  __shared__ double piv;
  for (int e = threadIdx.x; e < r * 2 * r; e += kEt) {
    const int i = e / (2 * r), j = e % (2 * r);
    a[i][j] = j < r ? G[i * kp + j] : (j - r == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int p = 0; p < r; ++p) {
    if (threadIdx.x == 0) piv = a[p][p];
    __syncthreads();
    const double pv = piv;
    if (!(pv > 0.0)) {
      if (threadIdx.x == 0 && bad != nullptr) *bad = 1;
      return;   // uniform: every thread read the same pivot
    }
    for (int j = threadIdx.x; j < 2 * r; j += kEt) a[p][j] /= pv;
    __syncthreads();
    for (int e = threadIdx.x; e < r * 2 * r; e += kEt) {
      const int i = e / (2 * r), j = e % (2 * r);
      if (i != p) a[i][j] = fma(-a[i][p], a[p][j], a[i][j]);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < r * r; e += kEt) Ginv[(e / r) * kp + e % r] = a[e / r][r + e % r];
}

// X0 = M o X (unobserved entries zero), float32.
__global__ __launch_bounds__(kEt) void k_mask_x(const float* __restrict__ X, int64_t m, int64_t n,
                                                int64_t ld, const uint32_t* __restrict__ bits,
                                                int64_t ldm, float* __restrict__ out) {
  const int64_t count = m * n;
  for (int64_t e = (int64_t)blockIdx.x * kEt + threadIdx.x; e < count; e += (int64_t)gridDim.x * kEt) {
    const int64_t i = e / n, j = e % n;
    const bool obs = (bits[i * ldm + (j >> 5)] >> (j & 31)) & 1u;
    out[e] = obs ? X[i * ld + j] : 0.f;
  }
}

// Check partials of the rows of A with grad = -(sum of the partials of R):
// per block {|proj grad|^2, |A|^2, |min(A, 0)|^2, #negative, min A}.
__global__ __launch_bounds__(kEt) void k_enmc_check(const float* __restrict__ A, int64_t rows, int r,
                                                    const float* __restrict__ Rp, int nsplit,
                                                    int64_t pstride, double* __restrict__ part) {
  __shared__ double sh[5 * (kEt / kWave)];
  double v[5] = {0.0, 0.0, 0.0, 0.0, INFINITY};
  const int64_t count = rows * r;
  for (int64_t o = (int64_t)blockIdx.x * kEt + threadIdx.x; o < count; o += (int64_t)gridDim.x * kEt) {
    float R = Rp[o];
    for (int s = 1; s < nsplit; ++s) R += Rp[s * pstride + o];
    const double g = -(double)R;
    const double a = (double)A[o];
    const double pg = a > 0.0 ? g : fmin(g, 0.0);
    v[0] = fma(pg, pg, v[0]);
    v[1] = fma(a, a, v[1]);
    if (a < 0.0) { v[2] = fma(a, a, v[2]); v[3] += 1.0; }
    v[4] = fmin(v[4], a);
  }
  const int kind[5] = {0, 0, 0, 0, 2};
  double out[5];
  block_reduce_fields<kEt, 5>(v, kind, sh, out);
  if (threadIdx.x == 0)
    for (int f = 0; f < 5; ++f) part[(int64_t)blockIdx.x * 5 + f] = out[f];
}

// The check of the masked problem from the partials (in block order):
// f = 1/2 sum rss, relerr = sqrt(2 f) / |M o X|, and the normalised KKT
// residual of the eNMF readings with the masked gradients; stop when
// feasible and kappa <= kkt_tol, or on the final check.
__global__ __launch_bounds__(kWave) void k_enmc_finalize(const double* __restrict__ rss, int nrss,
                                                         const double* __restrict__ cu, int ncu,
                                                         const double* __restrict__ cv, int ncv,
                                                         int k, int final_check, EnmcState* st) {
  if (threadIdx.x != 0) return;
  double f2 = 0.0;
  for (int b = 0; b < nrss; ++b) f2 += rss[b];
  double a[2][5];
  for (int side = 0; side < 2; ++side) {
    const double* p = side == 0 ? cu : cv;
    const int nb = side == 0 ? ncu : ncv;
    a[side][0] = a[side][1] = a[side][2] = a[side][3] = 0.0;
    a[side][4] = INFINITY;
    for (int b = 0; b < nb; ++b) {
      for (int f = 0; f < 4; ++f) a[side][f] += p[b * 5 + f];
      a[side][4] = fmin(a[side][4], p[b * 5 + 4]);
    }
  }
  const double nx = sqrt(st->nx2);
  const double nU = sqrt(a[0][1]), nV = sqrt(a[1][1]);
  const double feas = fmax(nU > 0.0 ? sqrt(a[0][2]) / nU : 0.0, nV > 0.0 ? sqrt(a[1][2]) / nV : 0.0);
  const double pgu = (nV > 0.0 && nx > 0.0) ? sqrt(a[0][0]) / (nx * nV) : 0.0;
  const double pgv = (nU > 0.0 && nx > 0.0) ? sqrt(a[1][0]) / (nx * nU) : 0.0;
  const double kkt = fmax(feas, fmax(pgu, pgv));
  const double f = 0.5 * f2;
  st->f = f;
  st->relerr = nx > 0.0 ? sqrt(f2) / nx : 0.0;
  st->kkt = kkt;
  st->kkt_feas = feas;
  st->kkt_pg_u = pgu;
  st->kkt_pg_v = pgv;
  st->min_w = fmin(a[0][4], a[1][4]);
  st->negs = a[0][3] + a[1][3];
  st->negs_u = a[0][3];
  const bool feasible = st->negs == 0.0;
  const bool hit = feasible && st->kkt_tol >= 0.0 && kkt <= st->kkt_tol;
  const bool numerr = !isfinite(f) || !isfinite(kkt);
  if (numerr) st->numeric_error = 1;
  if (hit || numerr || final_check) {
    st->stop = 1;
    st->converged = hit ? 1 : 0;
    st->iters = k;
  } else {
    st->iters = k + 1;
  }
}

// out[e] = -(sum over s < nsplit of p[s * stride + e]), in split order.
__global__ __launch_bounds__(kEt) void k_sum_neg(const float* __restrict__ p, int nsplit,
                                                 int64_t stride, float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * kEt + threadIdx.x; e < stride; e += (int64_t)gridDim.x * kEt) {
    float v = p[e];
    for (int s = 1; s < nsplit; ++s) v += p[s * stride + e];
    out[e] = -v;
  }
}

template <int KP>
void mres_launch(int cols, dim3 g, const float* X, int64_t m, int64_t n, int64_t ld, int vec,
                 const uint32_t* bits, int64_t ldm, const float* U, const float* V, int r, int tps,
                 float* out, int64_t stride, double* rss, hipStream_t s) {
  if (cols)
    hipLaunchKernelGGL((k_mres<KP, 1>), g, dim3(kEt), 0, s, X, m, n, ld, vec, bits, ldm, U, V, r, tps, out, stride, rss);
  else
    hipLaunchKernelGGL((k_mres<KP, 0>), g, dim3(kEt), 0, s, X, m, n, ld, vec, bits, ldm, U, V, r, tps, out, stride, rss);
}

template <int KP>
void menergy_launch(int cols, dim3 g, int64_t m, int64_t n, const uint32_t* bits, int64_t ldm,
                    const float* U, const float* V, int r, const float* Rp, int nsplit,
                    int64_t pstride, int tps, double* out, int64_t ostride, hipStream_t s) {
  if (cols)
    hipLaunchKernelGGL((k_menergy<KP, 1>), g, dim3(kEt), 0, s, m, n, bits, ldm, U, V, r, Rp, nsplit, pstride, tps, out, ostride);
  else
    hipLaunchKernelGGL((k_menergy<KP, 0>), g, dim3(kEt), 0, s, m, n, bits, ldm, U, V, r, Rp, nsplit, pstride, tps, out, ostride);
}

int enmc_kp(int r) { return r <= 16 ? 16 : r <= 32 ? 32 : 64; }

}  // namespace

EnmcPlan enmc_plan(int64_t m, int64_t n, int cols) {
  EnmcPlan p;
  const int64_t out_tiles = cols ? (n + kTile - 1) / kTile : (m + kTile - 1) / kTile;
  const int64_t con_tiles = cols ? (m + kTile - 1) / kTile : (n + kTile - 1) / kTile;
  // about two blocks per compute unit, at least 4 contraction tiles per block
  const int64_t want = 512;
  int64_t splits = (want + out_tiles - 1) / out_tiles;
  const int64_t smax = (con_tiles + 3) / 4;
  if (splits > smax) splits = smax;
  if (splits < 1) splits = 1;
  p.tiles_per_split = (int)((con_tiles + splits - 1) / splits);
  p.splits = (int)((con_tiles + p.tiles_per_split - 1) / p.tiles_per_split);
  p.out_tiles = out_tiles;
  return p;
}

hipError_t launch_mres(int cols, const float* X, int64_t m, int64_t n, int64_t ld,
                       const uint32_t* bits, int64_t ldm, const float* U, const float* V, int r,
                       float* out, double* rss, hipStream_t s) {
  const EnmcPlan p = enmc_plan(m, n, cols);
  const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && (ld % 4 == 0);
  dim3 g((unsigned)p.out_tiles, (unsigned)p.splits);
  const int64_t stride = (cols ? n : m) * r;
  switch (enmc_kp(r)) {
    case 16: mres_launch<16>(cols, g, X, m, n, ld, vec, bits, ldm, U, V, r, p.tiles_per_split, out, stride, rss, s); break;
    case 32: mres_launch<32>(cols, g, X, m, n, ld, vec, bits, ldm, U, V, r, p.tiles_per_split, out, stride, rss, s); break;
    default: mres_launch<64>(cols, g, X, m, n, ld, vec, bits, ldm, U, V, r, p.tiles_per_split, out, stride, rss, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_menergy(int cols, int64_t m, int64_t n, const uint32_t* bits, int64_t ldm,
                          const float* U, const float* V, int r, const float* Rp, int nsplit,
                          double* out, hipStream_t s) {
  const EnmcPlan p = enmc_plan(m, n, cols);
  dim3 g((unsigned)p.out_tiles, (unsigned)p.splits);
  const int64_t pstride = (cols ? n : m) * r;
  const int64_t ostride = cols ? n : m;
  switch (enmc_kp(r)) {
    case 16: menergy_launch<16>(cols, g, m, n, bits, ldm, U, V, r, Rp, nsplit, pstride, p.tiles_per_split, out, ostride, s); break;
    case 32: menergy_launch<32>(cols, g, m, n, bits, ldm, U, V, r, Rp, nsplit, pstride, p.tiles_per_split, out, ostride, s); break;
    default: menergy_launch<64>(cols, g, m, n, bits, ldm, U, V, r, Rp, nsplit, pstride, p.tiles_per_split, out, ostride, s); break;
  }
  return hipGetLastError();
}

int enmc_push_blocks(int64_t count) {
  int64_t b = (count + kEt - 1) / kEt;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_enmc_push(float* A, int64_t count, double step, double* negs, hipStream_t s) {
  hipLaunchKernelGGL(k_enmc_push, dim3(enmc_push_blocks(count)), dim3(kEt), 0, s, A, count, step, negs);
  return hipGetLastError();
}

hipError_t launch_enmc_step(float* A, int64_t rows, int r, const float* Rp, int nsplit,
                            const double* Ep, int esplit, double dfix, hipStream_t s) {
  const dim3 g((unsigned)((rows + kEt - 1) / kEt));
  switch (enmc_kp(r)) {
    case 16: hipLaunchKernelGGL((k_enmc_step<16>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ep, esplit, rows, dfix); break;
    case 32: hipLaunchKernelGGL((k_enmc_step<32>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ep, esplit, rows, dfix); break;
    default: hipLaunchKernelGGL((k_enmc_step<64>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ep, esplit, rows, dfix); break;
  }
  return hipGetLastError();
}

hipError_t launch_als_step(float* A, int64_t rows, int r, const float* Rp, int nsplit,
                           const double* Ginv, int kp, hipStream_t s) {
  const dim3 g((unsigned)((rows + kEt - 1) / kEt));
  switch (enmc_kp(r)) {
    case 16: hipLaunchKernelGGL((k_als_step<16>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ginv, kp); break;
    case 32: hipLaunchKernelGGL((k_als_step<32>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ginv, kp); break;
    default: hipLaunchKernelGGL((k_als_step<64>), g, dim3(kEt), 0, s, A, rows, r, Rp, nsplit, rows * r, Ginv, kp); break;
  }
  return hipGetLastError();
}

hipError_t launch_spd_inverse(const double* G, int r, int kp, double* Ginv, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_spd_inverse, dim3(1), dim3(kEt), 0, s, G, r, kp, Ginv, bad);
  return hipGetLastError();
}

hipError_t launch_mask_x(const float* X, int64_t m, int64_t n, int64_t ld, const uint32_t* bits,
                         int64_t ldm, float* out, hipStream_t s) {
  int64_t b = (m * n + kEt - 1) / kEt;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_mask_x, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kEt), 0, s, X, m, n, ld, bits, ldm, out);
  return hipGetLastError();
}

int enmc_check_blocks(int64_t count) {
  int64_t b = (count + kEt - 1) / kEt;
  return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

hipError_t launch_enmc_check(const float* A, int64_t rows, int r, const float* Rp, int nsplit,
                             double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_enmc_check, dim3(enmc_check_blocks(rows * r)), dim3(kEt), 0, s, A, rows, r, Rp,
                     nsplit, rows * r, part);
  return hipGetLastError();
}

hipError_t launch_sum_neg(const float* p, int nsplit, int64_t stride, float* out, hipStream_t s) {
  int64_t b = (stride + kEt - 1) / kEt;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_sum_neg, dim3((unsigned)(b < 1 ? 1 : b)), dim3(kEt), 0, s, p, nsplit, stride, out);
  return hipGetLastError();
}

hipError_t launch_enmc_finalize(const double* rss, int nrss, const double* cu, int ncu,
                                const double* cv, int ncv, int k, int final_check, EnmcState* st,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_enmc_finalize, dim3(1), dim3(kWave), 0, s, rss, nrss, cu, ncu, cv, ncv, k,
                     final_check, st);
  return hipGetLastError();
}

}  // namespace enmf
