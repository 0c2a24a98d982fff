// Tall-skinny reductions and the small float64 linear algebra of the SVD
// initialisation and of the ADMM rotation:
//   * A^T B for tall A, B (the r x r Grams U^T U, V^T V, the Procrustes
//     matrix W^T B of the rotation, and the Grams of the range finder),
//     accumulated in float64 with per-block partials reduced in fixed order;
//   * a symmetric eigensolver (parallel cyclic Jacobi, one workgroup, LDS
//     resident, float64) and what is built on it: the orthonormalising
//     factor of the range finder, the SVD of the projected matrix, and the
//     polar factor of the Procrustes step;
//   * the row-parallel ADMM step (W R, the prox of eq. 7, the dual update).
#include <math.h>

#include "block_linalg.h"
#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kT = 256;
constexpr int kMaxW = ENMF_MAX_WIDTH;   // 80
using JacobiSmem = JacobiT<kMaxW>;

int grid_for(int64_t count, int threads = 256, int cap = 8192) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

template <typename T> __device__ __forceinline__ double ld64(const T* p) { return (double)*p; }

// part[block_offset + b][a * kb + c] = sum over the block's rows of A[i][a] * B[i][c].
// Rows are staged through LDS 32 at a time as float64 (products of float32
// inputs are exact); the 16 x 16 threads own a strided (KP/16) x (KP/16)
// tile of the output, so each staged row costs 2 KP/16 LDS reads per
// (KP/16)^2 FMAs.
template <typename TA, typename TB, int KP>
__global__ __launch_bounds__(kT) void k_tsgram(const TA* __restrict__ A, int64_t lda,
                                               const TB* __restrict__ B, int64_t ldb, int64_t rows,
                                               int ka, int kb, int64_t rows_per_block,
                                               double* __restrict__ part, int block_offset) {
  constexpr int TT = KP / 16;
  constexpr int RC = 32;
  __shared__ double sA[RC][KP];
  __shared__ double sB[RC][KP];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  double acc[TT][TT];
#pragma unroll
  for (int i = 0; i < TT; ++i)
#pragma unroll
    for (int j = 0; j < TT; ++j) acc[i][j] = 0.0;
  constexpr int PER = RC * KP / kT;   // staged elements per thread and operand
  static_assert(RC * KP % kT == 0, "row slab must split evenly over the block");
  for (int64_t t0 = r0; t0 < r1; t0 += RC) {
    const int nr = (int)(r1 - t0 < RC ? r1 - t0 : RC);
    // all of the slab's loads are in flight before the first is stored
    double va[PER], vb[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kT, row = e / KP, col = e % KP;
      const bool ok = row < nr;
      va[u] = (ok && col < ka) ? ld64(A + (t0 + row) * lda + col) : 0.0;
      vb[u] = (ok && col < kb) ? ld64(B + (t0 + row) * ldb + col) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kT;
      sA[e / KP][e % KP] = va[u];
      sB[e / KP][e % KP] = vb[u];
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      double av[TT], bv[TT];
#pragma unroll
      for (int i = 0; i < TT; ++i) av[i] = sA[rr][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < TT; ++j) bv[j] = sB[rr][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < TT; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
  double* o = part + (int64_t)(block_offset + blockIdx.x) * ka * kb;
#pragma unroll
  for (int i = 0; i < TT; ++i)
#pragma unroll
    for (int j = 0; j < TT; ++j) {
      const int a = ty + 16 * i, c = tx + 16 * j;
      if (a < ka && c < kb) o[a * kb + c] = acc[i][j];
    }
}

// out (kp x kp, zero padded) = sum_b part[b] (ka x kb).  One workgroup per
// group of 4 consecutive entries of the ka x kb partials; wave w of the 4
// takes the partials of the w-th quarter of [0, nparts), lane l of it adds
// partials l, l + 64, ... of that quarter in order (4 partials, 16 loads, in
// flight at a time), the wave sums each entry (wave_sum_last) and thread 0
// adds the four quarters in order, so the result does not depend on
// scheduling.  The padding entries are written as zeros by the grid.
__global__ __launch_bounds__(kT) void k_gram_finalize(const double* __restrict__ part, int nparts,
                                                      int ka, int kb, int kp,
                                                      double* __restrict__ out) {
  __shared__ double sq[kT / kWave][4];
  const int64_t ne = (int64_t)ka * kb;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kp * kp; e += gridDim.x * blockDim.x) {
    const int a = e / kp, c = e % kp;
    if (a >= ka || c >= kb) out[e] = 0.0;
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  constexpr int NW = kT / kWave;
  const int64_t e0 = 4 * (int64_t)blockIdx.x;
  if (e0 >= ne) return;   // whole blocks
  const int per = (nparts + NW - 1) / NW;
  const int b1 = (w + 1) * per < nparts ? (w + 1) * per : nparts;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b0 = w * per + lane; b0 < b1; b0 += 4 * kWave) {
    double v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * kWave;
      const double* src = part + (int64_t)(b < b1 ? b : 0) * ne;
#pragma unroll
      for (int c = 0; c < 4; ++c) v[u][c] = src[e0 + c < ne ? e0 + c : ne - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (b0 + u * kWave < b1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += v[u][c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) s[c] = wave_sum_last(s[c]);
  if (lane == kWave - 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) sq[w][c] = s[c];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    double t = sq[0][c];
#pragma unroll
    for (int q = 1; q < NW; ++q) t += sq[q][c];
    if (e0 + c < ne) {
      const int a = (int)((e0 + c) / kb), cc = (int)((e0 + c) % kb);
      out[a * kp + cc] = t;
    }
  }
}

// out[i][c] = sum_a A[i][a] T[a][c] for c < kb (float64 arithmetic).
template <typename TA, typename TO>
__global__ void k_apply_small(const TA* __restrict__ A, int64_t lda, int64_t rows, int ka,
                              const double* __restrict__ T, int ldt, int kb, TO* __restrict__ out,
                              int64_t ldo) {
  const int64_t count = rows * kb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kb;
    const int c = (int)(e % kb);
    const TA* a = A + i * lda;
    double s = 0.0;
    for (int q = 0; q < ka; ++q) s = fma((double)a[q], T[q * ldt + c], s);
    out[i * ldo + c] = (TO)s;
  }
}

// T with Q = A T orthonormal when A^T A = Gm (range finder orthonormalisation;
// only the span of Q is used).  Well-conditioned Gm: the Cholesky factor
// Gm = L L^T and T = L^-T (every pivot above 1e-10 of the largest diagonal
// entry).  Otherwise T = E diag(lambda^-1/2) from the eigenpairs (Jacobi),
// zero for lambda <= tau * lambda_max, which drops dependent directions.
__global__ __launch_bounds__(kT) void k_orth_factor(const double* __restrict__ Gm, int k, double tau,
                                                    double* __restrict__ T) {
  __shared__ JacobiSmem sm;
  __shared__ int fallback;
  __shared__ double dmax;
  constexpr int LD = JacobiSmem::LD;
  constexpr double kCholTau = 1e-10;
  for (int e = threadIdx.x; e < k * k; e += kT) sm.S[(e / k) * LD + e % k] = Gm[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    double d = 0.0;
    for (int a = 0; a < k; ++a) d = fmax(d, sm.S[a * LD + a]);
    dmax = d;
    fallback = d > 0.0 ? 0 : 1;
  }
  // right-looking Cholesky in the lower triangle
  for (int p = 0; p < k; ++p) {
    __syncthreads();
    if (threadIdx.x == 0 && !fallback) {
      const double d = sm.S[p * LD + p];
      if (d > kCholTau * dmax) sm.S[p * LD + p] = sqrt(d);
      else fallback = 1;
    }
    __syncthreads();
    if (fallback) break;
    const double piv = sm.S[p * LD + p];
    for (int i = p + 1 + threadIdx.x; i < k; i += kT) sm.S[i * LD + p] /= piv;
    __syncthreads();
    const int w = k - p - 1;
    for (int e = threadIdx.x; e < w * w; e += kT) {
      const int i = p + 1 + e / w, j = p + 1 + e % w;
      if (j <= i) sm.S[i * LD + j] = fma(-sm.S[i * LD + p], sm.S[j * LD + p], sm.S[i * LD + j]);
    }
  }
  __syncthreads();
  if (!fallback) {
    // column j of L^-1 by forward substitution (one thread per column); T[a][j] = (L^-1)[j][a]
    // (the column is kept in row j of the eigenvector array, unused on this path)
    if (threadIdx.x < k) {
      const int j = threadIdx.x;
      double* x = sm.E + j * LD;
      for (int i = 0; i < k; ++i) {
        double v = i == j ? 1.0 : 0.0;
        for (int l = j; l < i; ++l) v = fma(-sm.S[i * LD + l], x[l], v);
        x[i] = i < j ? 0.0 : v / sm.S[i * LD + i];
      }
      for (int i = 0; i < k; ++i) T[j * k + i] = x[i];
    }
    return;
  }
  for (int e = threadIdx.x; e < k * k; e += kT) sm.S[(e / k) * LD + e % k] = Gm[e];
  __syncthreads();
  jacobi_eig<kMaxW>(sm, k);
  const double lmax = eigval<kMaxW>(sm, 0);
  for (int e = threadIdx.x; e < k * k; e += kT) {
    const int a = e / k, j = e % k;
    const double l = eigval<kMaxW>(sm, j);
    const double sc = (l > tau * lmax && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
    T[e] = eigvec<kMaxW>(sm, a, j) * sc;
  }
}

// SVD of the projected matrix from C = Z^T Z (Z = X^T Q): eigenpairs
// (sigma_j^2, w_j) in descending order.  U = Q W, V = Z W / sigma; the sign
// of each pair makes the column sum of U (= colsum(Q) . w_j) positive; the
// balanced factors are U* = Q (W diag(s sqrt(sigma))), V* = Z (W diag(s / sqrt(sigma))).
__global__ __launch_bounds__(kT) void k_svd_factor(const double* __restrict__ C,
                                                   const double* __restrict__ colsum, int k, int r,
                                                   double* __restrict__ sigma,
                                                   double* __restrict__ TU,
                                                   double* __restrict__ TV) {
  __shared__ JacobiSmem sm;
  __shared__ double sgn[kMaxW];
  __shared__ double sq[kMaxW];
  for (int e = threadIdx.x; e < k * k; e += kT) sm.S[(e / k) * JacobiSmem::LD + e % k] = C[e];
  __syncthreads();
  jacobi_eig<kMaxW>(sm, k);
  if (threadIdx.x < r) {
    const int j = threadIdx.x;
    double cs = 0.0;
    for (int a = 0; a < k; ++a) cs = fma(colsum[a], eigvec<kMaxW>(sm, a, j), cs);
    sgn[j] = cs < 0.0 ? -1.0 : 1.0;
    const double l = eigval<kMaxW>(sm, j);
    const double sg = l > 0.0 ? sqrt(l) : 0.0;
    sigma[j] = sg;
    sq[j] = sqrt(sg);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * r; e += kT) {
    const int a = e / r, j = e % r;
    const double w = eigvec<kMaxW>(sm, a, j) * sgn[j];
    TU[e] = w * sq[j];
    TV[e] = sq[j] > 0.0 ? w / sq[j] : 0.0;
  }
}

// part[b][c] = sum over the block's rows of A[i][c] (float64 column sums).
__global__ __launch_bounds__(kT) void k_colsum(const double* __restrict__ A, int64_t lda,
                                               int64_t rows, int k, int64_t rows_per_block,
                                               double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  const int c = threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int64_t i = r0; i < r1; ++i) s += A[i * lda + c];
  part[(int64_t)blockIdx.x * k + c] = s;
}

// W = [U; V] as float64, kp columns (zero padded).
__global__ void k_pack_w(const float* __restrict__ U, int64_t m, const float* __restrict__ V,
                         int64_t n, int r, int kp, double* __restrict__ W) {
  const int64_t count = (m + n) * kp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kp;
    const int c = (int)(e % kp);
    double v = 0.0;
    if (c < r) v = i < m ? (double)U[i * r + c] : (double)V[(i - m) * r + c];
    W[e] = v;
  }
}

// part[b] = sum of squares over a contiguous chunk of W (float64).
__global__ __launch_bounds__(kT) void k_sumsq_f64(const double* __restrict__ W, int64_t count,
                                                  int64_t per_block, double* __restrict__ part) {
  __shared__ double sh[kT / kWave];
  const int64_t e0 = (int64_t)blockIdx.x * per_block;
  const int64_t e1 = e0 + per_block < count ? e0 + per_block : count;
  double s = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) s = fma(W[e], W[e], s);
  s = block_sum<kT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// rho = rho0 sqrt(N r) / ||W||_F (a reading: the paper gives rho as a symbol only).
__global__ void k_rho_init(const double* __restrict__ part, int nparts, int64_t N, int r,
                           double rho0, DevState* st) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[b];
  st->rho = s > 0.0 ? rho0 * sqrt((double)N * r) / sqrt(s) : 1.0;
  st->dR = INFINITY;
  st->rot_stop = 0;
  st->rot_steps = 0;
}

// One ADMM step of Algorithm 1 (eq. 7) on the rows of W = [U; V] (N x KP,
// float64, zero padded), fused with the Procrustes operand: per row block,
// W R (KP/8 threads per row, 8 columns each, R staged in LDS), then over the
// block's rows as one flat, coalesced range
//   Y <- Y + rho (Z - W R)  (Y = 0 at step 0),  b = W R - Y / rho,
//   Z <- prox of h at b (eq. 7),  B = Z + Y / rho.
// The multiplier and the split variable are carried as one array
// S = Y + rho Z (Y = S - rho W R at the next step), so a step reads W and S
// and writes S; B is only kept in LDS: the block adds the block's share of W^T B to its
// r x r float64 partial (on the float64 matrix cores, 16 x 16 tiles over
// 4-row steps; a thread per entry at KP = 8).  Blocks loop over row blocks
// (grid of admm_rows_blocks); part[b] receives block b's partial.
template <int KP> struct AdmmGeom {
  static constexpr int CG = KP / 8;        // threads per row
  static constexpr int RB = kT / CG;       // rows per row block
  static_assert(RB * KP <= 8 * kT, "a row block holds at most 8 state entries per thread");
};

template <int KP>
__global__ __launch_bounds__(kT) void k_admm_rows(const double* __restrict__ W, int64_t N, int r,
                                                  const double* __restrict__ R,
                                                  double* __restrict__ S,
                                                  const DevState* st, int step,
                                                  double* __restrict__ part) {
  using AG = AdmmGeom<KP>;
  constexpr int NE = (KP * KP + kT - 1) / kT;     // partial-Gram entries per thread (KP = 8)
  constexpr bool MF = KP % 16 == 0;               // partial Gram on the float64 matrix cores
  constexpr int RBP = (AG::RB + 3) / 4 * 4;       // rows padded to whole 4-row MFMA steps
  constexpr int NTL = KP / 16, NTILE = NTL * NTL, PERW = (NTILE + 3) / 4;
  typedef double d4 __attribute__((ext_vector_type(4)));
  if (st->rot_stop) return;   // the rotation stopped at an earlier check
  __shared__ double Rs[KP * KP];
  __shared__ double Ws[RBP * KP];
  __shared__ double Bs[RBP * KP];
  for (int e = threadIdx.x; e < KP * KP; e += kT) Rs[e] = R[e];
  const double rho = st->rho;
  const double irho = 1.0 / rho;
  const int rr = threadIdx.x / AG::CG, c0 = 8 * (threadIdx.x % AG::CG);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int li = lane % 16, lg = lane / 16;
  double gacc[MF ? 1 : NE];
#pragma unroll
  for (int q = 0; q < (MF ? 1 : NE); ++q) gacc[q] = 0.0;
  d4 macc[MF ? PERW : 1];
#pragma unroll
  for (int u = 0; u < (MF ? PERW : 1); ++u) macc[u] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t nrb = (N + AG::RB - 1) / AG::RB;
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t row0 = rb * AG::RB;
    const int64_t nrow = N - row0 < AG::RB ? N - row0 : AG::RB;
    const int cnt = (int)nrow * KP;
    double* Sb = S + row0 * KP;
    // the state entries this thread updates below (at most 8: RB KP <= 8 kT),
    // read now so that their latency overlaps the staging and W R
    double sv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = threadIdx.x + q * kT;
      sv[q] = step > 0 && e < cnt ? Sb[e] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RBP * KP; e += kT) {
      Ws[e] = e < nrow * KP ? W[row0 * KP + e] : 0.0;
      if (e >= AG::RB * KP) Bs[e] = 0.0;
    }
    __syncthreads();
    double wr[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) wr[e] = 0.0;
    if (rr < nrow) {
      const double* w = Ws + rr * KP;
      for (int a = 0; a < KP; ++a) {
        const double x = w[a];
        const double* rrow = Rs + a * KP + c0;
#pragma unroll
        for (int e = 0; e < 8; ++e) wr[e] = fma(x, rrow[e], wr[e]);
      }
    }
    if (rr < AG::RB) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[rr * KP + c0 + e] = wr[e];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = threadIdx.x + q * kT;
      if (e < cnt) {
        const double w = Bs[e];
        const double y = step > 0 ? sv[q] - rho * w : 0.0;
        const double b = w - y * irho;
        const double z = b > 0.0 ? b : (b >= -irho ? 0.0 : b + irho);
        Sb[e] = y + rho * z;
        Bs[e] = z + y * irho;
      }
    }
    __syncthreads();
    if constexpr (MF) {
      // tile (ti, tj) += sum over the block's rows of W[row][16 ti + i] B[row][16 tj + j];
      // lane (i, g) supplies W[k + g][16 ti + i] and B[k + g][16 tj + i] of each 4-row step;
      // a wave's tiles one after the other, each one chain over the rows
#pragma unroll
      for (int u = 0; u < PERW; ++u) {
        const int tile = wv + 4 * u;
        if (tile < NTILE) {
          const int ti = tile / NTL, tj = tile % NTL;
#pragma unroll
          for (int k0 = 0; k0 < RBP; k0 += 4)
            macc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ws[(k0 + lg) * KP + 16 * ti + li],
                                                           Bs[(k0 + lg) * KP + 16 * tj + li], macc[u],
                                                           0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int e = threadIdx.x + q * kT;
        if (e < KP * KP) {
          const int a = e / KP, c = e % KP;
          double s = gacc[q];
          for (int row = 0; row < (int)nrow; ++row) s = fma(Ws[row * KP + a], Bs[row * KP + c], s);
          gacc[q] = s;
        }
      }
    }
  }
  double* o = part + (int64_t)blockIdx.x * r * r;
  if constexpr (MF) {
    // lane (i, g) holds D[g + 4 v][i] of each of its tiles
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
      const int tile = wv + 4 * u;
      if (tile < NTILE) {
        const int ti = tile / NTL, tj = tile % NTL;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = 16 * ti + lg + 4 * v, c = 16 * tj + li;
          if (a < r && c < r) o[a * r + c] = macc[u][v];
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int e = threadIdx.x + q * kT;
      const int a = e / KP, c = e % KP;
      if (e < KP * KP && a < r && c < r) o[a * r + c] = gacc[q];
    }
  }
}

// R <- polar factor of M (r x r, leading dimension kp): the orthogonal
// Procrustes solution C D^T of section 3.1 (W^T B = C S D^T), by
// polar_ns_block.  Records ||R_new - R_old||_F in st->dR.  R is kp x kp,
// zero padded.
// Threads of k_polar_ns: one wave per 16 x 16 tile of the product (at least 4
// waves), so that each wave runs one short MFMA chain per product.
template <int KP> constexpr int polar_threads() {
  return (KP / 16) * (KP / 16) * kWave < kT ? kT : (KP / 16) * (KP / 16) * kWave;
}

template <int KP>
__global__ __launch_bounds__(polar_threads<KP>()) void k_polar_ns(const double* __restrict__ Mf, int r, int kp,
                                                 double* __restrict__ R, DevState* st,
                                                 double tol, int check_every, int step) {
  __shared__ double X[KP][KP + 1];
  __shared__ double T[KP][KP + 1];
  constexpr int NT = polar_threads<KP>();
  __shared__ double red[NT / kWave];
  if (st->rot_stop) return;
  // the change of R, and the tolerance stop at a check step (thread 0)
  auto record = [&](double dR) {
    st->dR = dR;
    if (tol > 0.0 && (step + 1) % check_every == 0 && dR <= tol) {
      st->rot_stop = 1;
      st->rot_steps = step + 1;
    }
  };
  for (int e = threadIdx.x; e < KP * KP; e += NT) {
    const int a = e / KP, c = e % KP;
    X[a][c] = (a < r && c < r) ? Mf[a * kp + c] : 0.0;
  }
  __syncthreads();
  if (!polar_ns_block<KP, NT>(X, T, red, (r + 3) / 4 * 4)) {
    if (threadIdx.x == 0) record(0.0);
    return;
  }
  double d2 = 0.0;
  for (int e = threadIdx.x; e < kp * kp; e += NT) {
    const int a = e / kp, c = e % kp;
    const double v = (a < r && c < r) ? X[a][c] : 0.0;
    const double dv = v - R[e];
    d2 = fma(dv, dv, d2);
    R[e] = v;
  }
  d2 = block_sum<NT>(d2, red);
  if (threadIdx.x == 0) record(sqrt(d2));
}

template <typename TA, typename TB, int KP>
void tsgram_launch_kp(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t rows, int ka,
                      int kb, int nblocks, double* part, int off, hipStream_t s) {
  const int64_t rpb = (rows + nblocks - 1) / nblocks;
  hipLaunchKernelGGL((k_tsgram<TA, TB, KP>), dim3(nblocks), dim3(kT), 0, s,
                     reinterpret_cast<const TA*>(A), lda, reinterpret_cast<const TB*>(B), ldb, rows,
                     ka, kb, rpb, part, off);
}

template <typename TA, typename TB>
void tsgram_launch(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t rows, int ka,
                   int kb, int nblocks, double* part, int off, hipStream_t s) {
  const int kq = pad_width(ka > kb ? ka : kb);
  switch (kq) {
    case 8:
    case 16: tsgram_launch_kp<TA, TB, 16>(A, lda, B, ldb, rows, ka, kb, nblocks, part, off, s); break;
    case 32: tsgram_launch_kp<TA, TB, 32>(A, lda, B, ldb, rows, ka, kb, nblocks, part, off, s); break;
    case 48: tsgram_launch_kp<TA, TB, 48>(A, lda, B, ldb, rows, ka, kb, nblocks, part, off, s); break;
    case 64: tsgram_launch_kp<TA, TB, 64>(A, lda, B, ldb, rows, ka, kb, nblocks, part, off, s); break;
    default: tsgram_launch_kp<TA, TB, 80>(A, lda, B, ldb, rows, ka, kb, nblocks, part, off, s); break;
  }
}

}  // namespace

int gram_blocks(int64_t rows) {
  int64_t b = (rows + 127) / 128;
  if (b > 256) b = 256;
  if (b < 1) b = 1;
  const int64_t rpb = (rows + b - 1) / b;
  return (int)((rows + rpb - 1) / rpb);
}

hipError_t launch_tsgram(const void* A, int a_is_f64, int64_t lda, const void* B, int b_is_f64,
                         int64_t ldb, int64_t rows, int ka, int kb, double* part, int block_offset,
                         int nblocks, hipStream_t s) {
  if (a_is_f64 && b_is_f64) tsgram_launch<double, double>(A, lda, B, ldb, rows, ka, kb, nblocks, part, block_offset, s);
  else if (a_is_f64) tsgram_launch<double, float>(A, lda, B, ldb, rows, ka, kb, nblocks, part, block_offset, s);
  else if (b_is_f64) tsgram_launch<float, double>(A, lda, B, ldb, rows, ka, kb, nblocks, part, block_offset, s);
  else tsgram_launch<float, float>(A, lda, B, ldb, rows, ka, kb, nblocks, part, block_offset, s);
  return hipGetLastError();
}

hipError_t launch_gram_finalize(const double* part, int nparts, int ka, int kb, int kp, double* out,
                                hipStream_t s) {
  const int groups = (ka * kb + 3) / 4;
  hipLaunchKernelGGL(k_gram_finalize, dim3(groups), dim3(kT), 0, s, part, nparts, ka, kb, kp, out);
  return hipGetLastError();
}

hipError_t launch_apply_small(const void* A, int a_is_f64, int64_t lda, int64_t rows, int ka,
                              const double* T, int ldt, int kb, void* out, int out_is_f64,
                              int64_t ldo, hipStream_t s) {
  dim3 g(grid_for(rows * kb)), b(256);
  if (a_is_f64 && out_is_f64)
    hipLaunchKernelGGL((k_apply_small<double, double>), g, b, 0, s, (const double*)A, lda, rows, ka, T, ldt, kb, (double*)out, ldo);
  else if (a_is_f64)
    hipLaunchKernelGGL((k_apply_small<double, float>), g, b, 0, s, (const double*)A, lda, rows, ka, T, ldt, kb, (float*)out, ldo);
  else if (out_is_f64)
    hipLaunchKernelGGL((k_apply_small<float, double>), g, b, 0, s, (const float*)A, lda, rows, ka, T, ldt, kb, (double*)out, ldo);
  else
    hipLaunchKernelGGL((k_apply_small<float, float>), g, b, 0, s, (const float*)A, lda, rows, ka, T, ldt, kb, (float*)out, ldo);
  return hipGetLastError();
}

hipError_t launch_orth_factor(const double* Gm, int k, double tau, double* T, hipStream_t s) {
  hipLaunchKernelGGL(k_orth_factor, dim3(1), dim3(kT), 0, s, Gm, k, tau, T);
  return hipGetLastError();
}

hipError_t launch_colsum(const double* A, int64_t lda, int64_t rows, int k, double* part, int* nparts,
                         hipStream_t s) {
  int64_t nb = (rows + 255) / 256;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  const int64_t rpb = (rows + nb - 1) / nb;
  nb = (rows + rpb - 1) / rpb;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)nb), dim3(kT), 0, s, A, lda, rows, k, rpb, part);
  *nparts = (int)nb;
  return hipGetLastError();
}

hipError_t launch_svd_factor(const double* C, const double* colsum, int k, int r, double* sigma,
                             double* TU, double* TV, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_factor, dim3(1), dim3(kT), 0, s, C, colsum, k, r, sigma, TU, TV);
  return hipGetLastError();
}

hipError_t launch_pack_w(const float* U, int64_t m, const float* V, int64_t n, int r, int kp,
                         double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_w, dim3(grid_for((m + n) * kp)), dim3(256), 0, s, U, m, V, n, r, kp, W);
  return hipGetLastError();
}

hipError_t launch_w_sumsq(const double* W, int64_t count, double* part, int* nparts, hipStream_t s) {
  int64_t nb = (count + 4095) / 4096;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  const int64_t per = (count + nb - 1) / nb;
  nb = (count + per - 1) / per;
  hipLaunchKernelGGL(k_sumsq_f64, dim3((unsigned)nb), dim3(kT), 0, s, W, count, per, part);
  *nparts = (int)nb;
  return hipGetLastError();
}

hipError_t launch_rho_init(const double* part, int nparts, int64_t N, int r, double rho0, DevState* st,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rho_init, dim3(1), dim3(64), 0, s, part, nparts, N, r, rho0, st);
  return hipGetLastError();
}

int admm_rows_blocks(int64_t N, int kp) {
  const int rb = kT / (kp / 8);
  const int64_t b = (N + rb - 1) / rb;
  return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_admm_rows(const double* W, int64_t N, int r, int kp, const double* R, double* S,
                            DevState* st, int step, double* part, hipStream_t s) {
  dim3 g((unsigned)admm_rows_blocks(N, kp)), b(kT);
  switch (kp) {
    case 8: hipLaunchKernelGGL((k_admm_rows<8>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
    case 16: hipLaunchKernelGGL((k_admm_rows<16>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
    case 32: hipLaunchKernelGGL((k_admm_rows<32>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
    case 48: hipLaunchKernelGGL((k_admm_rows<48>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
    case 64: hipLaunchKernelGGL((k_admm_rows<64>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
    default: hipLaunchKernelGGL((k_admm_rows<80>), g, b, 0, s, W, N, r, R, S, st, step, part); break;
  }
  return hipGetLastError();
}

hipError_t launch_polar(const double* Mf, int r, int kp, double* R, DevState* st, hipStream_t s,
                        double tol, int check_every, int step) {
  switch (pad_width(r)) {
    case 8:
    case 16:
      hipLaunchKernelGGL((k_polar_ns<16>), dim3(1), dim3(polar_threads<16>()), 0, s, Mf, r, kp, R, st,
                         tol, check_every, step);
      break;
    case 32:
      hipLaunchKernelGGL((k_polar_ns<32>), dim3(1), dim3(polar_threads<32>()), 0, s, Mf, r, kp, R, st,
                         tol, check_every, step);
      break;
    case 48:
      hipLaunchKernelGGL((k_polar_ns<48>), dim3(1), dim3(polar_threads<48>()), 0, s, Mf, r, kp, R, st,
                         tol, check_every, step);
      break;
    default:
      hipLaunchKernelGGL((k_polar_ns<64>), dim3(1), dim3(polar_threads<64>()), 0, s, Mf, r, kp, R, st,
                         tol, check_every, step);
      break;
  }
  return hipGetLastError();
}

}  // namespace enmf
