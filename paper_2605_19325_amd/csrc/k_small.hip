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

#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kT = 256;
constexpr int kMaxW = ENMF_MAX_WIDTH;   // 80
constexpr int kLdJ = kMaxW + 1;         // LDS leading dimension of the Jacobi matrices

int grid_for(int64_t count, int threads = 256, int cap = 8192) {
  int64_t g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  return (int)(g < cap ? g : cap);
}

template <typename T> __device__ __forceinline__ double ld64(const T* p) { return (double)*p; }

// part[block_offset + b][a * kb + c] = sum over the block's rows of A[i][a] * B[i][c].
template <typename TA, typename TB>
__global__ __launch_bounds__(kT) void k_tsgram(const TA* __restrict__ A, int64_t lda,
                                               const TB* __restrict__ B, int64_t ldb, int64_t rows,
                                               int ka, int kb, int64_t rows_per_block,
                                               double* __restrict__ part, int block_offset) {
  constexpr int kTile = 32;
  constexpr int kQ = (kMaxW * kMaxW + kT - 1) / kT;
  __shared__ double sA[kTile][kMaxW];
  __shared__ double sB[kTile][kMaxW];
  const int ne = ka * kb;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  int oa[kQ], ob[kQ];
  double acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int e = threadIdx.x + kT * q;
    oa[q] = e < ne ? e / kb : 0;
    ob[q] = e < ne ? e % kb : 0;
    acc[q] = 0.0;
  }
  for (int64_t t0 = r0; t0 < r1; t0 += kTile) {
    const int nr = (int)(r1 - t0 < kTile ? r1 - t0 : kTile);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * ka; e += kT) sA[e / ka][e % ka] = ld64(A + (t0 + e / ka) * lda + e % ka);
    for (int e = threadIdx.x; e < nr * kb; e += kT) sB[e / kb][e % kb] = ld64(B + (t0 + e / kb) * ldb + e % kb);
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) acc[q] = fma(sA[rr][oa[q]], sB[rr][ob[q]], acc[q]);
    }
  }
  double* o = part + (int64_t)(block_offset + blockIdx.x) * ne;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int e = threadIdx.x + kT * q;
    if (e < ne) o[e] = acc[q];
  }
}

// out (kp x kp, zero padded) = sum_b part[b] (ka x kb), b in order.
__global__ void k_gram_finalize(const double* __restrict__ part, int nparts, int ka, int kb, int kp,
                                double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kp * kp) return;
  const int a = e / kp, c = e % kp;
  double s = 0.0;
  if (a < ka && c < kb) {
    const int ne = ka * kb;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * ne + a * kb + c];
  }
  out[e] = s;
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

// ---------------------------------------------------------------------------
// Symmetric eigensolver: parallel cyclic Jacobi (Brent-Luk round-robin
// ordering) on an LDS-resident k x k float64 matrix S with eigenvector
// matrix E.  Each round applies n2/2 disjoint plane rotations, chosen with
// the stable formula of Golub & Van Loan (sym.schur2), first to the
// columns of S and E, then to the rows of S.  An odd k is padded with one
// zero row/column that no rotation ever touches.  On return diag(S) holds
// the eigenvalues and the columns of E the eigenvectors; perm lists the
// first k indices by descending eigenvalue.
// ---------------------------------------------------------------------------
struct JacobiSmem {
  double S[kMaxW * kLdJ];
  double E[kMaxW * kLdJ];
  double cs[kMaxW];
  double red[kT / kWave];
  int pq[kMaxW];
  int perm[kMaxW];
};

__device__ __forceinline__ int rr_player(int pos, int round, int n2) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (n2 - 1)) + 1;
}

__device__ void jacobi_eig(JacobiSmem& sm, int k) {
  const int n2 = k + (k & 1);
  double* S = sm.S;
  double* E = sm.E;
  for (int e = threadIdx.x; e < n2 * n2; e += kT) {
    const int a = e / n2, c = e % n2;
    E[a * kLdJ + c] = (a == c) ? 1.0 : 0.0;
    if (a >= k || c >= k) S[a * kLdJ + c] = 0.0;
  }
  __syncthreads();
  const int npairs = n2 / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < k * k; e += kT) {
      const int a = e / k, c = e % k;
      const double v = S[a * kLdJ + c];
      if (a == c) dia += v * v; else off += v * v;
    }
    off = block_sum<kT>(off, sm.red);
    dia = block_sum<kT>(dia, sm.red);
    if (!(off > 1e-30 * dia) || off == 0.0) break;
    for (int round = 0; round < n2 - 1; ++round) {
      if (threadIdx.x < npairs) {
        int p = rr_player(threadIdx.x, round, n2);
        int q = rr_player(n2 - 1 - threadIdx.x, round, n2);
        if (p > q) { const int t = p; p = q; q = t; }
        const double apq = S[p * kLdJ + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-300) {
          const double tau = (S[q * kLdJ + q] - S[p * kLdJ + p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        sm.pq[2 * threadIdx.x] = p;
        sm.pq[2 * threadIdx.x + 1] = q;
        sm.cs[2 * threadIdx.x] = c;
        sm.cs[2 * threadIdx.x + 1] = s;
      }
      __syncthreads();
      for (int task = threadIdx.x; task < npairs * n2; task += kT) {
        const int pr = task / n2, x = task % n2;
        const double c = sm.cs[2 * pr], s = sm.cs[2 * pr + 1];
        if (s == 0.0) continue;
        const int p = sm.pq[2 * pr], q = sm.pq[2 * pr + 1];
        double a = S[x * kLdJ + p], b = S[x * kLdJ + q];
        S[x * kLdJ + p] = c * a - s * b;
        S[x * kLdJ + q] = s * a + c * b;
        a = E[x * kLdJ + p];
        b = E[x * kLdJ + q];
        E[x * kLdJ + p] = c * a - s * b;
        E[x * kLdJ + q] = s * a + c * b;
      }
      __syncthreads();
      for (int task = threadIdx.x; task < npairs * n2; task += kT) {
        const int pr = task / n2, x = task % n2;
        const double c = sm.cs[2 * pr], s = sm.cs[2 * pr + 1];
        if (s == 0.0) continue;
        const int p = sm.pq[2 * pr], q = sm.pq[2 * pr + 1];
        const double a = S[p * kLdJ + x], b = S[q * kLdJ + x];
        S[p * kLdJ + x] = c * a - s * b;
        S[q * kLdJ + x] = s * a + c * b;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < k; ++i) sm.perm[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (S[sm.perm[j] * kLdJ + sm.perm[j]] > S[sm.perm[best] * kLdJ + sm.perm[best]]) best = j;
      const int t = sm.perm[i]; sm.perm[i] = sm.perm[best]; sm.perm[best] = t;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double eigval(const JacobiSmem& sm, int j) {
  return sm.S[sm.perm[j] * kLdJ + sm.perm[j]];
}
__device__ __forceinline__ double eigvec(const JacobiSmem& sm, int a, int j) {
  return sm.E[a * kLdJ + sm.perm[j]];
}

// T = E diag(lambda^-1/2) (zero for lambda <= tau * lambda_max): Q = A T has
// orthonormal columns when A^T A = Gm (range finder orthonormalisation).
__global__ __launch_bounds__(kT) void k_orth_factor(const double* __restrict__ Gm, int k, double tau,
                                                    double* __restrict__ T) {
  __shared__ JacobiSmem sm;
  for (int e = threadIdx.x; e < k * k; e += kT) sm.S[(e / k) * kLdJ + e % k] = Gm[e];
  __syncthreads();
  jacobi_eig(sm, k);
  const double lmax = eigval(sm, 0);
  for (int e = threadIdx.x; e < k * k; e += kT) {
    const int a = e / k, j = e % k;
    const double l = eigval(sm, j);
    const double sc = (l > tau * lmax && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
    T[e] = eigvec(sm, a, j) * sc;
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
  for (int e = threadIdx.x; e < k * k; e += kT) sm.S[(e / k) * kLdJ + e % k] = C[e];
  __syncthreads();
  jacobi_eig(sm, k);
  if (threadIdx.x < r) {
    const int j = threadIdx.x;
    double cs = 0.0;
    for (int a = 0; a < k; ++a) cs = fma(colsum[a], eigvec(sm, a, j), cs);
    sgn[j] = cs < 0.0 ? -1.0 : 1.0;
    const double l = eigval(sm, j);
    const double sg = l > 0.0 ? sqrt(l) : 0.0;
    sigma[j] = sg;
    sq[j] = sqrt(sg);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * r; e += kT) {
    const int a = e / r, j = e % r;
    const double w = eigvec(sm, a, j) * sgn[j];
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
}

// One row of the ADMM step (Algorithm 1): with WR = W R^k,
//   Y <- Y + rho (Z - WR)        (the dual update of the previous step; step > 0)
//   b = WR - Y / rho,  Z = prox_h(b) (eq. 7),  B = Z + Y / rho.
// R is kp x kp float64 (zero padded).  negpart[b] = sum h(WR) over the block.
template <int KP>
__global__ __launch_bounds__(kT) void k_admm_rows(const double* __restrict__ W, int64_t N,
                                                  const double* __restrict__ R,
                                                  double* __restrict__ Y, double* __restrict__ Z,
                                                  double* __restrict__ B, const DevState* st,
                                                  int step, double* __restrict__ negpart) {
  __shared__ double sh[kT / kWave];
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  const bool valid = i < N;
  const double rho = st->rho;
  const double irho = 1.0 / rho;
  double neg = 0.0;
  if (valid) {
    double w[KP];
#pragma unroll
    for (int c = 0; c < KP; ++c) w[c] = W[i * KP + c];
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      double wr = 0.0;
#pragma unroll
      for (int a = 0; a < KP; ++a) wr = fma(w[a], R[a * KP + c], wr);
      double y = 0.0;
      if (step > 0) y = Y[i * KP + c] + rho * (Z[i * KP + c] - wr);
      const double b = wr - y * irho;
      const double z = b > 0.0 ? b : (b >= -irho ? 0.0 : b + irho);
      Y[i * KP + c] = y;
      Z[i * KP + c] = z;
      B[i * KP + c] = z + y * irho;
      neg += wr < 0.0 ? -wr : 0.0;
    }
  }
  neg = block_sum<kT>(neg, sh);
  if (threadIdx.x == 0) negpart[blockIdx.x] = neg;
}

// R <- polar factor of M = sum_b Mpart[b] (r x r): with M^T M = E diag(l) E^T,
// R = M E diag(l^-1/2) E^T (the orthogonal Procrustes solution C D^T of
// section 3.1).  Records ||R_new - R_old||_F in st->dR.  R is kp x kp padded.
__global__ __launch_bounds__(kT) void k_polar(const double* __restrict__ Mpart, int nparts, int r,
                                              int kp, double* __restrict__ R, DevState* st) {
  __shared__ JacobiSmem sm;
  __shared__ double M[64 * 64];
  __shared__ double lam[64];
  __shared__ double red[kT / kWave];
  const int ne = r * r;
  for (int e = threadIdx.x; e < ne; e += kT) {
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += Mpart[(int64_t)b * ne + e];
    M[e] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ne; e += kT) {
    const int a = e / r, c = e % r;
    double s = 0.0;
    for (int q = 0; q < r; ++q) s = fma(M[q * r + a], M[q * r + c], s);
    sm.S[a * kLdJ + c] = s;
  }
  __syncthreads();
  jacobi_eig(sm, r);
  if (threadIdx.x < r) lam[threadIdx.x] = eigval(sm, threadIdx.x);
  __syncthreads();
  const double lmax = lam[0];
  // K = E diag(l^-1/2) E^T, written over S (no longer needed).
  for (int e = threadIdx.x; e < ne; e += kT) {
    const int a = e / r, c = e % r;
    double s = 0.0;
    for (int j = 0; j < r; ++j) {
      const double l = lam[j];
      const double sc = (l > 1e-28 * lmax && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
      s = fma(eigvec(sm, a, j) * sc, eigvec(sm, c, j), s);
    }
    sm.S[a * kLdJ + c] = s;
  }
  __syncthreads();
  double d2 = 0.0;
  for (int e = threadIdx.x; e < kp * kp; e += kT) {
    const int a = e / kp, c = e % kp;
    double v = 0.0;
    if (a < r && c < r) {
      for (int q = 0; q < r; ++q) v = fma(M[a * r + q], sm.S[q * kLdJ + c], v);
    }
    const double dv = v - R[e];
    d2 = fma(dv, dv, d2);
    R[e] = v;
  }
  d2 = block_sum<kT>(d2, red);
  if (threadIdx.x == 0) st->dR = sqrt(d2);
}

template <typename TA, typename TB>
void tsgram_launch(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t rows, int ka,
                   int kb, int nblocks, double* part, int off, hipStream_t s) {
  const int64_t rpb = (rows + nblocks - 1) / nblocks;
  hipLaunchKernelGGL((k_tsgram<TA, TB>), dim3(nblocks), dim3(kT), 0, s,
                     reinterpret_cast<const TA*>(A), lda, reinterpret_cast<const TB*>(B), ldb, rows,
                     ka, kb, rpb, part, off);
}

}  // namespace

int gram_blocks(int64_t rows) {
  int64_t b = (rows + 63) / 64;
  if (b > 240) b = 240;
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
  hipLaunchKernelGGL(k_gram_finalize, dim3((kp * kp + 255) / 256), dim3(256), 0, s, part, nparts, ka,
                     kb, kp, out);
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

hipError_t launch_admm_rows(const double* W, int64_t N, int r, int kp, const double* R, double* Y,
                            double* Z, double* B, DevState* st, int step, double* negpart,
                            hipStream_t s) {
  (void)r;
  dim3 g((unsigned)((N + kT - 1) / kT)), b(kT);
  switch (kp) {
    case 8: hipLaunchKernelGGL((k_admm_rows<8>), g, b, 0, s, W, N, R, Y, Z, B, st, step, negpart); break;
    case 16: hipLaunchKernelGGL((k_admm_rows<16>), g, b, 0, s, W, N, R, Y, Z, B, st, step, negpart); break;
    case 32: hipLaunchKernelGGL((k_admm_rows<32>), g, b, 0, s, W, N, R, Y, Z, B, st, step, negpart); break;
    case 48: hipLaunchKernelGGL((k_admm_rows<48>), g, b, 0, s, W, N, R, Y, Z, B, st, step, negpart); break;
    default: hipLaunchKernelGGL((k_admm_rows<64>), g, b, 0, s, W, N, R, Y, Z, B, st, step, negpart); break;
  }
  return hipGetLastError();
}

hipError_t launch_polar(const double* Mpart, int nparts, int r, int kp, double* R, DevState* st,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_polar, dim3(1), dim3(kT), 0, s, Mpart, nparts, r, kp, R, st);
  return hipGetLastError();
}

}  // namespace enmf
