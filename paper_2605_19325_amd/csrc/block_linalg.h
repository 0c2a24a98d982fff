// Block-level float64 linear algebra shared by the kernels of libenmf: one
// workgroup of kBlk threads owns a small matrix in LDS.
#pragma once

#include <math.h>

#include "dev_common.h"

namespace enmf {

constexpr int kBlk = 256;   // threads of the workgroups that call these routines

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
template <int MAXW>
struct JacobiT {
  static constexpr int LD = MAXW + 1;
  double S[MAXW * LD];
  double E[MAXW * LD];
  double cs[MAXW];
  double red[kBlk / kWave];
  int pq[MAXW];
  int perm[MAXW];
};

__device__ __forceinline__ int rr_player(int pos, int round, int n2) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (n2 - 1)) + 1;
}

template <int MAXW>
__device__ void jacobi_eig(JacobiT<MAXW>& sm, int k) {
  constexpr int kLdJ = JacobiT<MAXW>::LD;
  const int n2 = k + (k & 1);
  double* S = sm.S;
  double* E = sm.E;
  for (int e = threadIdx.x; e < n2 * n2; e += kBlk) {
    const int a = e / n2, c = e % n2;
    E[a * kLdJ + c] = (a == c) ? 1.0 : 0.0;
    if (a >= k || c >= k) S[a * kLdJ + c] = 0.0;
  }
  __syncthreads();
  const int npairs = n2 / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < k * k; e += kBlk) {
      const int a = e / k, c = e % k;
      const double v = S[a * kLdJ + c];
      if (a == c) dia += v * v; else off += v * v;
    }
    off = block_sum<kBlk>(off, sm.red);
    dia = block_sum<kBlk>(dia, sm.red);
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
      // S <- J^T S J in one pass: the pairs partition the indices, so every
      // 2 x 2 block (pair P1 rows, pair P2 columns) transforms on its own as
      // J1^T S_block J2.  E <- E J column pair by column pair.
      for (int task = threadIdx.x; task < npairs * npairs; task += kBlk) {
        const int P1 = task / npairs, P2 = task % npairs;
        const double c1 = sm.cs[2 * P1], s1 = sm.cs[2 * P1 + 1];
        const double c2 = sm.cs[2 * P2], s2 = sm.cs[2 * P2 + 1];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = sm.pq[2 * P1], q1 = sm.pq[2 * P1 + 1];
        const int p2 = sm.pq[2 * P2], q2 = sm.pq[2 * P2 + 1];
        const double a = S[p1 * kLdJ + p2], b = S[p1 * kLdJ + q2];
        const double cc = S[q1 * kLdJ + p2], d = S[q1 * kLdJ + q2];
        const double ra = c1 * a - s1 * cc, rb = c1 * b - s1 * d;     // rows: J1^T
        const double rc = s1 * a + c1 * cc, rd = s1 * b + c1 * d;
        double na = c2 * ra - s2 * rb, nb = s2 * ra + c2 * rb;        // columns: J2
        double nc = c2 * rc - s2 * rd, nd = s2 * rc + c2 * rd;
        if (P1 == P2) { nb = 0.0; nc = 0.0; }                        // the annihilated pair
        S[p1 * kLdJ + p2] = na;
        S[p1 * kLdJ + q2] = nb;
        S[q1 * kLdJ + p2] = nc;
        S[q1 * kLdJ + q2] = nd;
      }
      for (int task = threadIdx.x; task < npairs * n2; task += kBlk) {
        const int pr = task / n2, x = task % n2;
        const double c = sm.cs[2 * pr], s = sm.cs[2 * pr + 1];
        if (s == 0.0) continue;
        const int p = sm.pq[2 * pr], q = sm.pq[2 * pr + 1];
        const double a = E[x * kLdJ + p], b = E[x * kLdJ + q];
        E[x * kLdJ + p] = c * a - s * b;
        E[x * kLdJ + q] = s * a + c * b;
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

template <int MAXW>
__device__ __forceinline__ double eigval(const JacobiT<MAXW>& sm, int j) {
  return sm.S[sm.perm[j] * JacobiT<MAXW>::LD + sm.perm[j]];
}
template <int MAXW>
__device__ __forceinline__ double eigvec(const JacobiT<MAXW>& sm, int a, int j) {
  return sm.E[a * JacobiT<MAXW>::LD + sm.perm[j]];
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// One 16 x 16 output tile on the float64 matrix cores: acc + sum over q < N
// of the 16 x 4 by 4 x 16 steps whose operands ld(q, a, b) reads from LDS,
// as straight-line code (all reads issued first, each MFMA waits only for
// its own pair).
template <int N, typename LD>
__device__ __forceinline__ f64x4 tile_chain(const LD& ld, f64x4 acc) {
  double a[N], b[N];
#pragma unroll
  for (int q = 0; q < N; ++q) ld(q, a[q], b[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
  return acc;
}

// The same chain over n <= NK steps, n known only at run time (one
// straight-line chain per count, chosen by wave-uniform compares).
template <int NK, typename LD>
__device__ __forceinline__ f64x4 tile_chain_n(int n, const LD& ld, f64x4 acc) {
  if constexpr (NK == 0) {
    return acc;
  } else {
    if (n >= NK) return tile_chain<NK>(ld, acc);
    return tile_chain_n<NK - 1>(n, ld, acc);
  }
}

// Polar factor of the KP x KP matrix M held in X (zero padded past kc rows
// and columns; kc a multiple of 4), in place: the Newton-Schulz iteration
// with the scaling of Chen and Chow (2014).  From X0 = M / ||M||_F, whose
// singular values lie in (0, 1], step k is
//   X <- (a/2) X (3 I - a^2 X^T X),  a = sqrt(3 / (1 + l + l^2)),
// where [l, 1] is the interval the singular values are taken to lie in; the
// step maps it onto [l', 1] with l' = (a l / 2)(3 - a^2 l^2), so l grows
// about 2.6-fold per step while it is small and a falls to 1 (the plain
// Newton-Schulz step) as l reaches 1.  l0 = 1e-3; singular values below l0
// still converge, only later.  Every singular value is mapped into (0, 1]
// and tends to 1 while the singular vectors stay, so the limit is the polar
// factor of M.  The iteration stops after the step whose change
// ||X_{k+1} - X_k||_F^2 is at most 1e-20 (the convergence is quadratic, so
// the remaining error is of order 1e-20; the change is only summed once l has
// passed 0.999) or after 100 steps.  T is scratch.
// Returns false (X untouched) when ||M||_F is 0 or not finite.
//
// Both products run on v_mfma_f64_16x16x4f64, 16 x 16 output tiles dealt
// round robin to the NT / 64 waves of the workgroup (red: NT / 64 doubles),
// with the contraction over the kc leading rows or columns only, one
// straight-line chain per tile (tile_chain_n).  T = X^T X is
// symmetric: only its upper tiles are formed, each written to both halves.
// Lane (i, g) = (l % 16, l / 16) supplies A[i][g] and B[g][i] of each
// 16 x 4 by 4 x 16 step and receives D[g + 4 v][i] in accumulator element v.
template <int KP, int NT = kBlk>
__device__ bool polar_ns_block(double (*X)[KP + 1], double (*T)[KP + 1], double* red, int kc = KP) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NTL = KP / 16;                  // tiles per side
  constexpr int NTILE = NTL * NTL;
  constexpr int NSYM = NTL * (NTL + 1) / 2;     // upper tiles of T
  constexpr int NW = NT / kWave;                // waves
  constexpr int PERW = (NTILE + NW - 1) / NW;   // tiles per wave
  constexpr int PERWS = (NSYM + NW - 1) / NW;   // upper tiles per wave
  constexpr int NK = KP / 4;                    // contraction steps at most
  static_assert(KP % 16 == 0, "polar_ns_block needs KP a multiple of 16");
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  double nrm = 0.0;
  for (int e = threadIdx.x; e < KP * KP; e += NT) nrm = fma(X[e / KP][e % KP], X[e / KP][e % KP], nrm);
  nrm = sqrt(block_sum<NT>(nrm, red));
  if (!(nrm > 0.0) || !isfinite(nrm)) return false;
  const double sc = 1.0 / nrm;
  for (int e = threadIdx.x; e < KP * KP; e += NT) X[e / KP][e % KP] *= sc;
  __syncthreads();
  double l = 1e-3;
  for (int it = 0; it < 100; ++it) {
    const double a = sqrt(3.0 / (1.0 + l + l * l));
    const double c1 = 1.5 * a, c3 = 0.5 * a * a * a;
    // While a is away from 1 every singular value still moves by far more
    // than the stopping threshold, so the step change is summed only once
    // the interval's lower end has passed 0.999 (a within 5e-4 of 1).
    const bool look = l > 0.999;
    l = 0.5 * a * l * (3.0 - a * a * l * l);
    // T = X^T X: upper tile (ti, tj) = sum over k of X[k][16 ti + i] X[k][16 tj + j],
    // each tile one MFMA chain over the kc contraction rows.
#pragma unroll
    for (int u = 0; u < PERWS; ++u) {
      const int tile = w + NW * u;
      if (tile >= NSYM) break;   // wave-uniform
      int ti = 0, rem = tile;
      while (ti < NTL && rem >= NTL - ti) { rem -= NTL - ti; ++ti; }
      const int tj = ti + rem;
      const auto ld = [&](int q, double& a, double& b) {
        a = X[4 * q + g][16 * ti + i];
        b = X[4 * q + g][16 * tj + i];
      };
      const d4 acc = tile_chain_n<NK>(kc / 4, ld, d4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T[16 * ti + g + 4 * v][16 * tj + i] = acc[v];
        if (ti != tj) T[16 * tj + i][16 * ti + g + 4 * v] = acc[v];
      }
    }
    __syncthreads();
    // X_new = c1 X - c3 X T
    double xn[PERW][4];
    double d2 = 0.0;
    {
      d4 acc[PERW];
#pragma unroll
      for (int u = 0; u < PERW; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < PERW; ++u) {
        const int tile = w + NW * u;
        if (tile >= NTILE) break;   // wave-uniform
        const int ti = tile / NTL, tj = tile % NTL;
        const auto ld = [&](int q, double& a, double& b) {
          a = X[16 * ti + i][4 * q + g];
          b = T[4 * q + g][16 * tj + i];
        };
        acc[u] = tile_chain_n<NK>(kc / 4, ld, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < PERW; ++u) {
        const int tile = w + NW * u;
        if (tile < NTILE) {
          const int ti = tile / NTL, tj = tile % NTL;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double x = X[16 * ti + g + 4 * v][16 * tj + i];
            xn[u][v] = c1 * x - c3 * acc[u][v];
            d2 = fma(xn[u][v] - x, xn[u][v] - x, d2);
          }
        }
      }
    }
    if (look) d2 = block_sum<NT>(d2, red);   // also orders every read of X before the writes below
    else __syncthreads();
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
      const int tile = w + NW * u;
      if (tile < NTILE) {
        const int ti = tile / NTL, tj = tile % NTL;
#pragma unroll
        for (int v = 0; v < 4; ++v) X[16 * ti + g + 4 * v][16 * tj + i] = xn[u][v];
      }
    }
    __syncthreads();
    if (look && d2 <= 1e-20) break;
  }
  return true;
}

}  // namespace enmf
