// Row-team building blocks of the exterior-phase and HALS row updates (a
// team of KP/8 lanes owns one row of U or V, 8 columns per lane), shared by
// the per-iteration kernels and the serving kernel.
#pragma once

#include <math.h>

#include "dev_common.h"

namespace enmf {

// Team geometry: KP/8 lanes per row, teams aligned inside a wave.
template <int KP> struct Team {
  static constexpr int T = KP / 8;
  static constexpr int RB = T <= 4 ? 64 : 32;   // rows per block
  static constexpr int NT = RB * T;             // threads per block
};

template <int T>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
  for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// G (KP x KP float64) into LDS; all of a thread's loads are issued before
// the first is consumed.
template <int KP>
__device__ __forceinline__ void load_gram(const double* __restrict__ G, double* sG) {
  constexpr int NT = Team<KP>::NT;
  constexpr int PER = KP * KP / NT;
  static_assert(KP * KP % NT == 0, "Gram tile must split evenly over the block");
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = G[threadIdx.x + u * NT];
#pragma unroll
  for (int u = 0; u < PER; ++u) sG[threadIdx.x + u * NT] = v[u];
}

// The block's rows [row0, row0 + nrow) of a row-major rows x r float32
// matrix form one contiguous range of nrow * r floats.  stage_rows copies it
// into dst[row][col] (LDS, row pitch LD) with coalesced loads, summing
// `nsplit` partials of stride pstride in split order; columns >= r and rows
// >= nrow are zero filled.  Each thread owns at most KP / T = 8 elements.
template <int KP, int LD>
__device__ __forceinline__ void stage_rows(const float* __restrict__ src, int nsplit,
                                           int64_t pstride, int64_t row0, int nrow, int r,
                                           float (*dst)[LD]) {
  using TM = Team<KP>;
  constexpr int PER = TM::RB * KP / TM::NT;
  const int cnt = nrow * r;
  const float* base = src + row0 * r;
  float v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * TM::NT;
    v[u] = e < cnt ? base[e] : 0.f;
  }
  // partials in batches of SB splits, all of a batch's loads issued before
  // the first is added (the additions keep split order)
  constexpr int SB = 8;
  for (int sp0 = 1; sp0 < nsplit; sp0 += SB) {
    float w[SB][PER];
#pragma unroll
    for (int b = 0; b < SB; ++b) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * TM::NT;
        w[b][u] = (sp0 + b < nsplit && e < cnt) ? base[(int64_t)(sp0 + b) * pstride + e] : 0.f;
      }
    }
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      if (sp0 + b < nsplit) {
#pragma unroll
        for (int u = 0; u < PER; ++u) v[u] += w[b][u];
      }
    }
  }
  for (int e = threadIdx.x; e < TM::RB * KP; e += TM::NT) dst[e / KP][e % KP] = 0.f;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * TM::NT;
    if (e < cnt) dst[e / r][e % r] = v[u];
  }
  __syncthreads();
}

// A thread's PER elements of a block's contiguous range of cnt > 0 floats
// at base: element e(u, c) = 4 (threadIdx.x + u NT) + c, u < PER / 4,
// c < 4.  With VEC (base 16-byte aligned, cnt a multiple of 4) each group
// of four is one 16-byte load.  Addresses past the range are clamped into
// it, so every load is issued unconditionally and all stay in flight
// together; the values of elements e >= cnt are unspecified and callers
// never store them (scatter_quads).
template <int NT, int PER, bool VEC>
__device__ __forceinline__ void load_quads(const float* __restrict__ base, int cnt, float* v) {
  static_assert(PER % 4 == 0, "whole quads per thread");
#pragma unroll
  for (int u = 0; u < PER / 4; ++u) {
    const int e = 4 * ((int)threadIdx.x + u * NT);
    if constexpr (VEC) {
      const float4 x = *reinterpret_cast<const float4*>(base + (e < cnt ? e : 0));
      v[4 * u] = x.x;
      v[4 * u + 1] = x.y;
      v[4 * u + 2] = x.z;
      v[4 * u + 3] = x.w;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[4 * u + c] = base[e + c < cnt ? e + c : 0];
    }
  }
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

// Scatter of a thread's load_quads elements e < cnt into LDS rows of width r.
template <int NT, int PER, int LD>
__device__ __forceinline__ void scatter_quads(float (*dst)[LD], const float* v, int cnt, int r) {
#pragma unroll
  for (int u = 0; u < PER / 4; ++u) {
    const int e = 4 * ((int)threadIdx.x + u * NT);
    if (e < cnt) {
      int row = e / r, col = e - row * r;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (e + c < cnt) dst[row][col] = v[4 * u + c];
        if (++col == r) { col = 0; ++row; }
      }
    }
  }
}

// One row block's inputs: G (KP x KP float64; G and sG 16-byte aligned)
// into sG, the block's rows of A into sa and (with_g, as for G) the summed
// split partials of P into sp; columns >= r and rows >= nrow are zero
// (nrow >= 1).  The loads of G, A, the first partial and the first batch of
// SB further partials are issued together, with no branch between them.
// Once G and A are in LDS, mid() runs (all threads; it may use sG and sa)
// while the partials are still in flight; then the partials are summed in
// split order and stored.  Rows and partials are read in 16-byte groups
// (load_quads) when their layout allows.
template <int KP, int LDA, int LDP, bool VEC, typename MID>
__device__ __forceinline__ void stage_block_impl(const double* __restrict__ G, double* sG,
                                                 const float* __restrict__ A, float (*sa)[LDA],
                                                 const float* __restrict__ P, int nsplit,
                                                 int64_t pstride, float (*sp)[LDP], int64_t row0,
                                                 int nrow, int r, bool with_g, MID&& mid) {
  using TM = Team<KP>;
  constexpr int PER = TM::RB * KP / TM::NT;
  constexpr int PG = KP * KP / TM::NT;   // Gram entries per thread, in pairs when even
  constexpr bool G2 = PG % 2 == 0;
  constexpr int SB = 8;
  static_assert(KP * KP % TM::NT == 0, "Gram tile must split evenly over the block");
  const int cnt = nrow * r;
  const float* abase = A + row0 * r;
  float av[PER];
  for (int e = threadIdx.x; e < TM::RB * KP; e += TM::NT) {
    sa[e / KP][e % KP] = 0.f;
    if (with_g) sp[e / KP][e % KP] = 0.f;
  }
  if (!with_g) {
    load_quads<TM::NT, PER, VEC>(abase, cnt, av);
    __syncthreads();
    scatter_quads<TM::NT, PER, LDA>(sa, av, cnt, r);
    __syncthreads();
    return;
  }
  const float* pbase = P + row0 * r;
  double gv[PG];
  float pv[PER], w[SB][PER];
  // partials in batches of SB splits, all of a batch's loads issued before
  // the first is added (the additions keep split order); splits past the
  // last re-read the last one and are not added
  auto load_batch = [&](int sp0) {
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int sb = sp0 + b < nsplit ? sp0 + b : nsplit - 1;
      load_quads<TM::NT, PER, VEC>(pbase + (int64_t)sb * pstride, cnt, w[b]);
    }
  };
  auto add_batch = [&](int sp0) {
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      if (sp0 + b < nsplit) {
#pragma unroll
        for (int u = 0; u < PER; ++u) pv[u] += w[b][u];
      }
    }
  };
  if constexpr (G2) {
#pragma unroll
    for (int u = 0; u < PG / 2; ++u) {
      const double2 x = reinterpret_cast<const double2*>(G)[threadIdx.x + u * TM::NT];
      gv[2 * u] = x.x;
      gv[2 * u + 1] = x.y;
    }
  } else {
#pragma unroll
    for (int u = 0; u < PG; ++u) gv[u] = G[threadIdx.x + u * TM::NT];
  }
  load_quads<TM::NT, PER, VEC>(abase, cnt, av);
  // G and A are issued first, so that their wait leaves the partials in flight
  __builtin_amdgcn_sched_barrier(0);
  load_quads<TM::NT, PER, VEC>(pbase, cnt, pv);
  load_batch(1);   // unconditional: a branch here would make the waits for G and A cover it
  if constexpr (G2) {
#pragma unroll
    for (int u = 0; u < PG / 2; ++u)
      reinterpret_cast<double2*>(sG)[threadIdx.x + u * TM::NT] = make_double2(gv[2 * u], gv[2 * u + 1]);
  } else {
#pragma unroll
    for (int u = 0; u < PG; ++u) sG[threadIdx.x + u * TM::NT] = gv[u];
  }
  __syncthreads();
  scatter_quads<TM::NT, PER, LDA>(sa, av, cnt, r);
  __syncthreads();
  mid();
  add_batch(1);
  for (int sp0 = 1 + SB; sp0 < nsplit; sp0 += SB) {
    load_batch(sp0);
    add_batch(sp0);
  }
  scatter_quads<TM::NT, PER, LDP>(sp, pv, cnt, r);
  __syncthreads();
}

template <int KP, int LDA, int LDP, typename MID>
__device__ __forceinline__ void stage_block(const double* __restrict__ G, double* sG,
                                            const float* __restrict__ A, float (*sa)[LDA],
                                            const float* __restrict__ P, int nsplit,
                                            int64_t pstride, float (*sp)[LDP], int64_t row0,
                                            int nrow, int r, bool with_g, MID&& mid) {
  // row0 is a multiple of the block's row count, so row0 * r keeps a
  // 16-byte aligned matrix aligned; the choice is the same for the whole
  // block, and each variant keeps all of its loads in flight together
  const bool vec = nrow * r % 4 == 0 && aligned16(A) &&
                   (!with_g || (aligned16(P) && pstride % 4 == 0));
  if (vec)
    stage_block_impl<KP, LDA, LDP, true>(G, sG, A, sa, P, nsplit, pstride, sp, row0, nrow, r, with_g, mid);
  else
    stage_block_impl<KP, LDA, LDP, false>(G, sG, A, sa, P, nsplit, pstride, sp, row0, nrow, r, with_g, mid);
}

// s[e] = sum_b row[b] G[b][c0+e] for the 8 columns c0..c0+7 (G symmetric).
template <int KP, typename RT>
__device__ __forceinline__ void row_times_g(const RT* row, const double* sG, int c0, double* s) {
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] = 0.0;
  for (int b = 0; b < KP; ++b) {
    const double x = (double)row[b];
    const double* g = sG + b * KP + c0;
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] = fma(x, g[e], s[e]);
  }
}

// sT[row][c] = sum_b A[row][b] G[b][c] for the RB rows of a block (A: LDS
// rows of float32, G: LDS KP x KP float64), on v_mfma_f64_16x16x4f64: the
// RB x KP result in 16 x 16 tiles dealt round robin to the block's waves.
// Lane (i, g) supplies A[i][g] and B[g][i] of each 16 x 4 by 4 x 16 step and
// receives D[g + 4 v][i].  Called by every thread of the block; barriers on
// entry and exit.
template <int KP, int LDA>
__device__ __forceinline__ void block_times_g(const float (*A)[LDA], const double* sG,
                                              double (*sT)[KP + 1]) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  using TM = Team<KP>;
  constexpr int TC = KP / 16;
  constexpr int NTILE = (TM::RB / 16) * TC;
  constexpr int NW = TM::NT / kWave;
  static_assert(KP % 16 == 0 && TM::RB % 16 == 0, "matrix-core row products need 16 | KP");
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  constexpr int PERW = (NTILE + NW - 1) / NW;
  __syncthreads();
  // a wave's tiles one after the other, each one chain over k
  d4 acc[PERW];
#pragma unroll
  for (int u = 0; u < PERW; ++u) {
    acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    const int tile = w + NW * u;
    if (tile < NTILE) {
      const int ti = tile / TC, tj = tile % TC;
#pragma unroll 4
      for (int k0 = 0; k0 < KP; k0 += 4)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)A[16 * ti + i][k0 + g],
                                                      sG[(k0 + g) * KP + 16 * tj + i], acc[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int u = 0; u < PERW; ++u) {
    const int tile = w + NW * u;
    if (tile < NTILE) {
      const int ti = tile / TC, tj = tile % TC;
#pragma unroll
      for (int v = 0; v < 4; ++v) sT[16 * ti + g + 4 * v][16 * tj + i] = acc[u][v];
    }
  }
  __syncthreads();
}

// Upper-triangle 4x4 tile `task` of a KP x KP matrix -> (ti, tj), ti <= tj.
template <int KP>
__device__ __forceinline__ void gram_tile(int task, int& ti, int& tj) {
  constexpr int NTILE = KP / 4;
  int i = 0, rem = task;
  while (rem >= NTILE - i) { rem -= NTILE - i; ++i; }
  ti = i;
  tj = i + rem;
}

// Check-record accumulators for one row: grad = a G - p (the gradient of
// eq. 1 through the Gram identity), projected gradient = grad where a > 0
// and min(grad, 0) where a <= 0 (the KKT appendix).
// q accumulates a . (a G), the row's share of <A^T A, G> (the quadratic
// term of the objective expansion).
struct CheckAcc {
  double pg2 = 0.0, sg = 0.0, mx = -INFINITY, ng2 = 0.0, sq = 0.0, ap = 0.0, nneg = 0.0,
         mn = INFINITY, q = 0.0;
  __device__ __forceinline__ void add(const float* a, const double* s, const double* p, int c0,
                                      int r) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (c0 + e < r) {
        const double gv = s[e] - p[e];
        const double av = (double)a[e];
        const double pgc = av > 0.0 ? gv : fmin(gv, 0.0);
        pg2 = fma(pgc, pgc, pg2);
        sg = fma(av, gv, sg);
        mx = fmax(mx, av * gv);
        if (av < 0.0) { ng2 = fma(av, av, ng2); nneg += 1.0; }
        sq = fma(av, av, sq);
        ap = fma(av, p[e], ap);
        mn = fmin(mn, av);
        q = fma(av, s[e], q);
      }
    }
  }
};

// Fixed-order reduction of NF per-thread values over a block of NT threads
// (every thread active).  kind[f]: 0 sum, 1 max, 2 min.  Each wave reduces
// every field with wave_reduce_last (register lane moves; the fields'
// moves are independent and overlap), lane 63 stores the wave's values, and
// thread 0 combines the waves in wave order.  The result lands in out[] of
// thread 0.
template <int NT, int NF>
__device__ __forceinline__ void block_reduce_fields(double* v, const int* kind, double* sh,
                                                    double* out) {
  constexpr int NW = NT / kWave;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int f = 0; f < NF; ++f)
    v[f] = kind[f] == 1 ? wave_reduce_last<1>(v[f])
                        : (kind[f] == 2 ? wave_reduce_last<2>(v[f]) : wave_reduce_last<0>(v[f]));
  __syncthreads();
  if (lane == kWave - 1) {
#pragma unroll
    for (int f = 0; f < NF; ++f) sh[f * NW + w] = v[f];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      double t = sh[f * NW];
      for (int i = 1; i < NW; ++i)
        t = kind[f] == 1 ? fmax(t, sh[f * NW + i]) : (kind[f] == 2 ? fmin(t, sh[f * NW + i]) : t + sh[f * NW + i]);
      out[f] = t;
    }
  }
}

}  // namespace enmf
