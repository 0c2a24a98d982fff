// Row-local kernels of the exterior phase and of HALS, the KKT check and
// the per-iteration bookkeeping (sections 3.2-3.3, Algorithms 2-3, the KKT
// appendix).  One thread owns one row of the factor being updated: the
// paper notes that the PBCD updates of different rows are independent, and
// the HALS column update is row-local too.  The r x r Gram (G = V^T V for the
// U half, H = U^T U for the V half) is zero padded to KP x KP float64 and read
// with wave-uniform loads.  Row state is float32; every dot product, step and
// reduction is float64.
#include <math.h>

#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kT = 256;

// part[b] = {#negative, min, sum x^2, sum max(0,-x)} over a contiguous chunk.
__global__ __launch_bounds__(kT) void k_factor_stats(const float* __restrict__ A, int64_t count,
                                                     int64_t per_block, double* __restrict__ part,
                                                     int block_offset) {
  __shared__ double sh[kT / kWave];
  const int64_t e0 = (int64_t)blockIdx.x * per_block;
  const int64_t e1 = e0 + per_block < count ? e0 + per_block : count;
  double neg = 0.0, mn = INFINITY, sq = 0.0, nm = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) {
    const double v = A[e];
    neg += v < 0.0 ? 1.0 : 0.0;
    mn = fmin(mn, v);
    sq = fma(v, v, sq);
    nm += v < 0.0 ? -v : 0.0;
  }
  neg = block_sum<kT>(neg, sh);
  mn = block_min<kT>(mn, sh);
  sq = block_sum<kT>(sq, sh);
  nm = block_sum<kT>(nm, sh);
  if (threadIdx.x == 0) {
    double* o = part + 4 * (int64_t)(block_offset + blockIdx.x);
    o[0] = neg; o[1] = mn; o[2] = sq; o[3] = nm;
  }
}

// Initial state of an iterate call: ||X||^2, push sizes resolved from the
// input (eq. negup has a fixed step the paper does not give; the reading is
// max(-min, 0) / (ext_iters - 0.5)), and the negative count of U and V.
__global__ void k_setup_state(const double* __restrict__ stat, int nbU, int nbV,
                              const double* __restrict__ xpart, int nx, double step_u,
                              double step_v, int ext_iters, DevState* st,
                              double* __restrict__ negpart, int nneg) {
  if (threadIdx.x == 0) {
    double nx2 = 0.0;
    for (int b = 0; b < nx; ++b) nx2 += xpart[b];
    double negs = 0.0, mnU = INFINITY, mnV = INFINITY;
    for (int b = 0; b < nbU; ++b) { negs += stat[4 * b]; mnU = fmin(mnU, stat[4 * b + 1]); }
    for (int b = nbU; b < nbU + nbV; ++b) { negs += stat[4 * b]; mnV = fmin(mnV, stat[4 * b + 1]); }
    const double d = (double)ext_iters - 0.5;
    st->nx2 = nx2;
    st->step[0] = step_u > 0.0 ? step_u : fmax(-mnU, 0.0) / d;
    st->step[1] = step_v > 0.0 ? step_v : fmax(-mnV, 0.0) / d;
    st->phase = negs > 0.0 ? kPhaseExt : kPhaseHals;
    st->negs = (int)negs;
    st->stop = 0;
    st->converged = 0;
    st->iters = 0;
    st->ext_done = 0;
    st->ntrace = 0;
    st->numeric_error = 0;
    st->pbcd_done[0] = st->pbcd_done[1] = 0;
    negpart[0] = negs;
  }
  for (int b = 1 + threadIdx.x; b < nneg; b += blockDim.x) negpart[3 * b] = 0.0;
}

// Top of an outer iteration: the phase is EXT while U or V has a negative
// entry (Algorithm 3 repeats the exterior block until U, V >= 0), else HALS.
// negpart holds the row-update partial records (3 doubles per block, the
// negative count first) of the U half followed by those of the V half.
__global__ __launch_bounds__(kT) void k_head(const double* __restrict__ negpart, int nparts,
                                             DevState* st) {
  __shared__ double sh[kT / kWave];
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kT) s += negpart[3 * b];
  s = block_sum<kT>(s, sh);
  if (threadIdx.x == 0 && !st->stop) {
    st->negs = (int)s;
    st->phase = s > 0.0 ? kPhaseExt : kPhaseHals;
    st->pbcd_done[0] = st->pbcd_done[1] = 0;
  }
}

// Row state in LDS: each thread keeps its row in 8-column blocks
// (layout [block][thread][8]) so that the loops over column blocks can be
// runtime loops around fully unrolled 8 x 8 bodies.
constexpr int kRT = 128;   // threads (rows) per row-update / check block

struct F8 { float v[8]; };

__device__ __forceinline__ F8 ld8(const float* base, int blk, int t) {
  F8 r;
  const float4* p = reinterpret_cast<const float4*>(base + ((int64_t)blk * kRT + t) * 8);
  const float4 x = p[0], y = p[1];
  r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
  r.v[4] = y.x; r.v[5] = y.y; r.v[6] = y.z; r.v[7] = y.w;
  return r;
}

__device__ __forceinline__ void st8(float* base, int blk, int t, const F8& r) {
  float4* p = reinterpret_cast<float4*>(base + ((int64_t)blk * kRT + t) * 8);
  p[0] = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  p[1] = make_float4(r.v[4], r.v[5], r.v[6], r.v[7]);
}

// s[e] = sum_b a_b G[b][cb*8+e] - p[e] for the 8 columns of block cb
// (G symmetric, KP x KP, zero padded).
template <int KP>
__device__ __forceinline__ void grad_block(const float* sa, int t, const double* __restrict__ G,
                                           int cb, const double* pv, double* s) {
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] = -pv[e];
  for (int bb = 0; bb < KP / 8; ++bb) {
    const F8 av = ld8(sa, bb, t);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double ai = (double)av.v[i];
#pragma unroll
      for (int e = 0; e < 8; ++e) s[e] = fma(ai, G[(bb * 8 + i) * KP + cb * 8 + e], s[e]);
    }
  }
}

__device__ __forceinline__ void load_p8(const float* __restrict__ P, bool valid, int64_t i, int r,
                                        int cb, double* pv) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = cb * 8 + e;
    pv[e] = (valid && c < r) ? (double)P[i * r + c] : 0.0;
  }
}

// One half of an outer iteration on the rows of A (U with P = X V, G = V^T V,
// or V with P = X^T U, G = U^T U), in the phase chosen by k_head.
//   HALS: for j = 1..r, a_j <- max(0, a_j + (p_j - a . G_:j) / G_jj), skipped
//         when G_jj = 0 (textbook HALS, Gauss-Seidel over columns).
//   EXT:  (first launch) push negatives by the step (eq. negup); mask of
//         nonnegative entries; then `sweeps` PBCD sweeps (eqs. pbcdu, d_i):
//         g = M o (a G - p), d = |g|^2 / (g G g^T) (0 if not positive),
//         a <- (a - d g)_+ on the mask, unmasked entries unchanged.
// part[b] = {#negative after the update, |M o grad|^2 before the sweeps,
//            |M o grad|^2 after the sweeps}.
template <int KP>
__global__ __launch_bounds__(kRT) void k_rowupdate(float* __restrict__ A, int64_t rows, int r,
                                                   const float* __restrict__ P,
                                                   const double* __restrict__ G, DevState* st,
                                                   int half, int sweeps, int first, int want_pg,
                                                   double* __restrict__ part) {
  constexpr int NB = KP / 8;
  __shared__ __align__(16) float sa[NB * kRT * 8];
  __shared__ __align__(16) float sg[NB * kRT * 8];
  __shared__ double sh[kRT / kWave];
  if (st->stop) return;
  const int phase = st->phase;
  if (!first && (phase == kPhaseHals || st->pbcd_done[half])) return;
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kRT + t;
  const bool valid = i < rows;
  const int64_t ic = valid ? i : 0;

  for (int cb = 0; cb < NB; ++cb) {
    F8 x;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = cb * 8 + e;
      x.v[e] = (valid && c < r) ? A[ic * r + c] : 0.f;
    }
    st8(sa, cb, t, x);
  }
  double negc = 0.0, gi2 = 0.0, pg2 = 0.0;

  if (phase == kPhaseHals) {
    for (int j = 0; j < r; ++j) {
      const double gjj = G[j * KP + j];
      if (gjj > 0.0) {
        double s = 0.0;
        for (int cb = 0; cb < NB; ++cb) {
          const F8 av = ld8(sa, cb, t);
#pragma unroll
          for (int e = 0; e < 8; ++e) s = fma((double)av.v[e], G[(cb * 8 + e) * KP + j], s);
        }
        float* aj = sa + ((int64_t)(j / 8) * kRT + t) * 8 + (j % 8);
        const double pj = valid ? (double)P[ic * r + j] : 0.0;
        const double v = (double)*aj + (pj - s) / gjj;
        *aj = (float)(v > 0.0 ? v : 0.0);
      }
    }
  } else {
    if (first) {
      const double step = st->step[half];
      for (int cb = 0; cb < NB; ++cb) {
        F8 x = ld8(sa, cb, t);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (x.v[e] < 0.f) x.v[e] = (float)((double)x.v[e] + step);
        st8(sa, cb, t, x);
      }
    }
    // mask M = (a >= 0); padded columns carry zeros and stay inert.
    for (int sw = 0; sw < sweeps; ++sw) {
      double num = 0.0;
      for (int cb = 0; cb < NB; ++cb) {
        double pv[8], s[8];
        load_p8(P, valid, ic, r, cb, pv);
        grad_block<KP>(sa, t, G, cb, pv, s);
        const F8 av = ld8(sa, cb, t);
        F8 g;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          g.v[e] = av.v[e] >= 0.f ? (float)s[e] : 0.f;
          num = fma((double)g.v[e], (double)g.v[e], num);
        }
        st8(sg, cb, t, g);
      }
      if (sw == 0 && first) gi2 = num;
      double den = 0.0;
      for (int cb = 0; cb < NB; ++cb) {
        double h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = 0.0;
        for (int bb = 0; bb < NB; ++bb) {
          const F8 gv = ld8(sg, bb, t);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double gq = (double)gv.v[q];
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = fma(G[(bb * 8 + q) * KP + cb * 8 + e], gq, h[e]);
          }
        }
        const F8 gc = ld8(sg, cb, t);
#pragma unroll
        for (int e = 0; e < 8; ++e) den = fma((double)gc.v[e], h[e], den);
      }
      const double d = den > 0.0 ? num / den : 0.0;
      for (int cb = 0; cb < NB; ++cb) {
        F8 av = ld8(sa, cb, t);
        const F8 gv = ld8(sg, cb, t);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (av.v[e] >= 0.f) {
            const double v = (double)av.v[e] - d * (double)gv.v[e];
            av.v[e] = (float)(v > 0.0 ? v : 0.0);
          }
        }
        st8(sa, cb, t, av);
      }
    }
    if (want_pg) {
      for (int cb = 0; cb < NB; ++cb) {
        double pv[8], s[8];
        load_p8(P, valid, ic, r, cb, pv);
        grad_block<KP>(sa, t, G, cb, pv, s);
        const F8 av = ld8(sa, cb, t);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (av.v[e] >= 0.f) pg2 = fma(s[e], s[e], pg2);
      }
    }
  }
  if (valid) {
    for (int cb = 0; cb < NB; ++cb) {
      const F8 av = ld8(sa, cb, t);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = cb * 8 + e;
        if (c < r) {
          A[i * r + c] = av.v[e];
          negc += av.v[e] < 0.f ? 1.0 : 0.0;
        }
      }
    }
  }
  negc = block_sum<kRT>(negc, sh);
  gi2 = block_sum<kRT>(gi2, sh);
  pg2 = block_sum<kRT>(pg2, sh);
  if (t == 0) {
    double* o = part + 3 * (int64_t)blockIdx.x;
    if (first) o[0] = negc;   // later sweeps never change the sign pattern
    o[1] = gi2;
    o[2] = pg2;
  }
}

// PBCD stop test of Algorithm 2 between sweep launches:
// stop when |M o grad| < eps |M o grad_init|.
__global__ __launch_bounds__(kT) void k_pbcd_decide(const double* __restrict__ part, int nparts,
                                                    int half, int first, DevState* st) {
  __shared__ double sh[kT / kWave];
  double gi = 0.0, pg = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kT) {
    gi += part[3 * b + 1];
    pg += part[3 * b + 2];
  }
  gi = block_sum<kT>(gi, sh);
  pg = block_sum<kT>(pg, sh);
  if (threadIdx.x == 0 && !st->stop && st->phase == kPhaseExt && !st->pbcd_done[half]) {
    if (first) st->thr2[half] = st->pbcd_eps * st->pbcd_eps * gi;
    if (pg < st->thr2[half]) st->pbcd_done[half] = 1;
  }
}

// Per-block KKT partials.  Blocks [0, nbU) cover the rows of U with
// (P = X V, G = V^T V); blocks [nbU, nbU + nbV) the rows of V with
// (Q = X^T U, H = U^T U).  grad = a G - p (the gradient of eq. 1 through the
// Gram identity), projected gradient = grad where a > 0, min(grad, 0) where
// a <= 0.  Record: {|pg|^2, sum a grad, max a grad, |min(a,0)|^2, |a|^2,
// sum a p, #negative, min a, 0...}.
template <int KP>
__global__ __launch_bounds__(kRT) void k_check(const float* __restrict__ U, int64_t m,
                                               const float* __restrict__ P,
                                               const double* __restrict__ G,
                                               const float* __restrict__ V, int64_t n,
                                               const float* __restrict__ Q,
                                               const double* __restrict__ H, int r, int nbU,
                                               const DevState* st, double* __restrict__ part) {
  constexpr int NB = KP / 8;
  __shared__ __align__(16) float sa[NB * kRT * 8];
  __shared__ double sh[kRT / kWave];
  if (st->stop) return;
  const bool isU = (int)blockIdx.x < nbU;
  const float* A = isU ? U : V;
  const float* Pm = isU ? P : Q;
  const double* Gm = isU ? G : H;
  const int64_t rows = isU ? m : n;
  const int t = threadIdx.x;
  const int64_t i = (int64_t)(isU ? blockIdx.x : blockIdx.x - nbU) * kRT + t;
  const bool valid = i < rows;
  const int64_t ic = valid ? i : 0;
  for (int cb = 0; cb < NB; ++cb) {
    F8 x;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = cb * 8 + e;
      x.v[e] = (valid && c < r) ? A[ic * r + c] : 0.f;
    }
    st8(sa, cb, t, x);
  }
  double pg2 = 0.0, sg = 0.0, mx = -INFINITY, ng2 = 0.0, sq = 0.0, ap = 0.0, nneg = 0.0,
         mn = INFINITY;
  if (valid) {
    for (int cb = 0; cb < NB; ++cb) {
      double pv[8], s[8];
      load_p8(Pm, valid, ic, r, cb, pv);
      grad_block<KP>(sa, t, Gm, cb, pv, s);
      const F8 av = ld8(sa, cb, t);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (cb * 8 + e < r) {
          const double a = (double)av.v[e];
          const double pgc = a > 0.0 ? s[e] : fmin(s[e], 0.0);
          pg2 = fma(pgc, pgc, pg2);
          sg = fma(a, s[e], sg);
          mx = fmax(mx, a * s[e]);
          if (a < 0.0) { ng2 = fma(a, a, ng2); nneg += 1.0; }
          sq = fma(a, a, sq);
          ap = fma(a, pv[e], ap);
          mn = fmin(mn, a);
        }
      }
    }
  }
  pg2 = block_sum<kRT>(pg2, sh);
  sg = block_sum<kRT>(sg, sh);
  mx = block_max<kRT>(mx, sh);
  ng2 = block_sum<kRT>(ng2, sh);
  sq = block_sum<kRT>(sq, sh);
  ap = block_sum<kRT>(ap, sh);
  nneg = block_sum<kRT>(nneg, sh);
  mn = block_min<kRT>(mn, sh);
  if (t == 0) {
    double* o = part + (int64_t)blockIdx.x * kCheckFields;
    o[0] = pg2; o[1] = sg; o[2] = mx; o[3] = ng2; o[4] = sq; o[5] = ap; o[6] = nneg; o[7] = mn;
    o[8] = 0.0; o[9] = 0.0; o[10] = 0.0; o[11] = 0.0;
  }
}

// Combine the KKT partials (fixed order), evaluate f through the expansion
// 1/2||X||^2 - <U, X V> + 1/2 <U^T U, V^T V>, the relative error, the KKT
// residual of the KKT appendix (normalised as documented in enmf.h), decide
// whether to stop, and append a trace record.
__global__ __launch_bounds__(kT) void k_check_finalize(const double* __restrict__ part, int nbU,
                                                       int nbV, const double* __restrict__ G,
                                                       const double* __restrict__ H, int kp, int k,
                                                       int final_check, DevState* st,
                                                       double* __restrict__ trace) {
  __shared__ double sh[kT / kWave];
  __shared__ double acc[2][8];
  if (st->stop) return;
  for (int side = 0; side < 2; ++side) {
    const int b0 = side == 0 ? 0 : nbU;
    const int b1 = side == 0 ? nbU : nbU + nbV;
    for (int f = 0; f < 8; ++f) {
      double v = (f == 2) ? -INFINITY : (f == 7 ? INFINITY : 0.0);
      for (int b = b0 + threadIdx.x; b < b1; b += kT) {
        const double x = part[(int64_t)b * kCheckFields + f];
        v = (f == 2) ? fmax(v, x) : (f == 7 ? fmin(v, x) : v + x);
      }
      v = (f == 2) ? block_max<kT>(v, sh) : (f == 7 ? block_min<kT>(v, sh) : block_sum<kT>(v, sh));
      if (threadIdx.x == 0) acc[side][f] = v;
    }
  }
  double hg = 0.0;
  for (int e = threadIdx.x; e < kp * kp; e += kT) hg = fma(H[e], G[e], hg);
  hg = block_sum<kT>(hg, sh);
  if (threadIdx.x != 0) return;
  const double nx2 = st->nx2;
  const double f = 0.5 * nx2 - acc[0][5] + 0.5 * hg;
  const double nx = sqrt(nx2);
  const double nU = sqrt(acc[0][4]), nV = sqrt(acc[1][4]);
  const double feas = fmax(nU > 0.0 ? sqrt(acc[0][3]) / nU : 0.0, nV > 0.0 ? sqrt(acc[1][3]) / nV : 0.0);
  const double pgu = (nV > 0.0 && nx > 0.0) ? sqrt(acc[0][0]) / (nx * nV) : 0.0;
  const double pgv = (nU > 0.0 && nx > 0.0) ? sqrt(acc[1][0]) / (nx * nU) : 0.0;
  const double kkt = fmax(feas, fmax(pgu, pgv));
  const double relerr = nx > 0.0 ? sqrt(fmax(2.0 * f, 0.0)) / nx : 0.0;
  const double negs = acc[0][6] + acc[1][6];
  st->f = f;
  st->relerr = relerr;
  st->kkt = kkt;
  st->kkt_feas = feas;
  st->kkt_pg_u = pgu;
  st->kkt_pg_v = pgv;
  st->delta_w = fmax(acc[0][2], acc[1][2]);
  st->sigma_u = acc[0][1];
  st->sigma_v = acc[1][1];
  st->sigma_w = acc[0][1] + acc[1][1];
  st->min_w = fmin(acc[0][7], acc[1][7]);
  st->re_paper = st->relerr_svd > 0.0 ? relerr / st->relerr_svd : NAN;
  const bool feasible = negs == 0.0;
  const bool hit = feasible && ((st->kkt_tol >= 0.0 && kkt <= st->kkt_tol) ||
                                (st->relerr_tol >= 0.0 && relerr - st->relerr_svd <= st->relerr_tol) ||
                                st->mode == 3);
  if (!isfinite(f) || !isfinite(kkt)) st->numeric_error = 1;
  if (trace != nullptr && st->ntrace < st->trace_cap) {
    double* o = trace + (int64_t)st->ntrace * kTraceFields;
    o[0] = (double)k; o[1] = f; o[2] = relerr; o[3] = kkt; o[4] = st->min_w;
    o[5] = (double)(negs > 0.0 ? kPhaseExt : kPhaseHals);
    o[6] = (double)wall_clock64() * st->ns_per_tick;
    o[7] = negs;
    st->ntrace += 1;
  }
  if (hit || final_check || st->numeric_error) {
    st->stop = 1;
    st->converged = hit ? 1 : 0;
  }
}

// Counts a completed outer iteration (runs after the V half).
__global__ void k_tail(DevState* st) {
  if (threadIdx.x != 0 || st->stop) return;
  st->iters += 1;
  if (st->phase == kPhaseExt) st->ext_done += 1;
}

__global__ void k_clip(float* __restrict__ A, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    A[e] = A[e] > 0.f ? A[e] : 0.f;
}

}  // namespace

int factor_blocks(int64_t count) {
  int64_t nb = (count + 4095) / 4096;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  const int64_t per = (count + nb - 1) / nb;
  return (int)((count + per - 1) / per);
}

hipError_t launch_factor_stats(const float* A, int64_t count, int r, double* part, int block_offset,
                               int nblocks, hipStream_t s) {
  (void)r;
  const int64_t per = (count + nblocks - 1) / nblocks;
  hipLaunchKernelGGL(k_factor_stats, dim3(nblocks), dim3(kT), 0, s, A, count, per, part,
                     block_offset);
  return hipGetLastError();
}

hipError_t launch_setup_state2(const double* statpart, int nbU, int nbV, const double* xpart,
                               int nxpart, double step_u, double step_v, int ext_iters,
                               DevState* st, double* negpart, int nneg, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_state, dim3(1), dim3(256), 0, s, statpart, nbU, nbV, xpart, nxpart,
                     step_u, step_v, ext_iters, st, negpart, nneg);
  return hipGetLastError();
}

hipError_t launch_head(const double* negpart, int nparts, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_head, dim3(1), dim3(kT), 0, s, negpart, nparts, st);
  return hipGetLastError();
}

hipError_t launch_tail(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_tail, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

int rowupdate_blocks(int64_t rows) { return (int)((rows + kRT - 1) / kRT); }

hipError_t launch_rowupdate(float* A, int64_t rows, int r, int kp, const float* P, const double* G,
                            DevState* st, int half, int sweeps, int first, int want_pg,
                            double* part, hipStream_t s) {
  dim3 g((unsigned)rowupdate_blocks(rows)), b(kRT);
  switch (kp) {
    case 8: hipLaunchKernelGGL((k_rowupdate<8>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first, want_pg, part); break;
    case 16: hipLaunchKernelGGL((k_rowupdate<16>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first, want_pg, part); break;
    case 32: hipLaunchKernelGGL((k_rowupdate<32>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first, want_pg, part); break;
    case 48: hipLaunchKernelGGL((k_rowupdate<48>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first, want_pg, part); break;
    default: hipLaunchKernelGGL((k_rowupdate<64>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first, want_pg, part); break;
  }
  return hipGetLastError();
}

hipError_t launch_pbcd_decide(const double* part, int nparts, int half, int first, DevState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pbcd_decide, dim3(1), dim3(kT), 0, s, part, nparts, half, first, st);
  return hipGetLastError();
}

hipError_t launch_check(const float* U, int64_t m, const float* P, const double* G, const float* V,
                        int64_t n, const float* Q, const double* H, int r, int kp, double* part,
                        int* nbU, int* nbV, DevState* st, hipStream_t s) {
  const int bu = (int)((m + kRT - 1) / kRT), bv = (int)((n + kRT - 1) / kRT);
  *nbU = bu;
  *nbV = bv;
  dim3 g((unsigned)(bu + bv)), b(kRT);
  switch (kp) {
    case 8: hipLaunchKernelGGL((k_check<8>), g, b, 0, s, U, m, P, G, V, n, Q, H, r, bu, st, part); break;
    case 16: hipLaunchKernelGGL((k_check<16>), g, b, 0, s, U, m, P, G, V, n, Q, H, r, bu, st, part); break;
    case 32: hipLaunchKernelGGL((k_check<32>), g, b, 0, s, U, m, P, G, V, n, Q, H, r, bu, st, part); break;
    case 48: hipLaunchKernelGGL((k_check<48>), g, b, 0, s, U, m, P, G, V, n, Q, H, r, bu, st, part); break;
    default: hipLaunchKernelGGL((k_check<64>), g, b, 0, s, U, m, P, G, V, n, Q, H, r, bu, st, part); break;
  }
  return hipGetLastError();
}

hipError_t launch_check_finalize(const double* part, int nbU, int nbV, const double* G,
                                 const double* H, int kp, int k, int final_check, DevState* st,
                                 double* trace, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finalize, dim3(1), dim3(kT), 0, s, part, nbU, nbV, G, H, kp, k,
                     final_check, st, trace);
  return hipGetLastError();
}

hipError_t launch_clip(float* A, int64_t count, hipStream_t s) {
  int64_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_clip, dim3((unsigned)g), dim3(256), 0, s, A, count);
  return hipGetLastError();
}

}  // namespace enmf
