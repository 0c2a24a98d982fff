// Row-local kernels of the exterior phase and of HALS, the KKT check and
// the per-iteration bookkeeping (sections 3.2-3.3, Algorithms 2-3, the KKT
// appendix).  The paper notes that the PBCD updates of different rows are
// independent, and the HALS column update is row-local too, so rows are the
// unit of parallelism: a team of KP/8 consecutive lanes owns one row, each
// lane holding 8 of its columns in registers.  The r x r Gram (G = V^T V for
// the U half, H = U^T U for the V half) is zero padded to KP x KP float64 and
// staged in LDS; the team exchanges row vectors through LDS and reduces with
// xor shuffles.  Row state is float32; dot products, steps and reductions
// are float64.
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

template <int KP>
__device__ __forceinline__ void load_gram(const double* __restrict__ G, double* sG) {
  for (int e = threadIdx.x; e < KP * KP; e += Team<KP>::NT) sG[e] = G[e];
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

// One half of an outer iteration on the rows of A (U with P = X V, G = V^T V,
// or V with P = X^T U, G = U^T U), in the phase chosen by k_head.
//   HALS: for j = 1..r, a_j <- max(0, a_j + (p_j - a . G_:j) / G_jj), skipped
//         when G_jj = 0 (textbook HALS, Gauss-Seidel over columns).  The
//         team keeps t = a G up to date: the owner of column j computes the
//         change of a_j from t_j and the others add it times row j of G.
//   EXT:  (first launch) push negatives by the step (eq. negup); mask of
//         nonnegative entries; then `sweeps` PBCD sweeps (eqs. pbcdu, d_i):
//         g = M o (a G - p), d = |g|^2 / (g G g^T) (0 if not positive),
//         a <- (a - d g)_+ on the mask, unmasked entries unchanged.
// part[b] = {#negative after the update, |M o grad|^2 before the sweeps,
//            |M o grad|^2 after the sweeps}.
template <int KP>
__global__ __launch_bounds__(Team<KP>::NT) void k_rowupdate(float* __restrict__ A, int64_t rows,
                                                            int r, const float* __restrict__ P,
                                                            const double* __restrict__ G,
                                                            DevState* st, int half, int sweeps,
                                                            int first, int want_pg,
                                                            double* __restrict__ part) {
  using TM = Team<KP>;
  constexpr int T = TM::T;
  __shared__ double sG[KP * KP];
  __shared__ float sa[TM::RB][KP + 1];
  __shared__ float sgv[TM::RB][KP + 1];
  __shared__ double sh[(TM::NT + kWave - 1) / kWave];
  if (st->stop) return;
  const int phase = st->phase;
  if (!first && (phase == kPhaseHals || st->pbcd_done[half])) return;
  const int team = threadIdx.x / T, q = threadIdx.x % T, c0 = 8 * q;
  const int64_t i = (int64_t)blockIdx.x * TM::RB + team;
  const bool valid = i < rows;
  const int64_t ic = valid ? i : 0;
  load_gram<KP>(G, sG);

  float a[8];
  double p[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = c0 + e;
    a[e] = (valid && c < r) ? A[ic * r + c] : 0.f;
    p[e] = (valid && c < r) ? (double)P[ic * r + c] : 0.0;
  }
  double negc = 0.0, gi2 = 0.0, pg2 = 0.0;

  if (phase == kPhaseHals) {
#pragma unroll
    for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
    __syncthreads();
    double t[8];
    row_times_g<KP>(sa[team], sG, c0, t);
    const int base = (threadIdx.x % kWave) - q;
    for (int j = 0; j < r; ++j) {
      const int o = j / 8, ej = j % 8;
      double delta = 0.0;
      if (q == o) {
        const double gjj = sG[j * KP + j];
        if (gjj > 0.0) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (e == ej) {
              const double v = (double)a[e] + (p[e] - t[e]) / gjj;
              const float nv = (float)(v > 0.0 ? v : 0.0);
              delta = (double)nv - (double)a[e];
              a[e] = nv;
            }
          }
        }
      }
      delta = __shfl(delta, base + o);
      const double* gj = sG + j * KP + c0;
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = fma(delta, gj[e], t[e]);
    }
  } else {
    if (first) {
      const double step = st->step[half];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (a[e] < 0.f) a[e] = (float)((double)a[e] + step);
    }
    // mask M = (a >= 0); padded columns carry zeros and stay inert.
    for (int sw = 0; sw < sweeps; ++sw) {
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      double s[8];
      row_times_g<KP>(sa[team], sG, c0, s);
      float g[8];
      double num = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        g[e] = a[e] >= 0.f ? (float)(s[e] - p[e]) : 0.f;
        num = fma((double)g[e], (double)g[e], num);
        sgv[team][c0 + e] = g[e];
      }
      if (sw == 0 && first) gi2 = num;
      __syncthreads();
      double h[8];
      row_times_g<KP>(sgv[team], sG, c0, h);
      double den = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) den = fma((double)g[e], h[e], den);
      num = team_sum<T>(num);
      den = team_sum<T>(den);
      const double d = den > 0.0 ? num / den : 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (a[e] >= 0.f) {
          const double v = (double)a[e] - d * (double)g[e];
          a[e] = (float)(v > 0.0 ? v : 0.0);
        }
      }
    }
    if (want_pg) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      double s[8];
      row_times_g<KP>(sa[team], sG, c0, s);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double gv = s[e] - p[e];
        if (a[e] >= 0.f) pg2 = fma(gv, gv, pg2);
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      if (c < r) {
        A[i * r + c] = a[e];
        negc += a[e] < 0.f ? 1.0 : 0.0;
      }
    }
  }
  negc = block_sum<TM::NT>(negc, sh);
  gi2 = block_sum<TM::NT>(gi2, sh);
  pg2 = block_sum<TM::NT>(pg2, sh);
  if (threadIdx.x == 0) {
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
__global__ __launch_bounds__(Team<KP>::NT) void k_check(const float* __restrict__ U, int64_t m,
                                                        const float* __restrict__ P,
                                                        const double* __restrict__ G,
                                                        const float* __restrict__ V, int64_t n,
                                                        const float* __restrict__ Q,
                                                        const double* __restrict__ H, int r,
                                                        int nbU, const DevState* st,
                                                        double* __restrict__ part) {
  using TM = Team<KP>;
  constexpr int T = TM::T;
  __shared__ double sG[KP * KP];
  __shared__ float sa[TM::RB][KP + 1];
  __shared__ double sh[(TM::NT + kWave - 1) / kWave];
  if (st->stop) return;
  const bool isU = (int)blockIdx.x < nbU;
  const float* A = isU ? U : V;
  const float* Pm = isU ? P : Q;
  const int64_t rows = isU ? m : n;
  const int team = threadIdx.x / T, q = threadIdx.x % T, c0 = 8 * q;
  const int64_t i = (int64_t)(isU ? blockIdx.x : blockIdx.x - nbU) * TM::RB + team;
  const bool valid = i < rows;
  const int64_t ic = valid ? i : 0;
  load_gram<KP>(isU ? G : H, sG);
  float a[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = c0 + e;
    a[e] = (valid && c < r) ? A[ic * r + c] : 0.f;
    sa[team][c] = a[e];
  }
  __syncthreads();
  double s[8];
  row_times_g<KP>(sa[team], sG, c0, s);
  double pg2 = 0.0, sg = 0.0, mx = -INFINITY, ng2 = 0.0, sq = 0.0, ap = 0.0, nneg = 0.0,
         mn = INFINITY;
  if (valid) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c0 + e;
      if (c < r) {
        const double pc = (double)Pm[ic * r + c];
        const double gv = s[e] - pc;
        const double av = (double)a[e];
        const double pgc = av > 0.0 ? gv : fmin(gv, 0.0);
        pg2 = fma(pgc, pgc, pg2);
        sg = fma(av, gv, sg);
        mx = fmax(mx, av * gv);
        if (av < 0.0) { ng2 = fma(av, av, ng2); nneg += 1.0; }
        sq = fma(av, av, sq);
        ap = fma(av, pc, ap);
        mn = fmin(mn, av);
      }
    }
  }
  pg2 = block_sum<TM::NT>(pg2, sh);
  sg = block_sum<TM::NT>(sg, sh);
  mx = block_max<TM::NT>(mx, sh);
  ng2 = block_sum<TM::NT>(ng2, sh);
  sq = block_sum<TM::NT>(sq, sh);
  ap = block_sum<TM::NT>(ap, sh);
  nneg = block_sum<TM::NT>(nneg, sh);
  mn = block_min<TM::NT>(mn, sh);
  if (threadIdx.x == 0) {
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

template <int KP>
void rowupdate_launch(float* A, int64_t rows, int r, const float* P, const double* G, DevState* st,
                      int half, int sweeps, int first, int want_pg, double* part, hipStream_t s) {
  using TM = Team<KP>;
  dim3 g((unsigned)((rows + TM::RB - 1) / TM::RB)), b(TM::NT);
  hipLaunchKernelGGL((k_rowupdate<KP>), g, b, 0, s, A, rows, r, P, G, st, half, sweeps, first,
                     want_pg, part);
}

template <int KP>
void check_launch(const float* U, int64_t m, const float* P, const double* G, const float* V,
                  int64_t n, const float* Q, const double* H, int r, double* part, int* nbU,
                  int* nbV, DevState* st, hipStream_t s) {
  using TM = Team<KP>;
  const int bu = (int)((m + TM::RB - 1) / TM::RB), bv = (int)((n + TM::RB - 1) / TM::RB);
  *nbU = bu;
  *nbV = bv;
  hipLaunchKernelGGL((k_check<KP>), dim3((unsigned)(bu + bv)), dim3(TM::NT), 0, s, U, m, P, G, V, n,
                     Q, H, r, bu, st, part);
}

}  // namespace

int row_pad(int r) {
  if (r <= 8) return 8;
  if (r <= 16) return 16;
  if (r <= 32) return 32;
  return 64;
}

int factor_blocks(int64_t count) {
  int64_t nb = (count + 4095) / 4096;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  const int64_t per = (count + nb - 1) / nb;
  return (int)((count + per - 1) / per);
}

int rowupdate_blocks(int64_t rows, int kp) {
  const int rb = kp / 8 <= 4 ? 64 : 32;
  return (int)((rows + rb - 1) / rb);
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

hipError_t launch_rowupdate(float* A, int64_t rows, int r, int kp, const float* P, const double* G,
                            DevState* st, int half, int sweeps, int first, int want_pg,
                            double* part, hipStream_t s) {
  switch (kp) {
    case 8: rowupdate_launch<8>(A, rows, r, P, G, st, half, sweeps, first, want_pg, part, s); break;
    case 16: rowupdate_launch<16>(A, rows, r, P, G, st, half, sweeps, first, want_pg, part, s); break;
    case 32: rowupdate_launch<32>(A, rows, r, P, G, st, half, sweeps, first, want_pg, part, s); break;
    default: rowupdate_launch<64>(A, rows, r, P, G, st, half, sweeps, first, want_pg, part, s); break;
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
  switch (kp) {
    case 8: check_launch<8>(U, m, P, G, V, n, Q, H, r, part, nbU, nbV, st, s); break;
    case 16: check_launch<16>(U, m, P, G, V, n, Q, H, r, part, nbU, nbV, st, s); break;
    case 32: check_launch<32>(U, m, P, G, V, n, Q, H, r, part, nbU, nbV, st, s); break;
    default: check_launch<64>(U, m, P, G, V, n, Q, H, r, part, nbU, nbV, st, s); break;
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
