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
#include "decide.h"
#include "row_team.h"

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

// Initial state of an iterate call: ||X||^2 and the push sizes resolved from
// the input (eq. negup has a fixed step the paper does not give; the reading
// is max(-min, 0) / (ext_iters - 0.5)).  The phase of the first iteration is
// decided later from the row-update records, like every other iteration's.
__global__ void k_setup_state(const double* __restrict__ stat, int nbU, int nbV,
                              const double* __restrict__ xpart, int nx, double step_u,
                              double step_v, int ext_iters, int check_every, DevState* st) {
  if (threadIdx.x != 0) return;
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
  st->check_every = check_every > 0 ? check_every : 1;
  st->kcur = 0;
}

// One half of an outer iteration on the rows of A (U with P = X V, G = V^T V,
// or V with P = X^T U, G = U^T U).  P arrives as `nsplit` float32 partial
// products (stride pstride) summed here in split order.
//   HALS: for j = 1..r, a_j <- max(0, a_j + (p_j - a . G_:j) / G_jj), skipped
//         when G_jj = 0 (textbook HALS, Gauss-Seidel over columns).  The
//         team keeps t = a G up to date: the owner of column j computes the
//         change of a_j from t_j and the others add it times row j of G.
//   EXT:  (first launch) push negatives by the step (eq. negup); mask of
//         nonnegative entries; then `sweeps` PBCD sweeps (eqs. pbcdu, d_i):
//         g = M o (a G - p), d = |g|^2 / (g G g^T) (0 if not positive),
//         a <- (a - d g)_+ on the mask, unmasked entries unchanged.  Mode 2
//         (the fixed-step ablation) takes d = 1/||G||_F for every row.
// Flags select the extra work fused into the pass:
//   kRowHead        phase of this iteration from the negative counts in the
//                   previous records of both halves (EXT while U or V has a
//                   negative entry, Algorithm 3); block 0 publishes it.
//   kRowWriteCheck  KKT-check partials of the rows, at the input state with
//                   kRowCheckPre, else at the output state.
//   kRowGram        this block's partial Gram (upper 4x4 tiles, float64) of
//                   the output rows, for k_gram_fin.
// With `pack`, the output rows are also written as the packed split factor
// the next matrix-core product reads (chunks of pc rows, width pkp <= KP,
// row pitch pldt; see store_split_run8), the last block zeroing the rest of
// the last chunk.
// The result goes to Aout (which may be A).  rec[b] = {#negative of the
// output, |M o grad|^2 before the sweeps, |M o grad|^2 after, 0, check...}.
template <int KP, bool LOOP>
__global__ __launch_bounds__(Team<KP>::NT, (KP >= 16 && (LOOP ? KP >= 32 : true)) ? 2 : 1) void k_rowupdate(
    const float* A, float* Aout, int64_t rows, int r,
    const float* __restrict__ P, int nsplit, int64_t pstride, const double* __restrict__ G,
    DevState* st, int half, int sweeps, int flags, double* __restrict__ rec,
    double* __restrict__ gpart, const double* __restrict__ headU, int nbU,
    const double* __restrict__ headV, int nbV, unsigned short* __restrict__ pack, int pkp, int pc,
    int pldt, float* __restrict__ padout, DecideArgs dec) {
  using TM = Team<KP>;
  constexpr int T = TM::T;
  constexpr int NW = TM::NT / kWave;
  constexpr int NF = 3 + kRecChkN;
  __shared__ __align__(16) double sG[KP * KP];
  __shared__ __align__(16) float sa[TM::RB][KP + 4];
  __shared__ float sgv[TM::RB][KP + 1];
  __shared__ double sT[KP >= 16 ? TM::RB : 1][KP + 1];
  __shared__ double sinv[KP];
  __shared__ double sh[(NF > 17 ? NF : 17) * NW];
  __shared__ int sflag;
  if (st->stop) return;
  if ((flags & kRowDecide) && check_decide<TM::NT>(dec, 0, st, blockIdx.x == 0, sh, &sflag)) return;
  const bool update = (flags & kRowUpdate) != 0;
  const bool first = (flags & kRowFirst) != 0;
  const bool chk = (flags & kRowWriteCheck) != 0;
  const bool pre = (flags & kRowCheckPre) != 0;
  const bool want_pg = (flags & kRowWantPg) != 0;
  int phase;
  if (flags & kRowHead) {
    phase = take_phase<TM::NT>(headU, nbU, headV, nbV, st, blockIdx.x == 0, sh);
  } else {
    phase = st->phase;
  }
  if (update && !first && (phase == kPhaseHals || st->pbcd_done[half])) return;
  const int team = threadIdx.x / T, q = threadIdx.x % T, c0 = 8 * q;
  const bool needG = update || chk;
  constexpr int NTILE = KP / 4;
  constexpr int NTASK = NTILE * (NTILE + 1) / 2;
  static_assert(NTASK <= TM::NT, "one Gram tile per thread");
  const bool gram = (flags & kRowGram) != 0;
  CheckAcc ck;
  double gi2 = 0.0, pg2 = 0.0, negc = 0.0;
  // blocks of TM::RB rows, grid-strided (LOOP) when there are more than
  // kRowBlocksMax of them: the records and partial Grams stay one per
  // launched block however many rows there are
  const int64_t nrb = (rows + TM::RB - 1) / TM::RB;
  for (int64_t rb = blockIdx.x; rb < nrb; rb = LOOP ? rb + gridDim.x : nrb) {
  const int64_t row0 = rb * TM::RB;
  const int nrow = (int)(rows - row0 < TM::RB ? rows - row0 : TM::RB);
  const bool valid = team < nrow;

  // out = (row of `src` owned by this team) G, through the matrix cores when KP >= 16
  auto times_g = [&](auto src, double* out) {
    if constexpr (KP >= 16) {
      block_times_g<KP>(src, sG, sT);
#pragma unroll
      for (int e = 0; e < 8; ++e) out[e] = sT[team][c0 + e];
    } else {
      row_times_g<KP>(src[team], sG, c0, out);
    }
  };
  float a[8];
  double p[8];
  double t[8];
  bool have_t = false;   // t == a G for the current a
  // t = a G for the input rows, when the check at the input state or HALS
  // wants it, is formed while the split partials of P are still arriving
  // (not in the looping variant, whose registers would spill)
  const bool early_t = !LOOP && needG && ((chk && pre) || (update && phase == kPhaseHals));
  stage_block<KP, KP + 4, KP + 1>(G, sG, A, sa, P, nsplit, pstride, sgv, row0, nrow, r, needG,
                                  [&] {
                                    if (early_t) {
                                      times_g(sa, t);
                                      have_t = true;
                                    }
                                  });
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = sa[team][c0 + e];
    p[e] = needG ? (double)sgv[team][c0 + e] : 0.0;
  }
  // reciprocals of the Gram diagonal for the HALS steps (0 skips a column)
  if (needG && threadIdx.x < KP) {
    const double gjj = sG[threadIdx.x * KP + threadIdx.x];
    sinv[threadIdx.x] = gjj > 0.0 ? 1.0 / gjj : 0.0;
  }
  __syncthreads();
  if (chk && pre) {
    if (!have_t) {
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      times_g(sa, t);
      have_t = true;
    }
    if (valid) ck.add(a, t, p, c0, r);
  }

  if (update && phase == kPhaseHals) {
    if (!have_t) {
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      times_g(sa, t);
    }
    // Columns in blocks of 8, one block per team lane: the owner runs the
    // block's steps on its own t (no exchange inside the block), then the
    // team takes the 8 changes at once and applies them in column order,
    // the same fma sequence as one column at a time.  Inside the block the
    // owner adds a change only to the columns still to come (the next step
    // waits on those) and adds it to the earlier columns after the block;
    // each t[e] still receives the changes in column order.  The steps are
    // branch-free so that the Gram rows can be read ahead: a padded column
    // (j >= r, zero Gram row and diagonal) or one with G_jj = 0 changes
    // nothing.  The other lanes' update is unconditional too (the owner adds
    // zeros), so that its Gram rows are read while the changes are exchanged.
    double ig[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) ig[e] = sinv[c0 + e];
    const int base = (threadIdx.x % kWave) - q;
    if constexpr (!LOOP) {
      // The lane's 8 x 8 block of Gram rows 8o..8o+7 at its own columns is
      // loaded into registers before the block's steps (for the owner it is
      // the diagonal block), so the chain of steps waits on no LDS read.
      // (Not in the looping variant, whose registers would spill.)
      for (int o = 0; 8 * o < r; ++o) {
        double g[8][8];
#pragma unroll
        for (int ej = 0; ej < 8; ++ej)
#pragma unroll
          for (int e = 0; e < 8; ++e) g[ej][e] = sG[(8 * o + ej) * KP + c0 + e];
        __builtin_amdgcn_sched_barrier(0);
        double dl[8];
#pragma unroll
        for (int ej = 0; ej < 8; ++ej) dl[ej] = 0.0;
        if (q == o) {
#pragma unroll
          for (int ej = 0; ej < 8; ++ej) {
            const bool on = ig[ej] > 0.0;
            const double v = (double)a[ej] + (p[ej] - t[ej]) * ig[ej];
            const float nv = (float)(v > 0.0 ? v : 0.0);
            const double d = on ? (double)nv - (double)a[ej] : 0.0;
            a[ej] = on ? nv : a[ej];
            dl[ej] = d;
#pragma unroll
            for (int e = ej + 1; e < 8; ++e) t[e] = fma(d, g[ej][e], t[e]);
          }
#pragma unroll
          for (int ej = 0; ej < 8; ++ej)
#pragma unroll
            for (int e = 0; e <= ej; ++e) t[e] = fma(dl[ej], g[ej][e], t[e]);
        }
#pragma unroll
        for (int ej = 0; ej < 8; ++ej) {
          const double x = __shfl(dl[ej], base + o);
          dl[ej] = q == o ? 0.0 : x;
        }
#pragma unroll
        for (int ej = 0; ej < 8; ++ej)
#pragma unroll
          for (int e = 0; e < 8; ++e) t[e] = fma(dl[ej], g[ej][e], t[e]);
      }
    } else
    for (int o = 0; 8 * o < r; ++o) {
      double dl[8];
#pragma unroll
      for (int ej = 0; ej < 8; ++ej) dl[ej] = 0.0;
      if (q == o) {
#pragma unroll
        for (int ej = 0; ej < 8; ++ej) {
          const double* gj = sG + (c0 + ej) * KP + c0;
          const bool on = ig[ej] > 0.0;
          const double v = (double)a[ej] + (p[ej] - t[ej]) * ig[ej];
          const float nv = (float)(v > 0.0 ? v : 0.0);
          const double d = on ? (double)nv - (double)a[ej] : 0.0;
          a[ej] = on ? nv : a[ej];
          dl[ej] = d;
#pragma unroll
          for (int e = ej + 1; e < 8; ++e) t[e] = fma(d, gj[e], t[e]);
        }
#pragma unroll
        for (int ej = 0; ej < 8; ++ej) {
          const double* gj = sG + (c0 + ej) * KP + c0;
#pragma unroll
          for (int e = 0; e <= ej; ++e) t[e] = fma(dl[ej], gj[e], t[e]);
        }
      }
#pragma unroll
      for (int ej = 0; ej < 8; ++ej) {
        const double x = __shfl(dl[ej], base + o);
        dl[ej] = q == o ? 0.0 : x;
      }
#pragma unroll
      for (int ej = 0; ej < 8; ++ej) {
        const double* gj = sG + (8 * o + ej) * KP + c0;
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = fma(dl[ej], gj[e], t[e]);
      }
    }
    have_t = true;
  } else if (update) {
    // mode 2, the fixed-step ablation: one row step 1/||G||_F in place of d
    double dfix = -1.0;
    if (st->mode == 2) {
      double ss = 0.0;
      for (int e = threadIdx.x; e < KP * KP; e += TM::NT) ss = fma(sG[e], sG[e], ss);
      ss = block_sum<TM::NT>(ss, sh);
      dfix = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    }
    if (first) {
      const double step = st->step[half];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (a[e] < 0.f) a[e] = (float)((double)a[e] + step);
    }
    // mask M = (a >= 0); padded columns carry zeros and stay inert.
    for (int sw = 0; sw < sweeps; ++sw) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      double s[8];
      times_g(sa, s);
      float g[8];
      double num = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        g[e] = a[e] >= 0.f ? (float)(s[e] - p[e]) : 0.f;
        num = fma((double)g[e], (double)g[e], num);
        sgv[team][c0 + e] = g[e];
      }
      if (sw == 0 && first) gi2 += num;
      __syncthreads();
      double h[8];
      times_g(sgv, h);
      double den = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) den = fma((double)g[e], h[e], den);
      num = team_sum<T>(num);
      den = team_sum<T>(den);
      const double d = dfix >= 0.0 ? dfix : (den > 0.0 ? num / den : 0.0);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (a[e] >= 0.f) {
          const double v = (double)a[e] - d * (double)g[e];
          a[e] = (float)(v > 0.0 ? v : 0.0);
        }
      }
    }
    have_t = false;
  }
  // gradient at the output state, when wanted
  if ((chk && !pre) || (want_pg && update && phase == kPhaseExt)) {
    if (!have_t) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[team][c0 + e] = a[e];
      __syncthreads();
      times_g(sa, t);
    }
    if (want_pg && update && phase == kPhaseExt) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double gv = t[e] - p[e];
        if (a[e] >= 0.f) pg2 = fma(gv, gv, pg2);
      }
    }
    if (chk && !pre && valid) ck.add(a, t, p, c0, r);
  }
  if (valid) {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (c0 + e < r) negc += a[e] < 0.f ? 1.0 : 0.0;
  }
  // output rows through LDS: coalesced stores, and the operand of the Gram
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 8; ++e) sa[team][c0 + e] = valid ? a[e] : 0.f;
  __syncthreads();
  if (update) {
    constexpr int PER = TM::RB * KP / TM::NT;
    const int cnt = nrow * r;
    float* base = Aout + row0 * r;
    if (!LOOP && cnt % 4 == 0 && aligned16(Aout)) {
      // 16-byte stores of four consecutive elements (row0 * r is a multiple
      // of 4); the looping variant keeps element stores for its registers
#pragma unroll
      for (int u = 0; u < PER / 4; ++u) {
        const int e = 4 * ((int)threadIdx.x + u * TM::NT);
        if (e < cnt) {
          int row = e / r, col = e - row * r;
          float x[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            x[c] = sa[row][col];
            if (++col == r) { col = 0; ++row; }
          }
          *reinterpret_cast<float4*>(base + e) = make_float4(x[0], x[1], x[2], x[3]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * TM::NT;
        if (e < cnt) base[e] = sa[e / r][e % r];
      }
    }
    if (padout != nullptr) {
      // rows of KP floats: the first r columns of the output, zeros after
      float* pb = padout + row0 * KP;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * TM::NT;
        if (e < nrow * KP) pb[e] = e % KP < r ? sa[e / KP][e % KP] : 0.f;
      }
    }
  }
  if (pack != nullptr) {
    const int64_t chunk_end = (rows + pc - 1) / pc * pc;
    const int64_t end = rb == nrb - 1 ? chunk_end : row0 + TM::RB;
    const int nruns = (int)((end - row0) / 8);
    const int64_t term = (int64_t)pkp * pldt;
    for (int task = threadIdx.x; task < pkp * nruns; task += TM::NT) {
      const int lr = 8 * (task % nruns), c = task / nruns;
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = lr < TM::RB ? sa[lr + u][c] : 0.f;
      const int64_t row = row0 + lr;
      store_split_run8(v, pack + (row / pc) * 3 * term + (int64_t)c * pldt + row % pc, term);
    }
  }
  if constexpr (KP >= 16) {
    if (gram) {
      // this row block's part, added to the block's running partial Gram:
      // the upper 16 x 16 tiles of sa^T sa on the matrix cores (one wave per
      // tile, round robin), stored as the upper 4 x 4 tiles that k_gram_fin
      // combines.  Lane (i, g) supplies sa[k0 + g][16 TI + i] and
      // sa[k0 + g][16 TJ + i] and receives entry (16 TI + g + 4 v, 16 TJ + i).
      typedef double d4 __attribute__((ext_vector_type(4)));
      constexpr int TB = KP / 16;
      constexpr int NBT = TB * (TB + 1) / 2;
      constexpr int NWG = TM::NT / kWave;
      const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
      const int i = lane % 16, g = lane / 16;
      double* ob = gpart + (int64_t)blockIdx.x * (16 * NTASK);
      const bool again = rb != blockIdx.x;
      for (int bt = wv; bt < NBT; bt += NWG) {
        int TI = 0, rem = bt;
        while (rem >= TB - TI) { rem -= TB - TI; ++TI; }
        const int TJ = TI + rem;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int k0 = 0; k0 < TM::RB; k0 += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)sa[k0 + g][16 * TI + i],
                                                     (double)sa[k0 + g][16 * TJ + i], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int R = 16 * TI + g + 4 * v, C = 16 * TJ + i;
          const int ti = R / 4, tj = C / 4;
          if (ti <= tj) {
            const int task = ti * NTILE - ti * (ti - 1) / 2 + (tj - ti);
            double* o = ob + 16 * task + 4 * (R % 4) + (C % 4);
            *o = again ? *o + acc[v] : acc[v];
          }
        }
      }
    }
  } else if (gram && threadIdx.x < NTASK) {
    // this row block's part, added to the block's running partial Gram
    int ti, tj;
    gram_tile<KP>(threadIdx.x, ti, tj);
    double gacc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) gacc[e] = 0.0;
    for (int row = 0; row < TM::RB; ++row) {
      const float4 x = *reinterpret_cast<const float4*>(&sa[row][4 * ti]);
      const float4 y = *reinterpret_cast<const float4*>(&sa[row][4 * tj]);
      const double xv[4] = {(double)x.x, (double)x.y, (double)x.z, (double)x.w};
      const double yv[4] = {(double)y.x, (double)y.y, (double)y.z, (double)y.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) gacc[4 * u + v] = fma(xv[u], yv[v], gacc[4 * u + v]);
    }
    double* o = gpart + (int64_t)blockIdx.x * (16 * NTASK) + 16 * threadIdx.x;
    const bool again = rb != blockIdx.x;
#pragma unroll
    for (int e = 0; e < 16; ++e) o[e] = again ? o[e] + gacc[e] : gacc[e];
  }
  __syncthreads();   // the next row block restages the shared arrays
  }  // row blocks
  double vals[NF] = {negc, gi2, pg2, ck.pg2, ck.sg, ck.mx, ck.ng2, ck.sq, ck.ap, ck.nneg, ck.mn, ck.q};
  const int kind[NF] = {0, 0, 0, 0, 0, 1, 0, 0, 0, 0, 2, 0};
  double red[NF];
  block_reduce_fields<TM::NT, NF>(vals, kind, sh, red);
  if (threadIdx.x == 0) {
    double* o = rec + (int64_t)blockIdx.x * kRecFields;
    o[kRecNeg] = red[0];
    o[kRecGi] = red[1];
    o[kRecPg] = red[2];
    if (chk) {
#pragma unroll
      for (int f = 0; f < kRecChkN; ++f) o[kRecChk + f] = red[3 + f];
    }
  }
}

// G (KP x KP, symmetric, zero padded) = sum over blocks of the partial Grams
// written by k_rowupdate, in block order (gram_combine: one wave per entry).
template <int KP>
__global__ __launch_bounds__(256) void k_gram_fin(const double* __restrict__ gpart, int nparts,
                                                  double* __restrict__ out) {
  gram_combine(gpart, nparts, KP, out, (int64_t)(blockIdx.x * blockDim.x + threadIdx.x) / kWave,
               (int64_t)gridDim.x * blockDim.x / kWave);
}

// PBCD stop test of Algorithm 2 between sweep launches:
// stop when |M o grad| < eps |M o grad_init|.
__global__ __launch_bounds__(kT) void k_pbcd_decide(const double* __restrict__ rec, int nparts,
                                                    int half, int first, DevState* st) {
  __shared__ double sh[kT / kWave];
  double gi = 0.0, pg = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kT) {
    gi += rec[(int64_t)b * kRecFields + kRecGi];
    pg += rec[(int64_t)b * kRecFields + kRecPg];
  }
  gi = block_sum<kT>(gi, sh);
  pg = block_sum<kT>(pg, sh);
  if (threadIdx.x == 0 && !st->stop && st->phase == kPhaseExt && !st->pbcd_done[half]) {
    if (first) st->thr2[half] = st->pbcd_eps * st->pbcd_eps * gi;
    if (pg < st->thr2[half]) st->pbcd_done[half] = 1;
  }
}

// The check and stop decision of iteration k as a launch of its own (the
// final check, and solves whose V pass does not carry kRowDecide).
__global__ __launch_bounds__(kT) void k_finalize(DecideArgs d, int final_check, DevState* st) {
  __shared__ double sh[17 * (kT / kWave)];
  __shared__ int flag;
  if (st->stop) return;
  (void)check_decide<kT>(d, final_check, st, true, sh, &flag);
}

__global__ void k_clip(float* __restrict__ A, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    A[e] = A[e] > 0.f ? A[e] : 0.f;
}

template <int KP>
void rowupdate_launch(const float* A, float* Aout, int64_t rows, int r, const float* P, int nsplit,
                      int64_t pstride, const double* G, DevState* st, int half, int sweeps,
                      int flags, double* rec, double* gpart, const double* headU, int nbU,
                      const double* headV, int nbV, const PackOut& po, const DecideArgs& dec,
                      hipStream_t s) {
  using TM = Team<KP>;
  const int nb = rowupdate_blocks(rows, KP);
  dim3 g((unsigned)nb), b(TM::NT);
  if ((int64_t)nb * TM::RB >= rows)
    hipLaunchKernelGGL((k_rowupdate<KP, false>), g, b, 0, s, A, Aout, rows, r, P, nsplit, pstride,
                       G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po.p, po.kp,
                       po.c, po.ldt, po.pad, dec);
  else
    hipLaunchKernelGGL((k_rowupdate<KP, true>), g, b, 0, s, A, Aout, rows, r, P, nsplit, pstride,
                       G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po.p, po.kp,
                       po.c, po.ldt, po.pad, dec);
}

template <int KP>
void gram_fin_launch(const double* gpart, int nparts, double* out, hipStream_t s) {
  constexpr int NE = 16 * ((KP / 4) * (KP / 4 + 1) / 2);
  hipLaunchKernelGGL((k_gram_fin<KP>), dim3((NE + 3) / 4), dim3(256), 0, s, gpart, nparts, out);
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
  const int64_t nrb = (rows + rb - 1) / rb;
  return (int)(nrb < kRowBlocksMax ? nrb : kRowBlocksMax);
}

hipError_t launch_factor_stats(const float* A, int64_t count, int r, double* part, int block_offset,
                               int nblocks, hipStream_t s) {
  (void)r;
  const int64_t per = (count + nblocks - 1) / nblocks;
  hipLaunchKernelGGL(k_factor_stats, dim3(nblocks), dim3(kT), 0, s, A, count, per, part,
                     block_offset);
  return hipGetLastError();
}

hipError_t launch_setup_state(const double* statpart, int nbU, int nbV, const double* xpart,
                              int nxpart, double step_u, double step_v, int ext_iters,
                              int check_every, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_state, dim3(1), dim3(64), 0, s, statpart, nbU, nbV, xpart, nxpart,
                     step_u, step_v, ext_iters, check_every, st);
  return hipGetLastError();
}

int gram_part_len(int kp) { return 16 * ((kp / 4) * (kp / 4 + 1) / 2); }

hipError_t launch_rowupdate(const float* A, float* Aout, int64_t rows, int r, int kp, const float* P,
                            int nsplit, int64_t pstride, const double* G, DevState* st, int half,
                            int sweeps, int flags, double* rec, double* gpart, const double* headU,
                            int nbU, const double* headV, int nbV, hipStream_t s,
                            const PackOut& po, const DecideArgs& dec) {
  if (G != nullptr && (reinterpret_cast<uintptr_t>(G) & 15) != 0) return hipErrorInvalidValue;
  if (po.p != nullptr && (po.kp < 1 || po.kp > kp || po.c < 8 || po.c % 8 != 0 || po.ldt < po.c ||
                          (po.ldt * 2) % 16 != 0))
    return hipErrorInvalidValue;
  switch (kp) {
    case 8: rowupdate_launch<8>(A, Aout, rows, r, P, nsplit, pstride, G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po, dec, s); break;
    case 16: rowupdate_launch<16>(A, Aout, rows, r, P, nsplit, pstride, G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po, dec, s); break;
    case 32: rowupdate_launch<32>(A, Aout, rows, r, P, nsplit, pstride, G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po, dec, s); break;
    default: rowupdate_launch<64>(A, Aout, rows, r, P, nsplit, pstride, G, st, half, sweeps, flags, rec, gpart, headU, nbU, headV, nbV, po, dec, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram_fin(const double* gpart, int nparts, int kp, double* out, hipStream_t s) {
  switch (kp) {
    case 8: gram_fin_launch<8>(gpart, nparts, out, s); break;
    case 16: gram_fin_launch<16>(gpart, nparts, out, s); break;
    case 32: gram_fin_launch<32>(gpart, nparts, out, s); break;
    default: gram_fin_launch<64>(gpart, nparts, out, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_pbcd_decide(const double* rec, int nparts, int half, int first, DevState* st,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pbcd_decide, dim3(1), dim3(kT), 0, s, rec, nparts, half, first, st);
  return hipGetLastError();
}

hipError_t launch_finalize(const DecideArgs& d, int final_check, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kT), 0, s, d, final_check, st);
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
