// The check and stop decision of one outer iteration (the KKT appendix and
// the stopping rule of Algorithm 3), taken by one whole workgroup from the
// per-block check records of both halves, and the phase decision at the start
// of an iteration.  Shared by the row passes and the matrix-core X^T U product,
// which takes the check as a side job (in its first workgroup, or for
// bfloat16 X in a workgroup of its own after the streaming ones).
#pragma once

#include <math.h>

#include "dev_common.h"
#include "enmf_internal.h"
#include "row_team.h"

namespace enmf {

// Check of iteration k (the KKT appendix): combine the check records of the
// U half (input state U^k) and of the V half (V^k) in block order, evaluate
// f through the expansion 1/2||X||^2 - <U, X V> + 1/2 <U^T U, V^T V> (the
// last term from the U records' a . (a G) shares), the relative error and
// the normalised KKT residual documented in enmf.h, decide whether to stop,
// append a trace record, and count the iteration.  `due` = 0 skips the
// evaluation (check_every > 1) and only counts.  Called by all NT threads of
// a block; every calling block reaches the same decision, and only the
// writer block updates the state.  sh: 17 NT/64 doubles; flag: one int (LDS).
template <int NT>
__device__ inline bool check_decide(const DecideArgs& d, int final_check, DevState* st, bool writer,
                             double* sh, int* flag) {
  constexpr int NF = 17;
  // k < 0 (a loop body replayed from a graph): the iteration comes from the
  // state, published by this iteration's U pass, and due from the check period
  const int k = d.k >= 0 ? d.k : st->kcur;
  const int due = d.k >= 0 ? d.due : (k % st->check_every == 0 ? 1 : 0);
  if (due || final_check) {
    double v[NF];
    // a thread's records of both halves, 4 per half, all loads in flight
    // together; further batches (more than 4 NT records) follow; combined in
    // block order
    double acc[2][kRecChkN];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int f = 0; f < kRecChkN; ++f) acc[side][f] = f == 2 ? -INFINITY : (f == 7 ? INFINITY : 0.0);
    }
    const int nbmax = d.nbU > d.nbV ? d.nbU : d.nbV;
    for (int b0 = threadIdx.x; b0 < nbmax; b0 += 4 * NT) {
      double w[2][4][kRecChkN];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const double* rc = side == 0 ? d.recU : d.recV;
        const int nb = side == 0 ? d.nbU : d.nbV;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int b = b0 + u * NT;
          const double* o = rc + (int64_t)(b < nb ? b : 0) * kRecFields + kRecChk;
#pragma unroll
          for (int f = 0; f < kRecChkN; ++f) w[side][u][f] = o[f];
        }
      }
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int nb = side == 0 ? d.nbU : d.nbV;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (b0 + u * NT < nb) {
#pragma unroll
            for (int f = 0; f < kRecChkN; ++f)
              acc[side][f] = f == 2 ? fmax(acc[side][f], w[side][u][f])
                                    : (f == 7 ? fmin(acc[side][f], w[side][u][f])
                                              : acc[side][f] + w[side][u][f]);
          }
        }
      }
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
#pragma unroll
      for (int f = 0; f < 8; ++f) v[8 * side + f] = acc[side][f];
    }
    v[16] = acc[0][8];
    const int kind[NF] = {0, 0, 1, 0, 0, 0, 0, 2, 0, 0, 1, 0, 0, 0, 0, 2, 0};
    double a[NF];
    block_reduce_fields<NT, NF>(v, kind, sh, a);
    if (threadIdx.x == 0) {
      const double nx2 = st->nx2;
      const double f = 0.5 * nx2 - a[5] + 0.5 * a[16];
      const double nx = sqrt(nx2);
      const double nU = sqrt(a[4]), nV = sqrt(a[12]);
      const double feas = fmax(nU > 0.0 ? sqrt(a[3]) / nU : 0.0, nV > 0.0 ? sqrt(a[11]) / nV : 0.0);
      const double pgu = (nV > 0.0 && nx > 0.0) ? sqrt(a[0]) / (nx * nV) : 0.0;
      const double pgv = (nU > 0.0 && nx > 0.0) ? sqrt(a[8]) / (nx * nU) : 0.0;
      const double kkt = fmax(feas, fmax(pgu, pgv));
      const double relerr = nx > 0.0 ? sqrt(fmax(2.0 * f, 0.0)) / nx : 0.0;
      const double negs = a[6] + a[14];
      const bool feasible = negs == 0.0;
      const bool hit = feasible && ((st->kkt_tol >= 0.0 && kkt <= st->kkt_tol) ||
                                    (st->relerr_tol >= 0.0 && relerr - st->relerr_svd <= st->relerr_tol) ||
                                    st->mode == 3);
      const bool numerr = !isfinite(f) || !isfinite(kkt);
      if (writer) {
        st->f = f;
        st->relerr = relerr;
        st->kkt = kkt;
        st->kkt_feas = feas;
        st->kkt_pg_u = pgu;
        st->kkt_pg_v = pgv;
        st->delta_w = fmax(a[2], a[10]);
        st->sigma_u = a[1];
        st->sigma_v = a[9];
        st->sigma_w = a[1] + a[9];
        st->min_w = fmin(a[7], a[15]);
        st->re_paper = st->relerr_svd > 0.0 ? relerr / st->relerr_svd : NAN;
        if (numerr) st->numeric_error = 1;
        if (d.trace != nullptr && st->ntrace < st->trace_cap) {
          double* o = d.trace + (int64_t)st->ntrace * kTraceFields;
          o[0] = (double)k; o[1] = f; o[2] = relerr; o[3] = kkt; o[4] = fmin(a[7], a[15]);
          o[5] = (double)(negs > 0.0 ? kPhaseExt : kPhaseHals);
          o[6] = (double)wall_clock64() * st->ns_per_tick;
          o[7] = negs;
          st->ntrace += 1;
        }
      }
      *flag = ((final_check != 0 || hit || numerr) ? 1 : 0) | (hit ? 2 : 0);
    }
  } else if (threadIdx.x == 0) {
    *flag = final_check != 0 ? 1 : 0;
  }
  __syncthreads();
  const int fl = *flag;
  if (writer && threadIdx.x == 0) {
    if (fl & 1) {
      st->stop = 1;
      st->converged = (fl & 2) ? 1 : 0;
      st->iters = k;
    } else {
      st->iters = k + 1;
      if (st->phase == kPhaseExt) st->ext_done += 1;
    }
  }
  return (fl & 1) != 0;
}

// Phase of an outer iteration (Algorithm 3): EXT while U or V has a negative
// entry, from the negative counts in the latest records of both halves
// (headU, headV).  The writer stores the phase and the count in st and clears
// the PBCD stop flags.  NT threads; sh holds NT / 64 doubles.
template <int NT>
__device__ inline int take_phase(const double* headU, int nbU, const double* headV, int nbV,
                                 DevState* st, bool writer, double* sh) {
  // counts are whole numbers, so the order of the sum does not matter; the
  // loads of both halves, two strides at a time, are in flight together
  double s = 0.0;
  const int nbmax = nbU > nbV ? nbU : nbV;
  for (int b0 = threadIdx.x; b0 < nbmax; b0 += 2 * NT) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int b = b0 + u * NT;
      x[2 * u] = b < nbU ? headU[(int64_t)b * kRecFields + kRecNeg] : 0.0;
      x[2 * u + 1] = b < nbV ? headV[(int64_t)b * kRecFields + kRecNeg] : 0.0;
    }
    s += (x[0] + x[1]) + (x[2] + x[3]);
  }
  s = block_sum<NT>(s, sh);
  const int phase = s > 0.0 ? kPhaseExt : kPhaseHals;
  if (writer && threadIdx.x == 0) {
    st->negs = (int)s;
    st->phase = phase;
    st->pbcd_done[0] = st->pbcd_done[1] = 0;
    st->kcur = st->iters;   // the iteration this U pass belongs to
  }
  return phase;
}

}  // namespace enmf
