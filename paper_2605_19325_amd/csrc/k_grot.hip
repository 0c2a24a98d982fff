// Generalized rotation (the appendix section on exact NMF: problem eq5 in the
// split form eq:admm_form_2, Algorithm alg:rsr).  Orthogonal R1, R2 and a
// positive diagonal Lambda move (U* R1 Lambda R2, V* R1 Lambda^-1 R2) toward
// the nonnegative orthant.  The instances this is meant for are small (the
// appendix: m + n of 90 to 180 rows, r of 10 and 20), so one workgroup runs
// the whole ADMM, every step, in a single launch: R1, R2 in LDS, the six
// N x KP float64 split and dual arrays in a global workspace that stays in
// the caches, Procrustes by the Newton-Schulz polar factor, the quartic of
// each lambda by bracketing and bisection.
#include "block_linalg.h"
#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kG = kBlk;

// Stationary point of g(l) = a l^2 - 2 b l - 2 c / l + d / l^2 (the gamma
// terms of f3 for one column, up to constants) with the least g over l > 0.
// The stationary points are the positive roots of
// q(l) = a l^4 - b l^3 + c l - d; q''(l) = 6 l (2 a l - b), so q' is monotone
// on (0, b / 2a] and on [b / 2a, inf) and has at most two positive roots,
// which split (0, inf) into at most three intervals where q is monotone.
// Each interval with a sign change holds one root, found by bisection.
// a = 0 or d = 0 keeps lam_old.
__device__ double lambda_min(double a, double b, double c, double d, double lam_old) {
  if (!(a > 0.0) || !(d > 0.0)) return lam_old;
  auto q = [&](double l) { return ((a * l - b) * l * l + c) * l - d; };
  auto dq = [&](double l) { return (4.0 * a * l - 3.0 * b) * l * l + c; };
  auto g = [&](double l) { return (a * l - 2.0 * b) * l + (d / l - 2.0 * c) / l; };
  auto bisect = [](auto f, double lo, double hi) {
    const double flo = f(lo);
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      const double fm = f(mid);
      if ((fm < 0.0) == (flo < 0.0)) lo = mid;
      else hi = mid;
    }
    return 0.5 * (lo + hi);
  };
  // every positive root of q and of q' lies below the Cauchy bound of q
  const double hi = 1.0 + fmax(fabs(b), fmax(fabs(c), d)) / a;
  // critical points e1 <= e2 of q in (0, hi) (absent ones at hi)
  double e1 = hi, e2 = hi;
  const double l0 = b > 0.0 ? b / (2.0 * a) : 0.0;
  if (l0 > 0.0) {
    const bool dip = dq(l0) < 0.0;
    if (dip && c > 0.0) e1 = bisect(dq, 0.0, l0);
    if (dip) {
      const double x = bisect(dq, l0, hi);
      if (e1 < hi) e2 = x;
      else e1 = x;
    }
  } else if (c < 0.0) {
    e1 = bisect(dq, 0.0, hi);
  }
  double best = lam_old, gbest = INFINITY;
  // the monotone pieces (0, e1], [e1, e2], [e2, hi]; q(0) = -d < 0
  auto piece = [&](double lo, double qlo, double up) {
    if (!(up > lo)) return;
    const double qhi = q(up);
    double l;
    if (qhi == 0.0) l = up;
    else if ((qlo < 0.0) == (qhi < 0.0) && qlo != 0.0) return;
    else if (qlo == 0.0) l = lo;
    else l = bisect(q, lo, up);
    if (!(l > 0.0)) return;
    const double gl = g(l);
    if (gl < gbest) {
      gbest = gl;
      best = l;
    }
  };
  piece(0.0, -d, e1);
  piece(e1, q(e1), e2);
  piece(e2, q(e2), hi);
  return best;
}

// LDS of one solve.
template <int KP>
struct GrotShared {
  double R1[KP][KP + 1];
  double R2[KP][KP + 1];
  double X[KP][KP + 1];     // Procrustes operand, then its polar factor
  double T[KP][KP + 1];     // Newton-Schulz scratch
  double lam[KP];
  double stat[4][KP];       // per column: |W11|^2, (W21 + N1).W11, (W22 + N2).W12, |W12|^2
  double red[kG / kWave];
};

// S.X[a][b] = sum over rows i of A[i][a] (B[i][b] + C[i][b]) (zero padded
// past r), on the float64 matrix cores: chunks of KP rows of both operands
// are staged in S.X and S.T (free until the Procrustes step), and each wave
// accumulates its 16 x 16 tiles over the chunks (lane (i, g) = (l % 16, l / 16)
// supplies A[k][16 ti + i] and B[k][16 tj + i] of each 4-row step and receives
// D[g + 4 v][i] in accumulator element v).
template <int KP>
__device__ void cross_gram(const double* A, const double* B, const double* C, int64_t N, int r,
                           GrotShared<KP>& S) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NTL = KP / 16;
  constexpr int NTILE = NTL * NTL;
  constexpr int PERW = (NTILE + 3) / 4;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  d4 acc[PERW];
#pragma unroll
  for (int u = 0; u < PERW; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t row0 = 0; row0 < N; row0 += KP) {
    __syncthreads();
    for (int e = threadIdx.x; e < KP * KP; e += kG) {
      const int rr = e / KP, c = e % KP;
      const int64_t row = row0 + rr;
      const bool in = row < N && c < r;
      S.X[rr][c] = in ? A[row * KP + c] : 0.0;
      S.T[rr][c] = in ? B[row * KP + c] + C[row * KP + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int k0 = 0; k0 < KP; k0 += 4) {
#pragma unroll
      for (int u = 0; u < PERW; ++u) {
        const int tile = w + 4 * u;
        if (tile < NTILE) {
          const int ti = tile / NTL, tj = tile % NTL;
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(S.X[k0 + g][16 * ti + i],
                                                        S.T[k0 + g][16 * tj + i], acc[u], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PERW; ++u) {
    const int tile = w + 4 * u;
    if (tile < NTILE) {
      const int ti = tile / NTL, tj = tile % NTL;
#pragma unroll
      for (int v = 0; v < 4; ++v) S.X[16 * ti + g + 4 * v][16 * tj + i] = acc[u][v];
    }
  }
}

// Polar factor of S.X into R (kept when the factor cannot be formed); returns
// ||R_new - R_old||_F^2.
template <int KP>
__device__ double procrustes_into(double (*R)[KP + 1], int r, GrotShared<KP>& S) {
  __syncthreads();
  const bool ok = polar_ns_block<KP>(S.X, S.T, S.red);
  double d2 = 0.0;
  if (ok) {
    for (int e = threadIdx.x; e < KP * KP; e += kG) {
      const int a = e / KP, b = e % KP;
      const double v = (a < r && b < r) ? S.X[a][b] : 0.0;
      d2 = fma(v - R[a][b], v - R[a][b], d2);
      R[a][b] = v;
    }
  }
  d2 = block_sum<kG>(d2, S.red);
  return d2;
}

__device__ __forceinline__ double prox_h(double b, double t) {
  const double it = 1.0 / t;
  return b > 0.0 ? b : (b >= -it ? 0.0 : b + it);
}

template <int KP>
__global__ __launch_bounds__(kG) void k_grot(const float* __restrict__ U, int64_t m,
                                             const float* __restrict__ V, int64_t n, int r,
                                             double rho0, double tol, int max_iter,
                                             double* __restrict__ ws, float* __restrict__ Uout,
                                             float* __restrict__ Vout, double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  GrotShared<KP>& S = *reinterpret_cast<GrotShared<KP>*>(smem);
  const int64_t N = m + n;
  const int64_t NK = N * KP;
  double* Ws = ws;
  double* W1 = ws + NK;
  double* W2 = ws + 2 * NK;
  double* W3 = ws + 3 * NK;
  double* Md = ws + 4 * NK;
  double* Nd = ws + 5 * NK;
  double* Pd = ws + 6 * NK;
  const int64_t cnt = N * r;
  // W_svd = [U; V] in float64, W1 = W2 = W3 = W_svd, duals 0, R1 = R2 = I, lambda = 1
  double ss = 0.0, neg0 = 0.0;
  for (int64_t e = threadIdx.x; e < NK; e += kG) {
    const int64_t i = e / KP;
    const int j = (int)(e % KP);
    double w = 0.0;
    if (j < r) w = i < m ? (double)U[i * r + j] : (double)V[(i - m) * r + j];
    Ws[e] = w;
    W1[e] = w;
    W2[e] = w;
    W3[e] = w;
    Md[e] = 0.0;
    Nd[e] = 0.0;
    Pd[e] = 0.0;
    ss = fma(w, w, ss);
    neg0 += w < 0.0 ? -w : 0.0;
  }
  for (int e = threadIdx.x; e < KP * KP; e += kG) {
    const int a = e / KP, b = e % KP;
    S.R1[a][b] = (a == b && a < r) ? 1.0 : 0.0;
    S.R2[a][b] = S.R1[a][b];
  }
  if (threadIdx.x < KP) S.lam[threadIdx.x] = 1.0;
  ss = block_sum<kG>(ss, S.red);
  neg0 = block_sum<kG>(neg0, S.red);
  // rho = gamma = t = rho0 sqrt(N r) / ||W_svd||_F
  const double pen = ss > 0.0 ? rho0 * sqrt((double)N * r) / sqrt(ss) : 1.0;
  const double rho = pen, gam = pen, tp = pen;
  int steps = 0;
  for (int k = 0; k < max_iter; ++k) {
    // f1: W3 = prox(W2 R2 - P), W1 elementwise; both from the previous W2, R1, R2, lambda
    for (int64_t e = threadIdx.x; e < cnt; e += kG) {
      const int64_t i = e / r;
      const int j = (int)(e % r);
      const int64_t o = i * KP + j;
      double w2r2 = 0.0, wr1 = 0.0;
      for (int a = 0; a < r; ++a) {
        w2r2 = fma(W2[i * KP + a], S.R2[a][j], w2r2);
        wr1 = fma(Ws[i * KP + a], S.R1[a][j], wr1);
      }
      W3[o] = prox_h(w2r2 - Pd[o], tp);
      const double A = wr1 - Md[o], C = W2[o] + Nd[o], l = S.lam[j];
      W1[o] = i < m ? (rho * A + gam * l * C) / (rho + gam * l * l)
                    : (rho * A + (gam / l) * C) / (rho + gam / (l * l));
    }
    __syncthreads();
    // f2: R1 = polar(W_svd^T (W1 + M)); W2 from W1, N, W3 + P and the previous R2, lambda
    cross_gram<KP>(Ws, W1, Md, N, r, S);
    for (int64_t e = threadIdx.x; e < cnt; e += kG) {
      const int64_t i = e / r;
      const int j = (int)(e % r);
      const int64_t o = i * KP + j;
      double tr = 0.0;
      for (int a = 0; a < r; ++a) tr = fma(W3[i * KP + a] + Pd[i * KP + a], S.R2[j][a], tr);
      const double l = S.lam[j];
      const double w1l = i < m ? W1[o] * l : W1[o] / l;
      W2[o] = (gam * w1l - gam * Nd[o] + tp * tr) / (gam + tp);
    }
    const double d1 = procrustes_into<KP>(S.R1, r, S);
    // f3: R2 = polar(W2^T (W3 + P)); lambda per column from W1, W2 + N
    cross_gram<KP>(W2, W3, Pd, N, r, S);
    for (int e = threadIdx.x; e < 4 * KP; e += kG) {
      const int f = e / KP, j = e % KP;
      double s = 0.0;
      if (j < r) {
        const int64_t i0 = f < 2 ? 0 : m, i1 = f < 2 ? m : N;
        for (int64_t i = i0; i < i1; ++i) {
          const int64_t o = i * KP + j;
          const double w1 = W1[o];
          s = fma((f == 0 || f == 3) ? w1 : W2[o] + Nd[o], w1, s);
        }
      }
      S.stat[f][j] = s;
    }
    const double d2 = procrustes_into<KP>(S.R2, r, S);
    double dl = 0.0;
    if (threadIdx.x < r) {
      const int j = threadIdx.x;
      const double ln = lambda_min(S.stat[0][j], S.stat[1][j], S.stat[2][j], S.stat[3][j], S.lam[j]);
      dl = (ln - S.lam[j]) * (ln - S.lam[j]);
      S.lam[j] = ln;
    }
    dl = block_sum<kG>(dl, S.red);
    // duals with the new R1, Lambda, R2
    for (int64_t e = threadIdx.x; e < cnt; e += kG) {
      const int64_t i = e / r;
      const int j = (int)(e % r);
      const int64_t o = i * KP + j;
      double wr1 = 0.0, w2r2 = 0.0;
      for (int a = 0; a < r; ++a) {
        wr1 = fma(Ws[i * KP + a], S.R1[a][j], wr1);
        w2r2 = fma(W2[i * KP + a], S.R2[a][j], w2r2);
      }
      const double l = S.lam[j];
      Md[o] += W1[o] - wr1;
      Nd[o] += W2[o] - (i < m ? W1[o] * l : W1[o] / l);
      Pd[o] += W3[o] - w2r2;
    }
    __syncthreads();
    steps = k + 1;
    const double change = sqrt(d1) + sqrt(d2) + sqrt(dl);
    if (tol > 0.0 && change <= tol) break;
  }
  // outputs: U* R1 Lambda R2 and V* R1 Lambda^-1 R2, rounded to float32
  double neg1 = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += kG) {
    const int64_t i = e / r;
    const int j = (int)(e % r);
    double s = 0.0;
    for (int b = 0; b < r; ++b) {
      double t = 0.0;
      for (int a = 0; a < r; ++a) t = fma(Ws[i * KP + a], S.R1[a][b], t);
      t = i < m ? t * S.lam[b] : t / S.lam[b];
      s = fma(t, S.R2[b][j], s);
    }
    neg1 += s < 0.0 ? -s : 0.0;
    if (i < m) Uout[i * r + j] = (float)s;
    else Vout[(i - m) * r + j] = (float)s;
  }
  neg1 = block_sum<kG>(neg1, S.red);
  if (threadIdx.x == 0) {
    out[0] = neg0;
    out[1] = neg1;
    out[2] = (double)steps;
  }
  for (int e = threadIdx.x; e < r * r; e += kG) {
    out[4 + e] = S.R1[e / r][e % r];
    out[4 + r * r + e] = S.R2[e / r][e % r];
  }
  if (threadIdx.x < r) out[4 + 2 * r * r + threadIdx.x] = S.lam[threadIdx.x];
}

template <int KP>
hipError_t grot_launch(const float* U, int64_t m, const float* V, int64_t n, int r, double rho0,
                       double tol, int max_iter, double* ws, float* Uout, float* Vout, double* out,
                       hipStream_t s) {
  const size_t lds = sizeof(GrotShared<KP>);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_grot<KP>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_grot<KP>), dim3(1), dim3(kG), lds, s, U, m, V, n, r, rho0, tol, max_iter, ws,
                     Uout, Vout, out);
  return hipGetLastError();
}

}  // namespace

int grot_pad(int r) { return r <= 16 ? 16 : (r <= 32 ? 32 : 64); }

hipError_t launch_grot(const float* U, int64_t m, const float* V, int64_t n, int r, double rho0,
                       double tol, int max_iter, double* ws, float* Uout, float* Vout, double* out,
                       hipStream_t s) {
  switch (grot_pad(r)) {
    case 16: return grot_launch<16>(U, m, V, n, r, rho0, tol, max_iter, ws, Uout, Vout, out, s);
    case 32: return grot_launch<32>(U, m, V, n, r, rho0, tol, max_iter, ws, Uout, Vout, out, s);
    default: return grot_launch<64>(U, m, V, n, r, rho0, tol, max_iter, ws, Uout, Vout, out, s);
  }
}

}  // namespace enmf
