// Serving loop: many independent eNMF solves of uneven shape, advanced
// together one launch ("tick") at a time.  One workgroup owns one request and
// runs its whole solve as a resumable state machine: the randomized SVD
// initialisation (section 3 opening, Algorithm 3 step 2), the ADMM rotation
// (section 3.1, Algorithm 1), the exterior phase and HALS (sections 3.2-3.3,
// Algorithms 2-3) with the KKT check of every iteration, and the final
// objective.  Everything that survives a tick lives in device memory (the
// slot's state and workspace), so a request computes the same numbers
// whether it runs alone or beside others, and however long its ticks are.
//
// Within a workgroup every step is a block-level routine: tall-skinny
// products X B and X^T A stream X in LDS tiles and accumulate in float32
// (X is float32, bfloat16 or float16); Grams and cross products are float64
// with fixed-order combination; the range finder orthonormalises with the
// eigenpairs of the Gram (Jacobi in LDS); the Procrustes step takes the
// Newton-Schulz polar factor; row updates reuse the row-team code of the
// per-iteration kernels at a padded width of 32.
#include <math.h>

#include "block_linalg.h"
#include "dev_common.h"
#include "enmf_internal.h"
#include "mfma_common.h"
#include "row_team.h"
#include "serve_internal.h"

namespace enmf {

namespace {

constexpr int SNT = kBlk;        // threads per serving workgroup
constexpr int SKP = kServeKP;    // padded factor width
constexpr int SKB = kServeKK;    // padded range-finder width
constexpr double kOrthTau = 1e-15;

template <int XT> using XE = typename XElem<XT>::T;

// LDS of the phases; one union per workgroup.
struct ProdSmem {
  float X[128 * 33];
  float B[32 * SKB];
};
struct GramSmem {
  double A[32 * SKB];
  double B[32 * SKB];
};
struct RowSmem {
  double G[SKP * SKP];
  __align__(16) float a[64][SKP + 4];
  float g[64][SKP + 1];
  double sh[16 * (SNT / kWave)];
  double out[16];
};
struct EigSmem {
  JacobiT<SKB> j;
  double aux[2 * SKB];
};
constexpr int kAdmmRB = 128;  // rows per block of the served ADMM step
struct AdmmSmem {
  double R[SKP * SKP];
  double red[SNT / kWave];
  union {
    struct {                     // the polar step
      double X[SKP][SKP + 1];
      double T[SKP][SKP + 1];
    };
    struct {                     // the row blocks of the ADMM step
      float Wb[kAdmmRB * SKP];   // a row block of W = [U*; V*] (row pitch SKP)
      double Sb[kAdmmRB * SKP];  // its rows of the ADMM state (row pitch r)
    };
  };
};
constexpr int kSvBLd = 72;   // LDS row pitch of a 64-row factor chunk of X B (matrix cores)
constexpr int kSvALd = 40;   // LDS row pitch of a 32-row factor chunk of X^T A (matrix cores)
struct MfmaSmem {
  __align__(16) unsigned short f[2 * 3 * SKB * kSvBLd];
};
union ServeSmem {
  ProdSmem p;
  MfmaSmem mf;
  GramSmem g;
  RowSmem w;
  EigSmem e;
  AdmmSmem a;
};

__device__ __forceinline__ int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// Tall-skinny products (float32 accumulation).  Tiles of 128 output rows; the
// contraction advances 32 at a time through LDS.  Thread t owns one output
// row and KB/2 of its columns; the next chunk's global loads are issued
// before the barrier that retires the current one.
// ---------------------------------------------------------------------------

// out (m x k, ld ldo) = X (m x n, ld) B (n x k, ld ldb).
template <int XT, int KB>
__device__ void bx_xb(const XE<XT>* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                      const float* __restrict__ B, int ldb, int k, float* __restrict__ out, int ldo,
                      ProdSmem& sm) {
  constexpr int CPT = KB / 2;
  constexpr int NB = 32 * KB / SNT;
  const int t = threadIdx.x, row = t & 127, cg = t >> 7;
  for (int64_t r0 = 0; r0 < m; r0 += 128) {
    float acc[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[c] = 0.f;
    for (int64_t j0 = 0; j0 < n; j0 += 32) {
      float xv[16], bv[NB];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + SNT * u, rr = e >> 5, cc = e & 31;
        const int64_t gi = r0 + rr, gj = j0 + cc;
        xv[u] = (gi < m && gj < n) ? to_f32<XT>(X[gi * ld + gj]) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int e = t + SNT * u, rr = e / KB, cc = e % KB;
        const int64_t gj = j0 + rr;
        bv[u] = (gj < n && cc < k) ? B[gj * ldb + cc] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + SNT * u;
        sm.X[(e >> 5) * 33 + (e & 31)] = xv[u];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) sm.B[t + SNT * u] = bv[u];
      __syncthreads();
#pragma unroll 8
      for (int kk = 0; kk < 32; ++kk) {
        const float x = sm.X[row * 33 + kk];
        const float* b = sm.B + kk * KB + cg * CPT;
#pragma unroll
        for (int c = 0; c < CPT; ++c) acc[c] = fmaf(x, b[c], acc[c]);
      }
    }
    const int64_t gi = r0 + row;
    if (gi < m) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = cg * CPT + c;
        if (col < k) out[gi * ldo + col] = acc[c];
      }
    }
  }
  __syncthreads();
}

// out (n x k, ld ldo) = X^T (X m x n, ld) A (m x k, ld lda).
template <int XT, int KB>
__device__ void bx_xta(const XE<XT>* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                       const float* __restrict__ A, int lda, int k, float* __restrict__ out, int ldo,
                       ProdSmem& sm) {
  constexpr int CPT = KB / 2;
  constexpr int NB = 32 * KB / SNT;
  const int t = threadIdx.x, jr = t & 127, cg = t >> 7;
  for (int64_t j0 = 0; j0 < n; j0 += 128) {
    float acc[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[c] = 0.f;
    for (int64_t i0 = 0; i0 < m; i0 += 32) {
      float xv[16], av[NB];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + SNT * u, ii = e >> 7, jj = e & 127;
        const int64_t gi = i0 + ii, gj = j0 + jj;
        xv[u] = (gi < m && gj < n) ? to_f32<XT>(X[gi * ld + gj]) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int e = t + SNT * u, rr = e / KB, cc = e % KB;
        const int64_t gi = i0 + rr;
        av[u] = (gi < m && cc < k) ? A[gi * lda + cc] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = t + SNT * u;
        sm.X[(e >> 7) * 129 + (e & 127)] = xv[u];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) sm.B[t + SNT * u] = av[u];
      __syncthreads();
#pragma unroll 8
      for (int kk = 0; kk < 32; ++kk) {
        const float x = sm.X[kk * 129 + jr];
        const float* a = sm.B + kk * KB + cg * CPT;
#pragma unroll
        for (int c = 0; c < CPT; ++c) acc[c] = fmaf(x, a[c], acc[c]);
      }
    }
    const int64_t gj = j0 + jr;
    if (gj < n) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = cg * CPT + c;
        if (col < k) out[gj * ldo + col] = acc[c];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// bfloat16 X on the matrix cores (v_mfma_f32_16x16x32_bf16).  The float32
// factor is split into three bfloat16 terms (hi + mid + lo, within 2^-24 of
// it; store_split_run8) as it is staged into LDS, so each 32-step of the
// contraction is three MFMAs per 16 x 16 output tile with float32
// accumulation, and X is exact in bfloat16.  The next factor chunk travels
// through registers and reaches the other LDS buffer after the current
// chunk's MFMAs.  Element v of lane (i, g) = (l % 16, l / 16) of an output
// tile is D[4g + v][i].
// ---------------------------------------------------------------------------

// Rows r0 .. r0 + 7 of column c of the rows x k float32 factor F (ld ldf),
// zero past its rows or columns.
__device__ __forceinline__ void fetch_run8(const float* __restrict__ F, int64_t rows, int ldf, int k,
                                           int64_t r0, int c, float (&v)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (r0 + e < rows && c < k) ? F[(r0 + e) * ldf + c] : 0.f;
}

// out (m x k, ld ldo) = X (m x n, ld) B (n x k, ld ldb), k <= KP.  Row groups
// of 256 (4 waves x 4 tiles of 16 rows); chunk = 64 columns of X (two
// 32-steps).  Lane (i, g) of row tile rt supplies X[row0 + 16 rt + i][64 ch +
// 32 s + 8g .. +7]; the B operand is Bt[term][16 nt + i][32 s + 8g .. +7] of
// the LDS chunk (factor column major, rows padded to 72).
template <int KP>
__device__ void sv_xb_bf16(const unsigned short* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                           const float* __restrict__ B, int ldb, int k, float* __restrict__ out,
                           int ldo, MfmaSmem& sm) {
  constexpr int NT = KP / 16, RT = 4, CH = 3 * KP * kSvBLd;
  constexpr int NTASK = KP * 8;   // runs of 8 rows of one column per chunk
  constexpr int NR = (NTASK + SNT - 1) / SNT;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  const bool vec = (reinterpret_cast<uintptr_t>(X) & 15) == 0 && ld % 8 == 0;
  const int64_t nch = (n + 63) / 64;
  float bv[NR][8];
  auto fetch_b = [&](int64_t ch) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int task = threadIdx.x + SNT * u;
      if (task < NTASK) fetch_run8(B, n, ldb, k, 64 * ch + 8 * (task / KP), task % KP, bv[u]);
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int task = threadIdx.x + SNT * u;
      if (task < NTASK)
        store_split_run8(bv[u], sm.f + buf * CH + (task % KP) * kSvBLd + 8 * (task / KP), KP * kSvBLd);
    }
  };
  uint4 xa[RT][2], xn[RT][2];
  auto load_x = [&](int64_t row0, int64_t ch, uint4 (&dst)[RT][2]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
        dst[rt][s2] = load16<unsigned short>(X, m, n, ld, row0 + 16 * rt + i, 64 * ch + 32 * s2 + 8 * g, vec);
  };
  for (int64_t rg = 0; rg < m; rg += 4 * 64) {
    const int64_t row0 = rg + 64 * w;
    const bool active = row0 < m;   // wave-uniform
    f32x4 acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = zero4();
    fetch_b(0);
    store_b(0);
    if (active) load_x(row0, 0, xa);
    int buf = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
      __syncthreads();
      const bool more = ch + 1 < nch;
      if (more) {
        fetch_b(ch + 1);
        if (active) load_x(row0, ch + 1, xn);
      }
      if (active) {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int hl = 0; hl < 3; ++hl) {
              const bf16x8 b = as_bf16x8(*reinterpret_cast<const uint4*>(
                  &sm.f[buf * CH + (hl * KP + 16 * nt + i) * kSvBLd + 32 * s2 + 8 * g]));
#pragma unroll
              for (int rt = 0; rt < RT; ++rt)
                acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(xa[rt][s2]), b, acc[rt][nt], 0, 0, 0);
            }
          }
        }
      }
      if (more) {
        store_b(buf ^ 1);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) { xa[rt][0] = xn[rt][0]; xa[rt][1] = xn[rt][1]; }
      }
      buf ^= 1;
    }
    if (active) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int col = 16 * nt + i;
          if (col < k) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int64_t row = row0 + 16 * rt + 4 * g + v;
              if (row < m) out[row * ldo + col] = acc[rt][nt][v];
            }
          }
        }
    }
    __syncthreads();   // the next row group restages chunk 0
  }
}

// out (n x k, ld ldo) = X^T (X m x n, ld) A (m x k, ld lda), k <= KP.  Column
// groups of 512 (4 waves x 128 columns); chunk = 32 rows of X (one 32-step).
// Lane (i, g) loads the 8 x 8 block X[32 ch + 8g + e][j0 + 8i .. 8i + 7] (e =
// 0..7) and transposes it in registers: operand t holds X[32 ch + 8g + 0..7]
// [j0 + 8i + t], so tile t covers the columns j0 + 8 mm + t (mm = 0..15).  The
// B operand is At[term][16 nt + i][8g .. 8g + 7] of the LDS chunk (rows
// padded to 40).  Element v of lane (i, g) in tile t is column j0 + 8 (4g +
// v) + t, factor column 16 nt + i.
template <int KP>
__device__ void sv_xta_bf16(const unsigned short* __restrict__ X, int64_t m, int64_t n, int64_t ld,
                            const float* __restrict__ A, int lda, int k, float* __restrict__ out,
                            int ldo, MfmaSmem& sm) {
  constexpr int NT = KP / 16, CH = 3 * KP * kSvALd;
  constexpr int NTASK = KP * 4;   // runs of 8 rows of one column per chunk
  constexpr int NR = (NTASK + SNT - 1) / SNT;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  const bool vec = (reinterpret_cast<uintptr_t>(X) & 15) == 0 && ld % 8 == 0;
  const int64_t nch = (m + 31) / 32;
  float av[NR][8];
  auto fetch_a = [&](int64_t ch) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int task = threadIdx.x + SNT * u;
      if (task < NTASK) fetch_run8(A, m, lda, k, 32 * ch + 8 * (task / KP), task % KP, av[u]);
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int task = threadIdx.x + SNT * u;
      if (task < NTASK)
        store_split_run8(av[u], sm.f + buf * CH + (task % KP) * kSvALd + 8 * (task / KP), KP * kSvALd);
    }
  };
  uint4 xa[8], xn[8];
  auto load_x = [&](int64_t j0, int64_t ch, uint4 (&dst)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[e] = load16<unsigned short>(X, m, n, ld, 32 * ch + 8 * g + e, j0 + 8 * i, vec);
  };
  for (int64_t cg = 0; cg < n; cg += 4 * 128) {
    const int64_t j0 = cg + 128 * w;
    const bool active = j0 < n;   // wave-uniform
    f32x4 acc[8][NT];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4();
    fetch_a(0);
    store_a(0);
    if (active) load_x(j0, 0, xa);
    int buf = 0;
    for (int64_t ch = 0; ch < nch; ++ch) {
      __syncthreads();
      const bool more = ch + 1 < nch;
      if (more) {
        fetch_a(ch + 1);
        if (active) load_x(j0, ch + 1, xn);
      }
      if (active) {
        // op[t] dword d = (X[2d][t], X[2d + 1][t]) of the lane's 8 x 8 block
        uint4 op[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          unsigned d[4];
#pragma unroll
          for (int dd = 0; dd < 4; ++dd) {
            const uint4& lo = xa[2 * dd];
            const uint4& hi = xa[2 * dd + 1];
            const unsigned a = (t / 2 == 0) ? lo.x : (t / 2 == 1) ? lo.y : (t / 2 == 2) ? lo.z : lo.w;
            const unsigned b = (t / 2 == 0) ? hi.x : (t / 2 == 1) ? hi.y : (t / 2 == 2) ? hi.z : hi.w;
            d[dd] = (t % 2 == 0) ? __builtin_amdgcn_perm(b, a, 0x05040100u)
                                 : __builtin_amdgcn_perm(b, a, 0x07060302u);
          }
          op[t] = make_uint4(d[0], d[1], d[2], d[3]);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
          for (int hl = 0; hl < 3; ++hl) {
            const bf16x8 b = as_bf16x8(*reinterpret_cast<const uint4*>(
                &sm.f[buf * CH + (hl * KP + 16 * nt + i) * kSvALd + 8 * g]));
#pragma unroll
            for (int t = 0; t < 8; ++t)
              acc[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(op[t]), b, acc[t][nt], 0, 0, 0);
          }
        }
      }
      if (more) {
        store_a(buf ^ 1);
#pragma unroll
        for (int e = 0; e < 8; ++e) xa[e] = xn[e];
      }
      buf ^= 1;
    }
    if (active) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int col = 16 * nt + i;
          if (col < k) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int64_t j = j0 + 8 * (4 * g + v) + t;
              if (j < n) out[j * ldo + col] = acc[t][nt][v];
            }
          }
        }
    }
    __syncthreads();   // the next column group restages chunk 0
  }
}

// Products of the serving steps: bfloat16 X on the matrix cores, float32 and
// float16 X on the vector ALU.
template <int XT>
__device__ void xb(const XE<XT>* X, int64_t m, int64_t n, int64_t ld, const float* B, int ldb, int k,
                   float* out, int ldo, ServeSmem& sm) {
  if constexpr (XT == 1) {
    if (k <= 16) sv_xb_bf16<16>(X, m, n, ld, B, ldb, k, out, ldo, sm.mf);
    else if (k <= 32) sv_xb_bf16<32>(X, m, n, ld, B, ldb, k, out, ldo, sm.mf);
    else sv_xb_bf16<48>(X, m, n, ld, B, ldb, k, out, ldo, sm.mf);
  } else {
    if (k <= 8) bx_xb<XT, 8>(X, m, n, ld, B, ldb, k, out, ldo, sm.p);
    else if (k <= 16) bx_xb<XT, 16>(X, m, n, ld, B, ldb, k, out, ldo, sm.p);
    else if (k <= 32) bx_xb<XT, 32>(X, m, n, ld, B, ldb, k, out, ldo, sm.p);
    else bx_xb<XT, 48>(X, m, n, ld, B, ldb, k, out, ldo, sm.p);
  }
}

template <int XT>
__device__ void xta(const XE<XT>* X, int64_t m, int64_t n, int64_t ld, const float* A, int lda, int k,
                    float* out, int ldo, ServeSmem& sm) {
  if constexpr (XT == 1) {
    if (k <= 16) sv_xta_bf16<16>(X, m, n, ld, A, lda, k, out, ldo, sm.mf);
    else if (k <= 32) sv_xta_bf16<32>(X, m, n, ld, A, lda, k, out, ldo, sm.mf);
    else sv_xta_bf16<48>(X, m, n, ld, A, lda, k, out, ldo, sm.mf);
  } else {
    if (k <= 8) bx_xta<XT, 8>(X, m, n, ld, A, lda, k, out, ldo, sm.p);
    else if (k <= 16) bx_xta<XT, 16>(X, m, n, ld, A, lda, k, out, ldo, sm.p);
    else if (k <= 32) bx_xta<XT, 32>(X, m, n, ld, A, lda, k, out, ldo, sm.p);
    else bx_xta<XT, 48>(X, m, n, ld, A, lda, k, out, ldo, sm.p);
  }
}

// ---------------------------------------------------------------------------
// out (KB x KB, ld KB) = A^T B for tall A (rows x ka), B (rows x kb), float64
// (products of the float32 inputs are exact).  Rows are staged 32 at a time;
// thread groups of RG consecutive lanes own one 4 x 4 output tile and take
// its rows round robin; the groups combine by butterfly, so every entry has
// a fixed summation order (and A^T A comes out exactly symmetric).
// ---------------------------------------------------------------------------
template <typename TA, typename TB, int KB>
__device__ void bx_cross(const TA* __restrict__ A, int lda, int ka, const TB* __restrict__ B,
                         int ldb, int kb, int64_t rows, double* __restrict__ out, GramSmem& sm) {
  constexpr int NTILE = KB / 4;
  constexpr int NTASK = NTILE * NTILE;
  constexpr int RG = NTASK >= SNT ? 1 : SNT / NTASK;
  constexpr int NL = 32 * KB / SNT;
  static_assert(RG == 1 || RG == 4 || RG == 16 || RG == 64, "row groups must tile a wave");
  const int t = threadIdx.x, task = t / RG, rg = t % RG;
  const bool act = task < NTASK;
  const int ti = act ? task / NTILE : 0, tj = act ? task % NTILE : 0;
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  for (int64_t i0 = 0; i0 < rows; i0 += 32) {
    double av[NL], bv[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = t + SNT * u, rr = e / KB, cc = e % KB;
      const int64_t gi = i0 + rr;
      av[u] = (gi < rows && cc < ka) ? (double)A[gi * lda + cc] : 0.0;
      bv[u] = (gi < rows && cc < kb) ? (double)B[gi * ldb + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      sm.A[t + SNT * u] = av[u];
      sm.B[t + SNT * u] = bv[u];
    }
    __syncthreads();
    if (act) {
      for (int rr = rg; rr < 32; rr += RG) {
        const double* x = sm.A + rr * KB + 4 * ti;
        const double* y = sm.B + rr * KB + 4 * tj;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[4 * u + v] = fma(x[u], y[v], acc[4 * u + v]);
      }
    }
  }
#pragma unroll
  for (int o = RG / 2; o > 0; o >>= 1)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] += __shfl_xor(acc[e], o);
  if (act && rg == 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(4 * ti + u) * KB + 4 * tj + v] = acc[4 * u + v];
  }
  __syncthreads();
}

// out[i][c] = sum_a A[i][a] T[a][c] for c < kb (T: LDS, ld KB), float64; a
// row is read whole before it is written, so out may alias A.  out32, when
// given, receives a float32 copy.
template <typename TA, typename TO, int KB>
__device__ void bx_apply(const TA* A, int lda, int ka, int64_t rows, const double* T, int kb, TO* out,
                         int ldo, float* out32 = nullptr, int ld32 = 0) {
  for (int64_t i = threadIdx.x; i < rows; i += SNT) {
    double a[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) a[q] = q < ka ? (double)A[i * lda + q] : 0.0;
    for (int c = 0; c < kb; ++c) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < KB; ++q) s = fma(a[q], T[q * KB + c], s);
      out[i * ldo + c] = (TO)s;
      if (out32) out32[i * ld32 + c] = (float)s;
    }
  }
  __syncthreads();
}

// sum over all threads, valid in every thread
__device__ __forceinline__ double bsum(double v, double* red) { return block_sum<SNT>(v, red); }

// ---------------------------------------------------------------------------
// Range finder
// ---------------------------------------------------------------------------

// Eigenpairs of the k x k Gram in `g` (global, ld SKB); leaves the sorted
// eigenvalues in aux[0..k) and the eigenvectors in the Jacobi state.
__device__ void eig_of(const double* g, int k, EigSmem& sm) {
  for (int e = threadIdx.x; e < k * k; e += SNT)
    sm.j.S[(e / k) * JacobiT<SKB>::LD + e % k] = g[(e / k) * SKB + e % k];
  __syncthreads();
  jacobi_eig<SKB>(sm.j, k);
  if (threadIdx.x < k) sm.aux[threadIdx.x] = eigval<SKB>(sm.j, threadIdx.x);
  __syncthreads();
}

// T (into the S area, ld SKB) = E diag(lambda^-1/2), zero for lambda <= tau lambda_max.
__device__ double* orth_factor_lds(int k, EigSmem& sm) {
  double* T = sm.j.S;
  const double lmax = sm.aux[0];
  for (int e = threadIdx.x; e < SKB * SKB; e += SNT) {
    const int a = e / SKB, j = e % SKB;
    double v = 0.0;
    if (a < k && j < k) {
      const double l = sm.aux[j];
      const double sc = (l > kOrthTau * lmax && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
      v = eigvec<SKB>(sm.j, a, j) * sc;
    }
    T[e] = v;
  }
  __syncthreads();
  return T;
}

// Orthonormal basis of the columns of A32 (rows x k): two passes of
// Q = A E diag(lambda^-1/2) with the eigenpairs of A^T A.  out64 (float64)
// and out32 (float32) both rows x k; out32 may alias A32.
__device__ void orth(const float* A32, int64_t rows, int k, double* out64, float* out32,
                     double* scratch, ServeSmem& sm) {
  bx_cross<float, float, SKB>(A32, k, k, A32, k, k, rows, scratch, sm.g);
  eig_of(scratch, k, sm.e);
  const double* T = orth_factor_lds(k, sm.e);
  bx_apply<float, double, SKB>(A32, k, k, rows, T, k, out64, k);
  bx_cross<double, double, SKB>(out64, k, k, out64, k, k, rows, scratch, sm.g);
  eig_of(scratch, k, sm.e);
  T = orth_factor_lds(k, sm.e);
  bx_apply<double, double, SKB>(out64, k, k, rows, T, k, out64, k, out32, k);
}

// ||X||_F^2 in float64.
template <int XT>
__device__ double sumsq_x(const XE<XT>* X, int64_t m, int64_t n, int64_t ld, double* red) {
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = threadIdx.x; j < n; j += SNT) {
      const double v = (double)to_f32<XT>(X[i * ld + j]);
      s = fma(v, v, s);
    }
  return bsum(s, red);
}

// 1/2 ||X - U V^T||_F^2 evaluated directly, float64 (U m x r, V n x r).
template <int XT>
__device__ double residual(const XE<XT>* X, int64_t m, int64_t n, int64_t ld, const float* U,
                           const float* V, int r, ProdSmem& sm, double* red) {
  // V chunk (32 rows) in sm.B as float; U row in registers.
  double s = 0.0;
  const int t = threadIdx.x;
  for (int64_t j0 = 0; j0 < n; j0 += 32) {
    __syncthreads();
    for (int e = t; e < 32 * SKP; e += SNT) {
      const int rr = e / SKP, cc = e % SKP;
      const int64_t gj = j0 + rr;
      sm.B[e] = (gj < n && cc < r) ? V[gj * r + cc] : 0.f;
    }
    __syncthreads();
    const int jn = (int)imin(32, n - j0);
    for (int64_t i = t; i < m; i += SNT) {
      double u[SKP];
#pragma unroll
      for (int c = 0; c < SKP; ++c) u[c] = c < r ? (double)U[i * r + c] : 0.0;
      for (int jj = 0; jj < jn; ++jj) {
        double e = (double)to_f32<XT>(X[i * ld + j0 + jj]);
        const float* v = sm.B + jj * SKP;
#pragma unroll
        for (int c = 0; c < SKP; ++c) e = fma(-u[c], (double)v[c], e);
        s = fma(e, e, s);
      }
    }
  }
  return 0.5 * bsum(s, red);
}

// ---------------------------------------------------------------------------
// Row passes (exterior phase / HALS / KKT partials) at padded width 32.
// ---------------------------------------------------------------------------

// One pass over the rows of A (rows x r, ld r) with P (rows x r, ld r) and
// the Gram already in sm.G.  update: the EXT (push, mask, `sweeps` PBCD
// sweeps; eqs. negup, pbcdu, d_i) or HALS update of every row, in place.
// pre: KKT partials at the input rows, else at the output rows.  Leaves in
// sm.out the 8 check fields (CheckAcc order) and the negative count of the
// output rows.
__device__ void row_pass(float* A, int64_t rows, int r, const float* P, RowSmem& sm, bool update,
                         bool pre, int phase, double step, int sweeps, bool fixed_step) {
  using TM = Team<SKP>;
  constexpr int T = TM::T;
  const int team = threadIdx.x / T, q = threadIdx.x % T, c0 = 8 * q;
  const double* sG = sm.G;
  CheckAcc ck;
  double negc = 0.0;
  // fixed-step ablation (mode 2): one row step 1/||G||_F in place of d
  double dfix = -1.0;
  if (update && phase == kPhaseExt && fixed_step) {
    double ss = 0.0;
    for (int e = threadIdx.x; e < SKP * SKP; e += SNT) ss = fma(sG[e], sG[e], ss);
    ss = block_sum<SNT>(ss, sm.sh);
    dfix = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  }
  for (int64_t row0 = 0; row0 < rows; row0 += TM::RB) {
    const int nrow = (int)imin(rows - row0, TM::RB);
    const bool valid = team < nrow;
    stage_rows<SKP, SKP + 4>(A, 1, 0, row0, nrow, r, sm.a);
    stage_rows<SKP, SKP + 1>(P, 1, 0, row0, nrow, r, sm.g);
    float a[8];
    double p[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = sm.a[team][c0 + e];
      p[e] = (double)sm.g[team][c0 + e];
    }
    __syncthreads();
    double t[8];
    bool have_t = false;
    if (pre) {
#pragma unroll
      for (int e = 0; e < 8; ++e) sm.a[team][c0 + e] = a[e];
      __syncthreads();
      row_times_g<SKP>(sm.a[team], sG, c0, t);
      have_t = true;
      if (valid) ck.add(a, t, p, c0, r);
    }
    if (update && phase == kPhaseHals) {
      if (!have_t) {
#pragma unroll
        for (int e = 0; e < 8; ++e) sm.a[team][c0 + e] = a[e];
        __syncthreads();
        row_times_g<SKP>(sm.a[team], sG, c0, t);
      }
      const int base = (threadIdx.x % kWave) - q;
      for (int j = 0; j < r; ++j) {
        const int o = j / 8, ej = j % 8;
        double delta = 0.0;
        if (q == o) {
          const double gjj = sG[j * SKP + j];
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
        const double* gj = sG + j * SKP + c0;
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = fma(delta, gj[e], t[e]);
      }
      have_t = true;
    } else if (update) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (a[e] < 0.f) a[e] = (float)((double)a[e] + step);
      for (int sw = 0; sw < sweeps; ++sw) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) sm.a[team][c0 + e] = a[e];
        __syncthreads();
        double s[8];
        row_times_g<SKP>(sm.a[team], sG, c0, s);
        float g[8];
        double num = 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          g[e] = a[e] >= 0.f ? (float)(s[e] - p[e]) : 0.f;
          num = fma((double)g[e], (double)g[e], num);
          sm.g[team][c0 + e] = g[e];
        }
        __syncthreads();
        double h[8];
        row_times_g<SKP>(sm.g[team], sG, c0, h);
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
    if (!pre) {
      if (!have_t) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) sm.a[team][c0 + e] = a[e];
        __syncthreads();
        row_times_g<SKP>(sm.a[team], sG, c0, t);
      }
      if (valid) ck.add(a, t, p, c0, r);
    }
    if (valid) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (c0 + e < r) negc += a[e] < 0.f ? 1.0 : 0.0;
    }
    if (update) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 8; ++e) sm.a[team][c0 + e] = valid ? a[e] : 0.f;
      __syncthreads();
      float* base = A + row0 * r;
      for (int e = threadIdx.x; e < nrow * r; e += SNT) base[e] = sm.a[e / r][e % r];
    }
    __syncthreads();
  }
  double vals[9] = {ck.pg2, ck.sg, ck.mx, ck.ng2, ck.sq, ck.ap, ck.nneg, ck.mn, negc};
  const int kind[9] = {0, 0, 1, 0, 0, 0, 0, 2, 0};
  block_reduce_fields<SNT, 9>(vals, kind, sm.sh, sm.out);
  __syncthreads();
}

__device__ void load_gram32(const double* G, RowSmem& sm) {
  for (int e = threadIdx.x; e < SKP * SKP; e += SNT) sm.G[e] = G[e];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One ADMM step of Algorithm 1 (eq. 7) over the N = m + n rows of W = [U*;
// V*] (the float32 factors), KR = r rounded up to 8.  Blocks of kAdmmRB rows
// pass through LDS: the next block's W and state rows are loaded into
// registers (flat, coalesced) while the current one is processed, and the
// new state goes straight back to global memory.  Thread
// (rl, c) = (t / r, t % r) keeps column c of R in registers and takes rows
// rl, rl + nl, ... (nl = 256 / r row lanes) of the block: w = (W R)[row][c]
// (float64, four interleaved partial sums), then the multiplier, prox and B
// updates with the state carried as S = Y + rho Z (Y = S - rho w; N x r
// float64, row pitch r), and B[row][c] W[row][:] added to its share of column
// c of M = W^T B.  The row lanes' shares are then added into X (the polar
// step's input, which shares LDS with the row blocks) in row-lane order.  R
// must be in sm.R; ends with a barrier.
template <int KR>
__device__ void admm_rows(const ServeReq& q, const ServeScalars& ctl, AdmmSmem& sm, int64_t m,
                          int64_t N, int r, int step) {
  constexpr int PW = kAdmmRB * KR / SNT;   // W elements per thread and block
  constexpr int PS = kAdmmRB * SKP / SNT;  // state elements per thread and block (at most)
  const double rho = ctl.rho, irho = 1.0 / rho;
  const int nl = SNT / r;
  const int rl = threadIdx.x / r, c = threadIdx.x % r;
  const bool act = rl < nl;
  __syncthreads();   // R staged
  double rc[KR], macc[KR];
#pragma unroll
  for (int a = 0; a < KR; ++a) {
    rc[a] = (act && a < r) ? sm.R[a * SKP + c] : 0.0;
    macc[a] = 0.0;
  }
  float wn[PW];
  double sn[PS];
  auto fetch = [&](int64_t row0) {
    const int nrow = (int)imin(N - row0, kAdmmRB);
#pragma unroll
    for (int u = 0; u < PW; ++u) {
      const int e = threadIdx.x + SNT * u;
      const int rr = e / KR, a = e % KR;
      const int64_t row = row0 + rr;
      float v = 0.f;
      if (rr < nrow && a < r) v = row < m ? q.U[row * r + a] : q.V[(row - m) * r + a];
      wn[u] = v;
    }
    if (step > 0) {
      const double* src = q.S + row0 * r;
#pragma unroll
      for (int u = 0; u < PS; ++u) {
        const int e = threadIdx.x + SNT * u;
        sn[u] = e < nrow * r ? src[e] : 0.0;
      }
    }
  };
  fetch(0);
  for (int64_t row0 = 0; row0 < N; row0 += kAdmmRB) {
    const int nrow = (int)imin(N - row0, kAdmmRB);
    __syncthreads();   // the previous block is consumed
#pragma unroll
    for (int u = 0; u < PW; ++u) {
      const int e = threadIdx.x + SNT * u;
      sm.Wb[(e / KR) * SKP + e % KR] = wn[u];
    }
    if (step > 0) {
#pragma unroll
      for (int u = 0; u < PS; ++u) sm.Sb[threadIdx.x + SNT * u] = sn[u];
    }
    __syncthreads();
    // the next block's loads are issued here, after the barrier (a barrier
    // waits for every load in flight), and meet the compute below
    if (row0 + kAdmmRB < N) fetch(row0 + kAdmmRB);
    if (act) {
      for (int rr = rl; rr < nrow; rr += nl) {
        double wv[KR];
#pragma unroll
        for (int a = 0; a < KR; ++a) wv[a] = (double)sm.Wb[rr * SKP + a];
        double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < KR; ++a) w4[a % 4] = fma(wv[a], rc[a], w4[a % 4]);
        const double w = (w4[0] + w4[1]) + (w4[2] + w4[3]);
        const double y = step > 0 ? sm.Sb[rr * r + c] - rho * w : 0.0;
        const double b = w - y * irho;
        const double z = b > 0.0 ? b : (b >= -irho ? 0.0 : b + irho);
        q.S[(row0 + rr) * r + c] = y + rho * z;   // consecutive across the wave
        const double bb = z + y * irho;
#pragma unroll
        for (int a = 0; a < KR; ++a) macc[a] = fma(wv[a], bb, macc[a]);
      }
    }
  }
  __syncthreads();   // the last block is consumed before X takes its LDS
  for (int e = threadIdx.x; e < SKP * (SKP + 1); e += SNT) sm.X[e / (SKP + 1)][e % (SKP + 1)] = 0.0;
  for (int l = 0; l < nl; ++l) {
    __syncthreads();
    if (rl == l) {
#pragma unroll
      for (int a = 0; a < KR; ++a)
        if (a < r) sm.X[a][c] += macc[a];
    }
  }
}

// ---------------------------------------------------------------------------
// The state machine.  Each call runs one step; thread 0 updates ctl, and
// every path ends at a barrier.
// ---------------------------------------------------------------------------
template <int XT>
__device__ void serve_step(const ServeReq& q, ServeState& st, ServeScalars& ctl, ServeSmem& sm,
                              double* red) {
  const XE<XT>* X = reinterpret_cast<const XE<XT>*>(q.X);
  const int64_t m = q.m, n = q.n, ld = q.ld;
  const int r = q.r, kk = q.kk;
  const int t0 = threadIdx.x == 0;
  const int stage = ctl.stage, sub = ctl.sub;

  if (stage == kStSvd) {
    const int last_orth = 2 * q.power_iters;   // subs 0..last_orth end with an orthonormalisation
    if (sub == 0) {
      xb<XT>(X, m, n, ld, q.omega, kk, kk, q.Y32, kk, sm);
      orth(q.Y32, m, kk, q.Qm64, q.Y32, st.scratch, sm);
    } else if (sub <= last_orth) {
      if (sub & 1) {
        xta<XT>(X, m, n, ld, q.Y32, kk, kk, q.Z32, kk, sm);
        orth(q.Z32, n, kk, q.Qn64, q.Z32, st.scratch, sm);
      } else {
        xb<XT>(X, m, n, ld, q.Z32, kk, kk, q.Y32, kk, sm);
        orth(q.Y32, m, kk, q.Qm64, q.Y32, st.scratch, sm);
      }
    } else if (sub == last_orth + 1) {
      // B = Q^T X through Z = X^T Q; SVD of B from the eigenpairs of Z^T Z
      xta<XT>(X, m, n, ld, q.Y32, kk, kk, q.Z32, kk, sm);
      bx_cross<float, float, SKB>(q.Z32, kk, kk, q.Z32, kk, kk, n, st.scratch, sm.g);
      eig_of(st.scratch, kk, sm.e);
      // column sums of Q (float64, fixed order per column)
      double* colsum = sm.e.aux + SKB;
      if (threadIdx.x < kk) {
        double cs = 0.0;
        for (int64_t i = 0; i < m; ++i) cs += q.Qm64[i * kk + threadIdx.x];
        colsum[threadIdx.x] = cs;
      }
      __syncthreads();
      // signs (column sum of U positive), sigma, TU into S, TV into scratch
      double* TU = sm.e.j.S;
      __shared__ double sgn[SKP], sq[SKP];
      if (threadIdx.x < r) {
        const int j = threadIdx.x;
        double cs = 0.0;
        for (int a = 0; a < kk; ++a) cs = fma(colsum[a], eigvec<SKB>(sm.e.j, a, j), cs);
        sgn[j] = cs < 0.0 ? -1.0 : 1.0;
        const double l = sm.e.aux[j];
        const double sg = l > 0.0 ? sqrt(l) : 0.0;
        st.sigma[j] = sg;
        sq[j] = sqrt(sg);
      }
      __syncthreads();
      for (int e = threadIdx.x; e < SKB * SKB; e += SNT) {
        const int a = e / SKB, j = e % SKB;
        double w = 0.0;
        if (a < kk && j < r) w = eigvec<SKB>(sm.e.j, a, j) * sgn[j];
        st.scratch[e] = (j < r && sq[j] > 0.0) ? w / sq[j] : 0.0;
        TU[e] = j < r ? w * sq[j] : 0.0;
      }
      __syncthreads();
      bx_apply<double, float, SKB>(q.Qm64, kk, kk, m, TU, r, q.U, r);
      for (int e = threadIdx.x; e < SKB * SKB; e += SNT) TU[e] = st.scratch[e];
      __syncthreads();
      bx_apply<float, float, SKB>(q.Z32, kk, kk, n, TU, r, q.V, r);
    } else {
      // Eckart-Young floor evaluated directly: ||X - U* V*^T|| / ||X||
      const double nx2 = sumsq_x<XT>(X, m, n, ld, red);
      const double f = residual<XT>(X, m, n, ld, q.U, q.V, r, sm.p, red);
      if (t0) {
        ctl.nx2 = nx2;
        ctl.relerr_svd = nx2 > 0.0 ? sqrt(2.0 * f / nx2) : 0.0;
      }
    }
    if (t0) {
      if (sub >= last_orth + 2) {
        ctl.stage = kStRot;
        ctl.sub = 0;
      } else {
        ctl.sub = sub + 1;
      }
    }
    __syncthreads();
    return;
  }

  if (stage == kStRot) {
    const int64_t N = m + n;
    double* Rs = sm.a.R;
    if (sub == 0) {
      // rho = rho0 sqrt(N r) / ||W||_F for W = [U*; V*] (the float32 factors,
      // read in float64 where needed), R = I
      double s2 = 0.0;
      for (int64_t e = threadIdx.x; e < m * r; e += SNT) s2 = fma((double)q.U[e], (double)q.U[e], s2);
      for (int64_t e = threadIdx.x; e < n * r; e += SNT) s2 = fma((double)q.V[e], (double)q.V[e], s2);
      s2 = bsum(s2, red);
      for (int e = threadIdx.x; e < SKP * SKP; e += SNT)
        st.R[e] = (e / SKP == e % SKP && e / SKP < r) ? 1.0 : 0.0;
      if (t0) {
        ctl.rho = s2 > 0.0 ? q.rho0 * sqrt((double)N * r) / sqrt(s2) : 1.0;
        ctl.dR = INFINITY;
        ctl.rot_steps = 0;
        if (q.rot_max_iter > 0) {
          ctl.sub = 1;
        } else {
          ctl.stage = kStSetup;
          ctl.sub = 0;
        }
      }
      __syncthreads();
      return;
    }
    if (sub == 1) {
      // one ADMM step (Algorithm 1): rows and M = W^T B (admm_rows), then R = polar(M)
      const int step = ctl.rot_steps;
      for (int e = threadIdx.x; e < SKP * SKP; e += SNT) Rs[e] = st.R[e];
      if (r <= 8) admm_rows<8>(q, ctl, sm.a, m, N, r, step);
      else if (r <= 16) admm_rows<16>(q, ctl, sm.a, m, N, r, step);
      else if (r <= 24) admm_rows<24>(q, ctl, sm.a, m, N, r, step);
      else admm_rows<32>(q, ctl, sm.a, m, N, r, step);
      __syncthreads();
      const bool ok = polar_ns_block<SKP>(sm.a.X, sm.a.T, sm.a.red, (r + 3) / 4 * 4);
      double d2 = 0.0;
      if (ok) {
        for (int e = threadIdx.x; e < SKP * SKP; e += SNT) {
          const int a = e / SKP, c = e % SKP;
          const double v = (a < r && c < r) ? sm.a.X[a][c] : 0.0;
          const double dv = v - st.R[e];
          d2 = fma(dv, dv, d2);
          st.R[e] = v;
        }
      }
      d2 = bsum(d2, red);
      if (t0) {
        ctl.dR = ok ? sqrt(d2) : 0.0;
        ctl.rot_steps = step + 1;
        const bool tol_hit = q.rot_tol > 0.0 && (step + 1) % q.rot_check_every == 0 && ctl.dR <= q.rot_tol;
        if (tol_hit || step + 1 >= q.rot_max_iter) ctl.sub = 2;
      }
      __syncthreads();
      return;
    }
    // U = W_U R, V = W_V R with the last R
    for (int e = threadIdx.x; e < SKP * SKP; e += SNT) Rs[e] = st.R[e];
    __syncthreads();
    // in place: each row is read whole before it is written
    bx_apply<float, float, SKP>(q.U, r, r, m, Rs, r, q.U, r);
    bx_apply<float, float, SKP>(q.V, r, r, n, Rs, r, q.V, r);
    if (t0) {
      ctl.stage = kStSetup;
      ctl.sub = 0;
    }
    __syncthreads();
    return;
  }

  if (stage == kStSetup) {
    // resolved push sizes, phase, H = U^T U, Q = X^T U, KKT partials of V
    if (q.mode == 1) {
      for (int64_t e = threadIdx.x; e < m * r; e += SNT) q.U[e] = q.U[e] > 0.f ? q.U[e] : 0.f;
      for (int64_t e = threadIdx.x; e < n * r; e += SNT) q.V[e] = q.V[e] > 0.f ? q.V[e] : 0.f;
      __syncthreads();
    }
    double mnU = INFINITY, mnV = INFINITY, negs = 0.0;
    for (int64_t e = threadIdx.x; e < m * r; e += SNT) {
      mnU = fmin(mnU, (double)q.U[e]);
      negs += q.U[e] < 0.f ? 1.0 : 0.0;
    }
    for (int64_t e = threadIdx.x; e < n * r; e += SNT) {
      mnV = fmin(mnV, (double)q.V[e]);
      negs += q.V[e] < 0.f ? 1.0 : 0.0;
    }
    mnU = block_min<SNT>(mnU, red);
    mnV = block_min<SNT>(mnV, red);
    negs = bsum(negs, red);
    bx_cross<float, float, SKP>(q.U, r, r, q.U, r, r, m, st.H, sm.g);
    xta<XT>(X, m, n, ld, q.U, r, r, q.Z32, r, sm);
    load_gram32(st.H, sm.w);
    row_pass(q.V, n, r, q.Z32, sm.w, false, false, kPhaseHals, 0.0, 0, false);
    if (t0) {
      const double d = (double)q.ext_iters - 0.5;
      ctl.step[0] = q.step_u > 0.0 ? q.step_u : fmax(-mnU, 0.0) / d;
      ctl.step[1] = q.step_v > 0.0 ? q.step_v : fmax(-mnV, 0.0) / d;
      ctl.iphase = negs > 0.0 ? kPhaseExt : kPhaseHals;
      for (int f = 0; f < 8; ++f) ctl.recV[f] = sm.w.out[f];
      ctl.negsV = sm.w.out[8];
      ctl.k = 0;
      ctl.iters = 0;
      ctl.ext_done = 0;
      ctl.stage = kStIter;
    }
    __syncthreads();
    return;
  }

  if (stage == kStIter) {
    const int k = ctl.k;
    // G = V^T V, P = X V, KKT partials of U^k (pre-update)
    bx_cross<float, float, SKP>(q.V, r, r, q.V, r, r, n, st.G, sm.g);
    xb<XT>(X, m, n, ld, q.V, r, r, q.Y32, r, sm);
    load_gram32(st.G, sm.w);
    row_pass(q.U, m, r, q.Y32, sm.w, false, true, kPhaseHals, 0.0, 0, false);
    // check of iteration k (the KKT appendix), same expressions as k_finalize
    double hg = 0.0;
    for (int e = threadIdx.x; e < SKP * SKP; e += SNT) hg = fma(st.H[e], st.G[e], hg);
    hg = bsum(hg, red);
    __shared__ int s_stop;
    if (t0) {
      const double* a = sm.w.out;       // U side
      const double* b = ctl.recV;       // V side
      const double negsU = a[8];
      const double nx2 = ctl.nx2;
      const double f = 0.5 * nx2 - a[5] + 0.5 * hg;
      const double nx = sqrt(nx2);
      const double nU = sqrt(a[4]), nV = sqrt(b[4]);
      const double feas = fmax(nU > 0.0 ? sqrt(a[3]) / nU : 0.0, nV > 0.0 ? sqrt(b[3]) / nV : 0.0);
      const double pgu = (nV > 0.0 && nx > 0.0) ? sqrt(a[0]) / (nx * nV) : 0.0;
      const double pgv = (nU > 0.0 && nx > 0.0) ? sqrt(b[0]) / (nx * nU) : 0.0;
      const double kkt = fmax(feas, fmax(pgu, pgv));
      const double relerr = nx > 0.0 ? sqrt(fmax(2.0 * f, 0.0)) / nx : 0.0;
      const double negs = a[6] + b[6];
      const bool due = (k % q.check_every == 0) || k == q.max_iter;
      bool stop = k >= q.max_iter;
      bool hit = false;
      if (due) {
        ctl.f = f;
        ctl.relerr = relerr;
        ctl.kkt = kkt;
        ctl.kkt_feas = feas;
        ctl.kkt_pg_u = pgu;
        ctl.kkt_pg_v = pgv;
        ctl.delta_w = fmax(a[2], b[2]);
        ctl.sigma_w = a[1] + b[1];
        ctl.min_w = fmin(a[7], b[7]);
        hit = negs == 0.0 && ((q.kkt_tol >= 0.0 && kkt <= q.kkt_tol) ||
                              (q.relerr_tol >= 0.0 && relerr - ctl.relerr_svd <= q.relerr_tol) ||
                              q.mode == 3);
        if (!isfinite(f) || !isfinite(kkt)) ctl.numeric_error = 1;
        if (hit || ctl.numeric_error) stop = true;
      }
      ctl.iphase = negsU + ctl.negsV > 0.0 ? kPhaseExt : kPhaseHals;
      if (stop) {
        ctl.converged = hit ? 1 : 0;
        ctl.iters = k;
        ctl.stage = kStFinal;
      }
      s_stop = stop ? 1 : 0;
    }
    __syncthreads();
    if (s_stop) return;
    const int phase = ctl.iphase;
    // U half: update in place, then H = U^T U and Q = X^T U
    row_pass(q.U, m, r, q.Y32, sm.w, true, true, phase, ctl.step[0], q.sweeps, q.mode == 2);
    bx_cross<float, float, SKP>(q.U, r, r, q.U, r, r, m, st.H, sm.g);
    xta<XT>(X, m, n, ld, q.U, r, r, q.Z32, r, sm);
    // V half with the new U; KKT partials of V^(k+1)
    load_gram32(st.H, sm.w);
    row_pass(q.V, n, r, q.Z32, sm.w, true, false, phase, ctl.step[1], q.sweeps, q.mode == 2);
    if (t0) {
      for (int f = 0; f < 8; ++f) ctl.recV[f] = sm.w.out[f];
      ctl.negsV = sm.w.out[8];
      if (phase == kPhaseExt) ctl.ext_done += 1;
      ctl.k = k + 1;
      ctl.iters = k + 1;
    }
    __syncthreads();
    return;
  }

  // final objective, evaluated directly
  const double f = residual<XT>(X, m, n, ld, q.U, q.V, r, sm.p, red);
  if (t0) {
    ctl.f = f;
    ctl.relerr = ctl.nx2 > 0.0 ? sqrt(2.0 * f / ctl.nx2) : 0.0;
    if (!isfinite(f)) ctl.numeric_error = 1;
    ctl.stage = kStDone;
  }
  __syncthreads();
}

template <int XT>
__global__ __launch_bounds__(SNT) void k_serve_tick(ServeSlot* __restrict__ slots,
                                                    ServeStatus* __restrict__ status, int nslots,
                                                    int64_t time_limit) {
  __shared__ ServeSmem sm;
  __shared__ ServeScalars ctl;
  __shared__ double red[SNT / kWave];
  const int b = blockIdx.x;
  if (b >= nslots) return;
  ServeStatus* stt = status + b;
  ServeSlot* sl = slots + b;
  if (stt->status != kSlotRunning || sl->q.xt != XT) return;
  if (threadIdx.x == 0) ctl = sl->s.c;
  __syncthreads();
  // steps until one ends past the slot's time in this tick, read by thread 0
  // from the constant 100 MHz clock and shared through LDS
  const long long t_start = wall_clock64();
  __shared__ int s_more;
  while (ctl.stage != kStDone) {
    serve_step<XT>(sl->q, sl->s, ctl, sm, red);
    if (threadIdx.x == 0) s_more = wall_clock64() - t_start < time_limit ? 1 : 0;
    __syncthreads();
    if (!s_more) break;
  }
  if (threadIdx.x == 0) {
    sl->s.c = ctl;
    const bool done = ctl.stage == kStDone;
    stt->stage = ctl.stage;
    stt->iters = ctl.iters;
    stt->ext_done = ctl.ext_done;
    stt->converged = ctl.converged;
    stt->phase = ctl.iphase;
    stt->rot_steps = ctl.rot_steps;
    stt->numeric_error = ctl.numeric_error;
    stt->f = ctl.f;
    stt->relerr = ctl.relerr;
    stt->kkt = ctl.kkt;
    stt->kkt_feas = ctl.kkt_feas;
    stt->kkt_pg_u = ctl.kkt_pg_u;
    stt->kkt_pg_v = ctl.kkt_pg_v;
    stt->delta_w = ctl.delta_w;
    stt->sigma_w = ctl.sigma_w;
    stt->step_u = ctl.step[0];
    stt->step_v = ctl.step[1];
    stt->relerr_svd = ctl.relerr_svd;
    stt->status = done ? kSlotDone : kSlotRunning;
  }
}

}  // namespace

namespace {

// Admission batch: workgroup b copies staged record b into its slot's record
// head and status (8-byte words).
__global__ __launch_bounds__(256) void k_serve_admit(const ServeAdmit* __restrict__ staged,
                                                     ServeSlot* __restrict__ slots,
                                                     ServeStatus* __restrict__ status) {
  const ServeAdmit& a = staged[blockIdx.x];
  const int slot = a.slot;
  const uint64_t* hs = reinterpret_cast<const uint64_t*>(a.head);
  uint64_t* hd = reinterpret_cast<uint64_t*>(slots + slot);
  for (int w = threadIdx.x; w < (int)(kSlotHeadBytes / 8); w += blockDim.x) hd[w] = hs[w];
  const uint64_t* ss = reinterpret_cast<const uint64_t*>(&a.status);
  uint64_t* sd = reinterpret_cast<uint64_t*>(status + slot);
  for (int w = threadIdx.x; w < (int)(sizeof(ServeStatus) / 8); w += blockDim.x) sd[w] = ss[w];
}

}  // namespace

hipError_t launch_serve_admit(const ServeAdmit* staged, int count, ServeSlot* slots, ServeStatus* status,
                              hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(k_serve_admit, dim3(count), dim3(256), 0, s, staged, slots, status);
  return hipGetLastError();
}

hipError_t launch_serve_tick(int xt, ServeSlot* slots, ServeStatus* status, int nslots,
                             int64_t time_limit, hipStream_t s) {
  if (nslots < 1) return hipSuccess;
  if (xt == ENMF_F32)
    hipLaunchKernelGGL((k_serve_tick<0>), dim3(nslots), dim3(SNT), 0, s, slots, status, nslots, time_limit);
  else if (xt == ENMF_BF16)
    hipLaunchKernelGGL((k_serve_tick<1>), dim3(nslots), dim3(SNT), 0, s, slots, status, nslots, time_limit);
  else
    hipLaunchKernelGGL((k_serve_tick<2>), dim3(nslots), dim3(SNT), 0, s, slots, status, nslots, time_limit);
  return hipGetLastError();
}

}  // namespace enmf
