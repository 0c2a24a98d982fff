// Matrix-core (MFMA) forms of the X-streaming products for ranks >= 16,
// where each product is a real dense contraction (appendix on complexity:
// X V and X^T U, O(mnr) per half-iteration).
//
//   float32 X: X and the factor each split into three bfloat16 terms on
//     v_mfma_f32_16x16x32_bf16 (six of the nine term products), float32
//     accumulate.
//   bfloat16 X: v_mfma_f32_16x16x32_bf16, float32 accumulate, with the float32
//     factor split into three bfloat16 terms (hi = rne(v), mid = rne(v - hi),
//     lo = rne(v - hi - mid), |v - hi - mid - lo| <= 2^-24 |v|), so that
//     X . v = X . hi + X . mid + X . lo keeps the factor to float32 precision
//     (the split-precision refinement of Henry et al. 2019); X itself is exact.
//
// MFMA 16x16 tiles on gfx950 (wave64): lane l = 16 g + i (i = l % 16,
// g = l / 16).  16x16x32 bf16: A = A[i][8g .. 8g+7], B = B[8g .. 8g+7][i].
// Result:
// D[4g + v][i] in accumulator element v.  The contraction index of a tile is
// free to be permuted as long as A and B agree, which lets every lane load
// contiguous runs of a row of X.
//
// X V  : lanes take rows of X (16 per tile); the factor chunk sits in LDS,
//        prefetched through registers.
// X^T U: lanes take 16-byte runs along a row of X; a tile covers a strided
//        set of 16 columns, so that each lane holds 8 rows of one column
//        (for bfloat16 the 8 x 8 blocks are transposed in registers, v_perm).
// Both split the contraction over blocks; partials are reduced in fixed
// order by the caller.
#include <stdint.h>

#include <map>
#include <mutex>

#include "dev_common.h"
#include "enmf_internal.h"
#include "decide.h"
#include "mfma_common.h"

namespace enmf {

namespace {


constexpr int kT = 256;




// Logical block (tile bx, contraction range by) of a tiles x splits product
// grid.  The dispatcher hands consecutive workgroups to the 8 XCDs in turn
// (workgroup L runs on XCD L % 8); each XCD here takes one contiguous range
// of the logical blocks in split-major order, so the blocks that read the
// same factor chunks share that XCD's L2.  Used by X B, whose packed factor
// outgrows one L2 and is read by every row tile; X^T A keeps the dispatch
// order (measured: its packed factor stays L2-resident and the remap only
// spreads its row bands).
__device__ __forceinline__ void xcd_block(int64_t& bx, int64_t& by) {
  const int64_t tiles = gridDim.x;
  const int64_t nb = tiles * gridDim.y;
  const int64_t L = blockIdx.x + tiles * blockIdx.y;
  const int64_t xcd = L % 8, slot = L / 8;
  const int64_t q = nb / 8, rem = nb % 8;
  const int64_t B = xcd * q + (xcd < rem ? xcd : rem) + slot;
  bx = B % tiles;
  by = B / tiles;
}


// Store a 16x16 accumulator tile: element v of lane (i, g) is D[4g + v][i],
// written to out[(row_of(4g+v)) * k + col0 + i].
__device__ __forceinline__ void store_tile_rows(float* __restrict__ out, int64_t m, int k,
                                                int64_t row0, int col0, const f32x4& d) {
  const int lane = threadIdx.x % kWave;
  const int i = lane % 16, g = lane / 16;
  const int col = col0 + i;
  if (col >= k) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = row0 + 4 * g + v;
    if (row < m) out[row * k + col] = d[v];
  }
}

// ---------------------------------------------------------------------------
// bfloat16 X: P = X B with B = Bhi + Bmid + Blo.  Block = 4 waves x 64 rows; chunk =
// 64 columns of X (two MFMA steps of 32).  Lane (i, g) of row tile rt loads
// X[row0 + 16 rt + i][kc + 32 s + 8g .. +7] (one A operand per step s).  The
// B operand is Bt[part][16 nt + i][32 s + 8g .. +7] of the LDS copy of the
// chunk, stored transposed (factor column major) with rows padded to 72.
// ---------------------------------------------------------------------------
constexpr int kBtLd = 72;   // padded LDS row (elements) of the transposed factor chunk, 64 rows

template <int KP>
__global__ __launch_bounds__(kT) void k_xv_bf16(const unsigned short* __restrict__ X, int64_t m,
                                                int64_t n, int64_t ld,
                                                const unsigned short* __restrict__ Bt, int k,
                                                int chunks_per_split, int64_t nchunks, int vec,
                                                float* __restrict__ out, int64_t split_stride,
    const int32_t* __restrict__ stop,
    const double* __restrict__ gsrc, int gparts, int gkp, double* __restrict__ gdst) {
  if (stop != nullptr && *stop) return;
  constexpr int NT = KP / 16;
  constexpr int RT = 4;
  constexpr int CH = 3 * KP * kBtLd;   // elements of one packed chunk (hi, mid, lo)
  __shared__ __align__(16) unsigned short Bs[2][CH];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  int64_t bx, by;
  xcd_block(bx, by);
  const int64_t row0 = bx * (4 * 64) + 64 * w;
  const int64_t c0 = by * chunks_per_split;
  const int64_t c1 = c0 + chunks_per_split < nchunks ? c0 + chunks_per_split : nchunks;

  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = zero4();

  uint4 xa[RT][2], xb[RT][2];
  auto load_x = [&](int64_t ch, uint4 (&dst)[RT][2]) {
    const bool interior = vec && row0 + 64 <= m && (ch + 1) * 64 <= n;   // wave-uniform
    if (interior) {
      const unsigned short* base = X + (row0 + i) * ld + ch * 64 + 8 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s = 0; s < 2; ++s) dst[rt][s] = ldg16(base + 16 * rt * ld + 32 * s);
    } else {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s = 0; s < 2; ++s)
          dst[rt][s] = load16<unsigned short>(X, m, n, ld, row0 + 16 * rt + i,
                                              ch * 64 + 32 * s + 8 * g, vec != 0);
    }
  };
  // The next chunk of the factor travels through registers and reaches LDS
  // only after the current chunk's MFMAs, so waiting for it never stalls the
  // X prefetch issued behind it.
  constexpr int NBQ = (CH / 8 + kT - 1) / kT;
  uint4 bq_next[NBQ];
  auto fetch_b = [&](int64_t ch) {
    const uint4* src = reinterpret_cast<const uint4*>(Bt + ch * CH);
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int e = threadIdx.x + u * kT;
      bq_next[u] = e < CH / 8 ? src[e] : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_b = [&](int buf) {
    uint4* dst = reinterpret_cast<uint4*>(Bs[buf]);
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int e = threadIdx.x + u * kT;
      if (e < CH / 8) dst[e] = bq_next[u];
    }
  };
  if (c0 < c1) {
    fetch_b(c0);
    load_x(c0, xa);
  }
  // side job: a Gram combine, one entry per wave, its loads behind the first chunk's
  const int64_t gwave = ((int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y) * (kT / kWave) + w;
  if (gsrc != nullptr) gram_combine(gsrc, gparts, gkp, gdst, gwave, (int64_t)gridDim.x * gridDim.y * (kT / kWave));
  if (c0 < c1) store_b(0);
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __syncthreads();
    const bool more = ch + 1 < c1;
    if (more) {
      fetch_b(ch + 1);
      load_x(ch + 1, xb);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
        for (int hl = 0; hl < 3; ++hl) {
          const uint4 bq = *reinterpret_cast<const uint4*>(
              &Bs[buf][(hl * KP + 16 * nt + i) * kBtLd + 32 * s + 8 * g]);
          const bf16x8 b = as_bf16x8(bq);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][nt] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(xa[rt][s]), b, acc[rt][nt], 0, 0, 0);
        }
      }
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) { xa[rt][0] = xb[rt][0]; xa[rt][1] = xb[rt][1]; }
    }
    buf ^= 1;
  }
  float* o = out + by * split_stride;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) store_tile_rows(o, m, k, row0 + 16 * rt, 16 * nt, acc[rt][nt]);
}

// ---------------------------------------------------------------------------
// float32 X through the bfloat16 matrix cores: X = x1 + x2 + x3 and
// B = b1 + b2 + b3 (three-term bfloat16 splits, |v - v1 - v2 - v3| <= 2^-24 |v|),
// and X B = sum of the six products xa bc with a + c <= 4; the three dropped
// ones together stay below 2^-23 |x||b|, so the result keeps float32
// accuracy while each 32-step costs six 16x16x32 bf16 MFMAs instead of eight
// 16x16x4 f32 ones of twice the cycles.  Block = 4 waves x 64 rows; chunk =
// 32 columns of X (one MFMA step).  Lane (i, g) of row tile rt loads
// X[row0 + 16 rt + i][kc + 8g .. +7] (two 16-byte loads) and splits it in
// registers; the factor chunk is Bt[part][16 nt + i][8g .. +7] in LDS,
// transposed with rows padded to 40, prefetched through registers like the
// bfloat16 kernel's.
// ---------------------------------------------------------------------------
constexpr int kBt32Ld = 40;

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned pk_bf16(f32x2 v) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// Eight floats (lo = elements 0..3, hi = 4..7) -> three packed bf16 terms.
__device__ __forceinline__ void split3(const uint4& lo, const uint4& hi, uint4& p1, uint4& p2,
                                       uint4& p3) {
  const unsigned w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  unsigned a[4], b[4], c[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const f32x2 x = {__uint_as_float(w[2 * d]), __uint_as_float(w[2 * d + 1])};
    const unsigned h = pk_bf16(x);
    const f32x2 fh = {__uint_as_float(h << 16), __uint_as_float(h & 0xffff0000u)};
    const f32x2 r = x - fh;
    const unsigned mm = pk_bf16(r);
    const f32x2 fm = {__uint_as_float(mm << 16), __uint_as_float(mm & 0xffff0000u)};
    const unsigned l = pk_bf16(r - fm);
    a[d] = h;
    b[d] = mm;
    c[d] = l;
  }
  p1 = make_uint4(a[0], a[1], a[2], a[3]);
  p2 = make_uint4(b[0], b[1], b[2], b[3]);
  p3 = make_uint4(c[0], c[1], c[2], c[3]);
}

template <int KP>
__global__ __launch_bounds__(kT) void k_xv_f32s(const float* __restrict__ X, int64_t m, int64_t n,
                                                int64_t ld, const unsigned short* __restrict__ Bt,
                                                int k, int chunks_per_split, int64_t nchunks,
                                                int vec, float* __restrict__ out,
                                                int64_t split_stride,
                                                const int32_t* __restrict__ stop,
    const double* __restrict__ gsrc, int gparts, int gkp, double* __restrict__ gdst) {
  if (stop != nullptr && *stop) return;
  constexpr int NT = KP / 16;
  constexpr int RT = 4;
  constexpr int CH = 3 * KP * kBt32Ld;   // elements of one packed chunk (three terms)
  __shared__ __align__(16) unsigned short Bs[2][CH];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  int64_t bx, by;
  xcd_block(bx, by);
  const int64_t row0 = bx * (4 * 64) + 64 * w;
  const int64_t c0 = by * chunks_per_split;
  const int64_t c1 = c0 + chunks_per_split < nchunks ? c0 + chunks_per_split : nchunks;

  f32x4 acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[rt][nt] = zero4();

  uint4 xa[RT][2], xb[RT][2];
  auto load_x = [&](int64_t ch, uint4 (&dst)[RT][2]) {
    const bool interior = vec && row0 + 64 <= m && (ch + 1) * 32 <= n;   // wave-uniform
    if (interior) {
      const float* base = X + (row0 + i) * ld + ch * 32 + 8 * g;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int h = 0; h < 2; ++h) dst[rt][h] = ldg16(base + 16 * rt * ld + 4 * h);
    } else {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          dst[rt][h] = load16<float>(X, m, n, ld, row0 + 16 * rt + i, ch * 32 + 8 * g + 4 * h,
                                     vec != 0);
    }
  };
  constexpr int NBQ = (CH / 8 + kT - 1) / kT;
  uint4 bq_next[NBQ];
  auto fetch_b = [&](int64_t ch) {
    const uint4* src = reinterpret_cast<const uint4*>(Bt + ch * CH);
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int e = threadIdx.x + u * kT;
      bq_next[u] = e < CH / 8 ? src[e] : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_b = [&](int buf) {
    uint4* dst = reinterpret_cast<uint4*>(Bs[buf]);
#pragma unroll
    for (int u = 0; u < NBQ; ++u) {
      const int e = threadIdx.x + u * kT;
      if (e < CH / 8) dst[e] = bq_next[u];
    }
  };
  if (c0 < c1) {
    fetch_b(c0);
    load_x(c0, xa);
  }
  // side job: a Gram combine, one entry per wave, its loads behind the first chunk's
  const int64_t gwave = ((int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y) * (kT / kWave) + w;
  if (gsrc != nullptr) gram_combine(gsrc, gparts, gkp, gdst, gwave, (int64_t)gridDim.x * gridDim.y * (kT / kWave));
  if (c0 < c1) store_b(0);
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __syncthreads();
    const bool more = ch + 1 < c1;
    if (more) {
      fetch_b(ch + 1);
      load_x(ch + 1, xb);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      uint4 x1, x2, x3;
      split3(xa[rt][0], xa[rt][1], x1, x2, x3);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const unsigned short* bp = &Bs[buf][(16 * nt + i) * kBt32Ld + 8 * g];
        const bf16x8 b1 = as_bf16x8(*reinterpret_cast<const uint4*>(bp));
        const bf16x8 b2 = as_bf16x8(*reinterpret_cast<const uint4*>(bp + KP * kBt32Ld));
        const bf16x8 b3 = as_bf16x8(*reinterpret_cast<const uint4*>(bp + 2 * KP * kBt32Ld));
        f32x4 a = acc[rt][nt];
        // smallest terms first
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x3), b1, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x2), b2, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1), b3, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x2), b1, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1), b2, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1), b1, a, 0, 0, 0);
        acc[rt][nt] = a;
      }
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) { xa[rt][0] = xb[rt][0]; xa[rt][1] = xb[rt][1]; }
    }
    buf ^= 1;
  }
  float* o = out + by * split_stride;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) store_tile_rows(o, m, k, row0 + 16 * rt, 16 * nt, acc[rt][nt]);
}

// Side jobs of the bfloat16 X^T A launch (the stop decision and a Gram
// combine), when it carries them, run in one extra row of workgroups at the
// end of the grid, which the dispatcher hands out after every streaming
// workgroup: block 0 of the row takes the check and stop decision of the
// iteration, the others the Gram combine (one entry group per wave; all of
// the row when it has one block).  Returns true in that row.  (The float32
// kernels keep their side jobs in their first workgroups, where the Gram
// combine overlaps the first chunk loads: the extra row measured slower for
// them and about 1% faster for bfloat16 X at the ratings shape.)
__device__ __forceinline__ bool xtu_side_row(const double* __restrict__ gsrc, int gparts, int gkp,
                                             double* __restrict__ gdst, const DecideArgs& dec,
                                             DevState* dst) {
  if ((gsrc == nullptr && dst == nullptr) || blockIdx.y != gridDim.y - 1) return false;
  const int w = threadIdx.x / kWave;
  if (dst != nullptr && blockIdx.x == 0) {
    __shared__ double dsh[17 * (kT / kWave)];
    __shared__ int dflag;
    (void)check_decide<kT>(dec, 0, dst, true, dsh, &dflag);
  }
  if (gsrc != nullptr) {
    const int g0 = (dst != nullptr && gridDim.x > 1) ? 1 : 0;
    if ((int)blockIdx.x >= g0)
      gram_combine(gsrc, gparts, gkp, gdst, (int64_t)(blockIdx.x - g0) * (kT / kWave) + w,
                   (int64_t)(gridDim.x - g0) * (kT / kWave));
  }
  return true;
}

// ---------------------------------------------------------------------------
// bfloat16 X: Q = X^T A with A = Ahi + Amid + Alo.  Block = 4 waves x 128 columns;
// chunk = 32 rows (one MFMA step).  Lane (i, g) loads the 8 x 8 block
// X[rc + 8g + e][j0 + 8i .. 8i+7] (e = 0..7) and transposes it in registers:
// operand t holds X[rc + 8g + 0..7][j0 + 8i + t], so tile t covers columns
// j0 + 8 mm + t.  B operand = At[part][16 nt + i][8g .. 8g+7] (transposed
// chunk in LDS, rows padded to 40).
// ---------------------------------------------------------------------------
constexpr int kAtLd = 40;   // LDS row pitch of the factor chunk (bank spread)
constexpr int64_t kNtMinBytes = (int64_t)512 << 20;   // X from which X^T A loads it non-temporally
constexpr int kAtG = 32;    // its row pitch in global memory (unpadded)

template <int KP, bool NTL>
__global__ __launch_bounds__(kT) void k_xtu_bf16(const unsigned short* __restrict__ X, int64_t m,
                                                 int64_t n, int64_t ld,
                                                 const unsigned short* __restrict__ At, int k,
                                                 int64_t chunks_per_split, int64_t nchunks, int vec,
                                                 float* __restrict__ out, int64_t split_stride,
    const int32_t* __restrict__ stop,
    const double* __restrict__ gsrc, int gparts, int gkp, double* __restrict__ gdst,
    DecideArgs dec, DevState* dst) {
  if (stop != nullptr && *stop) return;
  if (xtu_side_row(gsrc, gparts, gkp, gdst, dec, dst)) return;
  constexpr int NT = KP / 16;
  constexpr int CH = 3 * KP * kAtLd;    // LDS elements of one chunk
  constexpr int CHG = 3 * KP * kAtG;    // global elements of one chunk
  __shared__ __align__(16) unsigned short As[2][CH];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  const int64_t j0 = bx * (4 * 128) + 128 * w;
  const int64_t c0 = by * chunks_per_split;
  const int64_t c1 = c0 + chunks_per_split < nchunks ? c0 + chunks_per_split : nchunks;

  f32x4 acc[8][NT];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4();

  uint4 xa[8], xb[8];
  auto load_x = [&](int64_t ch, uint4 (&dst)[8]) {
    const bool interior = vec && (ch + 1) * 32 <= m && j0 + 128 <= n;   // wave-uniform
    if (interior) {
      const unsigned short* base = X + (ch * 32 + 8 * g) * ld + j0 + 8 * i;
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e] = NTL ? ldg16_nt(base + e * ld) : ldg16(base + e * ld);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        dst[e] = load16<unsigned short>(X, m, n, ld, ch * 32 + 8 * g + e, j0 + 8 * i, vec != 0);
    }
  };
  // factor chunk prefetched into registers, stored to LDS after the MFMAs
  // the chunk's 32-element rows are four 16-byte groups in global memory and
  // the first four of five in LDS
  constexpr int NAQ = (CHG / 8 + kT - 1) / kT;
  uint4 aq_next[NAQ];
  auto fetch_a = [&](int64_t ch) {
    const uint4* src = reinterpret_cast<const uint4*>(At + ch * CHG);
#pragma unroll
    for (int u = 0; u < NAQ; ++u) {
      const int e = threadIdx.x + u * kT;
      aq_next[u] = e < CHG / 8 ? src[e] : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_a = [&](int buf) {
    uint4* dst = reinterpret_cast<uint4*>(As[buf]);
#pragma unroll
    for (int u = 0; u < NAQ; ++u) {
      const int e = threadIdx.x + u * kT;
      if (e < CHG / 8) dst[(e / 4) * (kAtLd / 8) + e % 4] = aq_next[u];
    }
  };
  if (c0 < c1) {
    fetch_a(c0);
    load_x(c0, xa);
  }
  if (c0 < c1) store_a(0);
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __syncthreads();
    const bool more = ch + 1 < c1;
    if (more) {
      fetch_a(ch + 1);
      load_x(ch + 1, xb);
    }
    // transpose: op[t] dword d = (X[2d][t], X[2d+1][t]) of the lane's 8 x 8 block
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
        // low halves (t even) or high halves (t odd) of a and b, a in the low half of the result
        d[dd] = (t % 2 == 0) ? __builtin_amdgcn_perm(b, a, 0x05040100u)
                             : __builtin_amdgcn_perm(b, a, 0x07060302u);
      }
      op[t] = make_uint4(d[0], d[1], d[2], d[3]);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
      for (int hl = 0; hl < 3; ++hl) {
        const uint4 bq =
            *reinterpret_cast<const uint4*>(&As[buf][(hl * KP + 16 * nt + i) * kAtLd + 8 * g]);
        const bf16x8 b = as_bf16x8(bq);
#pragma unroll
        for (int t = 0; t < 8; ++t)
          acc[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(op[t]), b, acc[t][nt], 0, 0, 0);
      }
    }
    if (more) {
      store_a(buf ^ 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) xa[e] = xb[e];
    }
    buf ^= 1;
  }
  // element v of lane (i, g) in tile t is column j0 + 8 (4g + v) + t, factor column 16 nt + i
  float* o = out + by * split_stride;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + i;
      if (col < k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = j0 + 8 * (4 * g + v) + t;
          if (j < n) o[j * k + col] = acc[t][nt][v];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// float32 X through the bfloat16 matrix cores: Q = X^T A with X and A split
// into three bfloat16 terms each, six term products as in X B.  Block = 4
// waves x 64 columns; chunk = 32 rows (one MFMA step).  Lane (i, g) loads
// X[rc + 8g + e][j0 + 4i .. 4i+3] (e = 0..7); operand t gathers element t of
// the eight loads, so tile t covers the columns j0 + 4 mm + t (mm = 0..15)
// and needs no register transpose.  B operand = At[part][16 nt + i][8g ..
// 8g+7] (the transposed split chunk in LDS, rows padded to 40), read once per
// chunk and shared by the four tiles.
// ---------------------------------------------------------------------------
template <int KP, bool NTL>
__global__ __launch_bounds__(kT) void k_xtu_f32s(const float* __restrict__ X, int64_t m, int64_t n,
                                                 int64_t ld, const unsigned short* __restrict__ At,
                                                 int k, int chunks_per_split, int64_t nchunks,
                                                 int vec, float* __restrict__ out,
                                                 int64_t split_stride,
                                                 const int32_t* __restrict__ stop,
    const double* __restrict__ gsrc, int gparts, int gkp, double* __restrict__ gdst,
    DecideArgs dec, DevState* dst) {
  if (stop != nullptr && *stop) return;
  // side job of the first block, before its own loads: the check and stop
  // decision of the iteration (the blocks that start later see a stop and return)
  if (dst != nullptr && blockIdx.x == 0 && blockIdx.y == 0) {
    __shared__ double dsh[17 * (kT / kWave)];
    __shared__ int dflag;
    (void)check_decide<kT>(dec, 0, dst, true, dsh, &dflag);
  }
  constexpr int NT = KP / 16;
  constexpr int CH = 3 * KP * kAtLd;    // LDS elements of one chunk
  constexpr int CHG = 3 * KP * kAtG;    // global elements of one chunk
  __shared__ __align__(16) unsigned short As[2][CH];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int i = lane % 16, g = lane / 16;
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  const int64_t j0 = bx * (4 * 64) + 64 * w;
  const int64_t c0 = by * chunks_per_split;
  const int64_t c1 = c0 + chunks_per_split < nchunks ? c0 + chunks_per_split : nchunks;

  f32x4 acc[4][NT];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[t][nt] = zero4();

  uint4 xa[8], xb[8];
  auto load_x = [&](int64_t ch, uint4 (&dst)[8]) {
    const bool interior = vec && (ch + 1) * 32 <= m && j0 + 64 <= n;   // wave-uniform
    if (interior) {
      const float* base = X + (ch * 32 + 8 * g) * ld + j0 + 4 * i;
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e] = NTL ? ldg16_nt(base + e * ld) : ldg16(base + e * ld);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        dst[e] = load16<float>(X, m, n, ld, ch * 32 + 8 * g + e, j0 + 4 * i, vec != 0);
    }
  };
  // the chunk's 32-element rows are four 16-byte groups in global memory and
  // the first four of five in LDS
  constexpr int NAQ = (CHG / 8 + kT - 1) / kT;
  uint4 aq_next[NAQ];
  auto fetch_a = [&](int64_t ch) {
    const uint4* src = reinterpret_cast<const uint4*>(At + ch * CHG);
#pragma unroll
    for (int u = 0; u < NAQ; ++u) {
      const int e = threadIdx.x + u * kT;
      aq_next[u] = e < CHG / 8 ? src[e] : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store_a = [&](int buf) {
    uint4* dst = reinterpret_cast<uint4*>(As[buf]);
#pragma unroll
    for (int u = 0; u < NAQ; ++u) {
      const int e = threadIdx.x + u * kT;
      if (e < CHG / 8) dst[(e / 4) * (kAtLd / 8) + e % 4] = aq_next[u];
    }
  };
  if (c0 < c1) {
    fetch_a(c0);
    load_x(c0, xa);
  }
  // side job: a Gram combine, one entry per wave, its loads behind the first chunk's
  const int64_t gwave = ((int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y) * (kT / kWave) + w;
  if (gsrc != nullptr) gram_combine(gsrc, gparts, gkp, gdst, gwave, (int64_t)gridDim.x * gridDim.y * (kT / kWave));
  if (c0 < c1) store_a(0);
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __syncthreads();
    const bool more = ch + 1 < c1;
    if (more) {
      fetch_a(ch + 1);
      load_x(ch + 1, xb);
    }
    // split operands of the four tiles: element t of the eight row loads
    uint4 x1[4], x2[4], x3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint4 lo, hi;
      if (t == 0) { lo = make_uint4(xa[0].x, xa[1].x, xa[2].x, xa[3].x); hi = make_uint4(xa[4].x, xa[5].x, xa[6].x, xa[7].x); }
      if (t == 1) { lo = make_uint4(xa[0].y, xa[1].y, xa[2].y, xa[3].y); hi = make_uint4(xa[4].y, xa[5].y, xa[6].y, xa[7].y); }
      if (t == 2) { lo = make_uint4(xa[0].z, xa[1].z, xa[2].z, xa[3].z); hi = make_uint4(xa[4].z, xa[5].z, xa[6].z, xa[7].z); }
      if (t == 3) { lo = make_uint4(xa[0].w, xa[1].w, xa[2].w, xa[3].w); hi = make_uint4(xa[4].w, xa[5].w, xa[6].w, xa[7].w); }
      split3(lo, hi, x1[t], x2[t], x3[t]);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const unsigned short* bp = &As[buf][(16 * nt + i) * kAtLd + 8 * g];
      const bf16x8 b1 = as_bf16x8(*reinterpret_cast<const uint4*>(bp));
      const bf16x8 b2 = as_bf16x8(*reinterpret_cast<const uint4*>(bp + KP * kAtLd));
      const bf16x8 b3 = as_bf16x8(*reinterpret_cast<const uint4*>(bp + 2 * KP * kAtLd));
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 a = acc[t][nt];
        // smallest terms first
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x3[t]), b1, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x2[t]), b2, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1[t]), b3, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x2[t]), b1, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1[t]), b2, a, 0, 0, 0);
        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(x1[t]), b1, a, 0, 0, 0);
        acc[t][nt] = a;
      }
    }
    if (more) {
      store_a(buf ^ 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) xa[e] = xb[e];
    }
    buf ^= 1;
  }
  // element v of lane (i, g) in tile t is column j0 + 4 (4g + v) + t, factor column 16 nt + i
  float* o = out + by * split_stride;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = 16 * nt + i;
      if (col < k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = j0 + 4 * (4 * g + v) + t;
          if (j < n) o[j * k + col] = acc[t][nt][v];
        }
      }
    }
}

// Packs a float32 factor F (rows x k, leading dimension k) into transposed
// bfloat16 hi/mid/lo chunks: out[ch][part][c][kr] (row stride ldt) = split
// of F[ch * C + kr][c] for kr < C, c < KP (zero outside F).  A thread splits
// eight consecutive rows of one column and writes each term as one 16-byte
// run (C and ldt multiples of 8).
__global__ void k_pack_split_t(const float* __restrict__ F, int64_t rows, int k, int KP, int C,
                               int ldt, int64_t nchunks, unsigned short* __restrict__ out) {
  const int runs = C / 8;
  const int64_t count = nchunks * KP * runs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(e % runs);
    const int64_t rest = e / runs;
    const int c = (int)(rest % KP);
    const int64_t ch = rest / KP;
    const int64_t row0 = ch * C + 8 * q;
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t row = row0 + u;
      v[u] = (row < rows && c < k) ? F[row * k + c] : 0.f;
    }
    store_split_run8(v, out + ch * (int64_t)(3 * KP * ldt) + (int64_t)c * ldt + 8 * q,
                     (int64_t)KP * ldt);
  }
}

__global__ void k_reduce(const float* __restrict__ part, int splits, int64_t stride,
                         float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < stride;
       e += (int64_t)gridDim.x * blockDim.x) {
    float s = part[e];
    for (int q = 1; q < splits; ++q) s += part[q * stride + e];
    out[e] = s;
  }
}

int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g < 1) g = 1;
  return (int)(g < 8192 ? g : 8192);
}

int mfma_kp(int k) { return k <= 16 ? 16 : k <= 32 ? 32 : k <= 48 ? 48 : k <= 64 ? 64 : 80; }

bool aligned_rows(const void* X, int64_t ld, int esz) {
  return (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((ld * esz) % 16 == 0);
}

// Workgroups of `kernel` (256 threads) resident on the device at once.
int64_t resident_blocks(const void* kernel) {
  static std::mutex mu;
  static std::map<const void*, int64_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kT, 0) != hipSuccess) per = 1;
  (void)hipGetLastError();
  const int64_t v = (int64_t)(per > 0 ? per : 1) * (cus > 0 ? cus : 256);
  cache[kernel] = v;
  return v;
}

const void* xv_kernel(int xt, int KP) {
  if (xt == ENMF_F32) {
    switch (KP) {
      case 16: return reinterpret_cast<const void*>(&k_xv_f32s<16>);
      case 32: return reinterpret_cast<const void*>(&k_xv_f32s<32>);
      case 48: return reinterpret_cast<const void*>(&k_xv_f32s<48>);
      case 64: return reinterpret_cast<const void*>(&k_xv_f32s<64>);
      default: return reinterpret_cast<const void*>(&k_xv_f32s<80>);
    }
  }
  switch (KP) {
    case 16: return reinterpret_cast<const void*>(&k_xv_bf16<16>);
    case 32: return reinterpret_cast<const void*>(&k_xv_bf16<32>);
    case 48: return reinterpret_cast<const void*>(&k_xv_bf16<48>);
    case 64: return reinterpret_cast<const void*>(&k_xv_bf16<64>);
    default: return reinterpret_cast<const void*>(&k_xv_bf16<80>);
  }
}

const void* xtu_kernel(int xt, int KP) {
  if (xt == ENMF_F32) {
    switch (KP) {
      case 16: return reinterpret_cast<const void*>(&k_xtu_f32s<16, false>);
      case 32: return reinterpret_cast<const void*>(&k_xtu_f32s<32, false>);
      case 48: return reinterpret_cast<const void*>(&k_xtu_f32s<48, false>);
      case 64: return reinterpret_cast<const void*>(&k_xtu_f32s<64, false>);
      default: return reinterpret_cast<const void*>(&k_xtu_f32s<80, false>);
    }
  }
  switch (KP) {
    case 16: return reinterpret_cast<const void*>(&k_xtu_bf16<16, false>);
    case 32: return reinterpret_cast<const void*>(&k_xtu_bf16<32, false>);
    case 48: return reinterpret_cast<const void*>(&k_xtu_bf16<48, false>);
    case 64: return reinterpret_cast<const void*>(&k_xtu_bf16<64, false>);
    default: return reinterpret_cast<const void*>(&k_xtu_bf16<80, false>);
  }
}

// Grid plan of one product: `tiles` output blocks x `splits` contraction
// ranges of `cps` chunks each (nch chunks in all).
struct Plan {
  int64_t nch, tiles, cps, splits;
};

// Splits of the contraction, chosen by a model of the launch time in bytes
// moved at full bandwidth.  A full set of resident blocks is taken to keep
// HBM busy, so the streaming part is the larger of the X bytes and the
// rounds of resident blocks times the chunks of one block (plus one for its
// first load and write-out); every split adds its partial result, written
// here and read back by the consumer.  A larger count must win by 1%.
// chunk_bytes: X bytes one block reads per chunk; out_bytes: one partial.
Plan make_plan(int64_t nch, int64_t tiles, int64_t min_units, const void* kernel, int64_t smax_cap,
               double chunk_bytes, double out_bytes) {
  const int64_t capacity = resident_blocks(kernel);
  int64_t smax = (nch + min_units - 1) / min_units;
  if (smax > smax_cap) smax = smax_cap;
  if (smax < 1) smax = 1;
  const double xbytes = (double)nch * (double)tiles * chunk_bytes;
  Plan best{nch, tiles, nch, 1};
  double best_cost = -1.0;
  for (int64_t sp = 1; sp <= smax; ++sp) {
    const int64_t cps = (nch + sp - 1) / sp;
    const int64_t splits = (nch + cps - 1) / cps;
    const int64_t rounds = (tiles * splits + capacity - 1) / capacity;
    const double wave = (double)rounds * (double)(cps + 1) * (double)capacity * chunk_bytes;
    const double cost = (xbytes > wave ? xbytes : wave) +
                        (splits > 1 ? 2.0 * (double)splits : 1.0) * out_bytes;
    if (best_cost < 0.0 || cost < 0.99 * best_cost) {
      best_cost = cost;
      best = Plan{nch, tiles, cps, splits};
    }
  }
  return best;
}

// X B: tiles of 256 rows; f32 in 32-column chunks, bf16 in 64-column chunks.
Plan xv_plan(int xt, int64_t m, int64_t n, int k) {
  const int KP = mfma_kp(k);
  const double out = (double)m * k * 4;
  if (xt == ENMF_F32)
    return make_plan((n + 31) / 32, (m + 255) / 256, 4, xv_kernel(xt, KP), 64, 256.0 * 32 * 4, out);
  return make_plan((n + 63) / 64, (m + 255) / 256, 4, xv_kernel(xt, KP), 64, 256.0 * 64 * 2, out);
}

// X^T A: 32-row chunks; f32 tiles of 256 columns, bf16 tiles of 512 columns.
Plan xtu_plan(int xt, int64_t m, int64_t n, int k) {
  const int KP = mfma_kp(k);
  const double out = (double)n * k * 4;
  if (xt == ENMF_F32)
    return make_plan((m + 31) / 32, (n + 255) / 256, 4, xtu_kernel(xt, KP), 64, 32.0 * 256 * 4, out);
  return make_plan((m + 31) / 32, (n + 511) / 512, 4, xtu_kernel(xt, KP), 64, 32.0 * 512 * 2, out);
}

}  // namespace

void mfma_pack_layout(int xt, int xtu, int k, int* kp, int* c, int* ldt) {
  *kp = mfma_kp(k);
  if (xtu) { *c = 32; *ldt = kAtG; }
  else if (xt == ENMF_F32) { *c = 32; *ldt = kBt32Ld; }
  else { *c = 64; *ldt = kBtLd; }
}

bool mfma_eligible(int xt, int k) { return k >= 16 && k <= ENMF_MAX_WIDTH && (xt == ENMF_F32 || xt == ENMF_BF16); }

// Workspace (bytes) of the MFMA products: packed factor and split partials.
void mfma_xv_ws(int xt, int64_t m, int64_t n, int k, size_t* pack_bytes, size_t* part_bytes) {
  const int KP = mfma_kp(k);
  const Plan p = xv_plan(xt, m, n, k);
  *pack_bytes = xt == ENMF_F32 ? (size_t)p.nch * 3 * KP * kBt32Ld * 2 : (size_t)p.nch * 3 * KP * kBtLd * 2;
  *part_bytes = (size_t)p.splits * m * k * 4;
}

void mfma_xtu_ws(int xt, int64_t m, int64_t n, int k, size_t* pack_bytes, size_t* part_bytes) {
  const int KP = mfma_kp(k);
  const Plan p = xtu_plan(xt, m, n, k);
  *pack_bytes = (size_t)p.nch * 3 * KP * kAtG * 2;
  *part_bytes = (size_t)p.splits * n * k * 4;
}

// P = X B through the matrix cores.  pack and part are workspace of the
// sizes given by mfma_xv_ws.  reduce = 0 leaves the split partials unsummed
// and do_pack = 0 reuses the packed factor (instrumentation).
hipError_t launch_xv_mfma(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* B,
                          int k, void* pack, float* part, float* out, hipStream_t s, int reduce,
                          int do_pack, int* nsplit, const int32_t* stop,
                           hipEvent_t ev0, hipEvent_t ev1, const GramJob* gj) {
  const int KP = mfma_kp(k);
  const double* gsrc = gj ? gj->src : nullptr;
  const int gparts = gj ? gj->nparts : 0, gkp = gj ? gj->kp : 0;
  double* gdst = gj ? gj->dst : nullptr;
  const bool vec = aligned_rows(X, ld, xt == ENMF_F32 ? 4 : 2);
  int64_t eff = 1;
  if (xt == ENMF_F32) {
    const int64_t nch = (n + 31) / 32;
    const int64_t rb = (m + 255) / 256;
    if (do_pack)
      hipLaunchKernelGGL(k_pack_split_t, dim3(grid_for(nch * 4 * KP)), dim3(256), 0, s, B, n, k, KP, 32,
                         kBt32Ld, nch, (unsigned short*)pack);
    const Plan pl = xv_plan(xt, m, n, k);
    const int64_t cps = pl.cps;
    eff = pl.splits;
    float* dst = eff > 1 ? part : out;
    dim3 grid((unsigned)rb, (unsigned)eff);
    const float* Xf = reinterpret_cast<const float*>(X);
    const unsigned short* Bf = reinterpret_cast<const unsigned short*>(pack);
    if (ev0) (void)hipEventRecord(ev0, s);
    switch (KP) {
      case 16: hipLaunchKernelGGL((k_xv_f32s<16>), grid, dim3(kT), 0, s, Xf, m, n, ld, Bf, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 32: hipLaunchKernelGGL((k_xv_f32s<32>), grid, dim3(kT), 0, s, Xf, m, n, ld, Bf, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 48: hipLaunchKernelGGL((k_xv_f32s<48>), grid, dim3(kT), 0, s, Xf, m, n, ld, Bf, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 64: hipLaunchKernelGGL((k_xv_f32s<64>), grid, dim3(kT), 0, s, Xf, m, n, ld, Bf, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      default: hipLaunchKernelGGL((k_xv_f32s<80>), grid, dim3(kT), 0, s, Xf, m, n, ld, Bf, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
  } else {
    const int64_t nch = (n + 63) / 64;
    const int64_t rb = (m + 255) / 256;
    if (do_pack)
      hipLaunchKernelGGL(k_pack_split_t, dim3(grid_for(nch * 8 * KP)), dim3(256), 0, s, B, n, k, KP, 64,
                         kBtLd, nch, (unsigned short*)pack);
    const Plan pl = xv_plan(xt, m, n, k);
    const int64_t cps = pl.cps;
    eff = pl.splits;
    float* dst = eff > 1 ? part : out;
    dim3 grid((unsigned)rb, (unsigned)eff);
    const unsigned short* Xb = reinterpret_cast<const unsigned short*>(X);
    const unsigned short* Bt = reinterpret_cast<const unsigned short*>(pack);
    if (ev0) (void)hipEventRecord(ev0, s);
    switch (KP) {
      case 16: hipLaunchKernelGGL((k_xv_bf16<16>), grid, dim3(kT), 0, s, Xb, m, n, ld, Bt, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 32: hipLaunchKernelGGL((k_xv_bf16<32>), grid, dim3(kT), 0, s, Xb, m, n, ld, Bt, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 48: hipLaunchKernelGGL((k_xv_bf16<48>), grid, dim3(kT), 0, s, Xb, m, n, ld, Bt, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      case 64: hipLaunchKernelGGL((k_xv_bf16<64>), grid, dim3(kT), 0, s, Xb, m, n, ld, Bt, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
      default: hipLaunchKernelGGL((k_xv_bf16<80>), grid, dim3(kT), 0, s, Xb, m, n, ld, Bt, k, (int)cps, nch, (int)vec, dst, m * k, stop, gsrc, gparts, gkp, gdst); break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
  }
  hipError_t e = hipGetLastError();
  if (nsplit) *nsplit = (e == hipSuccess && !reduce) ? (int)eff : 1;
  if (e != hipSuccess || eff <= 1 || !reduce) return e;
  hipLaunchKernelGGL(k_reduce, dim3(grid_for(m * k)), dim3(256), 0, s, part, (int)eff, m * k, out);
  return hipGetLastError();
}

// Q = X^T A through the matrix cores (workspace from mfma_xtu_ws).
hipError_t launch_xtu_mfma(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* A,
                           int k, void* pack, float* part, float* out, hipStream_t s, int reduce,
                           int do_pack, int* nsplit, const int32_t* stop,
                           hipEvent_t ev0, hipEvent_t ev1, const GramJob* gj,
                           const DecideArgs* dec, DevState* st) {
  const int KP = mfma_kp(k);
  const DecideArgs da = dec ? *dec : DecideArgs();
  DevState* dst_state = dec ? st : nullptr;
  const double* gsrc = gj ? gj->src : nullptr;
  const int gparts = gj ? gj->nparts : 0, gkp = gj ? gj->kp : 0;
  double* gdst = gj ? gj->dst : nullptr;
  // 16-byte loads of X marked non-temporal only where X is far larger than
  // the last-level cache (where X fits it, the hint would evict the X that
  // the next product reads from there)
  const int64_t xbytes = m * n * (xt == ENMF_F32 ? 4 : 2);
  const int vec = aligned_rows(X, ld, xt == ENMF_F32 ? 4 : 2) ? 1 : 0;
  const bool ntl = xbytes >= kNtMinBytes;
  int64_t eff = 1;
  if (xt == ENMF_F32) {
    const int64_t nch = (m + 31) / 32;
    const int64_t tiles = (n + 255) / 256;
    if (do_pack)
      hipLaunchKernelGGL(k_pack_split_t, dim3(grid_for(nch * 4 * KP)), dim3(256), 0, s, A, m, k, KP, 32,
                         kAtG, nch, (unsigned short*)pack);
    const Plan pl = xtu_plan(xt, m, n, k);
    const int cps = (int)pl.cps;
    eff = pl.splits;
    float* dst = eff > 1 ? part : out;
    dim3 grid((unsigned)tiles, (unsigned)eff);
    const float* Xf = reinterpret_cast<const float*>(X);
    const unsigned short* At = reinterpret_cast<const unsigned short*>(pack);
    if (ev0) (void)hipEventRecord(ev0, s);
    switch (KP) {
      case 16: if (ntl) hipLaunchKernelGGL((k_xtu_f32s<16, true>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_f32s<16, false>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 32: if (ntl) hipLaunchKernelGGL((k_xtu_f32s<32, true>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_f32s<32, false>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 48: if (ntl) hipLaunchKernelGGL((k_xtu_f32s<48, true>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_f32s<48, false>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 64: if (ntl) hipLaunchKernelGGL((k_xtu_f32s<64, true>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_f32s<64, false>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      default: if (ntl) hipLaunchKernelGGL((k_xtu_f32s<80, true>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_f32s<80, false>), grid, dim3(kT), 0, s, Xf, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
  } else {
    const int64_t tiles = (n + 511) / 512;
    const int64_t nch = (m + 31) / 32;
    if (do_pack)
      hipLaunchKernelGGL(k_pack_split_t, dim3(grid_for(nch * 4 * KP)), dim3(256), 0, s, A, m, k, KP, 32,
                         kAtG, nch, (unsigned short*)pack);
    const Plan pl = xtu_plan(xt, m, n, k);
    const int64_t cps = pl.cps;
    eff = pl.splits;
    float* dst = eff > 1 ? part : out;
    // side jobs, if any, in one more grid row (xtu_side_row)
    const unsigned side = (gsrc != nullptr || dst_state != nullptr) ? 1u : 0u;
    dim3 grid((unsigned)tiles, (unsigned)eff + side);
    const unsigned short* Xb = reinterpret_cast<const unsigned short*>(X);
    const unsigned short* At = reinterpret_cast<const unsigned short*>(pack);
    if (ev0) (void)hipEventRecord(ev0, s);
    switch (KP) {
      case 16: if (ntl) hipLaunchKernelGGL((k_xtu_bf16<16, true>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_bf16<16, false>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 32: if (ntl) hipLaunchKernelGGL((k_xtu_bf16<32, true>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_bf16<32, false>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 48: if (ntl) hipLaunchKernelGGL((k_xtu_bf16<48, true>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_bf16<48, false>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      case 64: if (ntl) hipLaunchKernelGGL((k_xtu_bf16<64, true>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_bf16<64, false>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
      default: if (ntl) hipLaunchKernelGGL((k_xtu_bf16<80, true>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        else hipLaunchKernelGGL((k_xtu_bf16<80, false>), grid, dim3(kT), 0, s, Xb, m, n, ld, At, k, cps, nch, (int)vec, dst, n * k, stop, gsrc, gparts, gkp, gdst, da, dst_state);
        break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
  }
  hipError_t e = hipGetLastError();
  if (nsplit) *nsplit = (e == hipSuccess && !reduce) ? (int)eff : 1;
  if (e != hipSuccess || eff <= 1 || !reduce) return e;
  hipLaunchKernelGGL(k_reduce, dim3(grid_for(n * k)), dim3(256), 0, s, part, (int)eff, n * k, out);
  return hipGetLastError();
}

}  // namespace enmf
