// Sparse X (the sparse text collections of the experiments): the products
// X B and X^T A of the method on compressed rows, the squared norm of X and
// the cross term of the expanded objective.
//
// Product layout: the nonzeros of one orientation (CSR of X for X B, CSR of
// X^T for X^T A) are cut into work items of at most kSpChunk nonzeros, never
// spanning two rows or two panels of kSpPanel columns, and stored panel by
// panel (SparseForm): the blocks in flight then gather from one panel's rows
// of B, which stay in the last-level cache while X streams past.  A group of G lanes takes one item: the
// group loads G (index, value) pairs at a time with one coalesced load, hands
// them out lane to lane, and every lane gathers its column(s) c, c + G of the
// referenced rows of B, eight rows in flight.  Each output entry is a float32
// fused multiply-add chain over the item's nonzeros in storage order; the
// partial rows of a long row are then summed in slot order, so the result
// does not depend on scheduling.
#include "dev_common.h"
#include "enmf_internal.h"

namespace enmf {

namespace {

constexpr int kSt = 256;
constexpr int kUnroll = 8;

struct SpmmArgs {
  const int64_t* item_p0;
  const int64_t* item_p1;
  const int32_t* item_row;
  const int32_t* item_slot;
  const int32_t* idx;
  const float* val;
  int64_t nitems;
  const float* B;
  int k;
  float* part;
  float* out;
};

// Value of x in lane `src` of the caller's group of G lanes (src < G and the
// same in every lane of the group).
template <int G>
__device__ __forceinline__ int bcast(int x, int src) {
  if constexpr (G == kWave) return __builtin_amdgcn_readlane(x, src);
  else return __shfl(x, src, G);
}

template <int G>
__device__ __forceinline__ float bcast(float x, int src) {
  return __int_as_float(bcast<G>(__float_as_int(x), src));
}

template <int G, int KC>
__global__ __launch_bounds__(kSt) void k_spmm(SpmmArgs a) {
  constexpr int NG = kSt / G;
  static_assert(G % kUnroll == 0, "a group hands out whole runs of kUnroll nonzeros");
  const int lane = threadIdx.x % G;
  const int64_t it = (int64_t)blockIdx.x * NG + threadIdx.x / G;
  if (it >= a.nitems) return;
  const int64_t p0 = a.item_p0[it], p1 = a.item_p1[it];
  const int k = a.k;
  float acc[KC];
#pragma unroll
  for (int q = 0; q < KC; ++q) acc[q] = 0.f;
  for (int64_t base = p0; base < p1; base += G) {
    const int cnt = (int)(p1 - base < G ? p1 - base : G);
    // lanes past the end hold row 0 and a zero value; their products are skipped
    int mj = 0;
    float mv = 0.f;
    if (lane < cnt) {
      mj = a.idx[base + lane];
      mv = a.val[base + lane];
    }
    for (int t = 0; t < cnt; t += kUnroll) {
      int j[kUnroll];
      float v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        j[u] = bcast<G>(mj, t + u);
        v[u] = bcast<G>(mv, t + u);
      }
      float b[kUnroll][KC];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const float* Br = a.B + (int64_t)j[u] * k;
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          const int col = lane + q * G;
          b[u][q] = col < k ? Br[col] : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (t + u < cnt) {
#pragma unroll
          for (int q = 0; q < KC; ++q) acc[q] = fmaf(v[u], b[u][q], acc[q]);
        }
      }
    }
  }
  const int slot = a.item_slot[it];
  float* o = slot < 0 ? a.out + (int64_t)a.item_row[it] * k : a.part + (int64_t)slot * k;
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const int col = lane + q * G;
    if (col < k) o[col] = acc[q];
  }
}

// Rows cut into several items: out row = sum of its partial rows in slot order.
__global__ __launch_bounds__(kSt) void k_spmm_combine(const int32_t* __restrict__ split_row,
                                                      const int32_t* __restrict__ split_s0,
                                                      int64_t nsplit, const float* __restrict__ part,
                                                      int k, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kSt + threadIdx.x;
  const int64_t q = e / k;
  const int col = (int)(e % k);
  if (q >= nsplit) return;
  float s = 0.f;
  for (int32_t t = split_s0[q]; t < split_s0[q + 1]; ++t) s += part[(int64_t)t * k + col];
  out[(int64_t)split_row[q] * k + col] = s;
}

__global__ __launch_bounds__(kSt) void k_sp_sumsq(const float* __restrict__ v, int64_t nnz,
                                                  double* __restrict__ part) {
  __shared__ double sh[kSt / kWave];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kSt + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kSt)
    s = fma((double)v[e], (double)v[e], s);
  s = block_sum<kSt>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sum over the nonzeros of x_ij (x_ij - 2 u_i . v_j) = sum x^2 - 2 <U, X V>,
// with X V accumulated in float64: one wave per item (grid-stride over
// items), lane c holding column c of the item's partial row of X V, as in
// k_spmm; the lanes then take its dot product with u_i.  r <= 64.
__global__ __launch_bounds__(kSt) void k_sp_cross(const int64_t* __restrict__ item_p0,
                                                  const int64_t* __restrict__ item_p1,
                                                  const int32_t* __restrict__ item_row,
                                                  int64_t nitems, const int32_t* __restrict__ idx,
                                                  const float* __restrict__ val,
                                                  const float* __restrict__ U,
                                                  const float* __restrict__ V, int r,
                                                  double* __restrict__ part) {
  __shared__ double sh[kSt / kWave];
  const int lane = threadIdx.x % kWave;
  const int64_t nw = (int64_t)gridDim.x * (kSt / kWave);
  double sx2 = 0.0, s = 0.0;
  for (int64_t it = (int64_t)blockIdx.x * (kSt / kWave) + threadIdx.x / kWave; it < nitems;
       it += nw) {
    const int64_t p0 = item_p0[it], p1 = item_p1[it];
    const double u = lane < r ? (double)U[(int64_t)item_row[it] * r + lane] : 0.0;
    double acc = 0.0;
    for (int64_t base = p0; base < p1; base += kWave) {
      const int cnt = (int)(p1 - base < kWave ? p1 - base : kWave);
      int mj = 0;
      float mv = 0.f;
      if (lane < cnt) {
        mj = idx[base + lane];
        mv = val[base + lane];
      }
      sx2 = fma((double)mv, (double)mv, sx2);
      for (int t = 0; t < cnt; t += kUnroll) {
        float b[kUnroll], v[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          const int j = bcast<kWave>(mj, t + q);
          v[q] = bcast<kWave>(mv, t + q);
          b[q] = lane < r ? V[(int64_t)j * r + lane] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q)
          if (t + q < cnt) acc = fma((double)v[q], (double)b[q], acc);
      }
    }
    s = fma(u, acc, s);
  }
  const double tot = block_sum<kSt>(sx2 - 2.0 * s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kSt) void k_sp_objective(const double* __restrict__ part, int nparts,
                                                      const double* __restrict__ GU,
                                                      const double* __restrict__ GV, int r,
                                                      double* __restrict__ out) {
  __shared__ double sh[kSt / kWave];
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kSt) s += part[b];
  for (int e = threadIdx.x; e < r * r; e += kSt) s = fma(GU[e], GV[e], s);
  s = block_sum<kSt>(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

int reduce_blocks(int64_t work, int64_t per_block, int64_t cap) {
  const int64_t b = (work + per_block - 1) / per_block;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <int G, int KC>
hipError_t spmm_launch(const SpmmArgs& a, hipStream_t s) {
  constexpr int NG = kSt / G;
  const int64_t blocks = (a.nitems + NG - 1) / NG;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (blocks > 0) hipLaunchKernelGGL((k_spmm<G, KC>), dim3((unsigned)blocks), dim3(kSt), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_spmm(const SparseForm& f, const float* B, int k, float* part, float* out,
                       hipStream_t s) {
  if (k < 1 || k > 2 * kWave) return hipErrorInvalidValue;
  SpmmArgs a{f.item_p0, f.item_p1, f.item_row, f.item_slot, f.idx, f.val, f.nitems, B, k, part, out};
  hipError_t e;
  if (k <= 16) e = spmm_launch<16, 1>(a, s);
  else if (k <= 32) e = spmm_launch<32, 1>(a, s);
  else if (k <= 64) e = spmm_launch<64, 1>(a, s);
  else e = spmm_launch<64, 2>(a, s);
  if (e != hipSuccess || f.nsplit == 0) return e;
  const int64_t work = f.nsplit * k;
  hipLaunchKernelGGL(k_spmm_combine, dim3((unsigned)((work + kSt - 1) / kSt)), dim3(kSt), 0, s,
                     f.split_row, f.split_s0, f.nsplit, part, k, out);
  return hipGetLastError();
}

int launch_sparse_sumsq(const SparseForm& f, double* part, hipStream_t s) {
  const int nb = reduce_blocks(f.nnz, 4 * kSt, 1024);
  hipLaunchKernelGGL(k_sp_sumsq, dim3(nb), dim3(kSt), 0, s, f.val, f.nnz, part);
  return hipGetLastError() == hipSuccess ? nb : -1;
}

int launch_sparse_cross(const SparseForm& f, const float* U, const float* V, int r, double* part,
                        hipStream_t s) {
  const int nb = reduce_blocks(f.nitems, kSt / kWave, kSpCrossBlocks);
  hipLaunchKernelGGL(k_sp_cross, dim3(nb), dim3(kSt), 0, s, f.item_p0, f.item_p1, f.item_row,
                     f.nitems, f.idx, f.val, U, V, r, part);
  return hipGetLastError() == hipSuccess ? nb : -1;
}

hipError_t launch_sparse_objective(const double* part, int nparts, const double* GU,
                                   const double* GV, int r, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sp_objective, dim3(1), dim3(kSt), 0, s, part, nparts, GU, GV, r, out);
  return hipGetLastError();
}

}  // namespace enmf
