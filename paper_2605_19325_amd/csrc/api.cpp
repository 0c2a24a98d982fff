// Host side of libenmf: argument validation, context-owned device workspace
// and the launch sequences of the entry points declared in include/enmf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "enmf_internal.h"

using namespace enmf;

namespace {

enum Slot {
  S_BP, S_AP, S_SPLIT, S_P, S_Q, S_GPART, S_G, S_H, S_RUPART, S_XPART, S_U2, S_GPU, S_GPV, S_STAT, S_UD, S_RES,
  S_Y, S_QM64, S_QM32, S_Z, S_QN64, S_QN32, S_TMP64, S_T, S_C, S_COLP, S_COLS, S_SIG, S_TU, S_TV,
  S_W64, S_ADMM, S_R, S_WSQ, S_MPART,
  S_EX, S_ERU, S_ERV, S_EE, S_ERSS, S_ECU, S_ECV, S_EG, S_EGI, S_EST, S_ESTAT, S_SPX, S_SPG,
  S_GW, S_GOUT, S_XT, N_SLOTS
};

constexpr int kTimingPairs = 64;   // sampled launches per kind and iterate call

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct enmf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  Buf bufs[N_SLOTS];
  DevState* st = nullptr;
  double ns_per_tick = 10.0;
  bool use_mfma = true;   // ENMF_FORCE_VALU=1 at creation selects the vector-ALU products
  // X B of enmf_iterate through X^T A on a transposed copy of X when X holds at
  // least this many bytes (ENMF_XT_MIN_BYTES at creation; default 512 MiB)
  int64_t xt_min_bytes = int64_t(512) << 20;
  // in-solve sampling of the streaming kernels (enmf_kernel_timing)
  int timing_period = 0;
  std::vector<hipEvent_t> events;       // pool: [kind][pair][2]
  int pending[2] = {0, 0};              // pairs recorded in the current iterate call
  int pending_k[2][kTimingPairs] = {};            // outer iteration of each recorded pair
  double timing_sum[2] = {0.0, 0.0};
  int timing_n[2] = {0, 0};
  // the iterate loop's look at the device stop flag (pinned copy and its event)
  int32_t* stop_host = nullptr;
  hipEvent_t stop_ev = nullptr;
  // private stream on which the iterate loop body is captured into a graph
  hipStream_t cap_stream = nullptr;
};


int enmf::ctx_device(const enmf_ctx* c) { return c->device; }
hipStream_t enmf::ctx_stream(const enmf_ctx* c) { return c->stream; }
void enmf::ctx_set_error(enmf_ctx* c, const char* msg) { c->err = msg; }

namespace {

enmf_status fail(enmf_ctx* c, enmf_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

void* ws(enmf_ctx* c, int slot, size_t bytes) {
  Buf& b = c->bufs[slot];
  if (bytes < 256) bytes = 256;
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  const size_t want = bytes + bytes / 8;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.p;
}

#define CK(expr)                                                                          \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(c, ENMF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define WS(var, type, slot, bytes)                                                          \
  type* var = reinterpret_cast<type*>(ws(c, slot, (size_t)(bytes)));                       \
  if (!var) return fail(c, ENMF_ENOMEM, "device workspace allocation failed (" #var ")")

#define TRY(expr)                          \
  do {                                     \
    enmf_status s_ = (expr);               \
    if (s_ != ENMF_OK) return s_;          \
  } while (0)

int64_t esize(int dtype) { return dtype == ENMF_F32 ? 4 : 2; }

enmf_status check_ctx(enmf_ctx* c) {
  if (!c) return ENMF_EINVAL;
  c->err.clear();
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, ENMF_EDEVICE, "hipSetDevice failed");
  return ENMF_OK;
}

enmf_status check_matrix(enmf_ctx* c, const enmf_matrix* X) {
  if (!X || !X->data) return fail(c, ENMF_EINVAL, "X is null");
  if (X->m < 1 || X->n < 1) return fail(c, ENMF_EINVAL, "X must have m >= 1 and n >= 1");
  if (const SparseX* sp = sparse_of(X)) {
    if (sp->magic != kSparseMagic) return fail(c, ENMF_EINVAL, "X is not a sparse X handle");
    if (sp->device != c->device) return fail(c, ENMF_EINVAL, "sparse X lives on another device");
    if (sp->csr.rows != X->m || sp->csr.cols != X->n)
      return fail(c, ENMF_EINVAL, "X shape differs from the sparse X handle's");
    return ENMF_OK;
  }
  if (X->ld < X->n) return fail(c, ENMF_EINVAL, "X leading dimension must be >= n");
  if (X->dtype != ENMF_F32 && X->dtype != ENMF_BF16 && X->dtype != ENMF_F16)
    return fail(c, ENMF_EINVAL, "unsupported X dtype");
  if (reinterpret_cast<uintptr_t>(X->data) % esize(X->dtype) != 0)
    return fail(c, ENMF_EINVAL, "X data must be aligned to its element size");
  return ENMF_OK;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

bool use_mfma(const enmf_ctx* c, const enmf_matrix* X, int k) {
  return c->use_mfma && X->dtype != ENMF_CSR && mfma_eligible(X->dtype, k);
}

// A transposed copy of a dense X (n x m, leading dimension ld) that X B runs on.
struct XTCopy {
  const void* data = nullptr;
  int64_t ld = 0;
};

// X B through X^T A on a transposed copy: dense X on the matrix cores whose
// storage exceeds the last-level cache by far (xt_min_bytes).  The X^T A
// kernel reads X in whole row runs and streams it closer to the HBM roof
// than X B's operand-layout loads.
bool use_xt(const enmf_ctx* c, const enmf_matrix* X, int k) {
  if (!use_mfma(c, X, k) || c->xt_min_bytes <= 0) return false;
  const int64_t esz = X->dtype == ENMF_F32 ? 4 : 2;
  return X->m * X->n * esz >= c->xt_min_bytes;
}

// Split-partial bytes needed by either form of the products at width k.
size_t split_bytes(const enmf_ctx* c, const enmf_matrix* X, int k) {
  if (const SparseX* sp = sparse_of(X)) {
    const int64_t ns = sp->csr.nslots > sp->csc.nslots ? sp->csr.nslots : sp->csc.nslots;
    return (size_t)ns * k * 4;
  }
  size_t a = 0, b = 0, pa = 0, pb = 0;
  if (use_mfma(c, X, k)) {
    mfma_xv_ws(X->dtype, X->m, X->n, k, &pa, &a);
    mfma_xtu_ws(X->dtype, X->m, X->n, k, &pb, &b);
  } else {
    a = (size_t)xv_splits(X->m, X->n, X->dtype) * X->m * k * 4;
    b = (size_t)xtu_splits(X->m, X->n) * X->n * k * 4;
  }
  return a > b ? a : b;
}

// out = F B for one orientation of a sparse X.
enmf_status do_spmm(enmf_ctx* c, const enmf_matrix* X, const SparseForm& f, const float* B, int k,
                    float* out) {
  WS(part, float, S_SPLIT, split_bytes(c, X, k));
  CK(launch_spmm(f, B, k, part, out, c->stream));
  return ENMF_OK;
}

// P = X B (B: n x k, ld k).
enmf_status do_xv(enmf_ctx* c, const enmf_matrix* X, const float* B, int k, float* P) {
  if (const SparseX* sp = sparse_of(X)) return do_spmm(c, X, sp->csr, B, k, P);
  if (use_mfma(c, X, k)) {
    size_t pb = 0, sb = 0;
    mfma_xv_ws(X->dtype, X->m, X->n, k, &pb, &sb);
    WS(pack, void, S_BP, pb);
    WS(part, float, S_SPLIT, sb);
    CK(launch_xv_mfma(X->data, X->dtype, X->m, X->n, X->ld, B, k, pack, part, P, c->stream, 1, 1));
    return ENMF_OK;
  }
  const int kp = pad_width(k);
  const int64_t rows_pad = round_up(X->n, xv_tile_width(X->dtype));
  WS(Bp, float, S_BP, rows_pad * kp * 4);
  CK(launch_pad_rows_cols(B, X->n, k, kp, rows_pad, Bp, c->stream));
  const int splits = xv_splits(X->m, X->n, X->dtype);
  float* part = nullptr;
  if (splits > 1) {
    WS(pp, float, S_SPLIT, (int64_t)splits * X->m * k * 4);
    part = pp;
  }
  CK(launch_xv(X->data, X->dtype, X->m, X->n, X->ld, Bp, k, kp, splits, part, P, c->stream));
  return ENMF_OK;
}

// Q = X^T A (A: m x k, ld k).
enmf_status do_xtu(enmf_ctx* c, const enmf_matrix* X, const float* A, int k, float* Q) {
  if (const SparseX* sp = sparse_of(X)) return do_spmm(c, X, sp->csc, A, k, Q);
  if (use_mfma(c, X, k)) {
    size_t pb = 0, sb = 0;
    mfma_xtu_ws(X->dtype, X->m, X->n, k, &pb, &sb);
    WS(pack, void, S_AP, pb);
    WS(part, float, S_SPLIT, sb);
    CK(launch_xtu_mfma(X->data, X->dtype, X->m, X->n, X->ld, A, k, pack, part, Q, c->stream, 1, 1));
    return ENMF_OK;
  }
  const int kp = pad_width(k);
  WS(Ap, float, S_AP, X->m * kp * 4);
  CK(launch_pad_cols(A, X->m, k, kp, Ap, c->stream));
  const int splits = xtu_splits(X->m, X->n);
  float* part = nullptr;
  if (splits > 1) {
    WS(pp, float, S_SPLIT, (int64_t)splits * X->n * k * 4);
    part = pp;
  }
  CK(launch_xtu(X->data, X->dtype, X->m, X->n, X->ld, Ap, k, kp, splits, part, Q, c->stream));
  return ENMF_OK;
}

// A product left as split partials: value = sum over s < n of p[s * stride + e].
struct Parts {
  const float* p = nullptr;
  int n = 1;
  int64_t stride = 0;
};

// P = X B as partials (B: n x k, ld k); P_out receives the product when it
// is not split.
// packed = true: the matrix-core form takes B already packed in its slot
// (written by the row pass that produced B).
// gj: a Gram combine to run as well (inside the matrix-core product, else
// as a launch of its own after it).
enmf_status xv_parts(enmf_ctx* c, const enmf_matrix* X, const float* B, int k, float* P_out,
                     Parts* out, hipEvent_t* ev = nullptr, bool packed = false,
                     const GramJob* gj = nullptr, const XTCopy* xt = nullptr,
                     const float* prepadded = nullptr) {
  hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
  int ns = 1;
  if (xt != nullptr && xt->data != nullptr) {
    // P = X B = (X^T)^T B: the X^T A kernel on the transposed copy (n x m)
    size_t pb = 0, sb = 0;
    mfma_xtu_ws(X->dtype, X->n, X->m, k, &pb, &sb);
    WS(pack, void, S_BP, pb);
    WS(part, float, S_SPLIT, sb);
    CK(launch_xtu_mfma(xt->data, X->dtype, X->n, X->m, xt->ld, B, k, pack, part, P_out, c->stream, 0,
                       packed ? 0 : 1, &ns, &c->st->stop, e0, e1, gj, nullptr, nullptr));
    out->p = ns > 1 ? part : P_out;
  } else if (const SparseX* sp = sparse_of(X)) {
    if (e0) CK(hipEventRecord(e0, c->stream));
    TRY(do_spmm(c, X, sp->csr, B, k, P_out));
    if (e1) CK(hipEventRecord(e1, c->stream));
    out->p = P_out;
    if (gj) CK(launch_gram_fin(gj->src, gj->nparts, gj->kp, gj->dst, c->stream));
  } else if (use_mfma(c, X, k)) {
    size_t pb = 0, sb = 0;
    mfma_xv_ws(X->dtype, X->m, X->n, k, &pb, &sb);
    WS(pack, void, S_BP, pb);
    WS(part, float, S_SPLIT, sb);
    CK(launch_xv_mfma(X->data, X->dtype, X->m, X->n, X->ld, B, k, pack, part, P_out, c->stream, 0,
                      packed ? 0 : 1, &ns, &c->st->stop, e0, e1, gj));
    out->p = ns > 1 ? part : P_out;
  } else {
    const int kp = pad_width(k);
    const float* Bp = prepadded;
    if (Bp == nullptr) {
      const int64_t rows_pad = round_up(X->n, xv_tile_width(X->dtype));
      WS(Bw, float, S_BP, rows_pad * kp * 4);
      CK(launch_pad_rows_cols(B, X->n, k, kp, rows_pad, Bw, c->stream));
      Bp = Bw;
    }
    const int splits = xv_splits(X->m, X->n, X->dtype);
    WS(part, float, S_SPLIT, (int64_t)splits * X->m * k * 4);
    if (e0) CK(hipEventRecord(e0, c->stream));
    CK(launch_xv(X->data, X->dtype, X->m, X->n, X->ld, Bp, k, kp, splits, part, P_out, c->stream, 0,
                 &ns, gj));
    if (e1) CK(hipEventRecord(e1, c->stream));
    out->p = ns > 1 ? part : P_out;
  }
  out->n = ns;
  out->stride = X->m * k;
  return ENMF_OK;
}

// Q = X^T A as partials (A: m x k, ld k).
// dec: the check and stop decision of the iteration, taken inside the
// matrix-core product (see launch_xtu_mfma); ignored by the other forms.
enmf_status xtu_parts(enmf_ctx* c, const enmf_matrix* X, const float* A, int k, float* Q_out,
                      Parts* out, hipEvent_t* ev = nullptr, bool packed = false,
                      const GramJob* gj = nullptr, const DecideArgs* dec = nullptr,
                      const float* prepadded = nullptr) {
  hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
  int ns = 1;
  if (const SparseX* sp = sparse_of(X)) {
    if (e0) CK(hipEventRecord(e0, c->stream));
    TRY(do_spmm(c, X, sp->csc, A, k, Q_out));
    if (e1) CK(hipEventRecord(e1, c->stream));
    out->p = Q_out;
    if (gj) CK(launch_gram_fin(gj->src, gj->nparts, gj->kp, gj->dst, c->stream));
  } else if (use_mfma(c, X, k)) {
    size_t pb = 0, sb = 0;
    mfma_xtu_ws(X->dtype, X->m, X->n, k, &pb, &sb);
    WS(pack, void, S_AP, pb);
    WS(part, float, S_SPLIT, sb);
    CK(launch_xtu_mfma(X->data, X->dtype, X->m, X->n, X->ld, A, k, pack, part, Q_out, c->stream, 0,
                       packed ? 0 : 1, &ns, &c->st->stop, e0, e1, gj, dec, c->st));
    out->p = ns > 1 ? part : Q_out;
  } else {
    const int kp = pad_width(k);
    const float* Ap = prepadded;
    if (Ap == nullptr) {
      WS(Aw, float, S_AP, X->m * kp * 4);
      CK(launch_pad_cols(A, X->m, k, kp, Aw, c->stream));
      Ap = Aw;
    }
    const int splits = xtu_splits(X->m, X->n);
    WS(part, float, S_SPLIT, (int64_t)splits * X->n * k * 4);
    if (e0) CK(hipEventRecord(e0, c->stream));
    CK(launch_xtu(X->data, X->dtype, X->m, X->n, X->ld, Ap, k, kp, splits, part, Q_out, c->stream, 0,
                  &ns, gj));
    if (e1) CK(hipEventRecord(e1, c->stream));
    out->p = ns > 1 ? part : Q_out;
  }
  out->n = ns;
  out->stride = X->n * k;
  return ENMF_OK;
}

// out (kp x kp, zero padded) = A^T A for A (rows x k float32 or float64, ld lda).
enmf_status do_gram(enmf_ctx* c, const void* A, int a_f64, int64_t lda, int64_t rows, int k, int kp,
                    double* out) {
  const int nb = gram_blocks(rows);
  WS(part, double, S_GPART, (int64_t)nb * k * k * 8);
  CK(launch_tsgram(A, a_f64, lda, A, a_f64, lda, rows, k, k, part, 0, nb, c->stream));
  CK(launch_gram_finalize(part, nb, k, k, kp, out, c->stream));
  return ENMF_OK;
}

// Orthonormal basis of the columns of A32 (N x k float32), written to out64
// and out32 (N x k).  Passes of Q = A E diag(lambda^-1/2) with the eigenpairs
// of A^T A; directions with lambda <= tau lambda_max become zero columns.  One
// pass leaves an orthogonality error of order eps cond(A)^2, enough for the
// intermediate bases of the power iterations (only their span matters); the
// second pass brings it to eps.
enmf_status do_orth(enmf_ctx* c, const float* A32, int64_t N, int k, double* out64, float* out32,
                    int passes = 2) {
  const double tau = 1e-15;
  WS(G, double, S_C, k * k * 8);
  WS(T, double, S_T, k * k * 8);
  TRY(do_gram(c, A32, 0, k, N, k, k, G));
  CK(launch_orth_factor(G, k, tau, T, c->stream));
  if (passes < 2) {
    CK(launch_apply_small(A32, 0, k, N, k, T, k, k, out64, 1, k, c->stream));
    CK(launch_apply_small(A32, 0, k, N, k, T, k, k, out32, 0, k, c->stream));
    return ENMF_OK;
  }
  WS(tmp, double, S_TMP64, N * k * 8);
  CK(launch_apply_small(A32, 0, k, N, k, T, k, k, tmp, 1, k, c->stream));
  TRY(do_gram(c, tmp, 1, k, N, k, k, G));
  CK(launch_orth_factor(G, k, tau, T, c->stream));
  CK(launch_apply_small(tmp, 1, k, N, k, T, k, k, out64, 1, k, c->stream));
  CK(launch_apply_small(tmp, 1, k, N, k, T, k, k, out32, 0, k, c->stream));
  return ENMF_OK;
}

// Sparse X: f = 1/2 (sum over the nonzeros of x (x - 2 u_i . v_j) + <U^T U, V^T V>)
// in float64, synchronising.
enmf_status sparse_objective(enmf_ctx* c, const SparseX* sp, int r, const float* U, const float* V,
                             double* f) {
  hipStream_t s = c->stream;
  WS(part, double, S_SPX, (int64_t)kSpCrossBlocks * 8);
  WS(g, double, S_SPG, 2 * r * r * 8);
  WS(o, double, S_SIG, 64 * 8);
  TRY(do_gram(c, U, 0, r, sp->csr.rows, r, r, g));
  TRY(do_gram(c, V, 0, r, sp->csr.cols, r, r, g + r * r));
  const int np = launch_sparse_cross(sp->csr, U, V, r, part, s);
  if (np < 0) return fail(c, ENMF_EDEVICE, "sparse cross-term launch failed");
  CK(launch_sparse_objective(part, np, g, g + r * r, r, o, s));
  double v = 0.0;
  CK(hipMemcpyAsync(&v, o, 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  *f = 0.5 * v;
  return ENMF_OK;
}

// Direct residual f = 1/2 ||X - U V^T||^2 (float64), synchronising.
enmf_status direct_objective(enmf_ctx* c, const enmf_matrix* X, int r, const float* U,
                             const float* V, double* f) {
  if (const SparseX* sp = sparse_of(X)) return sparse_objective(c, sp, r, U, V, f);
  hipStream_t s = c->stream;
  const int kp = pad_width(r);
  WS(Ud, double, S_UD, X->m * kp * 8);
  CK(launch_pad_cols_f64(U, X->m, r, kp, Ud, s));
  const int64_t cb = (X->n + 255) / 256;
  WS(res, double, S_RES, (cb * 2048 + 4096) * 8);
  WS(o, double, S_SIG, 64 * 8);
  int np = 0;
  CK(launch_residual(X->data, X->dtype, X->m, X->n, X->ld, Ud, V, r, res, &np, s));
  CK(launch_sum_parts(res, np, 1, 1, o, s));
  double v = 0.0;
  CK(hipMemcpyAsync(&v, o, 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  *f = 0.5 * v;
  return ENMF_OK;
}

// Partials of ||X||^2 (at most 1024) into xp; *nx receives their count.
enmf_status sumsq_parts(enmf_ctx* c, const enmf_matrix* X, double* xp, int* nx) {
  if (const SparseX* sp = sparse_of(X)) {
    *nx = launch_sparse_sumsq(sp->csr, xp, c->stream);
    if (*nx < 0) return fail(c, ENMF_EDEVICE, "sparse sum-of-squares launch failed");
    return ENMF_OK;
  }
  CK(launch_sumsq_x(X->data, X->dtype, X->m, X->n, X->ld, xp, nx, c->stream));
  return ENMF_OK;
}

enmf_status read_sumsq_x(enmf_ctx* c, const enmf_matrix* X, double* nx2) {
  WS(xp, double, S_XPART, 1024 * 8);
  WS(o, double, S_SIG, 64 * 8);
  int nx = 0;
  TRY(sumsq_parts(c, X, xp, &nx));
  CK(launch_sum_parts(xp, nx, 1, 1, o, c->stream));
  CK(hipMemcpyAsync(nx2, o, 8, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return ENMF_OK;
}

}  // namespace

extern "C" {

int32_t enmf_version(void) { return 100; }

const char* enmf_status_string(int32_t s) {
  switch (s) {
    case ENMF_OK: return "ok";
    case ENMF_EINVAL: return "invalid argument";
    case ENMF_ENOMEM: return "out of device memory";
    case ENMF_EDEVICE: return "device error";
    case ENMF_ENUMERIC: return "non-finite objective";
    case ENMF_EBUSY: return "busy";
    case ENMF_ECLOSED: return "closed";
    default: return "unknown status";
  }
}

enmf_status enmf_create(enmf_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return ENMF_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return ENMF_EDEVICE;
  }
  if (device < 0 || device >= count) return ENMF_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return ENMF_EDEVICE;
  enmf_ctx* c = new enmf_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipMalloc(&c->st, sizeof(DevState)) != hipSuccess) {
    delete c;
    return ENMF_ENOMEM;
  }
  if (static_scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(c->st);
    delete c;
    return ENMF_EDEVICE;
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    c->ns_per_tick = 1e6 / (double)khz;
  const char* fv = std::getenv("ENMF_FORCE_VALU");
  c->use_mfma = !(fv && fv[0] == '1');
  if (const char* xb = std::getenv("ENMF_XT_MIN_BYTES")) c->xt_min_bytes = std::atoll(xb);
  *out = c;
  return ENMF_OK;
}

void enmf_destroy(enmf_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->bufs)
    if (b.p) (void)hipFree(b.p);
  if (c->st) (void)hipFree(c->st);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->stop_ev) (void)hipEventDestroy(c->stop_ev);
  if (c->stop_host) (void)hipHostFree(c->stop_host);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

const char* enmf_last_error(const enmf_ctx* c) { return c ? c->err.c_str() : "null context"; }

enmf_status enmf_set_stream(enmf_ctx* c, void* hip_stream) {
  if (!c) return ENMF_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return ENMF_OK;
}

enmf_status enmf_synchronize(enmf_ctx* c) {
  TRY(check_ctx(c));
  CK(hipStreamSynchronize(c->stream));
  return ENMF_OK;
}

enmf_status enmf_convert(enmf_ctx* c, const float* x32, int64_t m, int64_t n, int64_t ld_in,
                         int32_t to, void* out, int64_t ld_out) {
  TRY(check_ctx(c));
  if (!x32 || !out) return fail(c, ENMF_EINVAL, "null pointer");
  if (m < 1 || n < 1 || ld_in < n || ld_out < n) return fail(c, ENMF_EINVAL, "bad shape");
  if (to != ENMF_BF16 && to != ENMF_F16) return fail(c, ENMF_EINVAL, "target dtype must be BF16 or F16");
  CK(launch_convert(x32, m, n, ld_in, to, out, ld_out, c->stream));
  return ENMF_OK;
}

enmf_status enmf_xv(enmf_ctx* c, const enmf_matrix* X, const float* B, int32_t k, float* P) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!B || !P) return fail(c, ENMF_EINVAL, "null pointer");
  if (k < 1 || k > ENMF_MAX_WIDTH) return fail(c, ENMF_EINVAL, "k out of range");
  return do_xv(c, X, B, k, P);
}

enmf_status enmf_xv_static(enmf_ctx* c, const enmf_matrix* X, const float* B, int32_t k, float* P) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!B || !P) return fail(c, ENMF_EINVAL, "null pointer");
  if (k < 1 || k > ENMF_MAX_WIDTH) return fail(c, ENMF_EINVAL, "k out of range");
  if (sparse_of(X)) return fail(c, ENMF_EINVAL, "enmf_xv_static takes a dense X only");
  unsigned char* base = static_cast<unsigned char*>(static_scratch(c->device));
  if (!base) return fail(c, ENMF_EDEVICE, "static scratch not set up on this device");
  // the same kernels and launch plan as enmf_xv, with the packed factor and the
  // split partials carved out of the fixed scratch instead of the workspace
  const bool mf = use_mfma(c, X, k);
  size_t pack = 0, part = 0;
  int splits = 1, kp = 0;
  int64_t rows_pad = 0;
  if (mf) {
    mfma_xv_ws(X->dtype, X->m, X->n, k, &pack, &part);
  } else {
    kp = pad_width(k);
    rows_pad = round_up(X->n, xv_tile_width(X->dtype));
    pack = (size_t)rows_pad * kp * 4;
    splits = xv_splits(X->m, X->n, X->dtype);
    part = splits > 1 ? (size_t)splits * X->m * k * 4 : 0;
  }
  const size_t off = (pack + 255) / 256 * 256;
  if (off + part > kStaticScratchBytes)
    return fail(c, ENMF_ENOMEM,
                "enmf_xv_static needs " + std::to_string(off + part) + " bytes of scratch at this shape; "
                "the fixed scratch holds " + std::to_string(kStaticScratchBytes));
  float* pp = part ? reinterpret_cast<float*>(base + off) : nullptr;
  if (mf) {
    CK(launch_xv_mfma(X->data, X->dtype, X->m, X->n, X->ld, B, k, base, pp, P, c->stream, 1, 1));
  } else {
    float* Bp = reinterpret_cast<float*>(base);
    CK(launch_pad_rows_cols(B, X->n, k, kp, rows_pad, Bp, c->stream));
    CK(launch_xv(X->data, X->dtype, X->m, X->n, X->ld, Bp, k, kp, splits, pp, P, c->stream));
  }
  return ENMF_OK;
}

enmf_status enmf_xtu(enmf_ctx* c, const enmf_matrix* X, const float* A, int32_t k, float* Q) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!A || !Q) return fail(c, ENMF_EINVAL, "null pointer");
  if (k < 1 || k > ENMF_MAX_WIDTH) return fail(c, ENMF_EINVAL, "k out of range");
  return do_xtu(c, X, A, k, Q);
}

enmf_status enmf_gram(enmf_ctx* c, const float* A, int64_t rows, int32_t k, double* G) {
  TRY(check_ctx(c));
  if (!A || !G) return fail(c, ENMF_EINVAL, "null pointer");
  if (rows < 1 || k < 1 || k > ENMF_MAX_WIDTH) return fail(c, ENMF_EINVAL, "bad shape");
  return do_gram(c, A, 0, k, rows, k, k, G);
}

enmf_status enmf_svd_init(enmf_ctx* c, const enmf_matrix* X, int32_t r, const enmf_svd_opts* o,
                          float* U, float* V, double* sigma_host, double* relerr_host) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!o || !o->omega) return fail(c, ENMF_EINVAL, "svd opts with a device omega are required");
  if (!U || !V) return fail(c, ENMF_EINVAL, "null output pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  if (o->oversample < 0 || o->power_iters < 0) return fail(c, ENMF_EINVAL, "bad svd opts");
  const int k = r + o->oversample;
  if (k > ENMF_MAX_WIDTH) return fail(c, ENMF_EINVAL, "r + oversample exceeds ENMF_MAX_WIDTH");
  hipStream_t s = c->stream;

  WS(Y, float, S_Y, m * k * 4);
  WS(Qm64, double, S_QM64, m * k * 8);
  WS(Qm32, float, S_QM32, m * k * 4);
  WS(Z, float, S_Z, n * k * 4);
  WS(Qn64, double, S_QN64, n * k * 8);
  WS(Qn32, float, S_QN32, n * k * 4);

  TRY(do_xv(c, X, o->omega, k, Y));
  for (int it = 0; it < o->power_iters; ++it) {
    TRY(do_orth(c, Y, m, k, Qm64, Qm32, 1));
    TRY(do_xtu(c, X, Qm32, k, Z));
    TRY(do_orth(c, Z, n, k, Qn64, Qn32, 1));
    TRY(do_xv(c, X, Qn32, k, Y));
  }
  TRY(do_orth(c, Y, m, k, Qm64, Qm32));
  TRY(do_xtu(c, X, Qm32, k, Z));
  WS(C, double, S_C, k * k * 8);
  TRY(do_gram(c, Z, 0, k, n, k, k, C));
  WS(colp, double, S_COLP, 256 * k * 8);
  WS(cols, double, S_COLS, k * 8);
  int ncp = 0;
  CK(launch_colsum(Qm64, k, m, k, colp, &ncp, s));
  CK(launch_sum_parts(colp, ncp, k, k, cols, s));
  WS(sig, double, S_SIG, 64 * 8);
  WS(TU, double, S_TU, k * r * 8);
  WS(TV, double, S_TV, k * r * 8);
  CK(launch_svd_factor(C, cols, k, r, sig, TU, TV, s));
  CK(launch_apply_small(Qm64, 1, k, m, k, TU, r, r, U, 0, r, s));
  CK(launch_apply_small(Z, 0, k, n, k, TV, r, r, V, 0, r, s));

  std::vector<double> sg(r);
  CK(hipMemcpyAsync(sg.data(), sig, r * 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (sigma_host) std::memcpy(sigma_host, sg.data(), r * 8);
  if (relerr_host) {
    // Eckart-Young floor evaluated directly as ||X - U* V*^T|| / ||X|| in
    // float64: sqrt(||X||^2 - sum sigma^2) cancels catastrophically.
    double nx2 = 0.0, f = 0.0;
    TRY(read_sumsq_x(c, X, &nx2));
    TRY(direct_objective(c, X, r, U, V, &f));
    *relerr_host = nx2 > 0.0 ? std::sqrt(2.0 * f / nx2) : 0.0;
  }
  return ENMF_OK;
}

// The pinned word and event through which a loop looks at a device stop flag.
static enmf_status ensure_stop_copy(enmf_ctx* c) {
  if (!c->stop_host) {
    void* ph = nullptr;
    if (hipHostMalloc(&ph, 64) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, ENMF_ENOMEM, "pinned host allocation failed (stop flag)");
    }
    c->stop_host = static_cast<int32_t*>(ph);
  }
  if (!c->stop_ev) CK(hipEventCreateWithFlags(&c->stop_ev, hipEventDisableTiming));
  return ENMF_OK;
}

enmf_status enmf_rotate(enmf_ctx* c, int64_t m, int64_t n, int32_t r, float* U, float* V,
                        const enmf_rotate_opts* o, double* R_host, int32_t* steps_host,
                        double* neg_before_host, double* neg_after_host) {
  TRY(check_ctx(c));
  if (!U || !V) return fail(c, ENMF_EINVAL, "null pointer");
  if (m < 1 || n < 1 || r < 1 || r > ENMF_MAX_RANK) return fail(c, ENMF_EINVAL, "bad shape");
  enmf_rotate_opts d{1.0, 1e-10, 100, 10};
  if (o) d = *o;
  if (d.rho0 <= 0.0 || d.max_iter < 0 || d.tol < 0.0) return fail(c, ENMF_EINVAL, "bad rotate opts");
  if (d.check_every < 1) d.check_every = 1;
  hipStream_t s = c->stream;
  const int64_t N = m + n;
  const int kp = pad_width(r);
  WS(W, double, S_W64, N * kp * 8);
  WS(Sa, double, S_ADMM, N * kp * 8);
  WS(R, double, S_R, kp * kp * 8);
  WS(wsq, double, S_WSQ, 512 * 8);
  const int nbm = admm_rows_blocks(N, kp);
  WS(mpart, double, S_MPART, (int64_t)nbm * r * r * 8);
  WS(Mf, double, S_C, kp * kp * 8);
  WS(stat, double, S_STAT, 4 * 512 * 8);
  WS(tot, double, S_SIG, 64 * 8);

  // rotation objective before: sum h(W)
  const int fbU = factor_blocks(m * r), fbV = factor_blocks(n * r);
  CK(launch_factor_stats(U, m * r, r, stat, 0, fbU, s));
  CK(launch_factor_stats(V, n * r, r, stat, fbU, fbV, s));
  CK(launch_sum_parts(stat, fbU + fbV, 4, 4, tot, s));
  double before[4];
  CK(hipMemcpyAsync(before, tot, 32, hipMemcpyDeviceToHost, s));

  CK(launch_pack_w(U, m, V, n, r, kp, W, s));
  int nw = 0;
  CK(launch_w_sumsq(W, N * kp, wsq, &nw, s));
  CK(launch_rho_init(wsq, nw, N, r, d.rho0, c->st, s));
  std::vector<double> eye(kp * kp, 0.0);
  for (int i = 0; i < r; ++i) eye[i * kp + i] = 1.0;
  CK(hipMemcpyAsync(R, eye.data(), kp * kp * 8, hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));

  // The tolerance stop is taken on the device by the polar step of each check
  // step (later steps return at once).  The host looks at the stop flag one
  // check late, through a pinned copy, so that its look never drains the queue.
  TRY(ensure_stop_copy(c));
  bool stop_copied = false;
  int launched = 0;
  for (int t = 0; t < d.max_iter; ++t) {
    CK(launch_admm_rows(W, N, r, kp, R, Sa, c->st, t, mpart, s));
    CK(launch_gram_finalize(mpart, nbm, r, r, kp, Mf, s));
    CK(launch_polar(Mf, r, kp, R, c->st, s, d.tol, d.check_every, t));
    launched = t + 1;
    if (d.tol > 0.0 && (launched % d.check_every == 0)) {
      if (stop_copied) {
        CK(hipEventSynchronize(c->stop_ev));
        if (*c->stop_host) break;
      }
      CK(hipMemcpyAsync(c->stop_host, &c->st->rot_stop, 4, hipMemcpyDeviceToHost, s));
      CK(hipEventRecord(c->stop_ev, s));
      stop_copied = true;
    }
  }
  CK(launch_apply_small(W, 1, kp, m, r, R, kp, r, U, 0, r, s));
  CK(launch_apply_small(W + m * kp, 1, kp, n, r, R, kp, r, V, 0, r, s));
  CK(launch_factor_stats(U, m * r, r, stat, 0, fbU, s));
  CK(launch_factor_stats(V, n * r, r, stat, fbU, fbV, s));
  CK(launch_sum_parts(stat, fbU + fbV, 4, 4, tot, s));
  double after[4];
  CK(hipMemcpyAsync(after, tot, 32, hipMemcpyDeviceToHost, s));
  std::vector<double> Rh(kp * kp);
  CK(hipMemcpyAsync(Rh.data(), R, kp * kp * 8, hipMemcpyDeviceToHost, s));
  int32_t rs[2] = {0, 0};
  CK(hipMemcpyAsync(rs, &c->st->rot_stop, 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  const int steps = rs[0] ? rs[1] : launched;
  if (R_host)
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) R_host[a * r + b] = Rh[a * kp + b];
  if (steps_host) *steps_host = steps;
  if (neg_before_host) *neg_before_host = before[3];
  if (neg_after_host) *neg_after_host = after[3];
  return ENMF_OK;
}

enmf_status enmf_rotate_general(enmf_ctx* c, int64_t m, int64_t n, int32_t r, float* U, float* V,
                                const enmf_grot_opts* o, double* R1_host, double* lambda_host,
                                double* R2_host, int32_t* steps_host, double* neg_before_host,
                                double* neg_after_host) {
  TRY(check_ctx(c));
  if (!U || !V) return fail(c, ENMF_EINVAL, "null pointer");
  if (m < 1 || n < 1 || r < 1 || r > ENMF_MAX_RANK) return fail(c, ENMF_EINVAL, "bad shape");
  enmf_grot_opts d{1.0, 1e-10, 500, 0};
  if (o) d = *o;
  if (!(d.rho0 > 0.0) || d.max_iter < 0 || !(d.tol >= 0.0))
    return fail(c, ENMF_EINVAL, "bad generalized rotation opts");
  hipStream_t s = c->stream;
  const int kp = grot_pad(r);
  const int64_t N = m + n;
  WS(gw, double, S_GW, 7 * N * kp * 8);
  WS(out, double, S_GOUT, (4 + 2 * r * r + r) * 8);
  // U and V are read into float64 before any output row is written
  CK(launch_grot(U, m, V, n, r, d.rho0, d.tol, d.max_iter, gw, U, V, out, s));
  std::vector<double> h(4 + 2 * r * r + r);
  CK(hipMemcpyAsync(h.data(), out, h.size() * 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (neg_before_host) *neg_before_host = h[0];
  if (neg_after_host) *neg_after_host = h[1];
  if (steps_host) *steps_host = (int32_t)h[2];
  if (R1_host) std::memcpy(R1_host, h.data() + 4, r * r * 8);
  if (R2_host) std::memcpy(R2_host, h.data() + 4 + r * r, r * r * 8);
  if (lambda_host) std::memcpy(lambda_host, h.data() + 4 + 2 * r * r, r * 8);
  return ENMF_OK;
}

}  // extern "C"

namespace {

struct IterBufs {
  float *P, *Q, *U2;
  double *G, *H, *rec, *gpU, *gpV, *stat, *xpart;
  int nbU, nbV, fbU, fbV;
  double* recU(int slot) { return rec + (int64_t)slot * kRecFields * nbU; }
  double* recV(int slot) { return rec + (int64_t)kRecFields * (2 * nbU + slot * nbV); }
};

// Prepares DevState and the buffers shared by enmf_iterate and enmf_objective_kkt.
enmf_status iter_setup(enmf_ctx* c, const enmf_matrix* X, int r, const float* U, const float* V,
                       const enmf_iter_opts& o, IterBufs& b) {
  hipStream_t s = c->stream;
  const int64_t m = X->m, n = X->n;
  const int kp = row_pad(r);
  WS(P, float, S_P, m * r * 4);
  WS(Q, float, S_Q, n * r * 4);
  WS(U2, float, S_U2, m * r * 4);
  WS(G, double, S_G, kp * kp * 8);
  WS(H, double, S_H, kp * kp * 8);
  b.P = P; b.Q = Q; b.U2 = U2; b.G = G; b.H = H;
  b.nbU = rowupdate_blocks(m, kp);
  b.nbV = rowupdate_blocks(n, kp);
  WS(rec, double, S_RUPART, 2 * (int64_t)kRecFields * (b.nbU + b.nbV) * 8);
  WS(gpU, double, S_GPU, (int64_t)gram_part_len(kp) * b.nbU * 8);
  WS(gpV, double, S_GPV, (int64_t)gram_part_len(kp) * b.nbV * 8);
  b.rec = rec; b.gpU = gpU; b.gpV = gpV;
  b.fbU = factor_blocks(m * r);
  b.fbV = factor_blocks(n * r);
  WS(stat, double, S_STAT, 4 * (int64_t)(b.fbU + b.fbV + 512) * 8);
  WS(xp, double, S_XPART, 1024 * 8);
  b.stat = stat; b.xpart = xp;
  // pre-size the shared split buffers so the loop never reallocates
  if (sparse_of(X)) {
    if (!ws(c, S_SPLIT, split_bytes(c, X, r)))
      return fail(c, ENMF_ENOMEM, "device workspace allocation failed");
  } else {
    const int kpw = pad_width(r);
    const int64_t rows_pad = round_up(n, xv_tile_width(X->dtype));
    size_t pbx = (size_t)rows_pad * kpw * 4, pbu = (size_t)m * kpw * 4;
    size_t sbt = 0;
    if (use_mfma(c, X, r)) {
      size_t t = 0;
      mfma_xv_ws(X->dtype, m, n, r, &pbx, &t);
      mfma_xtu_ws(X->dtype, m, n, r, &pbu, &t);
      if (use_xt(c, X, r)) {
        size_t px = 0;
        mfma_xtu_ws(X->dtype, n, m, r, &px, &sbt);   // X B on the transposed copy
        if (px > pbx) pbx = px;
      }
    }
    if (!ws(c, S_BP, pbx) || !ws(c, S_AP, pbu))
      return fail(c, ENMF_ENOMEM, "device workspace allocation failed");
    size_t sb = split_bytes(c, X, r);
    if (sbt > sb) sb = sbt;
    const size_t sv = (size_t)xv_splits(m, n, X->dtype) * m * r * 4;
    const size_t su = (size_t)xtu_splits(m, n) * n * r * 4;
    if (!use_mfma(c, X, r)) sb = sv > su ? sv : su;
    if (!ws(c, S_SPLIT, sb)) return fail(c, ENMF_ENOMEM, "device workspace allocation failed");
  }

  DevState h;
  std::memset(&h, 0, sizeof(h));
  h.pbcd_eps = o.pbcd_eps;
  h.kkt_tol = o.kkt_tol;
  h.relerr_tol = o.relerr_tol;
  h.relerr_svd = o.relerr_svd;
  h.ns_per_tick = c->ns_per_tick;
  h.mode = o.mode;
  CK(hipMemcpyAsync(c->st, &h, sizeof(h), hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));
  int nx = 0;
  TRY(sumsq_parts(c, X, xp, &nx));
  CK(launch_factor_stats(U, m * r, r, stat, 0, b.fbU, s));
  CK(launch_factor_stats(V, n * r, r, stat, b.fbU, b.fbV, s));
  CK(launch_setup_state(stat, b.fbU, b.fbV, xp, nx, o.step_u, o.step_v, o.ext_iters, o.check_every,
                        c->st, s));
  return ENMF_OK;
}

enmf_status set_trace_cap(enmf_ctx* c, int cap) {
  CK(hipMemcpyAsync(&c->st->trace_cap, &cap, 4, hipMemcpyHostToDevice, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return ENMF_OK;
}

}  // namespace

extern "C" {

// Launch sequence of one solve (per outer iteration k):
//   xv(V^k), which also combines G^k from the partial Grams of V^k
//   rowupdate U: phase from the previous records, check partials of U^k,
//                update into the other U buffer, partial Grams of U^(k+1)
//                (and, for the matrix-core products, U^(k+1) packed for xtu)
//   xtu(U^(k+1)), which also combines H^(k+1)
//   rowupdate V: first the check of iteration k (stop, trace, iteration
//                count), then the update in place, check partials of
//                V^(k+1), its partial Grams (and V^(k+1) packed for xv).
// Without the matrix-core products the Gram combines are launches of their
// own.  The last iteration (k = max_iter) only checks.
// The U update of iteration k runs before its stop decision, into a second
// buffer, so a stop at k keeps U^k; U^k lives in buffer k mod 2.
enmf_status enmf_iterate(enmf_ctx* c, const enmf_matrix* X, int32_t r, float* U, float* V,
                         const enmf_iter_opts* opts, enmf_iter_report* rep, double* trace,
                         int32_t trace_cap) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!U || !V || !opts) return fail(c, ENMF_EINVAL, "null pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  enmf_iter_opts o = *opts;
  if (o.max_iter < 0) return fail(c, ENMF_EINVAL, "max_iter must be >= 0");
  if (o.ext_iters < 1) o.ext_iters = 10;
  if (o.pbcd_max_iter < 1) o.pbcd_max_iter = 5;
  if (o.check_every < 1) o.check_every = 1;
  if (o.pbcd_eps < 0.0) return fail(c, ENMF_EINVAL, "pbcd_eps must be >= 0");
  if (o.mode < 0 || o.mode > 3) return fail(c, ENMF_EINVAL, "unsupported mode");
  if (o.graph_replay != 0 && o.graph_replay != 1) return fail(c, ENMF_EINVAL, "graph_replay must be 0 or 1");
  if (trace && trace_cap < 0) return fail(c, ENMF_EINVAL, "bad trace capacity");
  hipStream_t s = c->stream;
  const int kp = row_pad(r);
  if (o.mode == 1) {
    CK(launch_clip(U, m * r, s));
    CK(launch_clip(V, n * r, s));
  }
  IterBufs b;
  TRY(iter_setup(c, X, r, U, V, o, b));
  TRY(set_trace_cap(c, trace ? trace_cap : 0));
  DevState* st = c->st;
  const bool fixed = o.pbcd_eps == 0.0;
  float* Ub[2] = {U, b.U2};
  Parts pp;
  c->pending[0] = c->pending[1] = 0;
  // matrix-core products: each row pass also writes its output rows as the
  // next product's packed factor (U for X^T U, V for X V)
  const bool mf = use_mfma(c, X, r);
  // X B through X^T A on a transposed copy of X, made once for the call
  XTCopy xtc;
  const bool tx = use_xt(c, X, r);
  if (tx) {
    // rows of the copy start on 128-byte lines (64 elements covers both
    // storage widths): a row pitch that is an odd multiple of 64 bytes makes
    // every other row's runs straddle one more line than they cover
    const int64_t ldt = round_up(m, 64);
    WS(xtb, unsigned char, S_XT, (size_t)n * ldt * esize(X->dtype));
    CK(launch_transpose(X->data, X->dtype, m, n, X->ld, xtb, ldt, s));
    xtc.data = xtb;
    xtc.ld = ldt;
  }
  const XTCopy* xtp = tx ? &xtc : nullptr;
  PackOut poU, poV;
  if (mf) {
    size_t pbx = 0, pbu = 0, t = 0;
    if (tx) mfma_xtu_ws(X->dtype, n, m, r, &pbx, &t);
    else mfma_xv_ws(X->dtype, m, n, r, &pbx, &t);
    mfma_xtu_ws(X->dtype, m, n, r, &pbu, &t);
    WS(bp, unsigned short, S_BP, pbx);
    WS(ap, unsigned short, S_AP, pbu);
    poV.p = bp;
    // V is packed for whichever kernel runs X B
    mfma_pack_layout(X->dtype, tx ? 1 : 0, r, &poV.kp, &poV.c, &poV.ldt);
    poU.p = ap;
    mfma_pack_layout(X->dtype, 1, r, &poU.kp, &poU.c, &poU.ldt);
  }
  // vector-ALU products: the row passes also write U and V zero-padded to the
  // products' width (rows of V up to the X B tile width), so no padding
  // launch precedes each product; the padding rows and columns stay zero
  float* padU = nullptr;
  float* padV = nullptr;
  if (!mf && !tx && X->dtype != ENMF_CSR && pad_width(r) == kp) {
    const int64_t rows_pad = round_up(n, xv_tile_width(X->dtype));
    WS(pv, float, S_BP, rows_pad * kp * 4);
    WS(pu, float, S_AP, m * kp * 4);
    CK(launch_pad_rows_cols(V, n, r, kp, rows_pad, pv, s));
    CK(launch_pad_cols(U, m, r, kp, pu, s));
    padV = poV.pad = pv;
    padU = poU.pad = pu;
  }

  TRY(ensure_stop_copy(c));
  bool stop_copied = false;

  auto sample = [&](int kind, int k) -> hipEvent_t* {
    if (c->timing_period <= 0 || k % c->timing_period != 0 || c->pending[kind] >= kTimingPairs)
      return nullptr;
    c->pending_k[kind][c->pending[kind]] = k;
    return &c->events[2 * (kind * kTimingPairs + c->pending[kind]++)];
  };

  // prologue: records and Grams of U^0 and V^0 (slot 1 = "iteration -1")
  GramJob gjG, gjH;
  gjG.src = b.gpV; gjG.nparts = b.nbV; gjG.kp = kp; gjG.dst = b.G;
  gjH.src = b.gpU; gjH.nparts = b.nbU; gjH.kp = kp; gjH.dst = b.H;
  CK(launch_rowupdate(U, U, m, r, kp, nullptr, 1, 0, nullptr, st, 0, 0, kRowGram, b.recU(1), b.gpU,
                      nullptr, 0, nullptr, 0, s, poU));
  TRY(xtu_parts(c, X, U, r, b.Q, &pp, nullptr, mf, &gjH, nullptr, padU));
  CK(launch_rowupdate(V, V, n, r, kp, pp.p, pp.n, pp.stride, b.H, st, 1, 0,
                      kRowGram | kRowWriteCheck, b.recV(1), b.gpV, nullptr, 0, nullptr, 0, s, poV));
  // One outer iteration k < max_iter, enqueued on c->stream.  devk: the
  // launches take k (and whether it is checked) from the device state, so
  // that the same launches can be replayed from a graph for any k of the same
  // parity; the U pass then always writes its check partials.
  auto body = [&](int k, bool devk) -> enmf_status {
    const hipStream_t s = c->stream;
    const int cur = k & 1, prev = cur ^ 1;
    const bool due = devk || (k % o.check_every == 0);
    DecideArgs dec;
    dec.recU = b.recU(cur); dec.nbU = b.nbU;
    dec.recV = b.recV(prev); dec.nbV = b.nbV;
    dec.k = devk ? -1 : k; dec.due = due ? 1 : 0; dec.trace = trace;
    TRY(xv_parts(c, X, V, r, b.P, &pp, devk ? nullptr : sample(0, k), mf, &gjG, xtp, padV));
    const int head = kRowHead | kRowCheckPre | (due ? kRowWriteCheck : 0);
    if (fixed) {
      CK(launch_rowupdate(Ub[cur], Ub[prev], m, r, kp, pp.p, pp.n, pp.stride, b.G, st, 0,
                          o.pbcd_max_iter, head | kRowUpdate | kRowFirst | kRowGram, b.recU(cur),
                          b.gpU, b.recU(prev), b.nbU, b.recV(prev), b.nbV, s, poU));
    } else {
      for (int t = 0; t < o.pbcd_max_iter; ++t) {
        const int fl = kRowUpdate | kRowWantPg | kRowGram | (t == 0 ? head | kRowFirst : 0);
        CK(launch_rowupdate(t == 0 ? Ub[cur] : Ub[prev], Ub[prev], m, r, kp, pp.p, pp.n, pp.stride,
                            b.G, st, 0, 1, fl, b.recU(cur), b.gpU, b.recU(prev), b.nbU,
                            b.recV(prev), b.nbV, s, poU));
        CK(launch_pbcd_decide(b.recU(cur), b.nbU, 0, t == 0, st, s));
      }
    }
    // X^T U^(k+1) runs before the check of iteration k.  The decision is
    // taken by a side workgroup of the matrix-core product, else at the head
    // of the V pass; either way the V pass leaves V^k in place on a stop.
    TRY(xtu_parts(c, X, Ub[prev], r, b.Q, &pp, devk ? nullptr : sample(1, k), mf, &gjH,
                  mf ? &dec : nullptr, padU));
    const int vdec = mf ? 0 : kRowDecide;
    if (fixed) {
      CK(launch_rowupdate(V, V, n, r, kp, pp.p, pp.n, pp.stride, b.H, st, 1, o.pbcd_max_iter,
                          vdec | kRowUpdate | kRowFirst | kRowGram | kRowWriteCheck,
                          b.recV(cur), b.gpV, nullptr, 0, nullptr, 0, s, poV, dec));
    } else {
      for (int t = 0; t < o.pbcd_max_iter; ++t) {
        const int fl = kRowUpdate | kRowWantPg | kRowGram | kRowWriteCheck |
                       (t == 0 ? kRowFirst | vdec : 0);
        CK(launch_rowupdate(V, V, n, r, kp, pp.p, pp.n, pp.stride, b.H, st, 1, 1, fl, b.recV(cur),
                            b.gpV, nullptr, 0, nullptr, 0, s, poV, dec));
        CK(launch_pbcd_decide(b.recV(cur), b.nbV, 1, t == 0, st, s));
      }
    }
    return ENMF_OK;
  };

  // graph_replay: the loop body of two iterations (odd k, then even k) is
  // captured once on a private stream and replayed for every pair after the
  // first iteration; the first, a trailing odd one and the final check are
  // launched directly.  Kernel sampling needs the events of each launch, so a
  // sampled call launches directly.
  const bool graphs = o.graph_replay == 1 && c->timing_period <= 0 && o.max_iter >= 5;
  hipGraphExec_t gx = nullptr;
  auto capture_pair = [&](int k) -> bool {
    if (!c->cap_stream &&
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      c->cap_stream = nullptr;
      return false;
    }
    const hipStream_t saved = c->stream;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    c->stream = c->cap_stream;
    enmf_status bs = body(k, true);
    if (bs == ENMF_OK) bs = body(k + 1, true);
    c->stream = saved;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (bs == ENMF_OK && e == hipSuccess) e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (bs != ENMF_OK || e != hipSuccess) {
      (void)hipGetLastError();
      c->err.clear();
      gx = nullptr;
      return false;
    }
    return true;
  };
  bool use_graph = graphs;
  int k = 0, next_look = 32;
  bool stopped = false;
  while (k < o.max_iter) {
    if (use_graph && (k & 1) && k + 1 < o.max_iter) {
      if (!gx && !capture_pair(k)) {
        use_graph = false;
        continue;
      }
      CK(hipGraphLaunch(gx, s));
      k += 2;
    } else {
      const enmf_status bs = body(k, false);
      if (bs != ENMF_OK) {
        if (gx) (void)hipGraphExecDestroy(gx);
        return bs;
      }
      k += 1;
    }
    if (k >= next_look) {
      next_look += 32;
      // The stop flag is copied to pinned memory here and looked at one check
      // later, once the device has passed this point, so the queue never drains
      // for the look; launches after a stop return at once on the device flag.
      if (stop_copied) {
        CK(hipEventSynchronize(c->stop_ev));
        if (*c->stop_host) {
          stopped = true;
          break;
        }
      }
      CK(hipMemcpyAsync(c->stop_host, &st->stop, 4, hipMemcpyDeviceToHost, s));
      CK(hipEventRecord(c->stop_ev, s));
      stop_copied = true;
    }
  }
  if (!stopped) {
    // the last check (k = max_iter) only: the state of the last iteration
    const int cur = o.max_iter & 1, prev = cur ^ 1;
    DecideArgs dec;
    dec.recU = b.recU(cur); dec.nbU = b.nbU;
    dec.recV = b.recV(prev); dec.nbV = b.nbV;
    dec.k = o.max_iter; dec.due = 1; dec.trace = trace;
    TRY(xv_parts(c, X, V, r, b.P, &pp, sample(0, o.max_iter), mf, &gjG, xtp));
    CK(launch_rowupdate(Ub[cur], Ub[cur], m, r, kp, pp.p, pp.n, pp.stride, b.G, st, 0, 0,
                        kRowHead | kRowCheckPre | kRowWriteCheck, b.recU(cur), b.gpU, b.recU(prev),
                        b.nbU, b.recV(prev), b.nbV, s));
    CK(launch_finalize(dec, 1, st, s));
  }
  DevState h;
  CK(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (gx) (void)hipGraphExecDestroy(gx);
  for (int kind = 0; kind < 2; ++kind) {
    for (int q = 0; q < c->pending[kind]; ++q) {
      float ms = 0.f;
      hipEvent_t* e = &c->events[2 * (kind * kTimingPairs + q)];
      // both products of the stopping iteration ran in full, later ones exit at once
      const int kq = c->pending_k[kind][q];
      const bool ran = kq <= h.iters;
      if (ran && hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) {
        c->timing_sum[kind] += ms;
        c->timing_n[kind] += 1;
      }
    }
    c->pending[kind] = 0;
  }
  (void)hipGetLastError();
  if (h.iters & 1) CK(hipMemcpyAsync(U, b.U2, m * r * 4, hipMemcpyDeviceToDevice, s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->iters = h.iters;
    rep->ext_iters_done = h.ext_done;
    rep->phase = h.negs > 0 ? kPhaseExt : kPhaseHals;
    rep->converged = h.converged;
    rep->step_u = h.step[0];
    rep->step_v = h.step[1];
    double f = 0.0;
    TRY(direct_objective(c, X, r, U, V, &f));
    rep->f = f;
    rep->relerr = h.nx2 > 0.0 ? std::sqrt(2.0 * f / h.nx2) : 0.0;
    rep->re_paper = o.relerr_svd > 0.0 ? rep->relerr / o.relerr_svd : NAN;
    rep->kkt = h.kkt;
    rep->kkt_feas = h.kkt_feas;
    rep->kkt_pg_u = h.kkt_pg_u;
    rep->kkt_pg_v = h.kkt_pg_v;
    rep->delta_w = h.delta_w;
    rep->sigma_w = h.sigma_w;
  } else {
    CK(hipStreamSynchronize(s));
  }
  if (h.numeric_error) return fail(c, ENMF_ENUMERIC, "non-finite objective or KKT residual");
  return ENMF_OK;
}

enmf_status enmf_objective_kkt(enmf_ctx* c, const enmf_matrix* X, int32_t r, const float* U,
                               const float* V, double relerr_svd, enmf_kkt* out) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (!U || !V || !out) return fail(c, ENMF_EINVAL, "null pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  hipStream_t s = c->stream;
  const int kp = row_pad(r);
  enmf_iter_opts o;
  std::memset(&o, 0, sizeof(o));
  o.kkt_tol = -1.0;
  o.relerr_tol = -1.0;
  o.relerr_svd = relerr_svd;
  o.ext_iters = 10;
  IterBufs b;
  TRY(iter_setup(c, X, r, U, V, o, b));
  TRY(set_trace_cap(c, 0));
  DevState* st = c->st;
  float* Uw = const_cast<float*>(U);   // never written: no kRowUpdate below
  float* Vw = const_cast<float*>(V);
  Parts pp;
  CK(launch_rowupdate(U, Uw, m, r, kp, nullptr, 1, 0, nullptr, st, 0, 0, kRowGram, b.recU(0), b.gpU,
                      nullptr, 0, nullptr, 0, s));
  CK(launch_gram_fin(b.gpU, b.nbU, kp, b.H, s));
  CK(launch_rowupdate(V, Vw, n, r, kp, nullptr, 1, 0, nullptr, st, 1, 0, kRowGram, b.recV(0), b.gpV,
                      nullptr, 0, nullptr, 0, s));
  CK(launch_gram_fin(b.gpV, b.nbV, kp, b.G, s));
  TRY(xtu_parts(c, X, U, r, b.Q, &pp));
  CK(launch_rowupdate(V, Vw, n, r, kp, pp.p, pp.n, pp.stride, b.H, st, 1, 0, kRowWriteCheck,
                      b.recV(0), b.gpV, nullptr, 0, nullptr, 0, s));
  TRY(xv_parts(c, X, V, r, b.P, &pp));
  CK(launch_rowupdate(U, Uw, m, r, kp, pp.p, pp.n, pp.stride, b.G, st, 0, 0,
                      kRowCheckPre | kRowWriteCheck, b.recU(0), b.gpU, nullptr, 0, nullptr, 0, s));
  DecideArgs dec;
  dec.recU = b.recU(0); dec.nbU = b.nbU;
  dec.recV = b.recV(0); dec.nbV = b.nbV;
  dec.k = 0; dec.due = 1;
  CK(launch_finalize(dec, 1, st, s));
  DevState h;
  CK(hipMemcpyAsync(&h, c->st, sizeof(h), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  double f = 0.0;
  TRY(direct_objective(c, X, r, U, V, &f));
  out->f = f;
  out->relerr = h.nx2 > 0.0 ? std::sqrt(2.0 * f / h.nx2) : 0.0;
  out->re_paper = relerr_svd > 0.0 ? out->relerr / relerr_svd : NAN;
  out->kkt = h.kkt;
  out->kkt_feas = h.kkt_feas;
  out->kkt_pg_u = h.kkt_pg_u;
  out->kkt_pg_v = h.kkt_pg_v;
  out->delta_w = h.delta_w;
  out->sigma_w = h.sigma_w;
  out->sigma_u = h.sigma_u;
  out->sigma_v = h.sigma_v;
  out->min_w = h.min_w;
  if (!std::isfinite(f)) return fail(c, ENMF_ENUMERIC, "non-finite objective");
  return ENMF_OK;
}

enmf_status enmf_kernel_timing(enmf_ctx* c, int32_t period, double* xv_ms, double* xtu_ms,
                               int32_t* samples) {
  TRY(check_ctx(c));
  if (period < 0) return fail(c, ENMF_EINVAL, "period must be >= 0");
  if (period > 0 && c->events.empty()) {
    c->events.resize(2 * 2 * kTimingPairs, nullptr);
    for (auto& e : c->events) CK(hipEventCreate(&e));
  }
  const int n0 = c->timing_n[0], n1 = c->timing_n[1];
  if (xv_ms) *xv_ms = n0 ? c->timing_sum[0] / n0 : 0.0;
  if (xtu_ms) *xtu_ms = n1 ? c->timing_sum[1] / n1 : 0.0;
  if (samples) *samples = n0 < n1 ? n0 : n1;
  c->timing_sum[0] = c->timing_sum[1] = 0.0;
  c->timing_n[0] = c->timing_n[1] = 0;
  c->timing_period = period;
  return ENMF_OK;
}

enmf_status enmf_time_products(enmf_ctx* c, const enmf_matrix* X, int32_t k, int32_t reps,
                               double* xv_ms, double* xtu_ms) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  if (k < 1 || k > ENMF_MAX_WIDTH || reps < 1) return fail(c, ENMF_EINVAL, "bad k or reps");
  hipStream_t s = c->stream;
  const int64_t m = X->m, n = X->n;
  const int kp = pad_width(k);
  const bool mf = use_mfma(c, X, k);
  const SparseX* sp = sparse_of(X);
  const int64_t rows_pad = sp ? n : round_up(n, xv_tile_width(X->dtype));
  size_t pbx = (size_t)rows_pad * kp * 4, pbu = (size_t)m * kp * 4, t = 0;
  if (mf) {
    mfma_xv_ws(X->dtype, m, n, k, &pbx, &t);
    mfma_xtu_ws(X->dtype, m, n, k, &pbu, &t);
  }
  WS(Bp, float, S_BP, pbx);
  WS(Ap, float, S_AP, pbu);
  WS(P, float, S_P, m * k * 4);
  WS(Q, float, S_Q, n * k * 4);
  WS(Z, float, S_Z, (m > n ? m : n) * k * 4);
  WS(part, float, S_SPLIT, split_bytes(c, X, k));
  CK(hipMemsetAsync(Z, 0, (m > n ? m : n) * k * 4, s));
  CK(hipMemsetAsync(Bp, 0, pbx, s));
  CK(hipMemsetAsync(Ap, 0, pbu, s));
  const int sx = sp ? 1 : xv_splits(m, n, X->dtype), su = sp ? 1 : xtu_splits(m, n);
  auto run_xv = [&](int pack) {
    if (sp) return launch_spmm(sp->csr, Z, k, part, P, s);
    return mf ? launch_xv_mfma(X->data, X->dtype, m, n, X->ld, Z, k, Bp, part, P, s, 0, pack)
              : launch_xv(X->data, X->dtype, m, n, X->ld, Bp, k, kp, sx, part, P, s, 0);
  };
  auto run_xtu = [&](int pack) {
    if (sp) return launch_spmm(sp->csc, Z, k, part, Q, s);
    return mf ? launch_xtu_mfma(X->data, X->dtype, m, n, X->ld, Z, k, Ap, part, Q, s, 0, pack)
              : launch_xtu(X->data, X->dtype, m, n, X->ld, Ap, k, kp, su, part, Q, s, 0);
  };
  hipEvent_t e0, e1, e2;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventCreate(&e2));
  // one untimed launch of each first (packs the zero operand)
  CK(run_xv(1));
  CK(run_xtu(1));
  CK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) CK(run_xv(0));
  CK(hipEventRecord(e1, s));
  for (int i = 0; i < reps; ++i) CK(run_xtu(0));
  CK(hipEventRecord(e2, s));
  CK(hipEventSynchronize(e2));
  float a = 0.f, b = 0.f;
  CK(hipEventElapsedTime(&a, e0, e1));
  CK(hipEventElapsedTime(&b, e1, e2));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  if (xv_ms) *xv_ms = a / reps;
  if (xtu_ms) *xtu_ms = b / reps;
  return ENMF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Exterior nonnegative matrix completion (the appendix "Exterior NMC
// algorithm"): host sequencing of the masked kernels of k_enmc.hip.
// ---------------------------------------------------------------------------
namespace {

enmf_status check_mask(enmf_ctx* c, const enmf_matrix* X, const enmf_mask* M) {
  if (!M || !M->bits) return fail(c, ENMF_EINVAL, "mask is null");
  if (M->ld_words < (X->n + 31) / 32) return fail(c, ENMF_EINVAL, "mask rows shorter than ceil(n/32) words");
  if (reinterpret_cast<uintptr_t>(M->bits) % 4 != 0) return fail(c, ENMF_EINVAL, "mask not 4-byte aligned");
  if (X->dtype != ENMF_F32) return fail(c, ENMF_EINVAL, "eNMC takes float32 X");
  return ENMF_OK;
}

// Buffers of the masked kernels at (m, n, r).
struct EnmcBufs {
  EnmcPlan pu, pv;
  float *RU, *RV;
  double *E, *rss, *cu, *cv, *G, *Gi;
  int* bad;
  EnmcState* st;
  int ncu, ncv;
};

enmf_status enmc_bufs(enmf_ctx* c, int64_t m, int64_t n, int r, EnmcBufs& b) {
  b.pu = enmc_plan(m, n, 0);
  b.pv = enmc_plan(m, n, 1);
  WS(RU, float, S_ERU, (int64_t)b.pu.splits * m * r * 4);
  WS(RV, float, S_ERV, (int64_t)b.pv.splits * n * r * 4);
  const int64_t ne = std::max((int64_t)b.pu.splits * m, (int64_t)b.pv.splits * n);
  WS(E, double, S_EE, ne * 8);
  WS(rss, double, S_ERSS, b.pu.out_tiles * b.pu.splits * 8);
  b.ncu = enmc_check_blocks(m * r);
  b.ncv = enmc_check_blocks(n * r);
  WS(cu, double, S_ECU, (int64_t)b.ncu * 5 * 8);
  WS(cv, double, S_ECV, (int64_t)b.ncv * 5 * 8);
  WS(G, double, S_EG, (int64_t)r * r * 8);
  WS(Gi, double, S_EGI, (int64_t)r * r * 8 + 256);
  WS(st, EnmcState, S_EST, sizeof(EnmcState));
  b.RU = RU; b.RV = RV; b.E = E; b.rss = rss; b.cu = cu; b.cv = cv; b.G = G; b.Gi = Gi;
  b.bad = reinterpret_cast<int*>(reinterpret_cast<char*>(Gi) + (int64_t)r * r * 8);
  b.st = st;
  return ENMF_OK;
}

// Ginv of the Gram of A (rows x r); sets *bad on a singular Gram.
enmf_status gram_inverse(enmf_ctx* c, const float* A, int64_t rows, int r, EnmcBufs& b) {
  TRY(do_gram(c, A, 0, r, rows, r, r, b.G));
  CK(launch_spd_inverse(b.G, r, r, b.Gi, b.bad, c->stream));
  return ENMF_OK;
}

// fhat = 1/2 sum of the masked squared residuals at (U, V).
enmf_status enmc_objective(enmf_ctx* c, const enmf_matrix* X, const enmf_mask* M, int r,
                           const float* U, const float* V, EnmcBufs& b, double* f) {
  CK(launch_mres(0, static_cast<const float*>(X->data), X->m, X->n, X->ld, M->bits, M->ld_words, U, V, r,
                 b.RU, b.rss, c->stream));
  const int64_t nr = b.pu.out_tiles * b.pu.splits;
  std::vector<double> h(nr);
  CK(hipMemcpyAsync(h.data(), b.rss, nr * 8, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  double sum = 0.0;
  for (double v : h) sum += v;
  *f = 0.5 * sum;
  return ENMF_OK;
}

}  // namespace

extern "C" {

enmf_status enmf_enmc_init(enmf_ctx* c, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                           const enmf_svd_opts* svd, int32_t als_iters, float* U, float* V,
                           double* fhat_host) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  TRY(check_mask(c, X, M));
  if (!U || !V || !svd) return fail(c, ENMF_EINVAL, "null pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  if (als_iters < 0) return fail(c, ENMF_EINVAL, "als_iters must be >= 0");
  hipStream_t s = c->stream;
  const float* Xf = static_cast<const float*>(X->data);
  WS(X0, float, S_EX, m * n * 4);
  CK(launch_mask_x(Xf, m, n, X->ld, M->bits, M->ld_words, X0, s));
  enmf_matrix Xz{X0, m, n, n, ENMF_F32, 0};
  std::vector<double> sg(r);
  double rsvd = 0.0;
  TRY(enmf_svd_init(c, &Xz, r, svd, U, V, sg.data(), &rsvd));
  EnmcBufs b;
  TRY(enmc_bufs(c, m, n, r, b));
  CK(hipMemsetAsync(b.bad, 0, 4, s));
  for (int it = 0; it < als_iters; ++it) {
    // U <- U + R_U (V^T V)^-1, then V <- V + R_V (U^T U)^-1 with the new U
    TRY(gram_inverse(c, V, n, r, b));
    CK(launch_mres(0, Xf, m, n, X->ld, M->bits, M->ld_words, U, V, r, b.RU, nullptr, s));
    CK(launch_als_step(U, m, r, b.RU, b.pu.splits, b.Gi, r, s));
    TRY(gram_inverse(c, U, m, r, b));
    CK(launch_mres(1, Xf, m, n, X->ld, M->bits, M->ld_words, U, V, r, b.RV, nullptr, s));
    CK(launch_als_step(V, n, r, b.RV, b.pv.splits, b.Gi, r, s));
  }
  int bad = 0;
  CK(hipMemcpyAsync(&bad, b.bad, 4, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (bad) return fail(c, ENMF_ENUMERIC, "singular Gram in softImpute-ALS");
  if (fhat_host) TRY(enmc_objective(c, X, M, r, U, V, b, fhat_host));
  return ENMF_OK;
}

enmf_status enmf_enmc_grad(enmf_ctx* c, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                           const float* U, const float* V, float* gU, float* gV, double* fhat_host) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  TRY(check_mask(c, X, M));
  if (!U || !V) return fail(c, ENMF_EINVAL, "null pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  hipStream_t s = c->stream;
  const float* Xf = static_cast<const float*>(X->data);
  EnmcBufs b;
  TRY(enmc_bufs(c, m, n, r, b));
  CK(launch_mres(0, Xf, m, n, X->ld, M->bits, M->ld_words, U, V, r, b.RU, b.rss, s));
  if (gU) CK(launch_sum_neg(b.RU, b.pu.splits, m * r, gU, s));
  if (gV) {
    CK(launch_mres(1, Xf, m, n, X->ld, M->bits, M->ld_words, U, V, r, b.RV, nullptr, s));
    CK(launch_sum_neg(b.RV, b.pv.splits, n * r, gV, s));
  }
  const int64_t nr = b.pu.out_tiles * b.pu.splits;
  std::vector<double> h(nr);
  CK(hipMemcpyAsync(h.data(), b.rss, nr * 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  double sum = 0.0;
  for (double v : h) sum += v;
  if (fhat_host) *fhat_host = 0.5 * sum;
  return ENMF_OK;
}

enmf_status enmf_enmc_iterate(enmf_ctx* c, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                              float* U, float* V, const enmf_iter_opts* opts,
                              enmf_iter_report* rep) {
  TRY(check_ctx(c));
  TRY(check_matrix(c, X));
  TRY(check_mask(c, X, M));
  if (!U || !V || !opts) return fail(c, ENMF_EINVAL, "null pointer");
  const int64_t m = X->m, n = X->n;
  if (r < 1 || r > ENMF_MAX_RANK || r > m || r > n) return fail(c, ENMF_EINVAL, "r out of range");
  enmf_iter_opts o = *opts;
  if (o.max_iter < 0) return fail(c, ENMF_EINVAL, "max_iter must be >= 0");
  if (o.pbcd_eps != 0.0 || o.mode != 0 || o.relerr_tol > 0.0)
    return fail(c, ENMF_EINVAL, "eNMC takes a fixed sweep count, mode 0 and no relerr stop");
  if (o.ext_iters < 1) o.ext_iters = 10;
  if (o.pbcd_max_iter < 1) o.pbcd_max_iter = 5;
  hipStream_t s = c->stream;
  const float* Xf = static_cast<const float*>(X->data);
  const uint32_t* bits = M->bits;
  const int64_t ldm = M->ld_words;
  EnmcBufs b;
  TRY(enmc_bufs(c, m, n, r, b));

  // ||M o X||^2 and the push sizes (as in enmf_iterate)
  WS(X0, float, S_EX, m * n * 4);
  CK(launch_mask_x(Xf, m, n, X->ld, bits, ldm, X0, s));
  enmf_matrix Xz{X0, m, n, n, ENMF_F32, 0};
  double nx2 = 0.0;
  TRY(read_sumsq_x(c, &Xz, &nx2));
  const int fbU = factor_blocks(m * r), fbV = factor_blocks(n * r);
  WS(stat, double, S_ESTAT, 4 * (int64_t)(fbU + fbV) * 8);
  CK(launch_factor_stats(U, m * r, r, stat, 0, fbU, s));
  CK(launch_factor_stats(V, n * r, r, stat, fbU, fbV, s));
  std::vector<double> hs(4 * (fbU + fbV));
  CK(hipMemcpyAsync(hs.data(), stat, hs.size() * 8, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  double mnU = INFINITY, mnV = INFINITY;
  for (int q = 0; q < fbU; ++q) mnU = std::min(mnU, hs[4 * q + 1]);
  for (int q = fbU; q < fbU + fbV; ++q) mnV = std::min(mnV, hs[4 * q + 1]);
  const double dd = (double)o.ext_iters - 0.5;
  const double su = o.step_u > 0.0 ? o.step_u : std::max(-mnU, 0.0) / dd;
  const double sv = o.step_v > 0.0 ? o.step_v : std::max(-mnV, 0.0) / dd;

  EnmcState h;
  std::memset(&h, 0, sizeof(h));
  h.nx2 = nx2;
  h.kkt_tol = o.kkt_tol;
  CK(hipMemcpyAsync(b.st, &h, sizeof(h), hipMemcpyHostToDevice, s));
  int ext_done = 0;
  const int64_t nrss = b.pu.out_tiles * b.pu.splits;
  for (int k = 0; k <= o.max_iter; ++k) {
    // check of (U^k, V^k)
    CK(launch_mres(0, Xf, m, n, X->ld, bits, ldm, U, V, r, b.RU, b.rss, s));
    CK(launch_mres(1, Xf, m, n, X->ld, bits, ldm, U, V, r, b.RV, nullptr, s));
    CK(launch_enmc_check(U, m, r, b.RU, b.pu.splits, b.cu, s));
    CK(launch_enmc_check(V, n, r, b.RV, b.pv.splits, b.cv, s));
    CK(launch_enmc_finalize(b.rss, (int)nrss, b.cu, b.ncu, b.cv, b.ncv, k, k == o.max_iter ? 1 : 0,
                            b.st, s));
    CK(hipMemcpyAsync(&h, b.st, sizeof(h), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (h.stop) break;
    if (h.negs > 0.0) ext_done += 1;
    // U half: push, then masked PBCD sweeps (the check's R_U serves the
    // first sweep when the push changed nothing)
    if (h.negs_u > 0.0) CK(launch_enmc_push(U, m * r, su, nullptr, s));
    for (int t = 0; t < o.pbcd_max_iter; ++t) {
      if (t > 0 || h.negs_u > 0.0)
        CK(launch_mres(0, Xf, m, n, X->ld, bits, ldm, U, V, r, b.RU, nullptr, s));
      CK(launch_menergy(0, m, n, bits, ldm, U, V, r, b.RU, b.pu.splits, b.E, s));
      CK(launch_enmc_step(U, m, r, b.RU, b.pu.splits, b.E, b.pu.splits, -1.0, s));
    }
    // V half with the new U
    if (h.negs - h.negs_u > 0.0) CK(launch_enmc_push(V, n * r, sv, nullptr, s));
    for (int t = 0; t < o.pbcd_max_iter; ++t) {
      CK(launch_mres(1, Xf, m, n, X->ld, bits, ldm, U, V, r, b.RV, nullptr, s));
      CK(launch_menergy(1, m, n, bits, ldm, U, V, r, b.RV, b.pv.splits, b.E, s));
      CK(launch_enmc_step(V, n, r, b.RV, b.pv.splits, b.E, b.pv.splits, -1.0, s));
    }
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->iters = h.iters;
    rep->ext_iters_done = ext_done;
    rep->phase = h.negs > 0.0 ? kPhaseExt : kPhaseHals;
    rep->converged = h.converged;
    rep->step_u = su;
    rep->step_v = sv;
    rep->f = h.f;
    rep->relerr = h.relerr;
    rep->re_paper = NAN;
    rep->kkt = h.kkt;
    rep->kkt_feas = h.kkt_feas;
    rep->kkt_pg_u = h.kkt_pg_u;
    rep->kkt_pg_v = h.kkt_pg_v;
  }
  if (h.numeric_error) return fail(c, ENMF_ENUMERIC, "non-finite objective or KKT residual");
  return ENMF_OK;
}

}  // extern "C"
