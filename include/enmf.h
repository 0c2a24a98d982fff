/*
 * enmf.h -- C ABI of the MI355X (gfx950) exterior-NMF library, libenmf.so.
 *
 * Problem (paper "An Exterior Method for Nonnegative Matrix Factorization",
 * problem statement, eq. 1): given X >= 0 (m x n) and a rank r, find U (m x r)
 * and V (n x r), both >= 0, minimising f(U,V) = 1/2 ||X - U V^T||_F^2.
 * The method (Algorithm 3) runs four blocks, one entry point each:
 *   enmf_svd_init      truncated (randomized) SVD, balanced factors      (section 3, Algorithm 3 step 2)
 *   enmf_rotate        ADMM rotation toward the nonnegative orthant       (section 3.1, Algorithm 1, eq. 7)
 *   enmf_iterate       exterior push + PBCD until feasible, then HALS     (sections 3.2-3.3, Algorithms 2-3)
 *   enmf_objective_kkt objective, relative errors and KKT residual        (appendix, eq. kkt-nmf)
 * plus the streaming products they are built from (enmf_xv, enmf_xtu, enmf_gram;
 * appendix on computational complexity: X V, X^T U and the r x r Grams).
 *
 * Conventions for every call
 *   - Matrices are dense, row-major.  X is described by enmf_matrix (leading
 *     dimension ld >= n, in elements).  Factor matrices are float32 with
 *     leading dimension r (row i of U starts at U + i*r).
 *   - Every pointer argument named *_host is host memory; every other pointer
 *     is device memory on the context's device.  All device buffers are owned
 *     by the caller; the library never frees them and keeps no pointer to
 *     them after a call returns.  Workspace is owned by the context.
 *   - Work is enqueued on the context's stream.  Calls that return host
 *     values synchronise that stream; no other stream is touched.
 *   - Calls return an enmf_status and never abort.  Arguments are validated
 *     on the host before anything is launched; enmf_last_error() then
 *     describes the failure.  X >= 0 is the caller's contract (eq. 1).
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef ENMF_H
#define ENMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ENMF_OK = 0,
  ENMF_EINVAL = 1,    /* bad argument: null pointer, bad shape, r out of range, bad dtype, ld < n */
  ENMF_ENOMEM = 2,    /* device workspace could not be allocated */
  ENMF_EDEVICE = 3,   /* a HIP runtime error (message in enmf_last_error) */
  ENMF_ENUMERIC = 4,  /* non-finite objective or residual; U, V hold the last iterate */
  ENMF_EBUSY = 5,     /* enmf_serve_poll: the request has not finished yet */
  ENMF_ECLOSED = 6    /* enmf_serve_submit after enmf_serve_stop began */
} enmf_status;

/* Storage of X.  ENMF_CSR: a sparse X uploaded with enmf_sparse_create. */
typedef enum { ENMF_F32 = 0, ENMF_BF16 = 1, ENMF_F16 = 2, ENMF_CSR = 3 } enmf_dtype;

/* Largest supported rank and oversampled width (r + oversample). */
#define ENMF_MAX_RANK 64
#define ENMF_MAX_WIDTH 80

typedef struct enmf_ctx enmf_ctx;

/* Data matrix X (eq. 1).  data: device pointer to m rows of ld elements of
 * the given dtype; only the first n of each row are read.  X >= 0.  Rows
 * that start on 128-byte lines (ld * element size a multiple of 128) are
 * streamed without fetching lines that straddle two rows' runs. 
 * dtype ENMF_CSR: data is an enmf_sparse handle (below) made on the same
 * device, m and n are its shape and ld is ignored. */
typedef struct {
  const void* data;
  int64_t m, n, ld;
  int32_t dtype;      /* enmf_dtype */
  int32_t reserved;
} enmf_matrix;

/* Library version (major*10000 + minor*100 + patch). */
int32_t enmf_version(void);

/* Static text for a status code. */
const char* enmf_status_string(int32_t status);

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the default stream).  Returns ENMF_EDEVICE when no usable device
 * exists.  *out is set to NULL on failure. */
enmf_status enmf_create(enmf_ctx** out, int32_t device, void* hip_stream);

/* Free the context and its workspace (synchronises its stream first). */
void enmf_destroy(enmf_ctx* ctx);

/* Message for the last failed call on this context (never NULL). */
const char* enmf_last_error(const enmf_ctx* ctx);

/* Change the stream later calls enqueue on. */
enmf_status enmf_set_stream(enmf_ctx* ctx, void* hip_stream);

/* Block until the context's stream is idle. */
enmf_status enmf_synchronize(enmf_ctx* ctx);

/* Round X (float32, m x n, leading dimension ld_in) to BF16 or FP16 storage
 * with round-to-nearest-even, writing m rows of ld_out elements (ld_out >= n)
 * to `out`.  This produces the reduced-storage form of X that every call
 * below accepts. */
enmf_status enmf_convert(enmf_ctx* ctx, const float* x32, int64_t m, int64_t n, int64_t ld_in,
                         int32_t to_dtype, void* out, int64_t ld_out);

/* ---- streaming products (appendix on complexity: the O(mnr) core kernel) ----
 * enmf_xv:  P = X B, B is n x k (leading dimension k), P is m x k.
 * enmf_xtu: Q = X^T A, A is m x k (leading dimension k), Q is n x k.
 * X is streamed once; products accumulate in float32 whatever X's storage.
 * 1 <= k <= ENMF_MAX_WIDTH. */
enmf_status enmf_xv(enmf_ctx* ctx, const enmf_matrix* X, const float* B, int32_t k, float* P);
enmf_status enmf_xtu(enmf_ctx* ctx, const enmf_matrix* X, const float* A, int32_t k, float* Q);

/* enmf_xv without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and result as enmf_xv (bitwise), dense
 * X only (float32, bfloat16 or float16).  The packed factor and the split
 * partials live in a fixed 64 MiB device array that the library holds on each
 * device from the first enmf_create on that device until the process ends;
 * nothing is allocated by the call.  A shape whose scratch would exceed
 * 64 MiB returns ENMF_ENOMEM before any launch (enmf_last_error gives the
 * bytes needed).  Every call on one device shares that array and leaves its
 * contents behind: calls that overlap on one device (two streams, two
 * threads, two contexts) race and must be serialised by the caller.  A sparse
 * X returns ENMF_EINVAL. */
enmf_status enmf_xv_static(enmf_ctx* ctx, const enmf_matrix* X, const float* B, int32_t k, float* P);

/* Gram matrix G = A^T A (k x k, float64, row-major) of the float32 rows x k
 * matrix A, accumulated in float64 (the r x r Grams V^T V, U^T U). */
enmf_status enmf_gram(enmf_ctx* ctx, const float* A, int64_t rows, int32_t k, double* G);

/* ---- block (i): truncated SVD (section 3; randomized variant, remark after Algorithm 3) ----
 * Randomized range finder with Gaussian test matrix omega (n x (r+oversample),
 * float32, leading dimension r+oversample, device, required) and power_iters
 * re-orthonormalised power iterations, then the SVD of the small projected
 * matrix.  Output: balanced factors U* = U Sigma^(1/2) (m x r) and
 * V* = V Sigma^(1/2) (n x r) in float32, each column pair signed so that the
 * column sum of U is positive; sigma_host (r values, descending) and
 * relerr_svd_host = ||X - U* V*^T||_F / ||X||_F, the Eckart-Young floor
 * sqrt(||X||^2 - sum sigma^2)/||X|| evaluated directly in float64 (either may be NULL).
 * Orthonormalisation and the small eigenproblem run in float64 on the GPU.
 * Requires 1 <= r <= min(m, n, ENMF_MAX_RANK) and r + oversample <= ENMF_MAX_WIDTH. */
typedef struct {
  const float* omega;
  int32_t oversample;    /* p, default 10 */
  int32_t power_iters;   /* q, default 2 */
} enmf_svd_opts;

enmf_status enmf_svd_init(enmf_ctx* ctx, const enmf_matrix* X, int32_t r, const enmf_svd_opts* opts,
                          float* U, float* V, double* sigma_host, double* relerr_svd_host);

/* ---- block (ii): rotation (section 3.1, Algorithm 1, eq. 7, Procrustes step) ----
 * ADMM on min_R sum h(W R) s.t. R^T R = I with W = [U; V], h(q) = max(0, -q).
 * rho = rho0 * sqrt((m+n) r) / ||W||_F, R0 = I, Y0 = 0.  Stops when
 * ||R_{k+1} - R_k||_F <= tol (tested every check_every steps) or after
 * max_iter steps; tol = 0 runs exactly max_iter steps.  U and V (float32,
 * in place) are replaced by U R and V R with the last R.  All ADMM state is
 * float64.  R_host (r x r, may be NULL), steps_host, neg_mass_*_host (the
 * rotation objective sum h before and after; may be NULL). */
typedef struct {
  double rho0;          /* default 1.0 */
  double tol;           /* default 1e-10 */
  int32_t max_iter;     /* default 100 */
  int32_t check_every;  /* default 10 */
} enmf_rotate_opts;

enmf_status enmf_rotate(enmf_ctx* ctx, int64_t m, int64_t n, int32_t r, float* U, float* V,
                        const enmf_rotate_opts* opts, double* R_host, int32_t* steps_host,
                        double* neg_mass_before_host, double* neg_mass_after_host);

/* ---- generalized rotation (the appendix section on exact NMF: eq5, its split
 * form eq:admm_form_2 and Algorithm alg:rsr) ----
 * Orthogonal R1, R2 and a positive diagonal Lambda minimising the negativity
 * mass sum h(.) of (U R1 Lambda R2, V R1 Lambda^-1 R2), h(q) = max(0, -q), a
 * pair with the same product U V^T.  ADMM on the split variables
 * W1 = [U; V] R1, W2 = [W11 Lambda; W12 Lambda^-1], W3 = W2 R2 with scaled
 * duals M, N, P: per step W3 (prox of h) and W1 (closed form), then R1
 * (Procrustes of [U; V]^T (W1 + M)) and W2 (closed form), then R2 (Procrustes
 * of W2^T (W3 + P)) and each lambda_i (the positive root of the appendix's
 * quartic with the least objective; a column whose U or V part is zero keeps
 * its lambda), then the duals.  rho = gamma = t = rho0 sqrt((m+n) r) / ||[U; V]||_F,
 * start R1 = R2 = I, Lambda = I, W1 = W2 = W3 = [U; V], duals 0.  Stops when
 * |R1' - R1|_F + |R2' - R2|_F + |lambda' - lambda|_2 <= tol, or after
 * max_iter steps (tol = 0 runs exactly max_iter).  All state is float64; one
 * workgroup runs every step in one launch, for the small exact-NMF instances
 * the method is meant for (m + n in the hundreds).  U (m x r) and V (n x r),
 * float32, are replaced in place.  Outputs (host, each may be NULL): R1 and R2
 * (r x r row-major), lambda (r), steps, and the negativity mass before and
 * after.  1 <= r <= ENMF_MAX_RANK.  Workspace: 7 (m + n) KP float64, KP = r
 * padded to 16, 32 or 64.  Synchronises the stream. */
typedef struct {
  double rho0;        /* default 1.0 */
  double tol;         /* default 1e-10 */
  int32_t max_iter;   /* default 500 */
  int32_t reserved;
} enmf_grot_opts;

enmf_status enmf_rotate_general(enmf_ctx* ctx, int64_t m, int64_t n, int32_t r, float* U, float* V,
                                const enmf_grot_opts* opts, double* R1_host, double* lambda_host,
                                double* R2_host, int32_t* steps_host, double* neg_mass_before_host,
                                double* neg_mass_after_host);

/* ---- blocks (iii)-(iv): exterior phase and HALS (sections 3.2-3.3, Algorithms 2-3) ----
 * One iteration = U half then V half (the V half uses the new U, eq. t_i).
 * Phase per iteration: EXT while U or V has a negative entry (push negatives
 * by step_u / step_v, eq. negup; mask of nonnegative entries; PBCD sweeps with
 * the optimal row step, eqs. pbcdu and d_i), else HALS (one Gauss-Seidel
 * sweep over columns per half).  The state after k iterations is checked when
 * k is a multiple of check_every and at k = max_iter; the run stops early when
 * U, V >= 0 and (kkt <= kkt_tol or relerr - relerr_svd <= relerr_tol).
 * U and V (float32) are updated in place.  trace_dev (optional, device,
 * trace_cap records of ENMF_TRACE_FIELDS float64) receives one record per check. */
typedef struct {
  double step_u, step_v;   /* push sizes; <= 0: max(-min, 0)/(ext_iters - 0.5) of the input */
  double pbcd_eps;         /* PBCD stop: ||M o grad|| < eps ||M o grad_init||; 0 = fixed count */
  double relerr_tol;       /* < 0: off */
  double kkt_tol;          /* < 0: off */
  double relerr_svd;       /* Eckart-Young floor from enmf_svd_init (for relerr_tol and re_paper) */
  int32_t ext_iters;       /* default 10 */
  int32_t pbcd_max_iter;   /* default 5 */
  int32_t max_iter;        /* outer iterations */
  int32_t check_every;     /* default 1 */
  int32_t mode;            /* 0 full eNMF; 1 project to the orthant then HALS; 2 fixed row step
                              1/||G||_F in the exterior phase (step-size ablation); 3 stop once
                              feasible (the ablations of the appendix tables and figure 5) */
  int32_t graph_replay;    /* 0: every kernel is launched directly; 1: the launches of two
                              iterations are captured once per call into a HIP graph (kernel
                              nodes only) and replayed for every later pair.  Same results bit
                              for bit.  Ignored by enmf_enmc_iterate and served requests. */
} enmf_iter_opts;

typedef struct {
  int32_t iters, ext_iters_done, phase, converged;
  double step_u, step_v;    /* resolved push sizes (pass them back to resume identically) */
  double f, relerr, re_paper, kkt, kkt_feas, kkt_pg_u, kkt_pg_v, delta_w, sigma_w;
} enmf_iter_report;

/* Trace record: k, f (expanded form), relerr, kkt, min(U,V), phase, device time (ns), negatives. */
#define ENMF_TRACE_FIELDS 8

enmf_status enmf_iterate(enmf_ctx* ctx, const enmf_matrix* X, int32_t r, float* U, float* V,
                         const enmf_iter_opts* opts, enmf_iter_report* report_host,
                         double* trace_dev, int32_t trace_cap);

/* ---- KKT check (appendix, eq. kkt-nmf; (delta_W, sigma_W) of the KKT table) ----
 * f = 1/2 ||X - U V^T||^2 summed directly in float64; relerr = sqrt(2f)/||X||;
 * re_paper = relerr / relerr_svd (NaN when relerr_svd <= 0); gradients
 * grad_U = U V^T V - X V, grad_V = V U^T U - X^T U; projected gradient (grad
 * where W > 0, min(grad, 0) where W <= 0); kkt_pg_u = ||pg_U||/(||X|| ||V||),
 * kkt_pg_v = ||pg_V||/(||X|| ||U||), kkt_feas = max ||min(W,0)||/||W||,
 * kkt = max of the three; delta_w = max(grad o W), sigma_w = sum(grad o W). */
typedef struct {
  double f, relerr, re_paper, kkt, kkt_feas, kkt_pg_u, kkt_pg_v;
  double delta_w, sigma_w, sigma_u, sigma_v, min_w;
} enmf_kkt;

enmf_status enmf_objective_kkt(enmf_ctx* ctx, const enmf_matrix* X, int32_t r, const float* U,
                               const float* V, double relerr_svd, enmf_kkt* out_host);

/* ---- sparse X (the sparse text collections of the experiments section and
 * the large sparse Reuters table, 97% to 99.84% zeros) ----
 * The method reads X only through X V, X^T U, ||X||_F^2 and the objective,
 * so a sparse X runs every call that takes an enmf_matrix except the eNMC
 * calls, enmf_convert and the server: enmf_xv, enmf_xtu, enmf_svd_init,
 * enmf_iterate, enmf_objective_kkt and the instrumentation.  Its products
 * accumulate in float32 in storage order (rows longer than 1024 nonzeros in
 * pieces of 1024, summed in order), with the same result on every run.  The
 * objective of a sparse X is evaluated in the expanded form
 * f = 1/2 (sum over the nonzeros of x (x - 2 u_i . v_j) + <U^T U, V^T V>)
 * in float64, whose rounding error is of order 1e-16 (||X||^2 + ||U V^T||^2)
 * rather than 1e-16 f.
 *
 * enmf_sparse_create copies X, given in compressed-sparse-row form in host
 * memory, to the context's device, in that form and transposed (compressed
 * columns), plus the work partition of the products.  rowptr_host: m + 1
 * offsets, rowptr[0] = 0, nondecreasing, rowptr[m] = nnz.  colind_host: nnz
 * column indices, strictly increasing within each row (no duplicates), in
 * [0, n).  vals_host: nnz finite values (X >= 0 is the caller's contract).
 * 1 <= m, n < 2^31, nnz >= 0.  The handle owns its device copies (about
 * 16 nnz + 16 (m + n) bytes) and keeps no pointer to the host arrays; it can
 * be used by any context on its device until enmf_sparse_destroy, which must
 * not be called while work that reads it is still queued.  ENMF_EINVAL for
 * a malformed matrix (the first offending row in enmf_last_error),
 * ENMF_ENOMEM if the device copies do not fit.  Synchronises the context's
 * stream.  *out is NULL on failure. */
typedef struct enmf_sparse enmf_sparse;

enmf_status enmf_sparse_create(enmf_ctx* ctx, int64_t m, int64_t n, int64_t nnz,
                               const int64_t* rowptr_host, const int32_t* colind_host,
                               const float* vals_host, enmf_sparse** out);

/* Free the device copies of a sparse X (NULL is ignored). */
void enmf_sparse_destroy(enmf_sparse* sp);

/* Exterior nonnegative matrix completion (eNMC; the appendix "Exterior NMC
 * algorithm").  fhat(U, V) = 1/2 ||M o (X - U V^T)||_F^2 over the entries
 * marked observed in M, with grad_U = (M o (U V^T - X)) V and
 * grad_V = (M o (U V^T - X))^T U.
 *
 * X: float32 (ENMF_F32 only).  The mask is one bit per entry, row-major:
 * bit (j % 32) of word bits[i * ld_words + j / 32] is 1 when X[i][j] is
 * observed; ld_words >= ceil(n / 32).  Unobserved entries of X are never
 * read as data (they may hold anything, NaN included). */
typedef struct {
  const uint32_t* bits;    /* device */
  int64_t ld_words;
} enmf_mask;

/* Line 2 of Algorithm eNMC: the rank-r randomized SVD (as enmf_svd_init) of
 * the zero-filled M o X, then als_iters softImpute-ALS iterations at
 * lambda = 0: U <- U + R_U (V^T V)^-1 with R_U = (M o (X - U V^T)) V, then the
 * same for V with the new U (an EM step on the imputed matrix).  U (m x r) and
 * V (n x r) are caller-owned device outputs.  fhat_host (optional) receives
 * fhat at the result.  Uses a workspace copy of M o X (m x n float32).
 * ENMF_ENUMERIC if a Gram is singular. */
enmf_status enmf_enmc_init(enmf_ctx* ctx, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                           const enmf_svd_opts* svd, int32_t als_iters, float* U, float* V,
                           double* fhat_host);

/* The masked gradients of fhat at (U, V): gU (m x r) = (M o (U V^T - X)) V
 * and gV (n x r) = (M o (U V^T - X))^T U, float32 accumulate in a fixed order
 * (either output may be NULL), and fhat (host, optional).  Synchronises. */
enmf_status enmf_enmc_grad(enmf_ctx* ctx, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                           const float* U, const float* V, float* gU, float* gV, double* fhat_host);

/* The loop of Algorithm eNMC from rotated factors (enmf_rotate): every
 * iteration pushes the negative entries of U by the fixed step (eq. negup;
 * step_u, or resolved as in enmf_iterate), then runs pbcd_max_iter masked
 * PBCD sweeps on U: g = M_U+ o grad_U, row step
 * d_i = |g_i|^2 / sum over observed j of (g_i . v_j)^2, U_i <- (U_i - d_i g_i)_+
 * on M_U+; then the same for V with the new U.  There is no HALS stage.
 * Every iteration is checked first (f, the error over the observed entries
 * |M o (X - U V^T)| / |M o X|, and the normalised KKT residual of enmf.h with
 * the masked gradients); the loop stops when U, V >= 0 and kkt <= kkt_tol, or
 * after max_iter iterations.  Uses opts->max_iter, ext_iters, pbcd_max_iter,
 * kkt_tol, step_u, step_v; the other fields must be zero.  U and V are
 * updated in place.  Synchronises once per iteration. */
enmf_status enmf_enmc_iterate(enmf_ctx* ctx, const enmf_matrix* X, const enmf_mask* M, int32_t r,
                              float* U, float* V, const enmf_iter_opts* opts,
                              enmf_iter_report* report_host);

/* ---- serving (many solves of uneven shape in flight together) ----
 * A server runs Algorithm 3 end to end (randomized SVD init, ADMM rotation,
 * exterior phase and HALS with the KKT check, final objective) for every
 * submitted request.  Requests are admitted into slots as slots and device
 * memory free up, and all admitted solves advance together: each tick gives
 * every running solve one workgroup for a bounded time (tick_time_us; the
 * solve yields after the first step that ends past it).  A worker thread replays a captured HIP graph of
 * ticks_per_launch ticks (kernel nodes only) again and again without waiting
 * for it: the slot status is copied to pinned host memory after each replay
 * and read one replay later, and newly admitted solves are uploaded between
 * replays, so requests that arrive while others run join at the next replay
 * and the device never idles on the host.  A solve's arithmetic does not
 * depend on what else is in flight, on the tick time or on the launch form.
 * Served solves take dense X and support r <= 32 and r + oversample <= 48, a fixed number of
 * PBCD sweeps (pbcd_eps = 0) and modes 0 to 3.  The request's trace is
 * not recorded.
 *
 * Wide requests (m n >= wide_min_elems) do not take a slot: each runs as one
 * device-wide solve (the kernels of enmf_svd_init, enmf_rotate and
 * enmf_iterate, whose products spread over every compute unit) on one of
 * wide_lanes host threads, each with its own context and stream, beside the
 * tick loop.  Their workspace lives in those contexts, outside
 * hbm_budget_bytes.  The path a request takes depends only on its shape, so its
 * result still does not depend on what else is in flight.
 *
 * Ownership: X, the omega of svd, U_out and V_out are caller-owned device
 * buffers that must stay valid and untouched until the request has finished
 * (enmf_serve_poll returned something other than ENMF_EBUSY).  U_out and
 * V_out receive the factors (m x r and n x r, float32).  The server owns a
 * device arena of hbm_budget_bytes for the solves' workspace; a request is
 * admitted only when its workspace fits in what is free, and one whose
 * workspace can never fit is refused at submission.  The server uses its
 * own stream on the context's device.  Submit and poll are thread-safe. */
typedef struct enmf_server enmf_server;

typedef struct {
  uint64_t hbm_budget_bytes;  /* device arena for admitted solves' workspace; 0 = 1 GiB */
  int32_t max_slots;          /* solves in flight, one workgroup each; 0 = 1024 */
  int32_t tick_time_us;       /* time a solve runs per tick before it yields, in microseconds of the
                                 device's constant 100 MHz clock (at least one step); 0 = 5000 */
  int32_t ticks_per_launch;   /* ticks per replay of the captured tick graph; 0 = 1 */
  int32_t direct_launch;      /* 0: each group of ticks is one replay of a captured HIP graph;
                                 1: the same kernels launched one by one (no graph) */
  int64_t wide_min_elems;     /* requests with m n at least this run on the device-wide path (below);
                                 0 = 3145728, < 0 = none */
  int32_t wide_lanes;         /* device-wide solves in flight at once; 0 = 2 */
  int32_t reserved;
} enmf_serve_opts;

typedef struct {
  enmf_matrix X;
  int32_t r;
  int32_t reserved;
  enmf_svd_opts svd;          /* omega required (n x (r + oversample)) */
  enmf_rotate_opts rot;
  enmf_iter_opts it;          /* pbcd_eps must be 0; relerr_svd is computed by the server */
  float* U_out;
  float* V_out;
} enmf_request;

/* Start a server on ctx's device (the context itself is not used afterwards
 * and may serve other calls).  ENMF_ENOMEM if the arena cannot be allocated. */
enmf_status enmf_serve_start(enmf_ctx* ctx, const enmf_serve_opts* opts, enmf_server** out);

/* Queue a request without blocking; *ticket identifies it.  ENMF_EINVAL for a
 * bad request, ENMF_ENOMEM if its workspace exceeds hbm_budget_bytes,
 * ENMF_ECLOSED after stop. */
enmf_status enmf_serve_submit(enmf_server* srv, const enmf_request* req, uint64_t* ticket_host);

/* ENMF_EBUSY while the request is queued or running.  Once finished: fills
 * *report_host (iters, phase, f, relerr, kkt, ...; re_paper = relerr /
 * relerr_svd) and *latency_s_host (seconds from submission to completion),
 * returns the solve's status (ENMF_OK, or ENMF_ENUMERIC), and forgets the
 * ticket.  ENMF_EINVAL for an unknown ticket. */
enmf_status enmf_serve_poll(enmf_server* srv, uint64_t ticket, enmf_iter_report* report_host,
                            double* latency_s_host);

/* Stop accepting requests, finish every queued and running one, then free
 * the server (results not yet polled are dropped). */
enmf_status enmf_serve_stop(enmf_server* srv);

/* Text of the server's last failed submit or poll. */
const char* enmf_serve_last_error(const enmf_server* srv);

/* ---- instrumentation ----
 * Average device time (ms) of one launch of the X B and of the X^T A
 * streaming kernels at width k, over `reps` back-to-back launches of each,
 * timed with HIP events on the context stream (operand padding and the
 * split-K reduction are excluded; operands are zero).  Either output may be
 * NULL.  Synchronises the stream. */
enmf_status enmf_time_products(enmf_ctx* ctx, const enmf_matrix* X, int32_t k, int32_t reps,
                               double* xv_ms_host, double* xtu_ms_host);

/* In-solve sampling of the two streaming kernels.  With period > 0, every
 * later enmf_iterate on this context brackets the X V and X^T U kernel
 * launches of every period-th outer iteration with HIP events on the context
 * stream (the events enclose the streaming kernel alone, not the factor
 * packing); period = 0 switches sampling off.  Each call returns the average
 * device time (ms) per sampled launch and the number of samples collected
 * since the previous call, then clears the accumulators.  Outputs may be
 * NULL. */
enmf_status enmf_kernel_timing(enmf_ctx* ctx, int32_t period, double* xv_ms_host,
                               double* xtu_ms_host, int32_t* samples_host);

#ifdef __cplusplus
}
#endif

#endif /* ENMF_H */
