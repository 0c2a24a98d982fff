// Internal declarations shared by the host library and the HIP kernels of libenmf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "enmf.h"

namespace enmf {

// Device-resident scalars of one solve.  Written and read by kernels only;
// the host copies it back once at the end of a call.
struct DevState {
  double nx2;            // ||X||_F^2
  double step[2];        // push sizes for U (0) and V (1)
  double rho;            // ADMM penalty
  double dR;             // ||R_new - R_old||_F of the last ADMM step
  double thr2[2];        // PBCD stop threshold eps^2 ||M o grad_init||^2, per half
  double relerr_svd;
  double ns_per_tick;    // device wall clock period
  double f, relerr, kkt, kkt_feas, kkt_pg_u, kkt_pg_v;
  double delta_w, sigma_w, sigma_u, sigma_v, min_w, re_paper;
  double neg_mass;       // rotation objective of the last rotated point
  double pbcd_eps;
  double kkt_tol, relerr_tol;
  int32_t phase;         // phase of the current iteration (0 EXT, 1 HALS)
  int32_t stop;          // set once the run has stopped; every kernel then returns at once
  int32_t converged;
  int32_t iters;         // completed outer iterations
  int32_t ext_done;
  int32_t pbcd_done[2];
  int32_t ntrace;
  int32_t trace_cap;
  int32_t mode;
  int32_t numeric_error;
  int32_t negs;          // negative entries in U and V at the last head
  int32_t rot_stop;      // set by a rotation step at a check within the tolerance; later steps return
  int32_t rot_steps;     // ADMM steps of the rotation when rot_stop was set
  int32_t check_every;   // check period of the iterate loop
  int32_t kcur;          // outer iteration in progress (published by the U pass's phase decision)
};

// Per-block record written by the row-update kernel (float64 fields):
// negative count of the output rows, PBCD gradient norms before/after the
// sweeps, and kRecChkN KKT-check partials starting at kRecChk (CheckAcc
// order: pg2, sg, mx, ng2, sq, ap, nneg, mn, q).
constexpr int kRecFields = 16;
constexpr int kRecNeg = 0;
constexpr int kRecGi = 1;
constexpr int kRecPg = 2;
constexpr int kRecChk = 4;
constexpr int kRecChkN = 9;
constexpr int kTraceFields = ENMF_TRACE_FIELDS;

// Work selected in one row-update launch (see k_rowupdate).
enum RowFlags {
  kRowUpdate = 1,       // apply the EXT or HALS update
  kRowFirst = 2,        // first launch of the half: push negatives, record |grad_0|
  kRowCheckPre = 4,     // check partials at the input state (else at the output)
  kRowHead = 8,         // decide the phase from the previous records
  kRowWantPg = 16,      // masked gradient norm after the sweeps (PBCD tolerance stop)
  kRowGram = 32,        // partial Gram of the output rows
  kRowWriteCheck = 64,  // write the check partials
  kRowDecide = 128,     // first: the check of iteration k and the stop decision (k_finalize's
                        // work, in every block; block 0 writes the state)
};

// Arguments of the stop decision folded into a row pass (kRowDecide).
struct DecideArgs {
  const double* recU = nullptr;   // check records of U^k (this iteration's U pass)
  int nbU = 0;
  const double* recV = nullptr;   // check records of V^k (the previous V pass)
  int nbV = 0;
  int k = 0, due = 0;     // k < 0: take k from DevState::kcur and due from its check period
  double* trace = nullptr;
};

constexpr int kPhaseExt = 0;
constexpr int kPhaseHals = 1;

// Padded widths the templated kernels are built for.
inline int pad_width(int k) {
  if (k <= 8) return 8;
  if (k <= 16) return 16;
  if (k <= 32) return 32;
  if (k <= 48) return 48;
  if (k <= 64) return 64;
  return 80;
}

// Fixed device scratch of the allocation-free product (static_scratch.hip):
// 64 MiB per device, held until the process ends.  static_scratch_setup takes
// the device's address of the array once (at context creation); static_scratch
// returns it, or null before the set-up.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch_setup(int device);
void* static_scratch(int device);

// Context accessors for the serving front end (api.cpp).
int ctx_device(const enmf_ctx* c);
hipStream_t ctx_stream(const enmf_ctx* c);
void ctx_set_error(enmf_ctx* c, const char* msg);

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All enqueue on `s`, return
// hipSuccess or the launch error.
// ---------------------------------------------------------------------------

// k_stream.hip
int64_t xv_tile_width(int xt);
int xv_splits(int64_t m, int64_t n, int xt);
int xtu_splits(int64_t m, int64_t n);
hipError_t launch_pad_cols(const float* in, int64_t rows, int k, int kp, float* out, hipStream_t s);
hipError_t launch_pad_rows_cols(const float* in, int64_t rows_in, int k, int kp, int64_t rows_out,
                                float* out, hipStream_t s);
hipError_t launch_pad_cols_f64(const float* in, int64_t rows, int k, int kp, double* out,
                               hipStream_t s);
// `reduce` = 0 launches only the streaming kernel (split partials are left in part).
// With reduce = 0 and nsplit != nullptr the product is left as *nsplit
// partials (part when *nsplit > 1, else out) of stride rows * k.

// A Gram combine (gram_combine) a product runs on the side:
// dst (kp x kp) = sum of the nparts partial Grams at src.
struct GramJob {
  const double* src = nullptr;
  int nparts = 0, kp = 0;
  double* dst = nullptr;
};
// With gj, the Gram combine runs as a side job in one more grid row.
hipError_t launch_xv(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* Bp, int k,
                     int kp, int splits, float* part, float* out, hipStream_t s, int reduce = 1,
                     int* nsplit = nullptr, const GramJob* gj = nullptr);
hipError_t launch_xtu(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* Ap, int k,
                      int kp, int splits, float* part, float* out, hipStream_t s, int reduce = 1,
                      int* nsplit = nullptr, const GramJob* gj = nullptr);
hipError_t launch_residual(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const double* Ud,
                           const float* V, int r, double* part, int* nparts, hipStream_t s);
hipError_t launch_sumsq_x(const void* X, int xt, int64_t m, int64_t n, int64_t ld, double* part,
                          int* nparts, hipStream_t s);
hipError_t launch_sum_parts(const double* part, int nparts, int stride, int nfields, double* out,
                            hipStream_t s);
// XT (n x m, leading dimension ldt) = X^T, X of storage type xt.
hipError_t launch_transpose(const void* X, int xt, int64_t m, int64_t n, int64_t ld, void* XT,
                            int64_t ldt, hipStream_t s);
hipError_t launch_convert(const float* x, int64_t m, int64_t n, int64_t ldi, int to, void* out,
                          int64_t ldo, hipStream_t s);

// k_mfma.hip (matrix-core products, k >= 16, float32 or bfloat16 X)
bool mfma_eligible(int xt, int k);
// Packed split-factor layout read by the matrix-core X B (xtu = 0) or X^T A
// (xtu = 1) at width k: padded width, rows per chunk, row pitch (elements).
void mfma_pack_layout(int xt, int xtu, int k, int* kp, int* c, int* ldt);
void mfma_xv_ws(int xt, int64_t m, int64_t n, int k, size_t* pack_bytes, size_t* part_bytes);
void mfma_xtu_ws(int xt, int64_t m, int64_t n, int k, size_t* pack_bytes, size_t* part_bytes);
hipError_t launch_xv_mfma(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* B,
                          int k, void* pack, float* part, float* out, hipStream_t s, int reduce,
                          int do_pack, int* nsplit = nullptr, const int32_t* stop = nullptr,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                          const GramJob* gj = nullptr);
// dec (with st): the check and stop decision of the iteration, taken as a side
// job (the row pass that follows then skips it): by the first block, or for
// bfloat16 X, together with gj's Gram combine, by an extra grid row.
hipError_t launch_xtu_mfma(const void* X, int xt, int64_t m, int64_t n, int64_t ld, const float* A,
                           int k, void* pack, float* part, float* out, hipStream_t s, int reduce,
                           int do_pack, int* nsplit = nullptr, const int32_t* stop = nullptr,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                           const GramJob* gj = nullptr, const DecideArgs* dec = nullptr,
                           DevState* st = nullptr);

// k_small.hip
int gram_blocks(int64_t rows);
hipError_t launch_tsgram(const void* A, int a_is_f64, int64_t lda, const void* B, int b_is_f64,
                         int64_t ldb, int64_t rows, int ka, int kb, double* part, int block_offset,
                         int nblocks, hipStream_t s);
hipError_t launch_gram_finalize(const double* part, int nparts, int ka, int kb, int kp, double* out,
                                hipStream_t s);
hipError_t launch_apply_small(const void* A, int a_is_f64, int64_t lda, int64_t rows, int ka,
                              const double* T, int ldt, int kb, void* out, int out_is_f64,
                              int64_t ldo, hipStream_t s);
hipError_t launch_orth_factor(const double* Gm, int k, double tau, double* T, hipStream_t s);
hipError_t launch_colsum(const double* A, int64_t lda, int64_t rows, int k, double* part, int* nparts,
                         hipStream_t s);
hipError_t launch_svd_factor(const double* C, const double* colsum, int k, int r, double* sigma,
                             double* TU, double* TV, hipStream_t s);
hipError_t launch_pack_w(const float* U, int64_t m, const float* V, int64_t n, int r, int kp,
                         double* W, hipStream_t s);
hipError_t launch_w_sumsq(const double* W, int64_t count, double* part, int* nparts, hipStream_t s);
hipError_t launch_rho_init(const double* part, int nparts, int64_t N, int r, double rho0, DevState* st,
                           hipStream_t s);
// Blocks (and partial Grams) of launch_admm_rows: one per row block, at most 1024.
int admm_rows_blocks(int64_t N, int kp);
// One ADMM step on W (N x kp float64) with the current R: updates the state
// S = Y + rho Z (N x kp float64; not read at step 0) in place and writes
// admm_rows_blocks(N, kp) partials (r x r float64 each) of W^T (Z + Y / rho)
// to part.
hipError_t launch_admm_rows(const double* W, int64_t N, int r, int kp, const double* R, double* S,
                            DevState* st, int step, double* part, hipStream_t s);
// R <- polar factor of Mf (r x r, leading dimension kp); R is kp x kp.
// tol > 0: at steps with (step + 1) % check_every == 0, a change ||R_new - R_old||_F <= tol
// sets st->rot_stop and st->rot_steps = step + 1.
hipError_t launch_polar(const double* Mf, int r, int kp, double* R, DevState* st, hipStream_t s,
                        double tol = 0.0, int check_every = 1, int step = 0);

// k_update.hip
int factor_blocks(int64_t count);
// Padded width of the r x r Grams consumed by the row-update and check kernels.
int row_pad(int r);
// Blocks of a row pass: one per block of rows, at most kRowBlocksMax (the
// blocks then loop over the row blocks).
constexpr int64_t kRowBlocksMax = 1024;
int rowupdate_blocks(int64_t rows, int kp);
// float64 entries of one block's partial Gram at padded width kp.
int gram_part_len(int kp);
hipError_t launch_factor_stats(const float* A, int64_t count, int r, double* part, int block_offset,
                               int nblocks, hipStream_t s);
hipError_t launch_setup_state(const double* statpart, int nbU, int nbV, const double* xpart,
                              int nxpart, double step_u, double step_v, int ext_iters,
                              int check_every, DevState* st, hipStream_t s);
// Destination of the packed split factor a row pass can write for the next
// matrix-core product (layout from mfma_pack_layout); p == nullptr: none.
struct PackOut {
  unsigned short* p = nullptr;
  int kp = 0, c = 0, ldt = 0;
  // the output rows also as float32 rows of the row pass's KP (columns past
  // r zero), the layout the vector-ALU products read
  float* pad = nullptr;
};
// One row pass (flags from RowFlags).  P: nsplit partials of stride pstride.
// rec: kRecFields doubles per block; gpart: gram_part_len(kp) doubles per
// block; headU/headV: the previous records of both halves (kRowHead).
hipError_t launch_rowupdate(const float* A, float* Aout, int64_t rows, int r, int kp, const float* P,
                            int nsplit, int64_t pstride, const double* G, DevState* st, int half,
                            int sweeps, int flags, double* rec, double* gpart, const double* headU,
                            int nbU, const double* headV, int nbV, hipStream_t s,
                            const PackOut& po = PackOut(), const DecideArgs& dec = DecideArgs());
hipError_t launch_gram_fin(const double* gpart, int nparts, int kp, double* out, hipStream_t s);
hipError_t launch_pbcd_decide(const double* rec, int nparts, int half, int first, DevState* st,
                              hipStream_t s);
hipError_t launch_finalize(const DecideArgs& d, int final_check, DevState* st, hipStream_t s);
hipError_t launch_clip(float* A, int64_t count, hipStream_t s);

// ---- sparse X (k_sparse.hip) ----
// One orientation of a sparse X on the device: `rows` compressed rows over
// `cols` columns (CSR of X, or CSR of X^T for the transposed product), and a
// partition of the nonzeros into work items.  Item t covers the nonzeros
// [item_p0[t], item_p1[t]) of row item_row[t]: a piece of the row that stays
// within one panel of kSpPanel columns and holds at most kSpChunk nonzeros.
// A row of one item writes its output row directly (item_slot = -1); the
// items of a longer row write partial rows to slots
// [split_s0[q], split_s0[q + 1]) of a workspace, summed in slot order into row
// split_row[q].  Every row, empty ones too, has at least one item, so every
// output row is written.  Items are stored panel by panel.
constexpr int64_t kSpChunk = 1024;
constexpr int64_t kSpPanel = 65536;
struct SparseForm {
  int64_t rows = 0, cols = 0, nnz = 0;
  int64_t* ptr = nullptr;      // rows + 1
  int32_t* idx = nullptr;      // nnz column indices, increasing within a row
  float* val = nullptr;        // nnz
  int64_t nitems = 0, nslots = 0, nsplit = 0;
  int64_t* item_p0 = nullptr;  // nitems
  int64_t* item_p1 = nullptr;  // nitems
  int32_t* item_row = nullptr;
  int32_t* item_slot = nullptr;
  int32_t* split_row = nullptr;   // nsplit
  int32_t* split_s0 = nullptr;    // nsplit + 1
};
// out (rows x k, leading dimension k) = F B with B (cols x k, leading
// dimension k), float32 accumulation in storage order; part: nslots * k
// floats of workspace.  1 <= k <= 128.
hipError_t launch_spmm(const SparseForm& f, const float* B, int k, float* part, float* out,
                       hipStream_t s);
// The two orientations of one sparse X (enmf_sparse_create).
constexpr uint64_t kSparseMagic = 0x656e6d6673707273ull;
struct SparseX {
  uint64_t magic = kSparseMagic;
  int device = 0;
  SparseForm csr;    // rows of X: X B
  SparseForm csc;    // rows of X^T: X^T A
};
// The sparse X of a matrix descriptor (dtype ENMF_CSR), or null.
const SparseX* sparse_of(const enmf_matrix* X);
// Partial sums (float64) of the squares of the stored values: returns the
// number of partials written to part (at most 1024).
int launch_sparse_sumsq(const SparseForm& f, double* part, hipStream_t s);
// Partials of sum over the nonzeros of x_ij (x_ij - 2 u_i . v_j) in float64
// (U: rows x r, V: cols x r, float32, r <= 64); returns the number written
// (at most kSpCrossBlocks).
constexpr int kSpCrossBlocks = 8192;
int launch_sparse_cross(const SparseForm& f, const float* U, const float* V, int r, double* part,
                        hipStream_t s);
// out[0] = sum of the nparts partials + sum_ab GU[a][b] GV[a][b] (r x r,
// leading dimension r): 2 f for the expanded objective.
hipError_t launch_sparse_objective(const double* part, int nparts, const double* GU,
                                   const double* GV, int r, double* out, hipStream_t s);

// ---- generalized rotation (k_grot.hip) ----
int grot_pad(int r);
// One workgroup runs every ADMM step of Algorithm alg:rsr.  ws: 7 (m + n)
// grot_pad(r) doubles; out: 4 + 2 r^2 + r doubles (negativity mass before,
// after, steps, unused, R1, R2, lambda).
hipError_t launch_grot(const float* U, int64_t m, const float* V, int64_t n, int r, double rho0,
                       double tol, int max_iter, double* ws, float* Uout, float* Vout, double* out,
                       hipStream_t s);

// ---- exterior nonnegative matrix completion (k_enmc.hip) ----
// State of an eNMC solve on the device (scalars of the last check).
struct EnmcState {
  double nx2, f, relerr, kkt, kkt_feas, kkt_pg_u, kkt_pg_v, min_w, negs, negs_u, kkt_tol;
  int32_t iters, stop, converged, numeric_error;
};
// Grid of a masked product: out_tiles 64-row (column) tiles x `splits`
// contraction ranges of tiles_per_split tiles.
struct EnmcPlan {
  int64_t out_tiles = 0;
  int splits = 1, tiles_per_split = 1;
};
EnmcPlan enmc_plan(int64_t m, int64_t n, int cols);
// cols = 0: out = (M o (X - U V^T)) V as plan.splits partials of m x r;
// cols = 1: out = (M o (X - U V^T))^T U as partials of n x r.  rss: one
// double per block (out_tiles x splits), or null.
hipError_t launch_mres(int cols, const float* X, int64_t m, int64_t n, int64_t ld,
                       const uint32_t* bits, int64_t ldm, const float* U, const float* V, int r,
                       float* out, double* rss, hipStream_t s);
// Masked row energies of the PBCD step (partials of m or n doubles).
hipError_t launch_menergy(int cols, int64_t m, int64_t n, const uint32_t* bits, int64_t ldm,
                          const float* U, const float* V, int r, const float* Rp, int nsplit,
                          double* out, hipStream_t s);
int enmc_push_blocks(int64_t count);
hipError_t launch_enmc_push(float* A, int64_t count, double step, double* negs, hipStream_t s);
hipError_t launch_enmc_step(float* A, int64_t rows, int r, const float* Rp, int nsplit,
                            const double* Ep, int esplit, double dfix, hipStream_t s);
hipError_t launch_als_step(float* A, int64_t rows, int r, const float* Rp, int nsplit,
                           const double* Ginv, int kp, hipStream_t s);
hipError_t launch_spd_inverse(const double* G, int r, int kp, double* Ginv, int* bad, hipStream_t s);
hipError_t launch_mask_x(const float* X, int64_t m, int64_t n, int64_t ld, const uint32_t* bits,
                         int64_t ldm, float* out, hipStream_t s);
hipError_t launch_sum_neg(const float* p, int nsplit, int64_t stride, float* out, hipStream_t s);
int enmc_check_blocks(int64_t count);
hipError_t launch_enmc_check(const float* A, int64_t rows, int r, const float* Rp, int nsplit,
                             double* part, hipStream_t s);
hipError_t launch_enmc_finalize(const double* rss, int nrss, const double* cu, int ncu,
                                const double* cv, int ncv, int k, int final_check, EnmcState* st,
                                hipStream_t s);

}  // namespace enmf

// The opaque handle of include/enmf.h.
struct enmf_sparse : enmf::SparseX {};
