// Device-memory records of the serving loop, shared by the host scheduler
// (serve.cpp) and the serving kernel (k_serve.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace enmf {

constexpr int kServeKP = 32;   // padded factor width of served solves (r <= 32)
constexpr int kServeKK = 48;   // padded range-finder width (r + oversample <= 48)

enum ServeStage { kStSvd = 0, kStRot = 1, kStSetup = 2, kStIter = 3, kStFinal = 4, kStDone = 5 };
enum ServeStatusCode { kSlotIdle = 0, kSlotRunning = 1, kSlotDone = 2, kSlotError = 3 };

// One admitted request, written by the host at admission and read-only on
// the device.  All pointers are device pointers; the workspace pointers
// index the slot's share of the server arena.
struct ServeReq {
  const void* X;
  int64_t m, n, ld;
  int32_t xt, r;
  const float* omega;          // n x kk
  int32_t kk, power_iters;     // kk = r + oversample
  double rho0, rot_tol;
  int32_t rot_max_iter, rot_check_every;
  double step_u, step_v, kkt_tol, relerr_tol;
  int32_t ext_iters, sweeps, max_iter, check_every, mode, pad0;
  float* U;                    // m x r, caller-owned output
  float* V;                    // n x r, caller-owned output
  float* Y32;                  // m x kk (range finder; later P = X V)
  double* Qm64;                // m x kk
  float* Z32;                  // n x kk (range finder; later Q = X^T U)
  double* Qn64;                // n x kk
  double* S;                   // (m + n) x r, rotation state (Y + rho Z)
};

// Scalar progress of one solve (copied to LDS for the length of a tick).
struct ServeScalars {
  int32_t stage, sub, k, iters, rot_steps, ext_done, converged, iphase, numeric_error, pad0;
  double nx2, relerr_svd, rho, dR, step[2];
  double f, relerr, kkt, kkt_feas, kkt_pg_u, kkt_pg_v, delta_w, sigma_w, min_w;
  double recV[8];              // KKT partials of the current V (see CheckAcc)
  double negsV;                // negative entries of the current V
};

// Progress of one solve; survives between ticks.
struct ServeState {
  ServeScalars c;
  double sigma[kServeKP];
  double R[kServeKP * kServeKP];
  double G[kServeKP * kServeKP];   // V^T V of the current V
  double H[kServeKP * kServeKP];   // U^T U of the current U
  double scratch[kServeKK * kServeKK];
};

struct ServeSlot {
  ServeReq q;
  ServeState s;
};

// Compact per-slot status the host reads back after every tick.
struct ServeStatus {
  int32_t status, stage, iters, ext_done, converged, phase, rot_steps, numeric_error;
  double f, relerr, kkt, kkt_feas, kkt_pg_u, kkt_pg_v, delta_w, sigma_w, step_u, step_v, relerr_svd;
};

// Bytes of a slot record the host writes at admission: the request and the
// scalar progress (the rest of the state is written by the solve itself).
constexpr size_t kSlotHeadBytes = offsetof(ServeSlot, s) + sizeof(ServeScalars);
static_assert(kSlotHeadBytes % 8 == 0 && sizeof(ServeStatus) % 8 == 0, "records copied in 8-byte words");

// One newly admitted solve as uploaded in a batch: its slot, its starting
// status and the head of its slot record.
struct ServeAdmit {
  int32_t slot, pad0;
  ServeStatus status;
  unsigned char head[kSlotHeadBytes];
};
static_assert(offsetof(ServeAdmit, status) % 8 == 0 && offsetof(ServeAdmit, head) % 8 == 0 &&
                  sizeof(ServeAdmit) % 8 == 0,
              "admission records copied in 8-byte words");

// Copy `count` staged admissions (device) into their slot records and
// statuses, one workgroup per admission.
hipError_t launch_serve_admit(const ServeAdmit* staged, int count, ServeSlot* slots, ServeStatus* status,
                              hipStream_t s);

// Launch one tick over nslots slots for X stored as xt (ENMF_F32/BF16/F16);
// slots of another storage type or not running are skipped.  A slot runs
// steps until one ends time_limit or more ticks of the device's constant
// 100 MHz clock after the slot started in this tick (at least one step runs).
hipError_t launch_serve_tick(int xt, ServeSlot* slots, ServeStatus* status, int nslots,
                             int64_t time_limit, hipStream_t s);

}  // namespace enmf
