// Host side of the serving loop: admission by device-memory footprint,
// slot assignment, and the launch loop that advances every running solve by
// ticks (k_serve.hip) until it finishes.  One worker thread per server
// drives the device: it replays a captured graph of a few ticks, copies the
// slot status to pinned memory behind it and reads that copy one replay
// later, so the device queue never drains for the host's look.  Wide
// requests bypass the slots: a few lane threads, each with its own context
// and stream, run them one at a time as device-wide solves beside the ticks.
// Submit and poll only touch the queues under the lock.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "enmf_internal.h"
#include "serve_internal.h"

using namespace enmf;

namespace {

using Clock = std::chrono::steady_clock;

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Workspace of one served solve, laid out in its arena block.
struct Layout {
  int64_t y32, qm64, z32, qn64, s, total;
};

Layout layout_for(int64_t m, int64_t n, int kk, int r) {
  Layout L;
  int64_t o = 0;
  L.y32 = o;  o += align256(m * kk * 4);
  L.qm64 = o; o += align256(m * kk * 8);
  L.z32 = o;  o += align256(n * kk * 4);
  L.qn64 = o; o += align256(n * kk * 8);
  L.s = o;    o += align256((m + n) * r * 8);
  L.total = o;
  return L;
}

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
 public:
  explicit Arena(int64_t size) : size_(size) { free_[0] = size; }
  int64_t alloc(int64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t size() const { return size_; }

 private:
  int64_t size_;
  std::map<int64_t, int64_t> free_;
};

struct Pending {
  uint64_t ticket;
  enmf_request req;
  Clock::time_point t_submit;
  int64_t bytes;
};

struct Running {
  bool used = false;
  uint64_t ticket = 0;
  int xt = 0;
  int64_t off = 0, bytes = 0;
  uint64_t admit_seq = 0;     // first replay that runs this solve
  Clock::time_point t_submit;
};

struct Result {
  enmf_status status;
  enmf_iter_report rep;
  double latency_s;
};

}  // namespace

struct enmf_server {
  int device = 0;
  hipStream_t stream = nullptr;
  int max_slots = 1024;
  int64_t tick_limit = 500000;   // constant-clock ticks (10 ns) a slot runs per tick
  char* arena_base = nullptr;
  Arena* arena = nullptr;
  ServeSlot* d_slots = nullptr;
  ServeStatus* d_status = nullptr;
  ServeStatus* h_ring[2] = {nullptr, nullptr};   // pinned status copies of alternate replays
  ServeStatus* h_init = nullptr;     // pinned: the status each newly admitted slot starts from
  ServeSlot* h_stage = nullptr;      // pinned staging of newly admitted slots, one per slot
  ServeAdmit* h_admit[2] = {nullptr, nullptr};   // pinned admission batches, used in turn
  hipEvent_t admit_ev[2] = {nullptr, nullptr};   // recorded after each batch's upload
  int admit_buf = 0;
  ServeAdmit* d_admit = nullptr;     // the batch on the device (one, read in stream order)
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ticks = 4;                     // ticks per replay
  bool direct = false;               // launch the ticks one by one instead of replaying a graph
  hipGraphExec_t graphs[8] = {};     // per set of X storage types in flight (bit per type)
  std::vector<Running> slots;
  std::deque<Pending> pending;
  int64_t wide_min = 3LL << 20;        // m n from which a request runs device-wide (0: never)
  std::vector<hipStream_t> wide_streams;
  std::vector<enmf_ctx*> wide_ctx;     // one context per lane
  std::vector<std::thread> wide_workers;
  std::deque<Pending> wide_pending;
  std::set<uint64_t> wide_running;
  std::condition_variable wcv;
  std::unordered_map<uint64_t, Result> done;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stopping = false;
  bool failed = false;
  std::string err;
  uint64_t next_ticket = 1;
};

namespace {

enmf_status fail_srv(enmf_server* s, enmf_status st, const std::string& msg) {
  s->err = msg;
  return st;
}

void fill_report(const ServeStatus& h, enmf_iter_report* rep) {
  std::memset(rep, 0, sizeof(*rep));
  rep->iters = h.iters;
  rep->ext_iters_done = h.ext_done;
  rep->phase = h.phase;
  rep->converged = h.converged;
  rep->step_u = h.step_u;
  rep->step_v = h.step_v;
  rep->f = h.f;
  rep->relerr = h.relerr;
  rep->re_paper = h.relerr_svd > 0.0 ? h.relerr / h.relerr_svd : NAN;
  rep->kkt = h.kkt;
  rep->kkt_feas = h.kkt_feas;
  rep->kkt_pg_u = h.kkt_pg_u;
  rep->kkt_pg_v = h.kkt_pg_v;
  rep->delta_w = h.delta_w;
  rep->sigma_w = h.sigma_w;
}

// Host image of a newly admitted slot: the request and a fresh state.
void build_slot(enmf_server* s, const Pending& p, int64_t off, ServeSlot* out) {
  const enmf_request& rq = p.req;
  const Layout L = layout_for(rq.X.m, rq.X.n, rq.r + rq.svd.oversample, rq.r);
  std::memset(out, 0, offsetof(ServeSlot, s) + sizeof(ServeScalars));
  ServeReq& q = out->q;
  char* base = s->arena_base + off;
  q.X = rq.X.data;
  q.m = rq.X.m;
  q.n = rq.X.n;
  q.ld = rq.X.ld;
  q.xt = rq.X.dtype;
  q.r = rq.r;
  q.omega = rq.svd.omega;
  q.kk = rq.r + rq.svd.oversample;
  q.power_iters = rq.svd.power_iters;
  q.rho0 = rq.rot.rho0;
  q.rot_tol = rq.rot.tol;
  q.rot_max_iter = rq.rot.max_iter;
  q.rot_check_every = rq.rot.check_every < 1 ? 1 : rq.rot.check_every;
  q.step_u = rq.it.step_u;
  q.step_v = rq.it.step_v;
  q.kkt_tol = rq.it.kkt_tol;
  q.relerr_tol = rq.it.relerr_tol;
  q.ext_iters = rq.it.ext_iters < 1 ? 10 : rq.it.ext_iters;
  q.sweeps = rq.it.pbcd_max_iter < 1 ? 5 : rq.it.pbcd_max_iter;
  q.max_iter = rq.it.max_iter;
  q.check_every = rq.it.check_every < 1 ? 1 : rq.it.check_every;
  q.mode = rq.it.mode;
  q.U = rq.U_out;
  q.V = rq.V_out;
  q.Y32 = reinterpret_cast<float*>(base + L.y32);
  q.Qm64 = reinterpret_cast<double*>(base + L.qm64);
  q.Z32 = reinterpret_cast<float*>(base + L.z32);
  q.Qn64 = reinterpret_cast<double*>(base + L.qn64);
  q.S = reinterpret_cast<double*>(base + L.s);
  out->s.c.stage = kStSvd;
}

void fail_all(enmf_server* s, const std::string& msg) {
  // called with the lock held
  s->failed = true;
  s->err = msg;
  Result r{};
  r.status = ENMF_EDEVICE;
  for (auto& p : s->pending) s->done[p.ticket] = r;
  s->pending.clear();
  for (auto& p : s->wide_pending) s->done[p.ticket] = r;
  s->wide_pending.clear();
  s->wcv.notify_all();
  for (auto& sl : s->slots)
    if (sl.used) {
      s->done[sl.ticket] = r;
      sl.used = false;
    }
  s->cv.notify_all();
}

// The ticks of one replay for the X storage types in `mask`: ticks x (one
// launch per type) over every slot; slots of another type or not running
// return at once, so the sequence does not change with the slots in flight.
hipError_t enqueue_ticks(enmf_server* s, int mask) {
  for (int t = 0; t < s->ticks; ++t)
    for (int xt = 0; xt < 3; ++xt)
      if (mask >> xt & 1) {
        const hipError_t e = launch_serve_tick(xt, s->d_slots, s->d_status, s->max_slots, s->tick_limit,
                                               s->stream);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

// One replay of the tick sequence: the captured graph for this set of
// storage types (captured and instantiated at its first use), or the same
// launches one by one.
hipError_t replay(enmf_server* s, int mask) {
  if (s->direct) return enqueue_ticks(s, mask);
  hipGraphExec_t& ex = s->graphs[mask];
  if (!ex) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = enqueue_ticks(s, mask);
    e = hipStreamEndCapture(s->stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ex = nullptr;
      return e;
    }
  }
  return hipGraphLaunch(ex, s->stream);
}

void worker_loop(enmf_server* s) {
  (void)hipSetDevice(s->device);
  std::vector<int> fresh;
  uint64_t seq = 0;          // replays enqueued so far
  int inflight = -1;         // ring entry of the replay whose status is not read yet
  uint64_t inflight_seq = 0;
  int cur = 0;
  for (;;) {
    int mask = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        // admit in arrival order while a slot and arena space are free
        fresh.clear();
        while (!s->pending.empty() && !s->failed) {
          int slot = -1;
          for (int i = 0; i < s->max_slots; ++i)
            if (!s->slots[i].used) { slot = i; break; }
          if (slot < 0) break;
          const Pending& p = s->pending.front();
          const int64_t off = s->arena->alloc(p.bytes);
          if (off < 0) break;
          Running& r = s->slots[slot];
          r.used = true;
          r.ticket = p.ticket;
          r.xt = p.req.X.dtype;
          r.off = off;
          r.bytes = p.bytes;
          r.t_submit = p.t_submit;
          r.admit_seq = seq;
          build_slot(s, p, off, &s->h_stage[slot]);
          fresh.push_back(slot);
          s->pending.pop_front();
        }
        for (int i = 0; i < s->max_slots; ++i)
          if (s->slots[i].used) mask |= 1 << s->slots[i].xt;
        if (mask || inflight >= 0) break;
        if (s->stopping && s->pending.empty()) return;
        s->cv.wait(lk);
      }
    }
    // upload the new slots and mark them running (ordered before the next
    // replay): one batch copy and one scatter launch, the pinned batch buffer
    // reused once the upload that last read it has run
    hipError_t e = hipSuccess;
    if (!fresh.empty()) {
      const int buf = s->admit_buf;
      s->admit_buf ^= 1;
      e = hipEventSynchronize(s->admit_ev[buf]);
      ServeAdmit* ha = s->h_admit[buf];
      for (size_t i = 0; i < fresh.size(); ++i) {
        const int slot = fresh[i];
        ha[i].slot = slot;
        ha[i].status = s->h_init[slot];
        std::memcpy(ha[i].head, &s->h_stage[slot], kSlotHeadBytes);
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_admit, ha, fresh.size() * sizeof(ServeAdmit), hipMemcpyHostToDevice,
                           s->stream);
      if (e == hipSuccess) e = launch_serve_admit(s->d_admit, (int)fresh.size(), s->d_slots, s->d_status, s->stream);
      if (e == hipSuccess) e = hipEventRecord(s->admit_ev[buf], s->stream);
    }
    int launched = -1;
    if (mask && e == hipSuccess) {
      e = replay(s, mask);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_ring[cur], s->d_status, s->max_slots * sizeof(ServeStatus),
                           hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipEventRecord(s->ev[cur], s->stream);
      if (e == hipSuccess) {
        launched = cur;
        ++seq;
      }
    }
    // read the status of the previous replay (finished, or about to, while
    // this one runs)
    int done_ring = inflight;
    const uint64_t done_seq = inflight_seq;
    if (e == hipSuccess && done_ring >= 0) e = hipEventSynchronize(s->ev[done_ring]);
    inflight = launched;
    inflight_seq = seq - 1;
    if (launched >= 0) cur ^= 1;
    const auto now = Clock::now();
    std::unique_lock<std::mutex> lk(s->mu);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(s->stream);
      (void)hipGetLastError();
      inflight = -1;
      fail_all(s, std::string("serving launch failed: ") + hipGetErrorString(e));
      if (s->stopping) return;
      continue;
    }
    if (done_ring < 0) continue;
    const ServeStatus* hs = s->h_ring[done_ring];
    bool finished = false;
    for (int i = 0; i < s->max_slots; ++i) {
      Running& r = s->slots[i];
      // a slot admitted after that replay still shows its previous occupant
      if (!r.used || r.admit_seq > done_seq || hs[i].status != kSlotDone) continue;
      Result res;
      fill_report(hs[i], &res.rep);
      res.status = hs[i].numeric_error ? ENMF_ENUMERIC : ENMF_OK;
      res.latency_s = std::chrono::duration<double>(now - r.t_submit).count();
      s->done[r.ticket] = res;
      s->arena->release(r.off, r.bytes);
      r.used = false;
      finished = true;
    }
    if (finished) s->cv.notify_all();
  }
}

// One request as a device-wide solve on the lane's context: the randomized
// SVD init, the rotation and the iterations with the request's options (the
// iterations measured against the init's error floor, kernels launched
// directly, no trace).
enmf_status solve_wide(enmf_ctx* c, const enmf_request& q, enmf_iter_report* rep) {
  double rsvd = 0.0;
  enmf_status st = enmf_svd_init(c, &q.X, q.r, &q.svd, q.U_out, q.V_out, nullptr, &rsvd);
  if (st != ENMF_OK) return st;
  st = enmf_rotate(c, q.X.m, q.X.n, q.r, q.U_out, q.V_out, &q.rot, nullptr, nullptr, nullptr, nullptr);
  if (st != ENMF_OK) return st;
  enmf_iter_opts it = q.it;
  it.relerr_svd = rsvd;
  it.graph_replay = 0;
  return enmf_iterate(c, &q.X, q.r, q.U_out, q.V_out, &it, rep, nullptr, 0);
}

// A wide lane: takes wide requests in arrival order until the server stops
// and nothing is left.
void wide_loop(enmf_server* s, int lane) {
  (void)hipSetDevice(s->device);
  enmf_ctx* c = s->wide_ctx[lane];
  for (;;) {
    Pending p;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->wcv.wait(lk, [&] { return !s->wide_pending.empty() || s->stopping; });
      if (s->wide_pending.empty()) return;
      p = s->wide_pending.front();
      s->wide_pending.pop_front();
      s->wide_running.insert(p.ticket);
    }
    Result res{};
    res.status = solve_wide(c, p.req, &res.rep);
    std::string msg = res.status == ENMF_OK ? std::string() : std::string(enmf_last_error(c));
    // the request is reported done only once nothing it queued on the
    // lane's stream can still be running
    const hipError_t e = hipStreamSynchronize(s->wide_streams[lane]);
    if (e != hipSuccess && res.status == ENMF_OK) {
      res.status = ENMF_EDEVICE;
      msg = std::string("wide-lane stream: ") + hipGetErrorString(e);
    }
    res.latency_s = std::chrono::duration<double>(Clock::now() - p.t_submit).count();
    std::lock_guard<std::mutex> lk(s->mu);
    s->wide_running.erase(p.ticket);
    if (!msg.empty()) s->err = msg;
    s->done[p.ticket] = res;
    s->cv.notify_all();
  }
}

enmf_status check_request(enmf_server* s, const enmf_request* q) {
  if (!q) return fail_srv(s, ENMF_EINVAL, "null request");
  const enmf_matrix& X = q->X;
  if (!X.data) return fail_srv(s, ENMF_EINVAL, "X is null");
  if (X.m < 1 || X.n < 1 || X.ld < X.n) return fail_srv(s, ENMF_EINVAL, "bad X shape");
  if (X.dtype != ENMF_F32 && X.dtype != ENMF_BF16 && X.dtype != ENMF_F16)
    return fail_srv(s, ENMF_EINVAL, "unsupported X dtype");
  const int esz = X.dtype == ENMF_F32 ? 4 : 2;
  if (reinterpret_cast<uintptr_t>(X.data) % esz != 0)
    return fail_srv(s, ENMF_EINVAL, "X data must be aligned to its element size");
  if (q->r < 1 || q->r > kServeKP || q->r > X.m || q->r > X.n)
    return fail_srv(s, ENMF_EINVAL, "served solves need 1 <= r <= min(m, n, 32)");
  if (!q->svd.omega) return fail_srv(s, ENMF_EINVAL, "svd.omega is required");
  if (q->svd.oversample < 0 || q->svd.power_iters < 0 || q->r + q->svd.oversample > kServeKK)
    return fail_srv(s, ENMF_EINVAL, "served solves need r + oversample <= 48");
  if (!(q->rot.rho0 > 0.0) || q->rot.max_iter < 0 || q->rot.tol < 0.0)
    return fail_srv(s, ENMF_EINVAL, "bad rotation options");
  const enmf_iter_opts& it = q->it;
  if (it.max_iter < 0) return fail_srv(s, ENMF_EINVAL, "max_iter must be >= 0");
  if (it.pbcd_eps != 0.0) return fail_srv(s, ENMF_EINVAL, "served solves use a fixed PBCD sweep count");
  if (it.mode < 0 || it.mode > 3) return fail_srv(s, ENMF_EINVAL, "unsupported mode");
  if (!q->U_out || !q->V_out) return fail_srv(s, ENMF_EINVAL, "null output pointer");
  return ENMF_OK;
}

}  // namespace

extern "C" {

enmf_status enmf_serve_start(enmf_ctx* c, const enmf_serve_opts* opts, enmf_server** out) {
  if (!out) return ENMF_EINVAL;
  *out = nullptr;
  if (!c) return ENMF_EINVAL;
  enmf_serve_opts o{};
  if (opts) o = *opts;
  if (o.max_slots < 0 || o.tick_time_us < 0 || o.ticks_per_launch < 0 || o.wide_lanes < 0 ||
      (o.direct_launch != 0 && o.direct_launch != 1))
    return ENMF_EINVAL;
  auto* s = new enmf_server();
  s->device = ctx_device(c);
  s->max_slots = o.max_slots > 0 ? o.max_slots : 1024;
  s->tick_limit = (int64_t)(o.tick_time_us > 0 ? o.tick_time_us : 5000) * 100;
  s->ticks = o.ticks_per_launch > 0 ? o.ticks_per_launch : 1;
  s->direct = o.direct_launch == 1;
  s->wide_min = o.wide_min_elems == 0 ? (3LL << 20) : (o.wide_min_elems < 0 ? 0 : o.wide_min_elems);
  const int lanes = s->wide_min > 0 ? (o.wide_lanes > 0 ? o.wide_lanes : 2) : 0;
  const int64_t arena_bytes = o.hbm_budget_bytes > 0 ? (int64_t)o.hbm_budget_bytes : (1LL << 30);
  auto bail = [&](enmf_status st, const char* msg) {
    ctx_set_error(c, msg);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->d_status) (void)hipFree(s->d_status);
    if (s->d_admit) (void)hipFree(s->d_admit);
    if (s->arena_base) (void)hipFree(s->arena_base);
    for (ServeStatus* h : {s->h_ring[0], s->h_ring[1], s->h_init})
      if (h) (void)hipHostFree(h);
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    for (ServeAdmit* h : s->h_admit)
      if (h) (void)hipHostFree(h);
    for (hipEvent_t ev : s->ev)
      if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : s->admit_ev)
      if (ev) (void)hipEventDestroy(ev);
    for (enmf_ctx* wc : s->wide_ctx) enmf_destroy(wc);
    for (hipStream_t ws : s->wide_streams) (void)hipStreamDestroy(ws);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return st;
  };
  if (hipSetDevice(s->device) != hipSuccess) return bail(ENMF_EDEVICE, "hipSetDevice failed");
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(ENMF_EDEVICE, "stream creation failed");
  if (hipMalloc(&s->arena_base, arena_bytes) != hipSuccess) {
    (void)hipGetLastError();
    s->arena_base = nullptr;
    return bail(ENMF_ENOMEM, "serving arena allocation failed");
  }
  if (hipMalloc(&s->d_slots, sizeof(ServeSlot) * s->max_slots) != hipSuccess ||
      hipMalloc(&s->d_status, sizeof(ServeStatus) * s->max_slots) != hipSuccess ||
      hipMalloc(&s->d_admit, sizeof(ServeAdmit) * s->max_slots) != hipSuccess) {
    (void)hipGetLastError();
    return bail(ENMF_ENOMEM, "serving slot allocation failed");
  }
  if (hipHostMalloc(&s->h_ring[0], sizeof(ServeStatus) * s->max_slots) != hipSuccess ||
      hipHostMalloc(&s->h_ring[1], sizeof(ServeStatus) * s->max_slots) != hipSuccess ||
      hipHostMalloc(&s->h_init, sizeof(ServeStatus) * s->max_slots) != hipSuccess ||
      hipHostMalloc(&s->h_stage, sizeof(ServeSlot) * s->max_slots) != hipSuccess ||
      hipHostMalloc(&s->h_admit[0], sizeof(ServeAdmit) * s->max_slots) != hipSuccess ||
      hipHostMalloc(&s->h_admit[1], sizeof(ServeAdmit) * s->max_slots) != hipSuccess) {
    (void)hipGetLastError();
    return bail(ENMF_ENOMEM, "pinned host allocation failed");
  }
  if (hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->admit_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->admit_ev[1], hipEventDisableTiming) != hipSuccess)
    return bail(ENMF_EDEVICE, "event creation failed");
  // every slot starts idle; a newly admitted slot's status is uploaded from h_init
  std::memset(s->h_init, 0, sizeof(ServeStatus) * s->max_slots);
  for (int i = 0; i < s->max_slots; ++i) s->h_init[i].status = kSlotRunning;
  std::memset(s->h_ring[0], 0, sizeof(ServeStatus) * s->max_slots);
  if (hipMemcpy(s->d_status, s->h_ring[0], sizeof(ServeStatus) * s->max_slots,
                hipMemcpyHostToDevice) != hipSuccess)
    return bail(ENMF_EDEVICE, "status initialisation failed");
  for (int l = 0; l < lanes; ++l) {
    hipStream_t ws = nullptr;
    if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess)
      return bail(ENMF_EDEVICE, "stream creation failed");
    s->wide_streams.push_back(ws);
    enmf_ctx* wc = nullptr;
    if (enmf_create(&wc, s->device, ws) != ENMF_OK) return bail(ENMF_EDEVICE, "wide-lane context creation failed");
    s->wide_ctx.push_back(wc);
  }
  s->arena = new Arena(arena_bytes);
  s->slots.resize(s->max_slots);
  s->worker = std::thread(worker_loop, s);
  for (int l = 0; l < lanes; ++l) s->wide_workers.emplace_back(wide_loop, s, l);
  *out = s;
  return ENMF_OK;
}

enmf_status enmf_serve_submit(enmf_server* s, const enmf_request* q, uint64_t* ticket) {
  if (!s || !ticket) return ENMF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail_srv(s, ENMF_ECLOSED, "server is stopping");
  if (s->failed) return fail_srv(s, ENMF_EDEVICE, s->err);
  const enmf_status v = check_request(s, q);
  if (v != ENMF_OK) return v;
  Pending p;
  p.req = *q;
  p.t_submit = Clock::now();
  if (s->wide_min > 0 && q->X.m * q->X.n >= s->wide_min) {
    p.ticket = s->next_ticket++;
    p.bytes = 0;
    s->wide_pending.push_back(p);
    *ticket = p.ticket;
    s->wcv.notify_one();
    return ENMF_OK;
  }
  const int64_t bytes = layout_for(q->X.m, q->X.n, q->r + q->svd.oversample, q->r).total;
  if (bytes > s->arena->size())
    return fail_srv(s, ENMF_ENOMEM, "request workspace exceeds the serving memory budget");
  p.ticket = s->next_ticket++;
  p.bytes = bytes;
  s->pending.push_back(p);
  *ticket = p.ticket;
  s->cv.notify_all();
  return ENMF_OK;
}

enmf_status enmf_serve_poll(enmf_server* s, uint64_t ticket, enmf_iter_report* rep, double* latency_s) {
  if (!s) return ENMF_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    const Result r = it->second;
    s->done.erase(it);
    if (rep) *rep = r.rep;
    if (latency_s) *latency_s = r.latency_s;
    if (r.status == ENMF_EDEVICE) s->err = s->err.empty() ? "device failure" : s->err;
    return r.status;
  }
  for (const auto& p : s->pending)
    if (p.ticket == ticket) return ENMF_EBUSY;
  for (const auto& r : s->slots)
    if (r.used && r.ticket == ticket) return ENMF_EBUSY;
  for (const auto& p : s->wide_pending)
    if (p.ticket == ticket) return ENMF_EBUSY;
  if (s->wide_running.count(ticket)) return ENMF_EBUSY;
  return fail_srv(s, ENMF_EINVAL, "unknown ticket");
}

const char* enmf_serve_last_error(const enmf_server* s) { return s ? s->err.c_str() : "null server"; }

enmf_status enmf_serve_stop(enmf_server* s) {
  if (!s) return ENMF_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  s->wcv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (std::thread& t : s->wide_workers)
    if (t.joinable()) t.join();
  for (enmf_ctx* wc : s->wide_ctx) enmf_destroy(wc);
  const bool failed = s->failed;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (hipGraphExec_t g : s->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  (void)hipFree(s->d_slots);
  (void)hipFree(s->d_status);
  (void)hipFree(s->d_admit);
  (void)hipFree(s->arena_base);
  for (ServeStatus* h : {s->h_ring[0], s->h_ring[1], s->h_init}) (void)hipHostFree(h);
  (void)hipHostFree(s->h_stage);
  for (ServeAdmit* h : s->h_admit) (void)hipHostFree(h);
  for (hipEvent_t ev : s->ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : s->admit_ev) (void)hipEventDestroy(ev);
  for (hipStream_t ws : s->wide_streams) (void)hipStreamDestroy(ws);
  (void)hipStreamDestroy(s->stream);
  delete s->arena;
  delete s;
  return failed ? ENMF_EDEVICE : ENMF_OK;
}

}  // extern "C"
