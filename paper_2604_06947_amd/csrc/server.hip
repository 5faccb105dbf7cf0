// server.hip -- continuous batching of solve requests.
//
// A worker thread owns the device stream.  Each tick it
//   1. admits queued requests, oldest first, whose device footprint fits the
//      free space of a preallocated arena (first fit: a smaller request may
//      pass a larger one that does not fit yet), and uploads their q0;
//   2. advances every admitted request by up to `tick_steps` steps:
//        - int32 scalar requests that fit a workgroup: one launch of the
//          register-resident batch kernel for all of them;
//        - Euler requests: launches of the multi-request step kernel, each
//          covering the tiles of every Euler request and advancing them up
//          to 8 steps;
//        - other scalar requests: their single-grid stepper;
//   3. copies finished states to the caller's buffers, stamps completion
//      times and frees their arena blocks.
// Requests that arrive during a tick join at the next one.  A request's
// integer trajectory does not depend on which others share its ticks: every
// kernel reads and writes only that request's own memory, and the integer
// state is the whole state, so splitting its steps across ticks changes
// nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace fqnm;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr size_t ARENA_ALIGN = 256;

// First-fit allocator over one device allocation.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    auto it = free_.emplace(off, n).first;
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
};

enum { R_RESIDENT = 0, R_EULER = 1, R_SINGLE = 2 };

struct SReq {
  uint64_t id = 0;
  fqnm_problem prob{};
  int comp = 1;
  size_t es = 4;
  std::vector<char> q0;
  int64_t steps = 0, done = 0;
  void* out = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = FQNM_OK;
  int path = R_SINGLE;
  int pol = 0;
  size_t bytes = 0, off = 0;
  char* buf[2] = {nullptr, nullptr};
  long long* ledger = nullptr;
  int parity = 0;
  fqnm_ctx* ctx = nullptr;
  int64_t tick_steps = 0;
  bool holds_arena = false;
  int64_t lo = 0, hi = 0;  // range of the initial state (component 0)
};

// Device bytes a request holds while admitted.  The layout inside the block
// is the one upload() builds: Euler = two state buffers, each rounded up to
// 256 bytes, then the 3-word ledger.
size_t state_bytes_rounded(const fqnm_problem& p, size_t es, int comp) {
  const size_t sb = static_cast<size_t>(comp) * static_cast<size_t>(p.n) * es;
  return (sb + 255) / 256 * 256;
}

// Single-grid requests (R_SINGLE) get their whole context -- both state
// buffers, ledger, reduction partials and, in table mode, the table over the
// initial range -- carved from their arena block, so the budget bounds all of
// the device memory the server's requests hold.
size_t footprint(const fqnm_problem& p, int path, size_t es, int comp, int64_t lo, int64_t hi) {
  const size_t n = static_cast<size_t>(p.n);
  if (path == R_RESIDENT) return (n + 4) * es;                           // in place + guard cells
  if (path == R_EULER) return 2 * state_bytes_rounded(p, es, comp) + 256;  // ping-pong + ledger
  return ctx_carved_bytes(p, lo, hi);
}

}  // namespace

struct fqnm_server {
  size_t budget = 0;
  int tick = 64;
  int device = 0;
  hipStream_t stream = nullptr;
  char* arena_base = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SReq*> pending;
  std::vector<SReq*> active;
  std::deque<fqnm_completion> done;
  std::thread worker;
  bool stop = false;
  bool poisoned = false;
  uint64_t next_id = 1;
  fqnm_server_stats stats{};
  // device tables (grown on demand)
  ResidentInst* d_rinst = nullptr;
  int32_t* d_rorder = nullptr;
  ResidentLauncher launcher;
  size_t rcap = 0, ocap = 0;
  EulerReq* d_ereq = nullptr;
  size_t ecap = 0;
  EulerTile* d_etile = nullptr;
  size_t tcap = 0;
  hipEvent_t ev = nullptr;
  std::string err;
};

namespace {

template <typename T>
bool grow(T** p, size_t* cap, size_t need) {
  if (need <= *cap) return true;
  size_t c = std::max<size_t>(need, *cap * 2 + 16);
  T* n = nullptr;
  if (hipMalloc(&n, sizeof(T) * c) != hipSuccess) return false;
  if (*p) (void)hipFree(*p);
  *p = n;
  *cap = c;
  return true;
}

void fail_all(fqnm_server* s, const char* what, hipError_t e) {
  s->poisoned = true;
  s->err = std::string(what) + ": " + hipGetErrorString(e);
}

// Zero a request's ledger and its range flag (the word after the ledger)
// with a tiny kernel (kept off memset nodes).
__global__ void k_zero3(long long* p) {
  if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

// Reserve arena space (worker thread only; cheap host bookkeeping).
bool reserve(fqnm_server* s, SReq* r) {
  r->off = 0;
  if (!s->arena.alloc(r->bytes, &r->off)) return false;
  r->holds_arena = true;
  return true;
}

// Upload q0 into the reserved block and set the request up for ticking.
void upload(fqnm_server* s, SReq* r) {
  char* base = s->arena_base + r->off;
  const size_t sb = r->comp * r->prob.n * r->es;
  hipError_t e = hipSuccess;
  r->buf[0] = base;
  if (r->path == R_EULER) {
    const size_t sbr = state_bytes_rounded(r->prob, r->es, r->comp);
    r->buf[1] = base + sbr;
    r->ledger = reinterpret_cast<long long*>(base + 2 * sbr);
  }
  e = hipMemcpyAsync(base, r->q0.data(), sb, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && r->path == R_EULER) {
    k_zero3<<<1, 64, 0, s->stream>>>(r->ledger);
    e = hipGetLastError();
  }
  if (e == hipSuccess && r->path == R_SINGLE) {
    fqnm_status st = ctx_create_carved(&r->prob, base, r->bytes, s->stream, &r->ctx);
    if (st) r->status = st;  // completes at once with this status
  }
  if (e != hipSuccess) {
    fail_all(s, "admit", e);
    r->status = FQNM_ERR_DEVICE;
  }
  r->parity = 0;
  std::vector<char>().swap(r->q0);  // the host copy is no longer needed
}

// Copy a finished request's state out and release its memory.
void retire(fqnm_server* s, SReq* r) {
  const size_t sb = r->comp * r->prob.n * r->es;
  hipError_t e = hipSuccess;
  if (r->status == FQNM_OK) {
    if (r->path == R_SINGLE) {
      fqnm_status st = fqnm_get_state(r->ctx, r->out);
      if (st) r->status = st;
    } else {
      const char* src = r->path == R_EULER ? r->buf[r->parity] : r->buf[0];
      int flag = 0;
      e = hipMemcpyAsync(r->out, src, sb, hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess && r->path == R_EULER)
        e = hipMemcpyAsync(&flag, r->ledger + 3, sizeof(int), hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) {
        fail_all(s, "retire", e);
        r->status = FQNM_ERR_DEVICE;
      } else if (flag) {
        r->status = FQNM_ERR_RANGE;  // a density or pressure became non-positive
      }
    }
  }
  if (r->ctx) fqnm_destroy(r->ctx);
  r->ctx = nullptr;
  if (r->holds_arena) s->arena.release(r->off, r->bytes);
  r->holds_arena = false;
  r->t_done = now_s();
}

// One tick over the active set; returns false on a device error.
bool run_tick(fqnm_server* s) {
  std::vector<ResidentInst> ri;
  std::vector<int32_t> rorder;
  std::vector<EulerReq> er;
  std::vector<EulerTile> et;
  std::vector<SReq*> singles;
  int emax = 0;
  for (SReq* r : s->active) {
    if (r->status != FQNM_OK) continue;
    r->tick_steps = std::min<int64_t>(s->tick, r->steps - r->done);
    if (r->tick_steps <= 0) continue;
    if (r->path == R_RESIDENT) {
      ResidentInst I;
      std::memset(&I, 0, sizeof I);
      I.off = static_cast<int64_t>((r->buf[0] - s->arena_base) / 4);
      I.n = static_cast<int32_t>(r->prob.n);
      I.steps = static_cast<int32_t>(r->tick_steps);
      I.pol = r->pol;
      resident_layout(r->prob.n, r->pol, &I.vec, &I.cls);
      I.bc = r->prob.bc;
      XParams x = xparams_of(r->prob);
      I.c = x.c;
      I.h = x.h;
      rorder.push_back(static_cast<int32_t>(ri.size()));
      ri.push_back(I);
    } else if (r->path == R_EULER) {
      EulerReq R;
      std::memset(&R, 0, sizeof R);
      R.buf0 = reinterpret_cast<int64_t*>(r->buf[0]);
      R.buf1 = reinterpret_cast<int64_t*>(r->buf[1]);
      R.n = r->prob.n;
      R.bc = r->prob.bc;
      R.steps = static_cast<int32_t>(r->tick_steps);
      R.parity = r->parity;
      R.ledger = r->ledger;
      R.E.delta = r->prob.delta;
      R.E.lambda = r->prob.lambda;
      R.E.g1 = r->prob.gamma - 1.0;
      R.E.fix = r->prob.flux == FQNM_FLUX_EULER_ROE_EF ||
                r->prob.flux == FQNM_FLUX_EULER_ROE_EF_DENSITY;
      R.E.dens = is_euler_density(r->prob.flux);
      R.E.err = reinterpret_cast<int*>(r->ledger + 3);
      const int32_t id = static_cast<int32_t>(er.size());
      er.push_back(R);
      const int64_t nt = euler_tiles(r->prob.n);
      for (int64_t t = 0; t < nt; ++t) et.push_back({id, 0, t * euler_tile_cells()});
      emax = std::max<int>(emax, static_cast<int>(r->tick_steps));
    } else {
      singles.push_back(r);
    }
  }
  hipError_t e = hipSuccess;
  if (!ri.empty()) {
    // longest work first within the tick
    std::stable_sort(rorder.begin(), rorder.end(), [&](int32_t a, int32_t b) {
      return int64_t(ri[a].n) * ri[a].steps > int64_t(ri[b].n) * ri[b].steps;
    });
    if (!grow(&s->d_rinst, &s->rcap, ri.size()) || !grow(&s->d_rorder, &s->ocap, rorder.size())) {
      fail_all(s, "table", hipErrorOutOfMemory);
      return false;
    }
    e = hipMemcpyAsync(s->d_rinst, ri.data(), sizeof(ResidentInst) * ri.size(),
                       hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_rorder, rorder.data(), sizeof(int32_t) * rorder.size(),
                         hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
      int32_t per_class[RCLASSES];
      resident_class_counts(ri.data(), static_cast<int32_t>(ri.size()), per_class);
      e = launch_resident(s->d_rinst, s->d_rorder, static_cast<int32_t>(ri.size()), per_class,
                          s->launcher, reinterpret_cast<int32_t*>(s->arena_base), s->stream);
    }
  }
  if (e == hipSuccess && !er.empty()) {
    if (!grow(&s->d_ereq, &s->ecap, er.size()) || !grow(&s->d_etile, &s->tcap, et.size())) {
      fail_all(s, "table", hipErrorOutOfMemory);
      return false;
    }
    e = hipMemcpyAsync(s->d_ereq, er.data(), sizeof(EulerReq) * er.size(), hipMemcpyHostToDevice,
                       s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_etile, et.data(), sizeof(EulerTile) * et.size(),
                         hipMemcpyHostToDevice, s->stream);
    const int ks = euler_steps_per_launch();
    for (int k = 0; k < emax && e == hipSuccess; k += ks)
      e = launch_euler_multi(s->d_etile, static_cast<int64_t>(et.size()), s->d_ereq, k, s->stream);
  }
  for (SReq* r : singles) {
    fqnm_status st = fqnm_step(r->ctx, r->tick_steps);
    if (st) r->status = st;
  }
  if (e == hipSuccess) e = hipEventRecord(s->ev, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(s->ev);
  if (e != hipSuccess) {
    fail_all(s, "tick", e);
    return false;
  }
  for (SReq* r : s->active) {
    if (r->status != FQNM_OK || r->tick_steps <= 0) continue;
    r->done += r->tick_steps;
    if (r->path == R_EULER) {  // every launch writes the other buffer
      const int64_t ks = euler_steps_per_launch();
      r->parity = static_cast<int>((r->parity + (r->tick_steps + ks - 1) / ks) & 1);
    }
    s->stats.cell_updates += static_cast<double>(r->prob.n) * r->tick_steps;
  }
  s->stats.ticks++;
  return true;
}

void worker_main(fqnm_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    std::vector<SReq*> admitted;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop) break;
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        if (!s->poisoned && reserve(s, *it)) {
          admitted.push_back(*it);
          it = s->pending.erase(it);
        } else {
          ++it;
        }
      }
      if (s->active.empty() && admitted.empty()) {
        s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    for (SReq* r : admitted) {
      upload(s, r);
      r->t_admit = now_s();
      s->active.push_back(r);
    }
    if (s->poisoned) {
      for (SReq* r : s->active) r->status = FQNM_ERR_DEVICE;
    } else {
      run_tick(s);
    }
    std::vector<SReq*> keep, fin;
    for (SReq* r : s->active)
      (r->status != FQNM_OK || r->done >= r->steps ? fin : keep).push_back(r);
    for (SReq* r : fin) retire(s, r);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->active.swap(keep);
      for (SReq* r : fin) {
        fqnm_completion c;
        std::memset(&c, 0, sizeof c);
        c.id = r->id;
        c.status = r->status;
        c.components = r->comp;
        c.n = r->prob.n;
        c.steps = r->done;
        c.t_submit = r->t_submit;
        c.t_admit = r->t_admit;
        c.t_done = r->t_done;
        s->done.push_back(c);
        s->stats.completed++;
        delete r;
      }
      s->stats.active = static_cast<int64_t>(s->active.size());
      s->stats.queued = static_cast<int64_t>(s->pending.size());
      size_t used = 0;
      for (SReq* r : s->active) used += r->bytes;
      s->stats.bytes_in_use = static_cast<int64_t>(used);
      s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, s->stats.bytes_in_use);
      s->stats.admitted += static_cast<int64_t>(admitted.size());
    }
    if (!fin.empty()) s->cv_done.notify_all();
  }
}

void server_free(fqnm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (SReq* r : s->active) {
    if (r->ctx) fqnm_destroy(r->ctx);
    delete r;
  }
  for (SReq* r : s->pending) delete r;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->arena_base) (void)hipFree(s->arena_base);
  if (s->d_rinst) (void)hipFree(s->d_rinst);
  if (s->d_rorder) (void)hipFree(s->d_rorder);
  resident_launcher_free(&s->launcher);
  if (s->d_ereq) (void)hipFree(s->d_ereq);
  if (s->d_etile) (void)hipFree(s->d_etile);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

double fqnm_server_now(void) { return now_s(); }

fqnm_status fqnm_server_create(size_t device_budget_bytes, int32_t tick_steps, void* hip_stream,
                               fqnm_server** out) {
  if (!out) return fail(FQNM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (device_budget_bytes < 4096) return fail(FQNM_ERR_ARG, "budget too small");
  if (tick_steps < 1) return fail(FQNM_ERR_ARG, "tick_steps must be >= 1");
  (void)hip_stream;  // the server owns its stream; results reach callers through host buffers
  fqnm_server* s = new fqnm_server();
  s->budget = device_budget_bytes;
  s->tick = tick_steps;
  (void)hipGetDevice(&s->device);
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) {
    server_free(s);
    return fail(FQNM_ERR_DEVICE, "stream/event creation failed");
  }
  if (hipMalloc(&s->arena_base, device_budget_bytes) != hipSuccess) {
    server_free(s);
    return fail(FQNM_ERR_OOM, "server arena allocation failed");
  }
  if (fqnm_status st = resident_launcher_init(&s->launcher)) {
    server_free(s);
    return st;
  }
  s->arena.init(device_budget_bytes);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return FQNM_OK;
}

fqnm_status fqnm_server_submit(fqnm_server* s, const fqnm_problem* prob, const void* q0_host,
                               int64_t n_steps, void* out_host, uint64_t* req_id) {
  if (!s || !prob || !q0_host || !out_host) return fail(FQNM_ERR_ARG, "NULL argument");
  if (n_steps < 0) return fail(FQNM_ERR_ARG, "n_steps must be >= 0");
  fqnm_status st = validate_problem(prob);
  if (st) return st;
  SReq* r = new SReq();
  r->prob = *prob;
  r->comp = is_euler(prob->flux) ? 3 : 1;
  r->es = prob->itype == FQNM_I32 ? 4 : 8;
  const size_t sb = r->comp * prob->n * r->es;
  r->q0.assign(static_cast<const char*>(q0_host), static_cast<const char*>(q0_host) + sb);
  // range checks on the host copy, as at create
  const int ncheck = is_euler_density(prob->flux) ? 1 : r->comp;  // m, E of density-only are FP64
  for (int c = 0; c < ncheck && st == FQNM_OK; ++c) {
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t i = 0; i < prob->n; ++i) {
      const int64_t v = r->es == 4 ? reinterpret_cast<const int32_t*>(r->q0.data())[i]
                                   : reinterpret_cast<const int64_t*>(r->q0.data())[c * prob->n + i];
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    st = validate_range(*prob, lo, hi);
    if (!st && r->comp == 3 && c == 0 && lo <= 0) st = fail(FQNM_ERR_RANGE, "density must be > 0");
    if (!st && r->comp == 1) st = validate_drift(*prob, lo, hi, n_steps);
    if (c == 0) {
      r->lo = lo;
      r->hi = hi;
    }
  }
  if (st) { delete r; return st; }
  r->steps = n_steps;
  r->out = out_host;
  r->pol = policy_of(*prob, false);
  r->path = r->comp == 3 ? R_EULER
                         : (resident_eligible(*prob, r->pol, n_steps) ? R_RESIDENT : R_SINGLE);
  if (r->path == R_SINGLE && prob->eval == FQNM_EVAL_LUT && r->hi - r->lo + 1 >= (int64_t(1) << 28)) {
    delete r;
    return fail(FQNM_ERR_RANGE, "LUT range too large");
  }
  r->bytes = footprint(*prob, r->path, r->es, r->comp, r->lo, r->hi);
  if (r->bytes > s->budget) {
    delete r;
    return fail(FQNM_ERR_OOM, "request footprint exceeds the server budget");
  }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->poisoned) { delete r; return fail(FQNM_ERR_DEVICE, "server is poisoned: " + s->err); }
    r->id = s->next_id++;
    if (req_id) *req_id = r->id;
    s->pending.push_back(r);
    s->stats.submitted++;
    s->stats.queued = static_cast<int64_t>(s->pending.size());
  }
  s->cv_work.notify_one();
  return FQNM_OK;
}

fqnm_status fqnm_server_poll(fqnm_server* s, fqnm_completion* out, int32_t max, int32_t* n_out) {
  if (!s || !n_out || (max > 0 && !out)) return fail(FQNM_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return FQNM_OK;
}

fqnm_status fqnm_server_drain(fqnm_server* s, double timeout_s) {
  if (!s) return fail(FQNM_ERR_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds(static_cast<int64_t>(timeout_s * 1e6));
  while (s->stats.completed < s->stats.submitted) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
        s->stats.completed < s->stats.submitted)
      return fail(FQNM_ERR_BUSY, "drain timed out");
  }
  return s->poisoned ? fail(FQNM_ERR_DEVICE, "server is poisoned: " + s->err) : FQNM_OK;
}

fqnm_status fqnm_server_stats_get(fqnm_server* s, fqnm_server_stats* out) {
  if (!s || !out) return fail(FQNM_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return FQNM_OK;
}

fqnm_status fqnm_server_destroy(fqnm_server* s) {
  server_free(s);
  return FQNM_OK;
}

}  // extern "C"
