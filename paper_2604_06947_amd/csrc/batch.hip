// batch.hip -- many independent instances advanced by one persistent launch.
//
// Every instance is a scalar problem of its own (flux kind, constants, size,
// boundary, step count).  Instances of int32 cells with n <= 512*128 run in
// the persistent kernel below: a 512-thread workgroup takes one instance at a
// time from a device work counter (longest first), loads all of its cells into
// registers (V consecutive cells per lane, V chosen per instance), advances
// them through every one of the instance's steps, and stores them once.  HBM
// is touched twice per instance, whatever its step count.
//
// Per step each lane needs the cell left of its first cell and right of its
// last one.  Inside a wavefront they arrive by cross-lane moves; across
// wavefronts each wavefront publishes its two edge cells in LDS (double
// buffered by step parity, one barrier per step).  With L = ceil(n/V) lanes
// in use, the last S = L*V - n lanes hold V-1 cells, so every lane's cells
// are contiguous, cell 0 is slot 0 of lane 0 and cell n-1 is the last real
// slot of lane L-1: the boundary neighbours (periodic wrap or outflow copy)
// come from fixed slots, with no data-dependent register indexing.
//
// Instances outside that envelope (int64 cells, larger n, tabulated maps,
// Lax-Friedrichs kinds) run as tiled work items: one launch per step block
// advances every such instance that still has steps in that block, one
// wavefront per (instance, tile), so they progress side by side rather than
// one after another; the launch boundary is the barrier between an
// instance's step blocks.  They run on a stream of their own, beside the
// persistent kernels.  The whole run is captured once into a HIP graph and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace fqnm {
namespace {

constexpr int BT = 512;            // threads of a persistent workgroup (classes 0 and 1)
constexpr int BT2 = 1024;          // threads of a class-2 workgroup
constexpr int BMAXW = BT2 / 64;    // most wavefronts per workgroup
constexpr int64_t BMAXN = int64_t(BT2) * 64;  // largest resident instance (split kinds)
constexpr int64_t BMAXN2 = int64_t(BT2) * 32;  // largest resident instance (two-point kinds)

template <int CLS>
constexpr int threads_of() { return CLS == 2 ? BT2 : BT; }

using BInst = ResidentInst;

template <int POL>
__device__ __forceinline__ void maps32(const XParams& P, int32_t q, int32_t& pp, int32_t& pm) {
  split_maps<int32_t, POL>(P, q, pp, pm);
}

template <int POL, int V, int NW>
__device__ __forceinline__ void run_resident(const BInst& I, int32_t* __restrict__ state,
                                             int32_t* s_first, int32_t* s_last, int32_t* s_q0,
                                             int32_t* s_qn1) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = I.n;
  const int L = (n + V - 1) / V;  // lanes in use
  const int S = L * V - n;        // the last S lanes hold V-1 cells ("short" lanes)
  const int wused = (L + 63) / 64;
  const bool periodic = I.bc == FQNM_BC_PERIODIC;
  const bool active = tid < L;
  const bool shortl = tid >= L - S;
  const int start = tid * V - (tid > L - S ? tid - (L - S) : 0);  // first cell of this lane
  int32_t* st = state + I.off;
  XParams P;
  P.c = I.c;
  P.h = I.h;
  int32_t q[V];
  if (active) {
    // V contiguous cells; the last slot of a short lane reads its right
    // neighbour (or the guard cells behind the instance) and is never stored
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = st[start + j];
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = 0;
  }
  for (int s = 0; s < I.steps; ++s) {
    const int b = s & 1;
    const int32_t mylast = shortl ? q[V - 2 >= 0 ? V - 2 : 0] : q[V - 1];
    if (wave < wused) {
      if (lane == 0) s_first[b * NW + wave] = q[0];
      if (lane == 63) s_last[b * NW + wave] = mylast;
      if (tid == 0) s_q0[b] = q[0];
      if (tid == L - 1) s_qn1[b] = mylast;
    }
    __syncthreads();
    if (wave >= wused) continue;
    int32_t qp = __shfl_up(mylast, 1, 64);
    int32_t qn = __shfl_down(q[0], 1, 64);
    if (lane == 0 && wave > 0) qp = s_last[b * NW + wave - 1];
    if (lane == 63 && wave + 1 < NW) qn = s_first[b * NW + wave + 1];
    if (tid == 0) qp = periodic ? s_qn1[b] : q[0];      // ghost left of cell 0
    if (tid == L - 1) qn = periodic ? s_q0[b] : mylast;  // ghost right of cell n-1
    if constexpr (IsSplit<POL>::value) {
      int32_t ppc, pmc, a, bb;
      maps32<POL>(P, q[0], ppc, pmc);
      maps32<POL>(P, qp, a, bb);
      int32_t Fprev = a + pmc;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        int32_t nxt = j + 1 < V ? q[j + 1] : qn;
        if (j == V - 2) nxt = shortl ? qn : nxt;
        int32_t ppn, pmn;
        maps32<POL>(P, nxt, ppn, pmn);
        const int32_t F = ppc + pmn;
        const int32_t v = wsub<int32_t>(q[j], wsub<int32_t>(F, Fprev));
        q[j] = (j == V - 1 && shortl) ? q[j] : v;
        Fprev = F;
        ppc = ppn;
      }
    } else {
      int32_t Fprev = transfer<int32_t, POL>(P, qp, q[0]);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        int32_t nxt = j + 1 < V ? q[j + 1] : qn;
        if (j == V - 2) nxt = shortl ? qn : nxt;
        const int32_t F = transfer<int32_t, POL>(P, q[j], nxt);
        const int32_t v = wsub<int32_t>(q[j], wsub<int32_t>(F, Fprev));
        q[j] = (j == V - 1 && shortl) ? q[j] : v;
        Fprev = F;
      }
    }
  }
  if (active) {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (j < V - 1 || !shortl) st[start + j] = q[j];
  }
}

// One persistent kernel per class of instance, so that the narrow variants
// are not held to the occupancy of the widest.  Class 0: at most 16384 cells,
// 512 threads, up to 32 cells per lane (86 VGPRs).  Class 1: split kinds of
// 16385..32768 cells, 512 threads, 64 cells per lane (80 VGPRs).  Class 2:
// larger split instances (64 cells per lane) and two-point instances above
// 16384 cells (32 cells per lane), on 1024 threads, so that no variant keeps
// more than 64 cells per lane in registers.  The kernels run side by side and
// each takes the instances of its own class from the shared order.
template <int POL, int CLS>
__device__ __forceinline__ void run_by_vec(const BInst& I, int32_t* state, int32_t* a,
                                           int32_t* b, int32_t* c, int32_t* d) {
  constexpr int NW = threads_of<CLS>() / 64;
  if constexpr (CLS == 2) {
    if constexpr (IsSplit<POL>::value) {
      run_resident<POL, 64, NW>(I, state, a, b, c, d);
    } else {
      run_resident<POL, 32, NW>(I, state, a, b, c, d);
    }
  } else if constexpr (CLS == 1) {
    if constexpr (IsSplit<POL>::value) run_resident<POL, 64, NW>(I, state, a, b, c, d);
  } else {
    switch (I.vec) {
      case 2: run_resident<POL, 2, NW>(I, state, a, b, c, d); break;
      case 4: run_resident<POL, 4, NW>(I, state, a, b, c, d); break;
      case 8: run_resident<POL, 8, NW>(I, state, a, b, c, d); break;
      case 16: run_resident<POL, 16, NW>(I, state, a, b, c, d); break;
      default: run_resident<POL, 32, NW>(I, state, a, b, c, d); break;
    }
  }
}

template <int CLS>
__global__ __launch_bounds__(threads_of<CLS>()) void k_batch_resident(
    const BInst* __restrict__ insts, const int32_t* __restrict__ order, int32_t count,
    int32_t* counter, int32_t* __restrict__ state) {
  constexpr int NW = threads_of<CLS>() / 64;
  __shared__ int32_t s_first[2 * NW], s_last[2 * NW], s_q0[2], s_qn1[2];
  __shared__ int32_t s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
    __syncthreads();
    // uniform: the instance record is read by scalar loads and kept in SGPRs
    const int32_t k = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();
    if (k >= count) return;  // every workgroup leaves once the counter passes the end
    const BInst I = insts[__builtin_amdgcn_readfirstlane(order[k])];
    if (I.cls != CLS) continue;  // another kernel's instance
    switch (I.pol) {
      case P_UPWIND_POS:
        run_by_vec<P_UPWIND_POS, CLS>(I, state, s_first, s_last, s_q0, s_qn1);
        break;
      case P_UPWIND_NEG:
        run_by_vec<P_UPWIND_NEG, CLS>(I, state, s_first, s_last, s_q0, s_qn1);
        break;
      case P_EO: run_by_vec<P_EO, CLS>(I, state, s_first, s_last, s_q0, s_qn1); break;
      case P_GODUNOV: run_by_vec<P_GODUNOV, CLS>(I, state, s_first, s_last, s_q0, s_qn1); break;
      default: run_by_vec<P_MURMAN_ROE, CLS>(I, state, s_first, s_last, s_q0, s_qn1); break;
    }
    __syncthreads();
  }
}

__global__ void k_zero_counter(int32_t* c) {
  if (threadIdx.x < RCLASSES && blockIdx.x == 0) c[threadIdx.x] = 0;
}

bool resident_policy(int pol) {
  return pol == P_UPWIND_POS || pol == P_UPWIND_NEG || pol == P_EO || pol == P_GODUNOV ||
         pol == P_MURMAN_ROE;
}

// cells per lane for an instance of n cells with at most `lanes` lanes in use
int pick_vec(int64_t n, int lanes) {
  for (int v = 2; v < 64; v *= 2)
    if ((n + v - 1) / v <= lanes) return v;
  return 64;
}

bool two_point(int pol) { return pol == P_GODUNOV || pol == P_MURMAN_ROE; }

int64_t resident_max_n(int pol) { return two_point(pol) ? BMAXN2 : BMAXN; }

}  // namespace

bool resident_eligible(const fqnm_problem& p, int pol, int64_t steps) {
  return p.itype == FQNM_I32 && p.n <= resident_max_n(pol) && p.eval != FQNM_EVAL_LUT &&
         resident_policy(pol) && steps <= INT32_MAX;
}

void resident_layout(int64_t n, int pol, int32_t* vec, int32_t* cls) {
  fqnm_batch_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  resident_layout_cfg(n, pol, cfg, vec, cls);
}

void resident_layout_cfg(int64_t n, int pol, const fqnm_batch_config& cfg, int32_t* vec,
                         int32_t* cls) {
  const int64_t c0max = cfg.class0_max_cells ? cfg.class0_max_cells : int64_t(BT) * 32;
  const int lanes = cfg.class0_lanes ? cfg.class0_lanes : BT;
  const bool wide = cfg.wide_split_class != 2;
  if (n <= c0max) {
    *cls = 0;
    *vec = pick_vec(n, lanes);
    if (*vec > 32) *vec = pick_vec(n, BT);  // class 0 keeps at most 32 cells per lane
  } else if (wide && !two_point(pol) && n <= int64_t(BT) * 64) {
    *cls = 1;
    *vec = 64;
  } else {
    *cls = 2;
    *vec = pick_vec(n, BT2);
  }
}

bool batch_config_valid(const fqnm_batch_config& c) {
  if (c.reserved != 0) return false;
  if (c.class0_max_cells < 0 || c.class0_max_cells > BT * 32) return false;
  if (c.class0_lanes != 0 && c.class0_lanes != 128 && c.class0_lanes != 256 &&
      c.class0_lanes != BT)
    return false;
  if (c.wide_split_class < 0 || c.wide_split_class > 2) return false;
  if (c.tiled_vec != 0 && c.tiled_vec != 4 && c.tiled_vec != 8) return false;
  if (c.tiled_depth < 0 || (c.tiled_depth > 0 && c.tiled_vec == 0)) return false;
  if (c.tiled_vec && c.tiled_depth &&
      64 * c.tiled_vec - 2 * scalar_halo(K_TBLOCK, c.tiled_vec, c.tiled_depth) < 2 * c.tiled_vec)
    return false;
  return true;
}

int resident_grid_of(int cls) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipError_t e = cls == 0   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_resident<0>, BT, 0)
                 : cls == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_resident<1>, BT, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_resident<2>, BT2, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return std::max(1, cus * per_cu);
}

void resident_class_counts(const ResidentInst* insts, int32_t count, int32_t* per_class) {
  for (int c = 0; c < RCLASSES; ++c) per_class[c] = 0;
  for (int32_t i = 0; i < count; ++i) ++per_class[insts[i].cls];
}

fqnm_status resident_launcher_init(ResidentLauncher* L) {
  *L = ResidentLauncher{};
  for (int c = 0; c < RCLASSES - 1; ++c)
    if (hipStreamCreateWithFlags(&L->side[c], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L->join[c], hipEventDisableTiming) != hipSuccess)
      return fail(FQNM_ERR_DEVICE, "resident launcher: stream/event creation failed");
  if (hipEventCreateWithFlags(&L->fork, hipEventDisableTiming) != hipSuccess)
    return fail(FQNM_ERR_DEVICE, "resident launcher: event creation failed");
  if (hipMalloc(&L->d_counters, RCLASSES * sizeof(int32_t)) != hipSuccess)
    return fail(FQNM_ERR_OOM, "resident launcher: counter allocation failed");
  return FQNM_OK;
}

void resident_launcher_free(ResidentLauncher* L) {
  for (int c = 0; c < RCLASSES - 1; ++c)
    if (L->side[c]) (void)hipStreamSynchronize(L->side[c]);
  if (L->d_counters) (void)hipFree(L->d_counters);
  if (L->fork) (void)hipEventDestroy(L->fork);
  for (int c = 0; c < RCLASSES - 1; ++c) {
    if (L->join[c]) (void)hipEventDestroy(L->join[c]);
    if (L->side[c]) (void)hipStreamDestroy(L->side[c]);
  }
  *L = ResidentLauncher{};
}

static hipError_t launch_class(int cls, int grid, const ResidentInst* d_insts,
                               const int32_t* d_order, int32_t count, int32_t* counter,
                               int32_t* d_state, hipStream_t s) {
  if (cls == 0)
    k_batch_resident<0><<<dim3(grid), dim3(BT), 0, s>>>(d_insts, d_order, count, counter, d_state);
  else if (cls == 1)
    k_batch_resident<1><<<dim3(grid), dim3(BT), 0, s>>>(d_insts, d_order, count, counter, d_state);
  else
    k_batch_resident<2><<<dim3(grid), dim3(BT2), 0, s>>>(d_insts, d_order, count, counter, d_state);
  return hipGetLastError();
}

hipError_t launch_resident(const ResidentInst* d_insts, const int32_t* d_order, int32_t count,
                           const int32_t* per_class, const ResidentLauncher& L, int32_t* d_state,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_zero_counter<<<1, 64, 0, s>>>(L.d_counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the widest nonempty class runs on the caller's stream and is launched
  // first (its instances are the longest, so its workgroups should take the
  // CUs first); the others run beside it on side streams forked from that
  // stream before it and joined back into it after
  int widest = -1, nonempty = 0;
  for (int cls = 0; cls < RCLASSES; ++cls)
    if (per_class[cls] > 0) {
      widest = cls;
      ++nonempty;
    }
  if (nonempty > 1 && (e = hipEventRecord(L.fork, s)) != hipSuccess) return e;
  if (widest >= 0) {
    const int grid = std::min(resident_grid_of(widest), static_cast<int>(per_class[widest]));
    if ((e = launch_class(widest, grid, d_insts, d_order, count, L.d_counters + widest, d_state,
                          s)) != hipSuccess)
      return e;
  }
  int used = 0;
  for (int cls = widest - 1; cls >= 0; --cls) {
    if (per_class[cls] <= 0) continue;
    hipStream_t st = L.side[used];
    if ((e = hipStreamWaitEvent(st, L.fork, 0)) != hipSuccess) return e;
    const int grid = std::min(resident_grid_of(cls), static_cast<int>(per_class[cls]));
    if ((e = launch_class(cls, grid, d_insts, d_order, count, L.d_counters + cls, d_state, st)) !=
        hipSuccess)
      return e;
    ++used;
  }
  for (int k = 0; k < used; ++k) {
    if ((e = hipEventRecord(L.join[k], L.side[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, L.join[k], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fqnm

using namespace fqnm;

struct fqnm_batch {
  hipStream_t user = nullptr;
  hipStream_t stream = nullptr;  // the library's capture/launch stream
  int32_t count = 0;
  std::vector<fqnm_problem> probs;
  std::vector<int64_t> steps;
  std::vector<int64_t> off;      // element offset of each instance
  std::vector<int> resident;     // 1 if run by the persistent kernel
  int64_t total = 0;             // elements
  void* d_state = nullptr;
  void* d_init = nullptr;
  BInst* d_insts = nullptr;
  int32_t* d_order = nullptr;
  ResidentLauncher launcher;
  int32_t n_resident = 0;
  int32_t n_class[RCLASSES] = {}; // resident instances per persistent kernel
  std::vector<fqnm_ctx*> big;    // single-grid contexts of the tiled instances (their slices,
  std::vector<int64_t> big_steps; // second buffers, tables and constants)
  // tiled work items: grids, per-launch entries, and the launches in order
  TileGrid* d_grids = nullptr;
  BlockGrid* d_entries = nullptr;
  struct TLaunch {
    int itype, pol, vec;
    int64_t entry0;
    int32_t nentries;
    int64_t nitems;
  };
  std::vector<TLaunch> tlaunch;
  std::vector<int32_t> copy_back;  // tiled instances whose last block wrote buf1
  std::vector<BInst> res_base;     // resident instances, before the layout fills vec, cls
  fqnm_batch_config cfg{};         // current layout
  bool direct = false;             // launches issued directly instead of a graph replay
  hipStream_t tstream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<fqnm_ctx*> solo;   // per-instance comparison contexts (created on demand)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool poisoned = false;
};

static size_t esize_of(const fqnm_problem& p) { return p.itype == FQNM_I32 ? 4 : 8; }

static void batch_free(fqnm_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto* c : b->big) fqnm_destroy(c);
  for (auto* c : b->solo) fqnm_destroy(c);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_state) (void)hipFree(b->d_state);
  if (b->d_init) (void)hipFree(b->d_init);
  if (b->d_insts) (void)hipFree(b->d_insts);
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_grids) (void)hipFree(b->d_grids);
  if (b->d_entries) (void)hipFree(b->d_entries);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->tstream) (void)hipStreamDestroy(b->tstream);
  resident_launcher_free(&b->launcher);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

#define B_HIP(call, what)              \
  do {                                 \
    hipError_t e_ = (call);            \
    if (e_ != hipSuccess) {            \
      b->poisoned = true;              \
      return hip_fail(e_, what);       \
    }                                  \
  } while (0)

// The tiled instances' step blocks: every instance takes its context's
// temporally blocked plan (cells per lane 4 or 8; else 4 for int32 and 8 for
// int64 with the default depth), and launch k of a (type, policy, cells per
// lane) group covers the tiles of every instance of the group that has a
// k-th step block.  Block k reads the instance's buffer k mod 2; an
// instance with an odd number of blocks ends in its second buffer and is
// copied back to its slice.
static fqnm_status batch_plan_tiles(fqnm_batch* b, const fqnm_batch_config& cfg) {
  struct G { int itype, pol, vec, depth, khalo; int64_t ntiles, nblocks, steps; };
  b->tlaunch.clear();
  b->copy_back.clear();
  if (b->d_grids) (void)hipFree(b->d_grids);
  if (b->d_entries) (void)hipFree(b->d_entries);
  b->d_grids = nullptr;
  b->d_entries = nullptr;
  std::vector<G> gs;
  std::vector<TileGrid> grids;
  int64_t maxblocks = 0;
  for (size_t i = 0; i < b->big.size(); ++i) {
    fqnm_ctx* c = b->big[i];
    const fqnm_plan dp = default_plan(c->prob, c->pol);
    int vec = c->plan.kernel == K_TBLOCK ? c->plan.vec : dp.vec;
    int depth = c->plan.kernel == K_TBLOCK ? c->plan.depth : dp.depth;
    if (vec != 4 && vec != 8) {  // tiled work items run 4 or 8 cells per lane
      vec = dp.vec == 4 ? 4 : 8;
      depth = dp.depth;
    }
    if (cfg.tiled_vec) vec = cfg.tiled_vec;
    if (cfg.tiled_depth) depth = cfg.tiled_depth;
    int kh = scalar_halo(K_TBLOCK, vec, depth);
    while (64 * vec - 2 * kh < 2 * vec && depth > 1) {  // keep some interior
      depth /= 2;
      kh = scalar_halo(K_TBLOCK, vec, depth);
    }
    if (!items_variant_available(c->prob.itype, c->pol, vec))
      return fail(FQNM_ERR_UNSUPPORTED, "no tiled variant for a batch instance");
    G g{c->prob.itype, c->pol, vec, depth, kh, 0, 0, b->big_steps[i]};
    const int64_t T = 64 * vec - 2 * kh;
    g.ntiles = (c->prob.n + T - 1) / T;
    g.nblocks = (g.steps + depth - 1) / depth;
    maxblocks = std::max(maxblocks, g.nblocks);
    gs.push_back(g);
    TileGrid tg;
    std::memset(&tg, 0, sizeof tg);
    tg.buf0 = c->buf[0];
    tg.buf1 = c->buf[1];
    tg.n = c->prob.n;
    tg.bc = c->prob.bc;
    tg.khalo = kh;
    tg.ledger = c->d_ledger;
    tg.P = c->xp;
    grids.push_back(tg);
    if (g.nblocks & 1) b->copy_back.push_back(static_cast<int32_t>(i));
  }
  // groups in a fixed order: (itype, pol, vec)
  std::vector<std::tuple<int, int, int>> keys;
  for (const G& g : gs) keys.emplace_back(g.itype, g.pol, g.vec);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::vector<BlockGrid> entries;
  for (int64_t k = 0; k < maxblocks; ++k) {
    for (const auto& key : keys) {
      fqnm_batch::TLaunch L{std::get<0>(key), std::get<1>(key), std::get<2>(key),
                            static_cast<int64_t>(entries.size()), 0, 0};
      for (size_t i = 0; i < gs.size(); ++i) {
        const G& g = gs[i];
        if (g.itype != L.itype || g.pol != L.pol || g.vec != L.vec || k >= g.nblocks) continue;
        BlockGrid e;
        std::memset(&e, 0, sizeof e);
        e.first = L.nitems;
        e.grid = static_cast<int32_t>(i);
        e.ksteps = static_cast<int32_t>(std::min<int64_t>(g.depth, g.steps - k * g.depth));
        e.parity = static_cast<int32_t>(k & 1);
        entries.push_back(e);
        L.nitems += g.ntiles;
        ++L.nentries;
      }
      if (L.nentries > 0) b->tlaunch.push_back(L);
    }
  }
  if (hipMalloc(&b->d_grids, sizeof(TileGrid) * grids.size()) != hipSuccess ||
      (!entries.empty() && hipMalloc(&b->d_entries, sizeof(BlockGrid) * entries.size()) != hipSuccess))
    return fail(FQNM_ERR_OOM, "batch tile table allocation failed");
  B_HIP(hipMemcpyAsync(b->d_grids, grids.data(), sizeof(TileGrid) * grids.size(),
                       hipMemcpyHostToDevice, b->stream), "copy tile grids");
  if (!entries.empty())
    B_HIP(hipMemcpyAsync(b->d_entries, entries.data(), sizeof(BlockGrid) * entries.size(),
                         hipMemcpyHostToDevice, b->stream), "copy tile entries");
  B_HIP(hipStreamSynchronize(b->stream), "sync");  // the host tables are freed on return
  if (!b->tstream) {
    B_HIP(hipStreamCreateWithFlags(&b->tstream, hipStreamNonBlocking), "stream");
    B_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming), "event");
    B_HIP(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming), "event");
  }
  return FQNM_OK;
}

// The resident instances' table under a layout: cells per lane and class of
// every instance, longest work first.
static fqnm_status batch_plan_resident(fqnm_batch* b, const fqnm_batch_config& cfg) {
  if (b->n_resident == 0) return FQNM_OK;
  std::vector<BInst> insts = b->res_base;
  for (BInst& I : insts) resident_layout_cfg(I.n, I.pol, cfg, &I.vec, &I.cls);
  std::vector<int32_t> order(b->n_resident);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return int64_t(insts[x].n) * insts[x].steps > int64_t(insts[y].n) * insts[y].steps;
  });
  if (!b->d_insts && (hipMalloc(&b->d_insts, sizeof(BInst) * insts.size()) != hipSuccess ||
                      hipMalloc(&b->d_order, sizeof(int32_t) * order.size()) != hipSuccess))
    return fail(FQNM_ERR_OOM, "batch table allocation failed");
  B_HIP(hipMemcpyAsync(b->d_insts, insts.data(), sizeof(BInst) * insts.size(),
                       hipMemcpyHostToDevice, b->stream), "copy batch table");
  B_HIP(hipMemcpyAsync(b->d_order, order.data(), sizeof(int32_t) * order.size(),
                       hipMemcpyHostToDevice, b->stream), "copy batch order");
  B_HIP(hipStreamSynchronize(b->stream), "sync");
  resident_class_counts(insts.data(), b->n_resident, b->n_class);
  return FQNM_OK;
}

static fqnm_status batch_build_graph(fqnm_batch* b);

// Lay the batch out under cfg: tables, tiled launches and the graph.
static fqnm_status batch_configure(fqnm_batch* b, const fqnm_batch_config& cfg) {
  if (!batch_config_valid(cfg)) return fail(FQNM_ERR_ARG, "invalid batch configuration");
  if (b->stream) B_HIP(hipStreamSynchronize(b->stream), "sync");
  fqnm_status st = batch_plan_resident(b, cfg);
  if (!st && !b->big.empty()) st = batch_plan_tiles(b, cfg);
  if (st) return st;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  st = batch_build_graph(b);
  if (!st) b->cfg = cfg;
  return st;
}

// In-process layout cache keyed by the shape of a batch: instance count,
// storage type, resident count and a histogram of log2 sizes (with the
// step counts' total, in powers of two).
static std::mutex g_bcfg_mu;
static std::map<std::string, fqnm_batch_config> g_bcfg;

static std::string batch_shape_key(const fqnm_batch* b) {
  std::vector<int> hist(40, 0);
  double work = 0.0;
  for (int32_t k = 0; k < b->count; ++k) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= b->probs[k].n && lg < 39) ++lg;
    ++hist[lg];
    work += static_cast<double>(b->probs[k].n) * static_cast<double>(b->steps[k]);
  }
  std::string key = "c" + std::to_string(b->count) + "_i" + std::to_string(b->probs[0].itype) +
                    "_r" + std::to_string(b->n_resident) + "_w" +
                    std::to_string(static_cast<int>(std::log2(work + 1.0)));
  for (int i = 0; i < 40; ++i)
    if (hist[i]) key += "_" + std::to_string(i) + ":" + std::to_string(hist[i]);
  return key;
}

static bool lookup_batch_config(const std::string& key, fqnm_batch_config* out) {
  std::lock_guard<std::mutex> g(g_bcfg_mu);
  auto it = g_bcfg.find(key);
  if (it == g_bcfg.end()) return false;
  *out = it->second;
  return true;
}

// The launches of one batched run, on b->stream (the tiled instances on
// their own stream, forked from it and joined back).
static hipError_t batch_issue(fqnm_batch* b) {
  hipError_t e = hipSuccess;
  const bool tiled = !b->tlaunch.empty() || !b->copy_back.empty();
  if (tiled) {
    e = hipEventRecord(b->ev_fork, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->tstream, b->ev_fork, 0);
  }
  if (e == hipSuccess && b->n_resident > 0)
    e = launch_resident(b->d_insts, b->d_order, b->n_resident, b->n_class, b->launcher,
                        static_cast<int32_t*>(b->d_state), b->stream);
  for (size_t i = 0; i < b->tlaunch.size() && e == hipSuccess; ++i) {
    const auto& L = b->tlaunch[i];
    e = launch_tile_items(L.itype, L.pol, L.vec, b->d_entries + L.entry0, L.nentries, L.nitems,
                          b->d_grids, b->tstream);
  }
  for (size_t i = 0; i < b->copy_back.size() && e == hipSuccess; ++i) {
    const fqnm_ctx* c = b->big[b->copy_back[i]];
    e = launch_copy(c->buf[1], c->buf[0], c->state_bytes(), b->tstream);
  }
  if (tiled && e == hipSuccess) {
    e = hipEventRecord(b->ev_join, b->tstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_join, 0);
  }
  return e;
}

// Capture the run once into a graph (unless the batch issues its launches
// directly, FQNM_BATCH_NO_GRAPH set at create: for profilers that cannot
// follow graph replays).
static fqnm_status batch_build_graph(fqnm_batch* b) {
  if (b->direct) return FQNM_OK;
  B_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  const hipError_t e = batch_issue(b);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); b->poisoned = true; return hip_fail(e, "batch launch"); }
  if (e2 != hipSuccess) { b->poisoned = true; return hip_fail(e2, "end capture"); }
  b->graph = g;
  B_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
  return FQNM_OK;
}

extern "C" {

fqnm_status fqnm_batch_create(const fqnm_problem* probs, const void* const* q0s,
                              const int64_t* steps, int32_t count, void* hip_stream,
                              fqnm_batch** out) {
  if (!out) return fail(FQNM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || !q0s || !steps || count < 1) return fail(FQNM_ERR_ARG, "empty or NULL batch");
  fqnm_batch* b = new fqnm_batch();
  b->user = static_cast<hipStream_t>(hip_stream);
  b->count = count;
  b->direct = std::getenv("FQNM_BATCH_NO_GRAPH") != nullptr;
  b->probs.assign(probs, probs + count);
  b->steps.assign(steps, steps + count);
  // validate and lay out: every instance starts on a 16-byte boundary
  for (int32_t k = 0; k < count; ++k) {
    const fqnm_problem& p = probs[k];
    fqnm_status st = validate_problem(&p);
    if (st == FQNM_OK && is_euler(p.flux)) st = fail(FQNM_ERR_ARG, "batches take scalar kinds");
    if (st == FQNM_OK && (steps[k] < 0 || !q0s[k])) st = fail(FQNM_ERR_ARG, "bad steps or q0");
    if (st == FQNM_OK && p.itype != probs[0].itype)
      st = fail(FQNM_ERR_ARG, "all instances of a batch share one itype");
    if (st) { batch_free(b); return st; }
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int64_t i = 0; i < p.n; ++i) {
      const int64_t v = p.itype == FQNM_I32 ? static_cast<const int32_t*>(q0s[k])[i]
                                            : static_cast<const int64_t*>(q0s[k])[i];
      lo = std::min(lo, v);
      hi = std::max(hi, v);
    }
    st = validate_range(p, lo, hi);
    if (!st) st = validate_drift(p, lo, hi, steps[k]);
    if (st) { batch_free(b); return st; }
    const int64_t per16 = 16 / esize_of(p);
    b->off.push_back(b->total);
    b->total += (p.n + 1 + per16 - 1) / per16 * per16;  // at least one guard cell behind
    const int pol = policy_of(p, false);
    const bool res = resident_eligible(p, pol, steps[k]);
    b->resident.push_back(res ? 1 : 0);
    if (res) {
      BInst I;
      std::memset(&I, 0, sizeof I);
      I.off = b->off.back();
      I.n = static_cast<int32_t>(p.n);
      I.steps = static_cast<int32_t>(steps[k]);
      I.pol = pol;
      I.bc = p.bc;
      XParams x = xparams_of(p);
      I.c = x.c;
      I.h = x.h;
      b->res_base.push_back(I);
    }
  }
  const size_t es = esize_of(probs[0]);
  fqnm_status st = FQNM_OK;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
    st = fail(FQNM_ERR_DEVICE, "stream/event creation failed");
  if (!st && (hipMalloc(&b->d_state, es * b->total) != hipSuccess ||
              hipMalloc(&b->d_init, es * b->total) != hipSuccess))
    st = fail(FQNM_ERR_OOM, "batch state allocation failed");
  if (!st) st = resident_launcher_init(&b->launcher);
  for (int32_t k = 0; k < count && !st; ++k) {
    if (hipMemcpyAsync(static_cast<char*>(b->d_init) + es * b->off[k], q0s[k],
                       es * probs[k].n, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      st = fail(FQNM_ERR_DEVICE, "copy q0");
  }
  if (!st && hipMemcpyAsync(b->d_state, b->d_init, es * b->total, hipMemcpyDeviceToDevice,
                            b->stream) != hipSuccess)
    st = fail(FQNM_ERR_DEVICE, "copy state");
  b->n_resident = static_cast<int32_t>(b->res_base.size());
  // instances outside the resident envelope: single-grid contexts on their slices
  for (int32_t k = 0; k < count && !st; ++k) {
    if (b->resident[k]) continue;
    fqnm_ctx* c = nullptr;
    st = fqnm_create_on_device(&probs[k], static_cast<char*>(b->d_state) + es * b->off[k],
                               b->stream, &c);
    if (!st) {
      b->big.push_back(c);
      b->big_steps.push_back(steps[k]);
    }
  }
  if (!st && hipStreamSynchronize(b->stream) != hipSuccess)
    st = fail(FQNM_ERR_DEVICE, "batch setup sync");
  if (!st) {
    fqnm_batch_config cfg;
    if (!lookup_batch_config(batch_shape_key(b), &cfg)) std::memset(&cfg, 0, sizeof cfg);
    st = batch_configure(b, cfg);
  }
  if (st) { batch_free(b); return st; }
  *out = b;
  return FQNM_OK;
}

fqnm_status fqnm_batch_reset(fqnm_batch* b) {
  if (!b) return fail(FQNM_ERR_ARG, "batch is NULL");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  const size_t es = esize_of(b->probs[0]);
  B_HIP(hipMemcpyAsync(b->d_state, b->d_init, es * b->total, hipMemcpyDeviceToDevice, b->user),
        "reset");
  return FQNM_OK;
}

fqnm_status fqnm_batch_run(fqnm_batch* b) {
  if (!b) return fail(FQNM_ERR_ARG, "batch is NULL");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  B_HIP(hipEventRecord(b->ev_in, b->user), "record");
  B_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0), "wait");
  if (b->direct) B_HIP(batch_issue(b), "batch launch");
  else B_HIP(hipGraphLaunch(b->exec, b->stream), "graph launch");
  B_HIP(hipEventRecord(b->ev_out, b->stream), "record");
  B_HIP(hipStreamWaitEvent(b->user, b->ev_out, 0), "wait");
  return FQNM_OK;
}

fqnm_status fqnm_batch_run_per_instance(fqnm_batch* b) {
  if (!b) return fail(FQNM_ERR_ARG, "batch is NULL");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  const size_t es = esize_of(b->probs[0]);
  if (b->solo.empty()) {
    for (int32_t k = 0; k < b->count; ++k) {
      fqnm_ctx* c = nullptr;
      fqnm_status st = fqnm_create_on_device(&b->probs[k],
                                             static_cast<char*>(b->d_state) + es * b->off[k],
                                             b->user, &c);
      if (st) return st;
      b->solo.push_back(c);
    }
  }
  for (int32_t k = 0; k < b->count; ++k) {
    fqnm_status st = fqnm_step(b->solo[k], b->steps[k]);
    if (st) return st;
  }
  return FQNM_OK;
}

fqnm_status fqnm_batch_get_state(fqnm_batch* b, int32_t idx, void* q_host) {
  if (!b || !q_host) return fail(FQNM_ERR_ARG, "NULL argument");
  if (idx < 0 || idx >= b->count) return fail(FQNM_ERR_ARG, "index out of range");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  const size_t es = esize_of(b->probs[idx]);
  B_HIP(hipStreamSynchronize(b->stream), "sync");
  B_HIP(hipMemcpyAsync(q_host, static_cast<char*>(b->d_state) + es * b->off[idx],
                       es * b->probs[idx].n, hipMemcpyDeviceToHost, b->user), "copy state");
  B_HIP(hipStreamSynchronize(b->user), "sync");
  return FQNM_OK;
}

fqnm_status fqnm_batch_destroy(fqnm_batch* b) {
  batch_free(b);
  return FQNM_OK;
}

fqnm_status fqnm_batch_get_config(fqnm_batch* b, fqnm_batch_config* out) {
  if (!b || !out) return fail(FQNM_ERR_ARG, "NULL argument");
  *out = b->cfg;
  return FQNM_OK;
}

fqnm_status fqnm_batch_set_config(fqnm_batch* b, const fqnm_batch_config* cfg) {
  if (!b || !cfg) return fail(FQNM_ERR_ARG, "NULL argument");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  return batch_configure(b, *cfg);
}

fqnm_status fqnm_batch_autotune(fqnm_batch* b) {
  if (!b) return fail(FQNM_ERR_ARG, "batch is NULL");
  if (b->poisoned) return fail(FQNM_ERR_DEVICE, "batch is poisoned");
  const size_t es = esize_of(b->probs[0]);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  B_HIP(hipEventCreate(&e0), "event");
  B_HIP(hipEventCreate(&e1), "event");
  // one configured run: reset from the initial states, replay, the better of two
  auto trial = [&](const fqnm_batch_config& c, float* ms) -> fqnm_status {
    fqnm_status st = batch_configure(b, c);
    if (st) return st;
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      B_HIP(hipMemcpyAsync(b->d_state, b->d_init, es * b->total, hipMemcpyDeviceToDevice,
                           b->stream), "reset");
      B_HIP(hipEventRecord(e0, b->stream), "record");
      if (b->direct) B_HIP(batch_issue(b), "batch launch");
      else B_HIP(hipGraphLaunch(b->exec, b->stream), "graph launch");
      B_HIP(hipEventRecord(e1, b->stream), "record");
      B_HIP(hipEventSynchronize(e1), "sync");
      float t = 0.f;
      B_HIP(hipEventElapsedTime(&t, e0, e1), "elapsed");
      best = t < best ? t : best;
    }
    *ms = best;
    return FQNM_OK;
  };
  fqnm_batch_config best;
  std::memset(&best, 0, sizeof best);
  float best_ms = 1e30f;
  fqnm_status st = FQNM_OK;
  if (b->n_resident > 0) {
    for (int c0 : {BT * 32, BT * 16})
      for (int lanes : {BT, 256, 128})
        for (int wide : {1, 2}) {
          fqnm_batch_config c = best;
          c.class0_max_cells = c0;
          c.class0_lanes = lanes;
          c.wide_split_class = wide;
          float ms = 0.f;
          if ((st = trial(c, &ms))) break;
          if (ms < best_ms) { best_ms = ms; best = c; }
        }
  }
  if (!st && !b->big.empty()) {
    const fqnm_batch_config base = best;
    best_ms = 1e30f;
    const int cand[][2] = {{0, 0}, {4, 24}, {4, 40}, {8, 24}, {8, 48}};
    for (const auto& vd : cand) {
      fqnm_batch_config c = base;
      c.tiled_vec = vd[0];
      c.tiled_depth = vd[1];
      if (!batch_config_valid(c)) continue;
      float ms = 0.f;
      if ((st = trial(c, &ms))) break;
      if (ms < best_ms) { best_ms = ms; best = c; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!st) st = batch_configure(b, best);
  if (!st && hipMemcpyAsync(b->d_state, b->d_init, es * b->total, hipMemcpyDeviceToDevice,
                            b->stream) != hipSuccess)
    st = fail(FQNM_ERR_DEVICE, "reset");
  if (!st && hipStreamSynchronize(b->stream) != hipSuccess) st = fail(FQNM_ERR_DEVICE, "sync");
  if (st) { b->poisoned = true; return st; }
  std::lock_guard<std::mutex> g(g_bcfg_mu);
  g_bcfg[batch_shape_key(b)] = best;
  return FQNM_OK;
}

}  // extern "C"
