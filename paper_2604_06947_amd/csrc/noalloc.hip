// noalloc.hip -- exact invariants of a context without allocating device
// memory, for callers that cannot allocate.
//
// fqnm_invariants_get reduces the state into per-block partial records held
// in a buffer the context allocates on its first call.  This variant keeps
// the partial records in a file-scope device array instead: at most
// NOALLOC_BLOCKS records (one block reduces ceil(n / NOALLOC_BLOCKS) cells, at
// least reduce_min_cells_per_block()), plus one combined record per integer
// component, i.e. (4096 + 3) * 48 bytes = 192 KiB per device, held from the
// library's first use of a device until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and that address is what the kernels and copies take.  Every
// call on one device shares the array and it keeps the last call's records,
// so two calls whose kernels overlapped on one device would race on it: the
// library holds a process-wide mutex from a call's first launch to its final
// stream synchronisation, so the calls of one process never overlap (each
// process has its own array).  No slot of the array needs to start at zero:
// every record is written before it is read.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "fqnm_internal.h"
#include "runtime.h"

constexpr int NOALLOC_BLOCKS = 4096;
constexpr int NOALLOC_RECORDS = NOALLOC_BLOCKS + 3;

static __device__ __align__(256) fqnm::ReducePartial scratch[NOALLOC_RECORDS];

namespace {

std::mutex g_mu;
std::vector<fqnm::ReducePartial*> g_ptr;  // per device, null until looked up

// Device address of the scratch array on `device` (current when called).
fqnm_status scratch_address(int device, fqnm::ReducePartial** out) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr.empty()) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return fqnm::hip_fail(e, "hipGetDeviceCount");
    g_ptr.assign(count > 0 ? count : 1, nullptr);
  }
  if (device < 0 || device >= static_cast<int>(g_ptr.size()))
    return fqnm::fail(FQNM_ERR_ARG, "device index out of range");
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fqnm::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_ptr[device] = static_cast<fqnm::ReducePartial*>(p);
  }
  *out = g_ptr[device];
  return FQNM_OK;
}

// Restores the caller's current device on every return path.
struct DeviceGuard {
  int saved = -1;
  bool switched = false;
  hipError_t enter(int device) {
    hipError_t e = hipGetDevice(&saved);
    if (e != hipSuccess) return e;
    if (saved != device) {
      e = hipSetDevice(device);
      if (e != hipSuccess) return e;
      switched = true;
    }
    return hipSuccess;
  }
  ~DeviceGuard() {
    if (switched) (void)hipSetDevice(saved);
  }
};

}  // namespace

using namespace fqnm;

extern "C" fqnm_status fqnm_invariants_get_noalloc(fqnm_ctx* ctx, fqnm_invariants* out) {
  if (!ctx || !out) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->classical) return fail(FQNM_ERR_UNSUPPORTED, "no integer invariants for the FP64 twin");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  const int64_t n = ctx->prob.n;
  const int64_t cpb0 = reduce_min_cells_per_block();
  int64_t cpb = (n + NOALLOC_BLOCKS - 1) / NOALLOC_BLOCKS;
  cpb = cpb < cpb0 ? cpb0 : cpb;
  const int64_t blocks = (n + cpb - 1) / cpb;
  if (blocks < 1 || blocks > NOALLOC_BLOCKS)  // not reachable for n <= 2^36
    return fail(FQNM_ERR_RANGE, "state too large for the static reduction scratch");
  DeviceGuard dg;
  hipError_t e = dg.enter(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "select the context's device");
  ReducePartial* ptr = nullptr;
  fqnm_status st = scratch_address(ctx->device, &ptr);
  if (st) return st;

  std::memset(out, 0, sizeof *out);
  const int ncomp = ctx->euler && ctx->eparams.dens ? 1 : ctx->comp;  // integer components
  out->components = ncomp;
  out->steps_done = ctx->steps_done;
  ReducePartial rec[3];
  long long led[3];
  {
    // the launches and copies below share the device's scratch array
    std::lock_guard<std::mutex> g(g_mu);
    for (int c = 0; c < ncomp; ++c) {
      const char* q = static_cast<const char*>(ctx->buf[ctx->cur]) + c * n * ctx->esize;
      e = launch_reduce_cpb(ctx->prob.itype, q, n, ctx->prob.bc == FQNM_BC_PERIODIC, cpb, ptr,
                            ctx->stream);
      if (e == hipSuccess)
        e = launch_reduce_final(ptr, static_cast<int>(blocks), ptr + NOALLOC_BLOCKS + c,
                                ctx->stream);
      if (e != hipSuccess) {
        ctx->poisoned = true;
        return hip_fail(e, "reduce");
      }
    }
    e = hipMemcpyAsync(rec, ptr + NOALLOC_BLOCKS, sizeof(ReducePartial) * ncomp,
                       hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(led, ctx->d_ledger, sizeof led, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      ctx->poisoned = true;
      return hip_fail(e, "copy invariants");
    }
  }
  for (int c = 0; c < ncomp; ++c) {
    out->sum_hi[c] = rec[c].sum_hi;
    out->sum_lo[c] = rec[c].sum_lo;
    // the 1-D total variation of the flat array means nothing in d-D
    out->tv_hi[c] = ctx->dim > 1 ? 0 : rec[c].tv_hi;
    out->tv_lo[c] = ctx->dim > 1 ? 0 : rec[c].tv_lo;
    out->qmin[c] = rec[c].qmin;
    out->qmax[c] = rec[c].qmax;
    out->ledger[c] = led[c];
  }
  return ctx_check_flag(ctx);
}
