// api.hip -- host runtime behind the C ABI of include/fqnm.h: validation,
// device memory, quantisation, LUT construction, the step loop, diagnostics,
// launch plans and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fqnm_internal.h"
#include "runtime.h"

namespace fqnm {

static thread_local std::string tl_error;
void set_error(const std::string& msg) { tl_error = msg; }

fqnm_status fail(fqnm_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

fqnm_status hip_fail(hipError_t e, const char* what) {
  return fail(FQNM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool is_euler(int flux) {
  return flux == FQNM_FLUX_EULER_ROE || flux == FQNM_FLUX_EULER_ROE_EF || is_euler_density(flux);
}
bool is_euler_density(int flux) {
  return flux == FQNM_FLUX_EULER_ROE_DENSITY || flux == FQNM_FLUX_EULER_ROE_EF_DENSITY;
}
bool is_burgers(int flux) {
  return flux == FQNM_FLUX_BURGERS_EO || flux == FQNM_FLUX_BURGERS_GODUNOV ||
         flux == FQNM_FLUX_BURGERS_MURMAN_ROE || flux == FQNM_FLUX_LF_BURGERS;
}
static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

fqnm_status validate_problem(const fqnm_problem* p) {
  if (!p) return fail(FQNM_ERR_ARG, "problem is NULL");
  if (p->abi_version != FQNM_ABI_VERSION) return fail(FQNM_ERR_ARG, "abi_version mismatch");
  if (p->flux < 0 || p->flux > FQNM_FLUX_EULER_ROE_EF_DENSITY)
    return fail(FQNM_ERR_ARG, "unknown flux kind");
  if (p->bc != FQNM_BC_PERIODIC && p->bc != FQNM_BC_OUTFLOW)
    return fail(FQNM_ERR_ARG, "unknown boundary kind");
  if (p->itype != FQNM_I32 && p->itype != FQNM_I64) return fail(FQNM_ERR_ARG, "unknown itype");
  if (p->eval < FQNM_EVAL_AUTO || p->eval > FQNM_EVAL_LUT)
    return fail(FQNM_ERR_ARG, "unknown eval mode");
  if (p->reserved != 0) return fail(FQNM_ERR_ARG, "reserved field must be 0");
  if (!finite_pos(p->delta) || !finite_pos(p->dx) || !finite_pos(p->lambda))
    return fail(FQNM_ERR_ARG, "delta, dx and lambda must be positive and finite");
  if (p->n < 1 || p->n > (int64_t(1) << 36)) return fail(FQNM_ERR_ARG, "n out of range");
  if (!std::isfinite(p->a)) return fail(FQNM_ERR_ARG, "a must be finite");
  if ((p->flux == FQNM_FLUX_LF_LINEAR || p->flux == FQNM_FLUX_LF_BURGERS) && !finite_pos(p->alpha))
    return fail(FQNM_ERR_ARG, "alpha must be positive for Lax-Friedrichs kinds");
  if (is_euler(p->flux)) {
    if (p->itype != FQNM_I64) return fail(FQNM_ERR_ARG, "Euler kinds need FQNM_I64 states");
    if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) return fail(FQNM_ERR_ARG, "gamma must be > 1");
    if (p->eval == FQNM_EVAL_LUT) return fail(FQNM_ERR_ARG, "Euler kinds have no LUT mode");
  }
  if (p->eval == FQNM_EVAL_LUT && p->flux != FQNM_FLUX_UPWIND && p->flux != FQNM_FLUX_BURGERS_EO)
    return fail(FQNM_ERR_ARG, "LUT mode is available for UPWIND and BURGERS_EO only");
  return FQNM_OK;
}

int policy_of(const fqnm_problem& p, bool lut) {
  if (lut) return P_LUT;
  switch (p.flux) {
    case FQNM_FLUX_UPWIND: return p.a >= 0.0 ? P_UPWIND_POS : P_UPWIND_NEG;
    case FQNM_FLUX_BURGERS_EO: return P_EO;
    case FQNM_FLUX_BURGERS_GODUNOV: return P_GODUNOV;
    case FQNM_FLUX_LF_LINEAR: return P_LF_LINEAR;
    case FQNM_FLUX_LF_BURGERS: return P_LF_BURGERS;
    case FQNM_FLUX_BURGERS_MURMAN_ROE: return P_MURMAN_ROE;
    default: return -1;
  }
}

int direct_split_policy(const fqnm_problem& p) {
  return p.flux == FQNM_FLUX_UPWIND ? (p.a >= 0.0 ? P_UPWIND_POS : P_UPWIND_NEG) : P_EO;
}

XParams xparams_of(const fqnm_problem& p) {
  XParams x;
  std::memset(&x, 0, sizeof x);
  x.c = p.a * p.lambda;
  x.h = (p.delta * p.lambda) * 0.5;
  x.a = p.a;
  x.alpha = p.alpha;
  x.delta = p.delta;
  x.lambda = p.lambda;
  return x;
}

// Host bound of |phi+-| on [lo, hi] for the range checks (the maps are monotone,
// so the extremes are at the end points; +1 covers rounding).
static double map_bound(const fqnm_problem& p, int64_t lo, int64_t hi) {
  const double qa = std::max(std::fabs((double)lo), std::fabs((double)hi));
  const double lam = p.lambda, d = p.delta;
  switch (p.flux) {
    case FQNM_FLUX_UPWIND: return std::fabs(p.a * lam) * qa + 1.0;
    case FQNM_FLUX_BURGERS_EO:
    case FQNM_FLUX_BURGERS_GODUNOV:
    case FQNM_FLUX_BURGERS_MURMAN_ROE: return 2.0 * ((d * lam) * 0.5 * qa * qa + 1.0);
    case FQNM_FLUX_LF_LINEAR: return 2.0 * ((std::fabs(p.a) + p.alpha) * 0.5 * lam * qa + 1.0);
    case FQNM_FLUX_LF_BURGERS:
      return 2.0 * ((0.5 * d * qa * qa + p.alpha * qa) * 0.5 * lam + 1.0);
    default: return 0.0;
  }
}

// CFL number of one direction on the state range (Sec. 2.2, eq:cfl_number):
// nu = dt/dx * max|f'| over |q| <= qa.
static fqnm_status cfl_number(const fqnm_problem& p, double qa, double* nu) {
  *nu = 0.0;
  switch (p.flux) {
    case FQNM_FLUX_UPWIND: *nu = std::fabs(p.a) * p.lambda; break;
    case FQNM_FLUX_BURGERS_EO:
    case FQNM_FLUX_BURGERS_GODUNOV:
    case FQNM_FLUX_BURGERS_MURMAN_ROE: *nu = p.lambda * (p.delta * qa); break;
    case FQNM_FLUX_LF_LINEAR:
      if (p.alpha < std::fabs(p.a)) return fail(FQNM_ERR_CFL, "LF needs alpha >= |a|");
      *nu = p.alpha * p.lambda;
      break;
    case FQNM_FLUX_LF_BURGERS:
      if (p.alpha < p.delta * qa) return fail(FQNM_ERR_CFL, "LF needs alpha >= max|u|");
      *nu = p.alpha * p.lambda;
      break;
  }
  return FQNM_OK;
}

static fqnm_status cfl_fail(double nu) {
  char b[128];
  std::snprintf(b, sizeof b, "CFL number %.6g exceeds 1", nu);
  return fail(FQNM_ERR_CFL, b);
}

fqnm_status validate_range(const fqnm_problem& p, int64_t lo, int64_t hi) {
  const double qa = std::max(std::fabs((double)lo), std::fabs((double)hi));
  if (qa >= 4503599627370496.0) return fail(FQNM_ERR_RANGE, "|q| must stay below 2^52");
  // the transfers of 64-bit states convert through the 1.5*2^52 bias
  if (p.itype == FQNM_I64 && qa >= 2251799813685248.0)
    return fail(FQNM_ERR_RANGE, "|q| must stay below 2^51 for int64 states");
  if (is_euler(p.flux)) return FQNM_OK;
  if (is_burgers(p.flux) && qa > 94906265.0)
    return fail(FQNM_ERR_RANGE, "Burgers kinds need q^2 < 2^53 (|q| <= 94906265)");
  double nu = 0.0;
  fqnm_status st = cfl_number(p, qa, &nu);
  if (st) return st;
  if (nu > 1.0) return cfl_fail(nu);
  const double lim = p.itype == FQNM_I32 ? 2147483647.0 : 4611686018427387904.0;
  if (qa + 2.0 * map_bound(p, lo, hi) >= lim)
    return fail(FQNM_ERR_RANGE, "states or transfers would overflow the storage type");
  return FQNM_OK;
}

fqnm_status validate_drift(const fqnm_problem& p, int64_t lo, int64_t hi, int64_t steps) {
  if (p.flux != FQNM_FLUX_LF_LINEAR && p.flux != FQNM_FLUX_LF_BURGERS) return FQNM_OK;
  const int64_t lim = int64_t(1) << 52;
  const int64_t d = steps > lim / 4 ? lim / 2 : 2 * steps;
  const int64_t a = lo - d < -lim ? -lim : lo - d;
  const int64_t b = hi + d > lim ? lim : hi + d;
  fqnm_status st = validate_range(p, a, b);
  if (st)
    set_error("after these steps the Lax-Friedrichs states may leave the checked range (they can "
              "move 2 counts per step past [min q0, max q0]): " + std::string(tl_error));
  return st;
}

// d-D (Thm dimension_extension): the summed CFL number of the directions must
// not exceed 1.  The composed quantised update has no exact maximum principle
// (rounding steps of several directions can add up), so int32 states keep a
// margin of 2^24 counts below the storage limit.
static fqnm_status validate_nd_range(const fqnm_problem* axes, int dim, int64_t lo, int64_t hi) {
  const double qa = std::max(std::fabs((double)lo), std::fabs((double)hi));
  const fqnm_problem& p = axes[0];
  if (qa >= 2251799813685248.0) return fail(FQNM_ERR_RANGE, "|q| must stay below 2^51");
  if (is_burgers(p.flux) && qa > 94906265.0)
    return fail(FQNM_ERR_RANGE, "Burgers kinds need q^2 < 2^53 (|q| <= 94906265)");
  double nu = 0.0, bound = 0.0;
  for (int m = 0; m < dim; ++m) {
    double num = 0.0;
    fqnm_status st = cfl_number(axes[m], qa, &num);
    if (st) return st;
    nu += num;
    bound += 2.0 * map_bound(axes[m], lo, hi);
  }
  if (nu > 1.0) return cfl_fail(nu);
  const double lim = p.itype == FQNM_I32 ? 2147483647.0 - 16777216.0 : 4611686018427387904.0;
  if (qa + bound >= lim)
    return fail(FQNM_ERR_RANGE, "states or transfers would overflow the storage type");
  return FQNM_OK;
}

// ---------------------------------------------------------------------------
// Plans and the in-process autotune cache.
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::string, fqnm_plan> g_tune;

std::string plan_key(const fqnm_problem& p, int pol) {
  char b[160];
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= p.n) ++lg;
  std::snprintf(b, sizeof b, "i%d_p%d_b%d_n2^%d", p.itype, pol, p.bc, lg);
  return b;
}

static void load_tune_file() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* f = std::getenv("FQNM_AUTOTUNE_CACHE");
  if (!f) return;
  FILE* fp = std::fopen(f, "r");
  if (!fp) return;
  char key[160];
  fqnm_plan pl;
  while (std::fscanf(fp, "%159s %d %d %d %d", key, &pl.kernel, &pl.vec, &pl.depth, &pl.eval) == 5)
    g_tune[key] = pl;
  std::fclose(fp);
}

static void save_tune_file() {
  const char* f = std::getenv("FQNM_AUTOTUNE_CACHE");
  if (!f) return;
  FILE* fp = std::fopen(f, "w");
  if (!fp) return;
  for (auto& kv : g_tune)
    std::fprintf(fp, "%s %d %d %d %d\n", kv.first.c_str(), kv.second.kernel, kv.second.vec,
                 kv.second.depth, kv.second.eval);
  std::fclose(fp);
}

bool lookup_plan(const std::string& key, fqnm_plan* out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

void store_plan(const std::string& key, const fqnm_plan& pl) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file();
  g_tune[key] = pl;
  save_tune_file();
}

fqnm_plan default_plan(const fqnm_problem& p, int pol) {
  fqnm_plan pl;
  pl.kernel = K_TBLOCK;
  pl.vec = p.itype == FQNM_I32 ? 4 : 8;
  pl.depth = p.itype == FQNM_I32 && p.eval == FQNM_EVAL_LUT ? 52 : 24;
  if (p.itype == FQNM_I64 && (pol == P_UPWIND_POS || pol == P_UPWIND_NEG)) {
    // 64-bit upwind windows step as exact doubles: wide tiles, deep passes
    pl.vec = 16;
    pl.depth = 48;
  }
  pl.eval = 0;
  return pl;
}

// SIMDs of a device (4 per compute unit), 0 if the runtime does not say.
static int64_t device_simds(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  return 4 * static_cast<int64_t>(cus > 0 ? cus : 0);
}

// A single grid small enough that a pass's wavefronts are about one per SIMD:
// there the extra halo of a deeper pass costs no time, while every pass saved
// saves a kernel boundary (about 3 us), so one solve of 1000 steps on 1024 to
// 65536 cells takes half the time at 96-120 steps per pass as at 24 (a third,
// for 64-bit upwind states, of the time of their wide default windows).  Takes
// the first plan of the list below whose tiles number at most 1.75 per SIMD
// and whose pass is deeper than the default plan's: 4-cell lanes from 120
// steps per pass down to 52, then, for 64-bit upwind states, exact-double
// windows of 16-cell lanes at 200 steps.
static void small_grid_plan(const fqnm_problem& p, int device, fqnm_plan* pl) {
  const int64_t simds = device_simds(device);
  if (simds <= 0) return;
  const bool wide = pl->vec == 16;  // the default of 64-bit upwind states
  static const int cands[][2] = {{4, 120}, {4, 96}, {4, 80}, {4, 64}, {4, 52}, {16, 200}};
  for (const auto& c : cands) {
    if ((c[0] == 16 && !wide) || c[1] <= pl->depth) continue;
    const int64_t T = 64 * c[0] - 2 * static_cast<int64_t>(scalar_halo(K_TBLOCK, c[0], c[1]));
    const int64_t tiles = (p.n + T - 1) / T;
    if (4 * tiles <= 7 * simds) {
      pl->kernel = K_TBLOCK;
      pl->vec = c[0];
      pl->depth = c[1];
      return;
    }
  }
}

}  // namespace fqnm

using namespace fqnm;

// ---------------------------------------------------------------------------
// Context.
// ---------------------------------------------------------------------------
#define CTX_HIP(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) {                        \
      ctx->poisoned = true;                        \
      return hip_fail(e_, what);                   \
    }                                              \
  } while (0)

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Device memory of a context: carved from its block if it has one, else
// allocated.
static bool ctx_dmalloc(fqnm_ctx* ctx, void** p, size_t bytes) {
  if (ctx->carve_base) {
    const size_t off = round256(ctx->carve_used);
    if (off + bytes > ctx->carve_size) return false;
    *p = ctx->carve_base + off;
    ctx->carve_used = off + bytes;
    return true;
  }
  return hipMalloc(p, bytes) == hipSuccess;
}

static void ctx_dfree(fqnm_ctx* ctx, void* p) {
  if (!p) return;
  const char* c = static_cast<const char*>(p);
  if (ctx->carve_base && c >= ctx->carve_base && c < ctx->carve_base + ctx->carve_size) return;
  (void)hipFree(p);
}

static fqnm_status ctx_alloc(fqnm_ctx* ctx, void* borrowed) {
  const size_t bytes = ctx->state_bytes();
  if (borrowed) {
    if ((reinterpret_cast<uintptr_t>(borrowed) & 15) != 0)
      return fail(FQNM_ERR_ARG, "device state must be 16-byte aligned");
    ctx->buf[0] = borrowed;
    ctx->borrowed = true;
  } else if (!ctx_dmalloc(ctx, &ctx->buf[0], bytes)) {
    return fail(FQNM_ERR_OOM, "allocation of the state failed");
  }
  if (!ctx_dmalloc(ctx, &ctx->buf[1], bytes))
    return fail(FQNM_ERR_OOM, "allocation of the second state buffer failed");
  void* led = nullptr;
  if (!ctx_dmalloc(ctx, &led, 3 * sizeof(long long)))
    return fail(FQNM_ERR_OOM, "allocation of the ledger failed");
  ctx->d_ledger = static_cast<long long*>(led);
  CTX_HIP(hipMemsetAsync(ctx->d_ledger, 0, 3 * sizeof(long long), ctx->stream), "ledger reset");
  return FQNM_OK;
}

static void ctx_free(fqnm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream_sync_on_free) (void)hipStreamSynchronize(ctx->stream);
  if (!ctx->borrowed) ctx_dfree(ctx, ctx->buf[0]);
  ctx_dfree(ctx, ctx->buf[1]);
  ctx_dfree(ctx, ctx->d_ledger);
  ctx_dfree(ctx, ctx->d_lut);
  ctx_dfree(ctx, ctx->d_u);
  ctx_dfree(ctx, ctx->d_red);
  ctx_dfree(ctx, ctx->d_err);
  ctx_dfree(ctx, ctx->d_ws);
  ctx_dfree(ctx, ctx->d_exch);
  ctx_dfree(ctx, ctx->d_perr);
  delete ctx;
}

// Exchange buffer and error flag of the persistent plan, grown on demand
// (zeroed: every word carries tag 0, below any pass tag).
static fqnm_status ctx_persist_buffers(fqnm_ctx* ctx, int vec, int depth) {
  int khalo = 0;
  int64_t ntiles = 0;
  if (!persist_geometry(ctx->prob.n, vec, depth, &khalo, &ntiles))
    return fail(FQNM_ERR_ARG, "the grid cannot be tiled for this persistent plan");
  const size_t need = sizeof(uint64_t) * 4 * static_cast<size_t>(ntiles) * khalo;
  if (!ctx->d_perr) {
    void* p = nullptr;
    if (!ctx_dmalloc(ctx, &p, sizeof(int))) return fail(FQNM_ERR_OOM, "allocation failed");
    ctx->d_perr = static_cast<int*>(p);
    CTX_HIP(hipMemsetAsync(ctx->d_perr, 0, sizeof(int), ctx->stream), "flag reset");
  }
  if (ctx->exch_bytes < need) {
    ctx_dfree(ctx, ctx->d_exch);
    ctx->d_exch = nullptr;
    ctx->exch_bytes = 0;
    void* p = nullptr;
    if (!ctx_dmalloc(ctx, &p, need)) return fail(FQNM_ERR_OOM, "allocation of the exchange buffer failed");
    ctx->d_exch = static_cast<uint64_t*>(p);
    ctx->exch_bytes = need;
    ctx->exch_tag = 0;
    CTX_HIP(hipMemsetAsync(ctx->d_exch, 0, need, ctx->stream), "exchange reset");
  }
  return FQNM_OK;
}

static bool persist_plan_ok(fqnm_ctx* ctx, const fqnm_plan& pl) {
  int khalo = 0;
  int64_t ntiles = 0;
  if (ctx->classical || ctx->euler || ctx->dim > 1) return false;
  if (!persist_available(ctx->prob.itype, ctx->pol, pl.vec, ctx->prob.bc)) return false;
  if (!persist_geometry(ctx->prob.n, pl.vec, pl.depth, &khalo, &ntiles)) return false;
  bool fits = false;
  return persist_fits(ctx->pol, pl.vec, ntiles, &fits) == hipSuccess && fits;
}

// Range of component 0 of the current state via the device reduction.
fqnm_status fqnm::ctx_minmax(fqnm_ctx* ctx, int comp, int64_t* lo, int64_t* hi) {
  const int64_t nb = reduce_blocks(ctx->prob.n);
  void* red = ctx->d_red;
  if (!red && !ctx_dmalloc(ctx, &red, sizeof(ReducePartial) * nb))
    return fail(FQNM_ERR_OOM, "allocation of reduction partials failed");
  ctx->d_red = static_cast<ReducePartial*>(red);
  const char* q = static_cast<const char*>(ctx->buf[ctx->cur]) +
                  comp * ctx->prob.n * ctx->esize;
  CTX_HIP(launch_reduce(ctx->prob.itype, q, ctx->prob.n, 0, ctx->d_red, ctx->stream), "reduce");
  std::vector<ReducePartial> h(nb);
  CTX_HIP(hipMemcpyAsync(h.data(), ctx->d_red, sizeof(ReducePartial) * nb, hipMemcpyDeviceToHost,
                         ctx->stream), "copy partials");
  CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
  int64_t a = INT64_MAX, b = INT64_MIN;
  for (auto& r : h) {
    a = std::min(a, r.qmin);
    b = std::max(b, r.qmax);
  }
  *lo = a;
  *hi = b;
  return FQNM_OK;
}

// Shared tail of the create calls: state is on the device in buf[0].
static fqnm_status ctx_finish(fqnm_ctx* ctx) {
  const fqnm_problem& p = ctx->prob;
  if (ctx->euler) {
    const bool dens = is_euler_density(p.flux);
    for (int c = 0; c < (dens ? 1 : 3); ++c) {  // density-only: m and E are FP64
      int64_t lo, hi;
      fqnm_status st = ctx_minmax(ctx, c, &lo, &hi);
      if (st) return st;
      st = validate_range(p, lo, hi);
      if (st) return st;
      if (c == 0 && lo <= 0) return fail(FQNM_ERR_RANGE, "density counts must be positive");
    }
    ctx->eparams.delta = p.delta;
    ctx->eparams.lambda = p.lambda;
    ctx->eparams.g1 = p.gamma - 1.0;
    ctx->eparams.fix = p.flux == FQNM_FLUX_EULER_ROE_EF || p.flux == FQNM_FLUX_EULER_ROE_EF_DENSITY;
    ctx->eparams.dens = dens;
    void* flag = ctx->d_err;
    if (!flag && !ctx_dmalloc(ctx, &flag, sizeof(int)))
      return fail(FQNM_ERR_OOM, "allocation of the error flag failed");
    ctx->d_err = static_cast<int*>(flag);
    CTX_HIP(hipMemsetAsync(ctx->d_err, 0, sizeof(int), ctx->stream), "flag reset");
    ctx->eparams.err = ctx->d_err;
    return FQNM_OK;
  }
  int64_t lo, hi;
  fqnm_status st = ctx_minmax(ctx, 0, &lo, &hi);
  if (st) return st;
  st = validate_range(p, lo, hi);
  if (st) return st;
  ctx->q0min = lo;
  ctx->q0max = hi;
  ctx->xp = xparams_of(p);
  const bool lut = p.eval == FQNM_EVAL_LUT;
  if (lut) {
    const int64_t count = hi - lo + 1;
    if (count >= (int64_t(1) << 28)) return fail(FQNM_ERR_RANGE, "LUT range too large");
    const size_t eb = p.itype == FQNM_I32 ? 8 : 16;
    if (!ctx_dmalloc(ctx, &ctx->d_lut, eb * count))
      return fail(FQNM_ERR_OOM, "allocation of the LUT failed");
    // the reduction partials (free again after ctx_minmax) hold the
    // certificate's violation flag
    int* viol = reinterpret_cast<int*>(ctx->d_red);
    CTX_HIP(hipMemsetAsync(viol, 0, sizeof(int), ctx->stream), "flag reset");
    CTX_HIP(launch_lut_build(p.itype, direct_split_policy(p), ctx->xp, ctx->d_lut, lo, count,
                             viol, ctx->stream), "LUT build");
    int violated = 1;
    CTX_HIP(hipMemcpyAsync(&violated, viol, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
            "copy flag");
    CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
    ctx->xp.lut = ctx->d_lut;
    ctx->xp.lut_lo = lo;
    ctx->xp.lut_last = count - 1;
    ctx->xp.lut_pol = direct_split_policy(p);
    // FQNM_TABLE_CLAMPED set: take the clamped reads even for a certified
    // table (for comparisons and tests of that path)
    ctx->xp.lut_mono = violated || std::getenv("FQNM_TABLE_CLAMPED") ? 0 : 1;
  }
  ctx->pol = policy_of(p, lut);
  ctx->direct_pol = policy_of(p, false);
  fqnm_plan pl;
  if (!lookup_plan(plan_key(p, ctx->pol), &pl)) {
    pl = default_plan(p, ctx->pol);
    small_grid_plan(p, ctx->device, &pl);
  }
  ctx->plan = pl;
  ctx->plan.eval = lut ? FQNM_EVAL_LUT : FQNM_EVAL_DIRECT;
  return FQNM_OK;
}

static fqnm_status ctx_new(const fqnm_problem* prob, void* stream, fqnm_ctx** out,
                           fqnm_ctx** made) {
  if (!out) return fail(FQNM_ERR_ARG, "out is NULL");
  *out = nullptr;
  fqnm_status st = validate_problem(prob);
  if (st) return st;
  fqnm_ctx* ctx = new fqnm_ctx();
  ctx->prob = *prob;
  ctx->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&ctx->device) != hipSuccess) ctx->device = 0;
  ctx->euler = is_euler(prob->flux);
  ctx->comp = ctx->euler ? 3 : 1;
  ctx->esize = prob->itype == FQNM_I32 ? 4 : 8;
  *made = ctx;
  return FQNM_OK;
}

// Plan-cache key of a d-D context: dimension, kind, storage, and the log2 of
// each extent with its boundary kind.
static std::string nd_plan_key(const fqnm_ctx* ctx) {
  std::string k = "nd" + std::to_string(ctx->dim) + "_" + plan_key(ctx->prob, ctx->pol);
  for (int m = 0; m < ctx->dim; ++m) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= ctx->nd.ax[m].n) ++lg;
    k += "_" + std::to_string(lg) + "b" + std::to_string(ctx->nd.ax[m].bc);
  }
  return k;
}

// Temporal-blocking plans of d-D contexts keep the steps per pass in the low
// 8 bits of `depth` and the rows per wavefront above them (0: chosen here so
// that the launch has about six wavefronts per SIMD).
static int nd_tb_depth(const fqnm_plan& pl) { return pl.depth & 0xFF; }
static int nd_tb_rows(const fqnm_ctx* ctx, const fqnm_plan& pl) {
  const int r = pl.depth >> 8;
  if (r > 0) return r;
  const int K = nd_tb_depth(pl), v = pl.vec;
  const int64_t W = 64 * v - 2 * ((K + v - 1) / v * v);
  const int64_t nstrips = (ctx->nd.ax[0].n + W - 1) / W;
  const int64_t want = nstrips * ctx->nd.ax[1].n / (6 * 1024);
  return static_cast<int>(std::max<int64_t>(8, std::min<int64_t>(64, want)));
}
static bool nd_plan_valid(const fqnm_ctx* ctx, const fqnm_plan& pl) {
  if (pl.kernel == K_ND_TB) {
    const int K = nd_tb_depth(pl);
    return K >= 1 && nd_tb_step_depth(K) == K &&
           nd_tb_valid(ctx->prob.itype, ctx->pol, pl.vec, ctx->nd);
  }
  return pl.kernel == K_ND_MARCH && pl.depth >= 1 &&
         nd_variant_available(ctx->prob.itype, ctx->pol, pl.vec);
}

extern "C" {

const char* fqnm_last_error(void) { return tl_error.c_str(); }
const char* fqnm_version(void) { return "fqnm-mi355x 1.0 (gfx950, ABI 1)"; }

fqnm_status fqnm_create(const fqnm_problem* prob, const void* q0_host, void* hip_stream,
                        fqnm_ctx** out) {
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(prob, hip_stream, out, &ctx);
  if (st) return st;
  if (!q0_host) { ctx_free(ctx); return fail(FQNM_ERR_ARG, "q0_host is NULL"); }
  st = ctx_alloc(ctx, nullptr);
  if (!st) {
    hipError_t e = hipMemcpyAsync(ctx->buf[0], q0_host, ctx->state_bytes(),
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) st = hip_fail(e, "copy q0");
  }
  if (!st) st = ctx_finish(ctx);
  if (st) { ctx_free(ctx); return st; }
  *out = ctx;
  return FQNM_OK;
}

fqnm_status fqnm_create_from_field(const fqnm_problem* prob, const double* u0_host,
                                   void* hip_stream, fqnm_ctx** out) {
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(prob, hip_stream, out, &ctx);
  if (st) return st;
  if (!u0_host) { ctx_free(ctx); return fail(FQNM_ERR_ARG, "u0_host is NULL"); }
  st = ctx_alloc(ctx, nullptr);
  const int64_t total = ctx->comp * prob->n;
  if (!st && hipMalloc(&ctx->d_u, sizeof(double) * total) != hipSuccess)
    st = fail(FQNM_ERR_OOM, "hipMalloc of the field failed");
  if (!st && hipMalloc(&ctx->d_err, sizeof(int)) != hipSuccess)
    st = fail(FQNM_ERR_OOM, "hipMalloc failed");
  if (!st) {
    hipError_t e = hipMemcpyAsync(ctx->d_u, u0_host, sizeof(double) * total,
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->d_err, 0, sizeof(int), ctx->stream);
    const bool dens = is_euler_density(prob->flux);
    if (e == hipSuccess)
      e = launch_quantise(prob->itype, ctx->d_u, ctx->buf[0], dens ? prob->n : total, prob->delta,
                          ctx->d_err, ctx->stream);
    if (e == hipSuccess && dens)  // momentum and energy stay real-valued
      e = hipMemcpyAsync(static_cast<char*>(ctx->buf[0]) + sizeof(double) * prob->n,
                         ctx->d_u + prob->n, sizeof(double) * 2 * prob->n,
                         hipMemcpyDeviceToDevice, ctx->stream);
    int herr = 0;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&herr, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) st = hip_fail(e, "quantise");
    else if (herr) st = fail(FQNM_ERR_RANGE, "u0/delta exceeds the storage range");
  }
  if (!st) st = ctx_finish(ctx);
  if (st) { ctx_free(ctx); return st; }
  *out = ctx;
  return FQNM_OK;
}

fqnm_status fqnm_create_on_device(const fqnm_problem* prob, void* d_q, void* hip_stream,
                                  fqnm_ctx** out) {
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(prob, hip_stream, out, &ctx);
  if (st) return st;
  if (!d_q) { ctx_free(ctx); return fail(FQNM_ERR_ARG, "d_q is NULL"); }
  st = ctx_alloc(ctx, d_q);
  if (!st) st = ctx_finish(ctx);
  if (st) { ctx_free(ctx); return st; }
  *out = ctx;
  return FQNM_OK;
}

}  // extern "C"

size_t fqnm::ctx_carved_bytes(const fqnm_problem& p, int64_t lo, int64_t hi) {
  const int comp = is_euler(p.flux) ? 3 : 1;
  const size_t sb = round256(static_cast<size_t>(comp) * p.n * (p.itype == FQNM_I32 ? 4 : 8));
  size_t b = 2 * sb + 256 + round256(sizeof(ReducePartial) * reduce_blocks(p.n));
  if (p.eval == FQNM_EVAL_LUT && !is_euler(p.flux))
    b += round256((p.itype == FQNM_I32 ? 8 : 16) * static_cast<size_t>(hi - lo + 1));
  return b;
}

fqnm_status fqnm::ctx_create_carved(const fqnm_problem* prob, char* block, size_t bytes,
                                    hipStream_t stream, fqnm_ctx** out) {
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(prob, stream, out, &ctx);
  if (st) return st;
  if (!block || (reinterpret_cast<uintptr_t>(block) & 255) != 0) {
    ctx_free(ctx);
    return fail(FQNM_ERR_ARG, "block must be 256-byte aligned");
  }
  ctx->carve_base = block;
  ctx->carve_size = bytes;
  st = ctx_alloc(ctx, nullptr);  // buf[0] is carved first: the state already there
  if (!st) st = ctx_finish(ctx);
  if (st) { ctx_free(ctx); return st; }
  *out = ctx;
  return FQNM_OK;
}

extern "C" {

fqnm_status fqnm_create_nd(const fqnm_problem* axes, int32_t dim, const void* q0_host,
                           void* hip_stream, fqnm_ctx** out) {
  if (!out) return fail(FQNM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!axes || !q0_host) return fail(FQNM_ERR_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(FQNM_ERR_ARG, "dim must be 2 or 3");
  int64_t total = 1;
  for (int m = 0; m < dim; ++m) {
    fqnm_status st = validate_problem(&axes[m]);
    if (st) return st;
    if (is_euler(axes[m].flux)) return fail(FQNM_ERR_UNSUPPORTED, "d-D grids take scalar kinds");
    if (axes[m].flux != axes[0].flux || axes[m].itype != axes[0].itype ||
        axes[m].delta != axes[0].delta)
      return fail(FQNM_ERR_ARG, "all axes must share flux kind, itype and delta");
    if (axes[m].eval == FQNM_EVAL_LUT)
      return fail(FQNM_ERR_UNSUPPORTED,
                  "no LUT mode in d-D: its table range rests on a maximum principle");
    if (axes[m].n > INT32_MAX) return fail(FQNM_ERR_ARG, "an axis holds more than 2^31 - 1 cells");
    if (total > (int64_t(1) << 36) / axes[m].n) return fail(FQNM_ERR_ARG, "grid too large");
    total *= axes[m].n;
  }
  fqnm_problem p0 = axes[0];
  p0.n = total;
  p0.eval = FQNM_EVAL_DIRECT;
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(&p0, hip_stream, out, &ctx);
  if (st) return st;
  ctx->dim = dim;
  ctx->nd.dim = dim;
  for (int m = 0; m < dim; ++m) {
    NdAxis& A = ctx->nd.ax[m];
    A.x = xparams_of(axes[m]);
    A.cp = A.x.c > 0.0 ? A.x.c : 0.0;
    A.cm = A.x.c < 0.0 ? A.x.c : 0.0;
    A.n = axes[m].n;
    A.bc = axes[m].bc;
  }
  st = ctx_alloc(ctx, nullptr);
  if (!st) {
    hipError_t e = hipMemcpyAsync(ctx->buf[0], q0_host, ctx->state_bytes(),
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) st = hip_fail(e, "copy q0");
  }
  int64_t lo = 0, hi = 0;
  if (!st) st = ctx_minmax(ctx, 0, &lo, &hi);
  if (!st) st = validate_nd_range(axes, dim, lo, hi);
  if (st) { ctx_free(ctx); return st; }
  ctx->q0min = lo;
  ctx->q0max = hi;
  ctx->xp = ctx->nd.ax[0].x;
  ctx->pol = p0.flux == FQNM_FLUX_UPWIND ? P_UPWIND_POS : policy_of(p0, false);
  ctx->direct_pol = ctx->pol;
  // 2-D grids default to 4 steps per pass, 2 cells per lane
  fqnm_plan pl{K_ND_MARCH, p0.itype == FQNM_I32 ? 4 : 2, 16, FQNM_EVAL_DIRECT};
  if (nd_tb_valid(p0.itype, ctx->pol, 2, ctx->nd)) pl = fqnm_plan{K_ND_TB, 2, 4, FQNM_EVAL_DIRECT};
  fqnm_plan cached;
  if (lookup_plan(nd_plan_key(ctx), &cached) && nd_plan_valid(ctx, cached)) pl = cached;
  ctx->plan = pl;
  *out = ctx;
  return FQNM_OK;
}

fqnm_status fqnm_create_classical(const fqnm_problem* prob, const double* u0_host,
                                  void* hip_stream, fqnm_ctx** out) {
  fqnm_ctx* ctx = nullptr;
  fqnm_status st = ctx_new(prob, hip_stream, out, &ctx);
  if (st) return st;
  if (!u0_host || ctx->euler) {
    ctx_free(ctx);
    return fail(FQNM_ERR_ARG, "u0_host is NULL, or an Euler kind (the twin is scalar)");
  }
  ctx->classical = true;
  ctx->esize = 8;
  // CFL on the range of the initial field (eq:cfl_number)
  double umax = 0.0;
  for (int64_t i = 0; i < prob->n; ++i) {
    if (!std::isfinite(u0_host[i])) { ctx_free(ctx); return fail(FQNM_ERR_ARG, "u0 must be finite"); }
    umax = std::max(umax, std::fabs(u0_host[i]));
  }
  double nu = 0.0;
  if (prob->flux == FQNM_FLUX_UPWIND) nu = std::fabs(prob->a) * prob->lambda;
  else if (prob->flux == FQNM_FLUX_LF_LINEAR || prob->flux == FQNM_FLUX_LF_BURGERS)
    nu = prob->alpha * prob->lambda;
  else nu = prob->lambda * umax;
  if (nu > 1.0) { ctx_free(ctx); return fail(FQNM_ERR_CFL, "CFL number exceeds 1"); }
  st = ctx_alloc(ctx, nullptr);
  if (!st) {
    hipError_t e = hipMemcpyAsync(ctx->buf[0], u0_host, ctx->state_bytes(),
                                  hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) st = hip_fail(e, "copy u0");
  }
  if (st) { ctx_free(ctx); return st; }
  ctx->xp = xparams_of(*prob);
  ctx->pol = policy_of(*prob, false);
  ctx->direct_pol = ctx->pol;
  ctx->plan.kernel = K_TBLOCK;
  ctx->plan.vec = 4;
  ctx->plan.depth = 24;
  ctx->plan.eval = FQNM_EVAL_DIRECT;
  *out = ctx;
  return FQNM_OK;
}

fqnm_status fqnm_destroy(fqnm_ctx* ctx) {
  if (!ctx) return FQNM_OK;
  ctx->stream_sync_on_free = true;
  ctx_free(ctx);
  return FQNM_OK;
}

}  // extern "C"

// Enqueue n_steps on the context's stream with its current plan.
fqnm_status fqnm::ctx_advance(fqnm_ctx* ctx, int64_t n_steps, void* const buf[2], int* cur,
                              const fqnm_plan& pl) {
  const fqnm_problem& p = ctx->prob;
  int64_t left = n_steps;
  while (left > 0) {
    const void* src = buf[*cur];
    void* dst = buf[1 - *cur];
    int64_t k = 1;
    hipError_t e;
    if (ctx->classical) {
      if (pl.kernel == K_STREAM) {
        e = launch_classical(ctx->pol, K_STREAM, pl.vec, static_cast<const double*>(src),
                             static_cast<double*>(dst), p.n, p.bc, 1, 0, ctx->xp, ctx->stream);
      } else {
        k = std::min<int64_t>(pl.depth, left);
        const int khalo = scalar_halo(K_TBLOCK, pl.vec, static_cast<int>(k));
        e = launch_classical(ctx->pol, K_TBLOCK, pl.vec, static_cast<const double*>(src),
                             static_cast<double*>(dst), p.n, p.bc, static_cast<int>(k), khalo,
                             ctx->xp, ctx->stream);
      }
    } else if (ctx->dim > 1 && pl.kernel == K_ND_TB) {
      k = nd_tb_step_depth(static_cast<int>(std::min<int64_t>(nd_tb_depth(pl), left)));
      e = launch_nd_tb(p.itype, ctx->pol, pl.vec, static_cast<int>(k), nd_tb_rows(ctx, pl), src,
                       dst, ctx->nd, ctx->d_ledger, ctx->stream);
    } else if (ctx->dim > 1) {
      e = launch_nd(p.itype, ctx->pol, pl.vec, pl.depth, src, dst, ctx->nd, ctx->d_ledger,
                    ctx->stream);
    } else if (ctx->euler) {
      k = std::min<int64_t>(euler_steps_per_launch(), left);
      e = launch_euler_step(static_cast<const int64_t*>(src), static_cast<int64_t*>(dst), p.n,
                            p.bc, ctx->eparams, static_cast<int>(k), ctx->d_ledger, ctx->stream);
    } else if (pl.kernel == K_TBLOCK_PERSIST) {
      // every pass in one cooperative launch
      k = left;
      fqnm_status st = ctx_persist_buffers(ctx, pl.vec, pl.depth);
      if (st) return st;
      const int64_t passes = (k + pl.depth - 1) / pl.depth;
      if (k > INT32_MAX || passes >= (int64_t(1) << 30))
        return fail(FQNM_ERR_ARG, "too many steps for one persistent launch");
      if (static_cast<uint64_t>(ctx->exch_tag) + passes >= (uint64_t(1) << 32)) {
        CTX_HIP(hipMemsetAsync(ctx->d_exch, 0, ctx->exch_bytes, ctx->stream), "exchange reset");
        ctx->exch_tag = 0;
      }
      e = launch_persist(ctx->pol, pl.vec, static_cast<const int32_t*>(src),
                         static_cast<int32_t*>(dst), p.n, static_cast<int>(k), pl.depth, ctx->xp,
                         ctx->d_exch, ctx->exch_tag, ctx->d_perr, 1 << 20, ctx->stream);
      ctx->exch_tag += static_cast<uint32_t>(passes);
    } else if (pl.kernel == K_TBLOCK_WG4 || pl.kernel == K_TBLOCK_WG8) {
      k = std::min<int64_t>(pl.depth, left);
      e = launch_tblock_wg(pl.kernel == K_TBLOCK_WG4 ? 4 : 8, pl.vec,
                           static_cast<const int32_t*>(src), static_cast<int32_t*>(dst), p.n,
                           static_cast<int>(k), ctx->xp, ctx->stream);
    } else if (pl.kernel == K_STREAM) {
      e = launch_scalar(p.itype, ctx->pol, K_STREAM, pl.vec, src, dst, p.n, p.bc, 1, 0, ctx->xp,
                        ctx->d_ledger, ctx->stream);
    } else {
      k = std::min<int64_t>(pl.depth, left);
      const int khalo = scalar_halo(pl.kernel, pl.vec, static_cast<int>(k));
      e = launch_scalar(p.itype, ctx->pol, pl.kernel, pl.vec, src, dst, p.n, p.bc,
                        static_cast<int>(k), khalo, ctx->xp, ctx->d_ledger, ctx->stream);
    }
    if (e != hipSuccess) {
      ctx->poisoned = true;
      return hip_fail(e, "step launch");
    }
    *cur = 1 - *cur;
    left -= k;
  }
  return FQNM_OK;
}

extern "C" {

fqnm_status fqnm_step(fqnm_ctx* ctx, int64_t n_steps) {
  if (!ctx) return fail(FQNM_ERR_ARG, "ctx is NULL");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned by an earlier device error");
  if (n_steps < 0) return fail(FQNM_ERR_ARG, "n_steps must be >= 0");
  if (ctx->range_error) return fail(FQNM_ERR_RANGE, "a density or pressure became non-positive");
  if (!ctx->euler && !ctx->classical && ctx->dim == 1) {
    fqnm_status st = validate_drift(ctx->prob, ctx->q0min, ctx->q0max, ctx->steps_done + n_steps);
    if (st) return st;
  }
  fqnm_status st = ctx_advance(ctx, n_steps, ctx->buf, &ctx->cur, ctx->plan);
  if (st) return st;
  ctx->steps_done += n_steps;
  if (ctx->borrowed && ctx->cur != 0) {
    CTX_HIP(hipMemcpyAsync(ctx->buf[0], ctx->buf[1], ctx->state_bytes(),
                           hipMemcpyDeviceToDevice, ctx->stream), "copy back");
    ctx->cur = 0;
  }
  return FQNM_OK;
}

}  // extern "C"

// Euler contexts: the kernels' sticky flag for a non-positive density or
// pressure (the transfers of such a step are meaningless).  Once raised, the
// context refuses every later call with FQNM_ERR_RANGE.
fqnm_status fqnm::ctx_check_flag(fqnm_ctx* ctx) {
  if (ctx->range_error) return fail(FQNM_ERR_RANGE, "a density or pressure became non-positive");
  if (ctx->d_perr) {
    int h = 0;
    CTX_HIP(hipMemcpyAsync(&h, ctx->d_perr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
            "copy flag");
    CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
    if (h) {
      ctx->poisoned = true;
      return fail(FQNM_ERR_DEVICE, "a persistent launch timed out waiting for a neighbouring tile");
    }
  }
  if (!ctx->euler || !ctx->d_err) return FQNM_OK;
  int h = 0;
  CTX_HIP(hipMemcpyAsync(&h, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
          "copy flag");
  CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
  if (h) {
    ctx->range_error = true;
    return fail(FQNM_ERR_RANGE, "a density or pressure became non-positive");
  }
  return FQNM_OK;
}

extern "C" {

fqnm_status fqnm_get_state(fqnm_ctx* ctx, void* q_host) {
  if (!ctx || !q_host) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  CTX_HIP(hipMemcpyAsync(q_host, ctx->buf[ctx->cur], ctx->state_bytes(), hipMemcpyDeviceToHost,
                         ctx->stream), "copy state");
  CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
  return ctx_check_flag(ctx);
}

fqnm_status fqnm_state_device(fqnm_ctx* ctx, void** d_q) {
  if (!ctx || !d_q) return fail(FQNM_ERR_ARG, "NULL argument");
  *d_q = ctx->buf[ctx->cur];
  return FQNM_OK;
}

fqnm_status fqnm_reconstruct_device(fqnm_ctx* ctx, double* d_u) {
  if (!ctx || !d_u) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  if (ctx->classical) {
    CTX_HIP(hipMemcpyAsync(d_u, ctx->buf[ctx->cur], ctx->state_bytes(), hipMemcpyDeviceToDevice,
                           ctx->stream), "copy field");
    return FQNM_OK;
  }
  if (ctx->euler && ctx->eparams.dens) {
    const int64_t n = ctx->prob.n;
    CTX_HIP(launch_reconstruct(ctx->prob.itype, ctx->buf[ctx->cur], d_u, n, ctx->prob.delta,
                               ctx->stream), "reconstruct");
    CTX_HIP(hipMemcpyAsync(d_u + n, static_cast<const char*>(ctx->buf[ctx->cur]) + 8 * n,
                           sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, ctx->stream),
            "copy m, E");
    return FQNM_OK;
  }
  CTX_HIP(launch_reconstruct(ctx->prob.itype, ctx->buf[ctx->cur], d_u, ctx->comp * ctx->prob.n,
                             ctx->prob.delta, ctx->stream), "reconstruct");
  return FQNM_OK;
}

fqnm_status fqnm_reconstruct(fqnm_ctx* ctx, double* u_host) {
  if (!ctx || !u_host) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  const int64_t total = ctx->comp * ctx->prob.n;
  if (!ctx->d_u && hipMalloc(&ctx->d_u, sizeof(double) * total) != hipSuccess)
    return fail(FQNM_ERR_OOM, "hipMalloc of the field failed");
  fqnm_status st = fqnm_reconstruct_device(ctx, ctx->d_u);
  if (st) return st;
  CTX_HIP(hipMemcpyAsync(u_host, ctx->d_u, sizeof(double) * total, hipMemcpyDeviceToHost,
                         ctx->stream), "copy field");
  CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
  return ctx_check_flag(ctx);
}

fqnm_status fqnm_invariants_get(fqnm_ctx* ctx, fqnm_invariants* out) {
  if (!ctx || !out) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->classical) return fail(FQNM_ERR_UNSUPPORTED, "no integer invariants for the FP64 twin");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  std::memset(out, 0, sizeof *out);
  const int ncomp = ctx->euler && ctx->eparams.dens ? 1 : ctx->comp;  // integer components
  out->components = ncomp;
  out->steps_done = ctx->steps_done;
  const int64_t n = ctx->prob.n;
  const int64_t nb = reduce_blocks(n);
  void* red = ctx->d_red;
  if (!red && !ctx_dmalloc(ctx, &red, sizeof(ReducePartial) * nb))
    return fail(FQNM_ERR_OOM, "allocation of reduction partials failed");
  ctx->d_red = static_cast<ReducePartial*>(red);
  std::vector<ReducePartial> h(nb);
  for (int c = 0; c < ncomp; ++c) {
    const char* q = static_cast<const char*>(ctx->buf[ctx->cur]) + c * n * ctx->esize;
    CTX_HIP(launch_reduce(ctx->prob.itype, q, n, ctx->prob.bc == FQNM_BC_PERIODIC, ctx->d_red,
                          ctx->stream), "reduce");
    CTX_HIP(hipMemcpyAsync(h.data(), ctx->d_red, sizeof(ReducePartial) * nb,
                           hipMemcpyDeviceToHost, ctx->stream), "copy partials");
    CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
    __int128 s = 0, tv = 0;
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (auto& r : h) {
      s += (static_cast<__int128>(r.sum_hi) << 64) | r.sum_lo;
      tv += (static_cast<__int128>(r.tv_hi) << 64) | r.tv_lo;
      lo = std::min(lo, r.qmin);
      hi = std::max(hi, r.qmax);
    }
    out->sum_hi[c] = static_cast<int64_t>(s >> 64);
    out->sum_lo[c] = static_cast<uint64_t>(s);
    if (ctx->dim > 1) tv = 0;  // the 1-D total variation of the flat array means nothing in d-D
    out->tv_hi[c] = static_cast<int64_t>(tv >> 64);
    out->tv_lo[c] = static_cast<uint64_t>(tv);
    out->qmin[c] = lo;
    out->qmax[c] = hi;
  }
  long long led[3];
  CTX_HIP(hipMemcpyAsync(led, ctx->d_ledger, sizeof led, hipMemcpyDeviceToHost, ctx->stream),
          "copy ledger");
  CTX_HIP(hipStreamSynchronize(ctx->stream), "sync");
  for (int c = 0; c < 3; ++c) out->ledger[c] = c < ncomp ? led[c] : 0;
  return ctx_check_flag(ctx);
}

fqnm_status fqnm_quantise(const double* u_host, int64_t n, double delta, int32_t itype,
                          void* q_host, void* hip_stream) {
  if (!u_host || !q_host || n < 0) return fail(FQNM_ERR_ARG, "NULL argument or negative n");
  if (!(std::isfinite(delta) && delta > 0.0)) return fail(FQNM_ERR_ARG, "delta must be > 0");
  if (itype != FQNM_I32 && itype != FQNM_I64) return fail(FQNM_ERR_ARG, "unknown itype");
  if (n == 0) return FQNM_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const size_t es = itype == FQNM_I32 ? 4 : 8;
  double* du = nullptr;
  void* dq = nullptr;
  int* derr = nullptr;
  fqnm_status st = FQNM_OK;
  if (hipMalloc(&du, sizeof(double) * n) != hipSuccess || hipMalloc(&dq, es * n) != hipSuccess ||
      hipMalloc(&derr, sizeof(int)) != hipSuccess)
    st = fail(FQNM_ERR_OOM, "hipMalloc failed");
  int herr = 0;
  if (!st) {
    hipError_t e = hipMemcpyAsync(du, u_host, sizeof(double) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(derr, 0, sizeof(int), s);
    if (e == hipSuccess) e = launch_quantise(itype, du, dq, n, delta, derr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(q_host, dq, es * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "quantise");
    else if (herr) st = fail(FQNM_ERR_RANGE, "u/delta exceeds the storage range");
  }
  if (du) (void)hipFree(du);
  if (dq) (void)hipFree(dq);
  if (derr) (void)hipFree(derr);
  return st;
}

fqnm_status fqnm_get_plan(fqnm_ctx* ctx, fqnm_plan* out) {
  if (!ctx || !out) return fail(FQNM_ERR_ARG, "NULL argument");
  *out = ctx->plan;
  if (ctx->euler) { out->kernel = K_STREAM; out->vec = 1; out->depth = euler_steps_per_launch(); }
  return FQNM_OK;
}

fqnm_status fqnm_set_plan(fqnm_ctx* ctx, const fqnm_plan* plan) {
  if (!ctx || !plan) return fail(FQNM_ERR_ARG, "NULL argument");
  if (ctx->euler) return fail(FQNM_ERR_UNSUPPORTED, "Euler contexts have a fixed plan");
  fqnm_plan pl = ctx->plan;
  if (ctx->dim > 1) {
    if (plan->kernel != 0 && plan->kernel != K_ND_MARCH && plan->kernel != K_ND_TB)
      return fail(FQNM_ERR_ARG, "d-D contexts run the marching kernels only");
    if (plan->kernel && plan->kernel != pl.kernel) {
      // a zero field of another kernel's plan takes that kernel's default
      pl.kernel = plan->kernel;
      pl.vec = pl.kernel == K_ND_TB ? 2 : (ctx->prob.itype == FQNM_I32 ? 4 : 2);
      pl.depth = pl.kernel == K_ND_TB ? 4 : 16;
    }
    if (plan->vec) pl.vec = plan->vec;
    if (plan->depth) pl.depth = plan->depth;
    if (pl.kernel == K_ND_TB) {
      if (!nd_tb_valid(ctx->prob.itype, ctx->pol, pl.vec, ctx->nd))
        return fail(FQNM_ERR_ARG, "temporal blocking needs a 2-D grid and vec 2 or 4 (int64: 2) "
                                  "dividing the first axis");
      const int K = nd_tb_depth(pl);
      if (pl.depth < 1 || K < 1 || nd_tb_step_depth(K) != K)
        return fail(FQNM_ERR_ARG, "steps per pass (depth & 0xFF) must be 1, 2, 4 or 8");
    } else {
      if (!nd_variant_available(ctx->prob.itype, ctx->pol, pl.vec))
        return fail(FQNM_ERR_ARG, "vec not available for this storage type");
      if (pl.depth < 1) return fail(FQNM_ERR_ARG, "depth (rows per wavefront) must be >= 1");
    }
    ctx->plan = pl;
    return FQNM_OK;
  }
  if ((plan->kernel >= K_STREAM && plan->kernel <= K_TBLOCK_B8) ||
      plan->kernel == K_TBLOCK_WG4 || plan->kernel == K_TBLOCK_WG8 ||
      plan->kernel == K_TBLOCK_PERSIST)
    pl.kernel = plan->kernel;
  else if (plan->kernel != 0) return fail(FQNM_ERR_ARG, "unknown kernel");
  if (plan->vec) pl.vec = plan->vec;
  if (plan->depth) pl.depth = plan->depth;
  if (pl.kernel == K_TBLOCK_PERSIST) {
    if (!persist_plan_ok(ctx, pl))
      return fail(FQNM_ERR_ARG, "the persistent plan needs int32 states on a periodic grid, a "
                                "table or direct split kind, vec 4 or 8, tiles of at least depth "
                                "cells and a grid that is resident at once");
    fqnm_status st = ctx_persist_buffers(ctx, pl.vec, pl.depth);
    if (st) return st;
    ctx->plan = pl;
    return FQNM_OK;
  }
  if (pl.kernel == K_TBLOCK_WG4 || pl.kernel == K_TBLOCK_WG8) {
    if (ctx->classical || ctx->prob.itype != FQNM_I32 || ctx->pol != P_LUT ||
        ctx->prob.bc != FQNM_BC_PERIODIC)
      return fail(FQNM_ERR_ARG, "overlapping-window tiles need int32 tables on a periodic grid");
    if (!tblock_wg_valid(pl.kernel == K_TBLOCK_WG4 ? 4 : 8, pl.vec, pl.depth))
      return fail(FQNM_ERR_ARG, "vec must be 2 or 4 and depth at most 64*vec - 16");
    ctx->plan = pl;
    return FQNM_OK;
  }
  if (ctx->classical ? !classical_variant_available(ctx->pol, pl.kernel, pl.vec)
                     : !scalar_variant_available(ctx->prob.itype, ctx->pol, pl.kernel, pl.vec))
    return fail(FQNM_ERR_ARG, "vec not available for this storage type");
  if (pl.kernel != K_STREAM) {
    if (pl.depth < 1) return fail(FQNM_ERR_ARG, "depth must be >= 1");
    const int kh = scalar_halo(pl.kernel, pl.vec, pl.depth);
    if (scalar_tile_positions(pl.kernel, pl.vec) - 2 * kh < pl.vec)
      return fail(FQNM_ERR_ARG, "depth too large for vec");
  }
  ctx->plan = pl;
  return FQNM_OK;
}

fqnm_status fqnm_autotune(fqnm_ctx* ctx, int64_t steps_per_trial) {
  if (!ctx) return fail(FQNM_ERR_ARG, "ctx is NULL");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  if (ctx->euler || ctx->classical) return FQNM_OK;
  if (steps_per_trial < 1) return fail(FQNM_ERR_ARG, "steps_per_trial must be >= 1");
  const size_t bytes = ctx->state_bytes();
  void* sb[2] = {nullptr, nullptr};
  long long* dled = nullptr;
  if (hipMalloc(&sb[0], bytes) != hipSuccess || hipMalloc(&sb[1], bytes) != hipSuccess ||
      hipMalloc(&dled, 3 * sizeof(long long)) != hipSuccess) {
    if (sb[0]) (void)hipFree(sb[0]);
    if (sb[1]) (void)hipFree(sb[1]);
    if (dled) (void)hipFree(dled);
    return fail(FQNM_ERR_OOM, "autotune scratch allocation failed");
  }
  long long* saved_ledger = ctx->d_ledger;
  ctx->d_ledger = dled;  // trials must not touch the real ledger
  std::vector<fqnm_plan> cand;
  const bool i32 = ctx->prob.itype == FQNM_I32;
  const std::vector<int> vecs32{4, 8, 16}, vecs64{2, 4, 8, 16};
  const int64_t simds = device_simds(ctx->device);
  if (ctx->dim > 1) {
    for (int v : {2, 4, 8})
      if (nd_variant_available(ctx->prob.itype, ctx->pol, v))
        for (int r : {4, 8, 16, 32, 64}) cand.push_back({K_ND_MARCH, v, r, 0});
    for (int v : {2, 4})
      if (nd_tb_valid(ctx->prob.itype, ctx->pol, v, ctx->nd))
        for (int K : {2, 4, 8})
          for (int r : {0, 16, 32, 64}) cand.push_back({K_ND_TB, v, K | (r << 8), 0});
  }
  for (int v : (i32 ? vecs32 : vecs64)) {
    if (ctx->dim > 1) break;
    const int PER = i32 ? 4 : 2;
    if (v >= 2 * PER) cand.push_back({K_STREAM, v, 1, 0});
    for (int d : {4, 8, 16, 32, 40, 48, 52, 56, 64, 96}) {
      const int kh = scalar_halo(K_TBLOCK, v, d);
      if (64 * v - 2 * kh >= 32 * v) cand.push_back({K_TBLOCK, v, d, 0});
    }
    // deeper passes with small tiles, for grids of about one wavefront per
    // SIMD (small_grid_plan)
    for (int d : {80, 96, 120, 160, 200, 240, 320, 400, 480}) {
      const int kh = scalar_halo(K_TBLOCK, v, d);
      const int64_t T = 64 * v - 2 * kh;
      if (T >= 8 && T < 32 * v && (ctx->prob.n + T - 1) / T <= 2 * simds)
        cand.push_back({K_TBLOCK, v, d, 0});
    }
    for (int kb : {K_TBLOCK_B2, K_TBLOCK_B4, K_TBLOCK_B8}) {
      for (int d : {24, 48, 64, 96}) {
        const int kh = scalar_halo(kb, v, d);
        if (scalar_tile_positions(kb, v) - 2 * kh >= scalar_tile_positions(kb, v) / 2)
          cand.push_back({kb, v, d, 0});
      }
    }
    if (v == 4 && ctx->prob.itype == FQNM_I32 && ctx->pol == P_LUT &&
        ctx->prob.bc == FQNM_BC_PERIODIC) {
      for (int kw : {K_TBLOCK_WG4, K_TBLOCK_WG8})
        for (int vv : {2, 4})
          for (int d : {24, 48, 64, 96})
            if (tblock_wg_valid(kw == K_TBLOCK_WG4 ? 4 : 8, vv, d)) cand.push_back({kw, vv, d, 0});
    }
    if (scalar_variant_available(ctx->prob.itype, ctx->pol, K_TBLOCK_IL, v)) {
      for (int d : {16, 32, 64, 128}) {
        const int kh = scalar_halo(K_TBLOCK_IL, v, d);
        if (64 * v - 2 * kh >= 32 * v) cand.push_back({K_TBLOCK_IL, v, d, 0});
      }
    }
    for (int d : {16, 24, 32, 40}) {
      const fqnm_plan pp{K_TBLOCK_PERSIST, v, d, 0};
      if (persist_plan_ok(ctx, pp)) cand.push_back(pp);
    }
  }
  // single-grid kernels exist for a subset of (storage type, policy, vec)
  cand.erase(std::remove_if(cand.begin(), cand.end(),
                            [&](const fqnm_plan& c) {
                              return c.kernel <= K_TBLOCK_B8 &&
                                     !scalar_variant_available(ctx->prob.itype, ctx->pol,
                                                               c.kernel, c.vec);
                            }),
             cand.end());
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best = 1e30f;
  fqnm_plan bestp = ctx->plan;
  fqnm_status st = FQNM_OK;
  for (const fqnm_plan& c : cand) {
    int cur = 0;
    if (hipMemcpyAsync(sb[0], ctx->buf[ctx->cur], bytes, hipMemcpyDeviceToDevice, ctx->stream) !=
        hipSuccess) { st = fail(FQNM_ERR_DEVICE, "autotune copy"); break; }
    st = ctx_advance(ctx, std::min<int64_t>(steps_per_trial, 4 * c.depth), sb, &cur, c);  // warm
    if (st) break;
    // the better of two timed trials, so that one noisy trial does not pick the plan
    float ms = 1e30f;
    for (int rep = 0; rep < 2 && !st; ++rep) {
      (void)hipEventRecord(e0, ctx->stream);
      st = ctx_advance(ctx, steps_per_trial, sb, &cur, c);
      if (st) break;
      (void)hipEventRecord(e1, ctx->stream);
      if (hipEventSynchronize(e1) != hipSuccess) { st = fail(FQNM_ERR_DEVICE, "autotune sync"); break; }
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = t < ms ? t : ms;
    }
    if (st) break;
    if (ms < best) { best = ms; bestp = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->d_ledger = saved_ledger;
  (void)hipFree(sb[0]);
  (void)hipFree(sb[1]);
  (void)hipFree(dled);
  if (st) return st;
  bestp.eval = ctx->plan.eval;
  ctx->plan = bestp;
  store_plan(ctx->dim > 1 ? nd_plan_key(ctx) : plan_key(ctx->prob, ctx->pol), bestp);
  return FQNM_OK;
}

}  // extern "C"
