// runtime.h -- host-side objects behind the C ABI (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "fqnm_internal.h"

struct fqnm_ctx {
  fqnm_problem prob{};
  bool euler = false;
  bool classical = false;  // FP64 finite-volume twin: the state holds doubles
  int comp = 1;        // components per cell
  size_t esize = 4;    // bytes per integer
  hipStream_t stream = nullptr;
  int device = 0;      // HIP device current at create
  void* buf[2] = {nullptr, nullptr};  // ping-pong states (buf[0] may be borrowed)
  bool borrowed = false;
  int cur = 0;                       // buffer holding the current state
  int64_t steps_done = 0;
  long long* d_ledger = nullptr;     // 3 int64 boundary ledgers
  void* d_lut = nullptr;
  double* d_u = nullptr;             // scratch field for quantise/reconstruct
  int* d_err = nullptr;
  fqnm::ReducePartial* d_red = nullptr;
  fqnm::XParams xp{};
  fqnm::EulerParams eparams{};
  int pol = 0;          // policy used by the stepper (P_LUT in LUT mode)
  int direct_pol = 0;   // the direct policy of the same flux
  fqnm_plan plan{};
  int64_t q0min = 0, q0max = 0;
  bool poisoned = false;
  bool stream_sync_on_free = false;
  void* d_ws = nullptr;  // diagnostics workspace, grown on demand, freed with the context
  size_t ws_bytes = 0;
  int dim = 1;           // > 1: d-dimensional grid, prob.n = total cells, axes in nd
  fqnm::NdParams nd{};

  size_t state_bytes() const { return static_cast<size_t>(comp) * prob.n * esize; }
};

namespace fqnm {

fqnm_status fail(fqnm_status st, const std::string& msg);
fqnm_status hip_fail(hipError_t e, const char* what);
fqnm_status validate_problem(const fqnm_problem* p);
fqnm_status validate_range(const fqnm_problem& p, int64_t lo, int64_t hi);
bool is_euler(int flux);
bool is_euler_density(int flux);  // Euler with only the density quantised
bool is_burgers(int flux);
int policy_of(const fqnm_problem& p, bool lut);
int direct_split_policy(const fqnm_problem& p);
XParams xparams_of(const fqnm_problem& p);
fqnm_plan default_plan(const fqnm_problem& p);
std::string plan_key(const fqnm_problem& p, int pol);
bool lookup_plan(const std::string& key, fqnm_plan* out);
void store_plan(const std::string& key, const fqnm_plan& pl);

// Range of component comp of the current state (device reduction, syncs).
fqnm_status ctx_minmax(fqnm_ctx* ctx, int comp, int64_t* lo, int64_t* hi);

// Enqueue n_steps of the context's problem from buf[*cur] with plan pl,
// flipping *cur once per launch.
fqnm_status ctx_advance(fqnm_ctx* ctx, int64_t n_steps, void* const buf[2], int* cur,
                        const fqnm_plan& pl);

}  // namespace fqnm
