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
  bool range_error = false;  // Euler: a density or pressure became non-positive
  bool stream_sync_on_free = false;
  void* d_ws = nullptr;  // diagnostics workspace, grown on demand, freed with the context
  // Device memory given to the context as one block (the server's arena):
  // buffers are carved from it instead of allocated, and not freed.
  char* carve_base = nullptr;
  size_t carve_size = 0, carve_used = 0;
  size_t ws_bytes = 0;
  int dim = 1;           // > 1: d-dimensional grid, prob.n = total cells, axes in nd
  // persistent plan (K_TBLOCK_PERSIST): halo exchange words, the next pass
  // tag, and the flag a launch raises when a neighbour wait times out
  uint64_t* d_exch = nullptr;
  size_t exch_bytes = 0;
  uint32_t exch_tag = 0;
  int* d_perr = nullptr;
  fqnm::NdParams nd{};

  size_t state_bytes() const { return static_cast<size_t>(comp) * prob.n * esize; }
};

namespace fqnm {

fqnm_status fail(fqnm_status st, const std::string& msg);
fqnm_status hip_fail(hipError_t e, const char* what);
fqnm_status validate_problem(const fqnm_problem* p);
fqnm_status validate_range(const fqnm_problem& p, int64_t lo, int64_t hi);
// Lax-Friedrichs kinds have no exact integer maximum principle: a step can
// move the extremes by up to 2 counts (the exact scheme keeps them, and the
// four roundings of a cell's update add at most 1/2 each).  Checks the range
// [lo - 2*steps, hi + 2*steps] that `steps` steps from [lo, hi] can reach.
// Other kinds: FQNM_OK.
fqnm_status validate_drift(const fqnm_problem& p, int64_t lo, int64_t hi, int64_t steps);
bool is_euler(int flux);
bool is_euler_density(int flux);  // Euler with only the density quantised
bool is_burgers(int flux);
int policy_of(const fqnm_problem& p, bool lut);
int direct_split_policy(const fqnm_problem& p);
XParams xparams_of(const fqnm_problem& p);
fqnm_plan default_plan(const fqnm_problem& p, int pol);
std::string plan_key(const fqnm_problem& p, int pol);
bool lookup_plan(const std::string& key, fqnm_plan* out);
void store_plan(const std::string& key, const fqnm_plan& pl);

// Device bytes a context of problem p with initial range [lo, hi] needs when
// all its buffers are carved from one block (state, second state, ledger,
// reduction partials and, in table mode, the table).
size_t ctx_carved_bytes(const fqnm_problem& p, int64_t lo, int64_t hi);
// Create a context whose memory is the block [block, block + bytes): the
// initial state must already be at its start (components*n integers).
fqnm_status ctx_create_carved(const fqnm_problem* prob, char* block, size_t bytes,
                              hipStream_t stream, fqnm_ctx** out);

// Euler contexts: FQNM_ERR_RANGE once the kernels have flagged a
// non-positive density or pressure (syncs the stream to read the flag).
fqnm_status ctx_check_flag(fqnm_ctx* ctx);

// Range of component comp of the current state (device reduction, syncs).
fqnm_status ctx_minmax(fqnm_ctx* ctx, int comp, int64_t* lo, int64_t* hi);

// Enqueue n_steps of the context's problem from buf[*cur] with plan pl,
// flipping *cur once per launch.
fqnm_status ctx_advance(fqnm_ctx* ctx, int64_t n_steps, void* const buf[2], int* cur,
                        const fqnm_plan& pl);

}  // namespace fqnm
