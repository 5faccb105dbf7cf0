// batch.hip -- batched execution of many independent instances (work in progress).
#include <hip/hip_runtime.h>

#include "runtime.h"

using namespace fqnm;

extern "C" {
fqnm_status fqnm_batch_create(const fqnm_problem*, const void* const*, const int64_t*, int32_t,
                              void*, fqnm_batch** out) {
  if (out) *out = nullptr;
  return fail(FQNM_ERR_UNSUPPORTED, "batching is not built yet");
}
fqnm_status fqnm_batch_reset(fqnm_batch*) { return fail(FQNM_ERR_UNSUPPORTED, "no batch"); }
fqnm_status fqnm_batch_run(fqnm_batch*) { return fail(FQNM_ERR_UNSUPPORTED, "no batch"); }
fqnm_status fqnm_batch_run_per_instance(fqnm_batch*) {
  return fail(FQNM_ERR_UNSUPPORTED, "no batch");
}
fqnm_status fqnm_batch_get_state(fqnm_batch*, int32_t, void*) {
  return fail(FQNM_ERR_UNSUPPORTED, "no batch");
}
fqnm_status fqnm_batch_destroy(fqnm_batch*) { return FQNM_OK; }
}
