// server.hip -- continuous-batching request server (work in progress).
#include <hip/hip_runtime.h>

#include <chrono>

#include "runtime.h"

using namespace fqnm;

extern "C" {
fqnm_status fqnm_server_create(size_t, int32_t, void*, fqnm_server** out) {
  if (out) *out = nullptr;
  return fail(FQNM_ERR_UNSUPPORTED, "serving is not built yet");
}
fqnm_status fqnm_server_submit(fqnm_server*, const fqnm_problem*, const void*, int64_t, void*,
                               uint64_t*) {
  return fail(FQNM_ERR_UNSUPPORTED, "no server");
}
fqnm_status fqnm_server_poll(fqnm_server*, fqnm_completion*, int32_t, int32_t* n) {
  if (n) *n = 0;
  return fail(FQNM_ERR_UNSUPPORTED, "no server");
}
fqnm_status fqnm_server_drain(fqnm_server*, double) { return fail(FQNM_ERR_UNSUPPORTED, "no server"); }
fqnm_status fqnm_server_stats_get(fqnm_server*, fqnm_server_stats*) {
  return fail(FQNM_ERR_UNSUPPORTED, "no server");
}
double fqnm_server_now(void) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
fqnm_status fqnm_server_destroy(fqnm_server*) { return FQNM_OK; }
}
