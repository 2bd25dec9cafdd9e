// Batched form (placeholder until the persistent work-queue kernel lands).
#include "arkcos_internal.h"

extern "C" {
arkcos_status_t arkcos_batch_plan(int32_t, const arkcos_plan_t*, arkcos_batch_t*) {
  return arkcos::fail(ARKCOS_ERR_NOT_SUPPORTED, "batched form not built yet");
}
arkcos_status_t arkcos_batch_workspace_size(arkcos_batch_t, size_t*) {
  return arkcos::fail(ARKCOS_ERR_NOT_SUPPORTED, "batched form not built yet");
}
arkcos_status_t arkcos_batch_convolve(arkcos_batch_t, const void* const*, void* const*, int32_t, void*,
                                      hipStream_t) {
  return arkcos::fail(ARKCOS_ERR_NOT_SUPPORTED, "batched form not built yet");
}
arkcos_status_t arkcos_batch_destroy(arkcos_batch_t) {
  return arkcos::fail(ARKCOS_ERR_NOT_SUPPORTED, "batched form not built yet");
}
}
