// Kernel-profile gradient (placeholder until the correlation kernels land).
#include "arkcos_internal.h"

namespace arkcos {

arkcos_status_t run_kernel_grad(arkcos_plan_s* P, const void* x, const void* r, double* grad,
                                void* ws, uint32_t flags, hipStream_t s) {
  (void)P; (void)x; (void)r; (void)grad; (void)ws; (void)flags; (void)s;
  return fail(ARKCOS_ERR_NOT_SUPPORTED, "knot gradient not built yet");
}

}  // namespace arkcos

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
