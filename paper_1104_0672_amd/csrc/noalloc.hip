// arkcos_convolve_noalloc: the forward convolution with its workspace (the
// extended input spectra and the output-ring coefficients) in a fixed device
// array of the library, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array.  Its name in host code is only a
// host-side stand-in for the symbol, not a device address: the device
// address is obtained once per device with hipGetSymbolAddress (with that
// device current) and only that address is ever passed to kernels.  Every
// call on one device shares that device's array and the array keeps the last
// call's contents; calls that may overlap in time on one device race.  No
// part of the array needs to start at zero: the ring transforms write every
// spectrum mode the accumulation reads, and the accumulation writes every
// coefficient the inverse transforms read.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "arkcos_internal.h"

namespace arkcos {

arkcos_status_t run_pipeline(arkcos_plan_s* P, const void* x, void* y, void* ws, int adjoint, hipStream_t s);
arkcos_status_t check_plan_maps(const arkcos_plan_s* P, const void* in, const void* out);

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (null: not looked up yet)

// The device address of this device's `scratch`, looked up on the first call
// with `dev` current.
arkcos_status_t scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ARKCOS_ERR_NOT_SUPPORTED, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ARKCOS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return ARKCOS_OK;
}

}  // namespace

}  // namespace arkcos

using namespace arkcos;

extern "C" {

arkcos_status_t arkcos_convolve_noalloc(arkcos_plan_t plan, const void* x, void* y, hipStream_t stream) {
  if (!plan) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan");
  const size_t need = workspace_bytes(plan);
  if (need > kScratchBytes)
    return fail(ARKCOS_ERR_NOT_SUPPORTED, "plan workspace of " + std::to_string(need) +
                                              " bytes exceeds the fixed scratch of " +
                                              std::to_string(kScratchBytes) + " bytes");
  arkcos_status_t st = check_plan_maps(plan, x, y);
  if (st != ARKCOS_OK) return st;
  void* ws = nullptr;
  st = scratch_ptr(plan->device, &ws);
  if (st != ARKCOS_OK) return st;
  return run_pipeline(plan, x, y, ws, 0, stream);
}

size_t arkcos_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
