// The extern "C" entry points declared in include/arkcos.h: argument checks
// on the host, then asynchronous launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "arkcos_internal.h"

namespace arkcos {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

arkcos_status_t fail(arkcos_status_t st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

arkcos_status_t build_plan(const arkcos_geometry_t* g, const arkcos_profile_t* prof, double R,
                           arkcos_dtype_t dtype, const arkcos_options_t* o, arkcos_plan_s** out);
hipError_t update_knots(arkcos_plan_s* P, const double* d_src, hipStream_t s);
arkcos_status_t run_kernel_grad(arkcos_plan_s* P, const void* x, const void* r, double* grad,
                                void* ws, uint32_t flags, hipStream_t s);

static size_t elem_size(const arkcos_plan_s* P) {
  return P->dtype == ARKCOS_F32 ? sizeof(float) : sizeof(double);
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

static arkcos_status_t check_device(const arkcos_plan_s* P) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(ARKCOS_ERR_DEVICE, "hipGetDevice failed");
  if (dev != P->device) return fail(ARKCOS_ERR_INVALID_VALUE, "plan was created on another device");
  return ARKCOS_OK;
}

// Maps only: non-null, disjoint, aligned, and the plan's device current.
arkcos_status_t check_plan_maps(const arkcos_plan_s* P, const void* in, const void* out) {
  if (!in || !out) return fail(ARKCOS_ERR_INVALID_VALUE, "null map pointer");
  const size_t bytes = (size_t)P->npix * elem_size(P);
  if (overlaps(in, bytes, out, bytes)) return fail(ARKCOS_ERR_INVALID_VALUE, "input and output maps overlap");
  if (reinterpret_cast<uintptr_t>(in) % elem_size(P) || reinterpret_cast<uintptr_t>(out) % elem_size(P))
    return fail(ARKCOS_ERR_INVALID_VALUE, "misaligned map pointer");
  return check_device(P);
}

static arkcos_status_t check_maps(const arkcos_plan_s* P, const void* in, const void* out, const void* ws) {
  if (!in || !out || !ws) return fail(ARKCOS_ERR_INVALID_VALUE, "null map or workspace pointer");
  const size_t bytes = (size_t)P->npix * elem_size(P);
  const size_t wsb = workspace_bytes(P);
  if (overlaps(in, bytes, ws, wsb) || overlaps(out, bytes, ws, wsb))
    return fail(ARKCOS_ERR_INVALID_VALUE, "workspace overlaps a map");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(ARKCOS_ERR_INVALID_VALUE, "workspace must be 256-byte aligned");
  return check_plan_maps(P, in, out);
}

void workspace_split(const arkcos_plan_s* P, void* ws, void** spec, void** bout) {
  const size_t csz = P->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  size_t a = ((size_t)std::max<int64_t>(P->spec_total, 1) * csz + 255) / 256 * 256;
  *spec = ws;
  *bout = static_cast<char*>(ws) + a;
}

#define LAUNCH(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

arkcos_status_t run_pipeline(arkcos_plan_s* P, const void* x, void* y, void* ws, int adjoint,
                             hipStream_t s) {
  void *spec, *bout;
  workspace_split(P, ws, &spec, &bout);
  const bool fix = P->geom.kind == 1 && P->opts.fix_pole_pixels;
  hipEvent_t* ev = nullptr;
  if (P->timing_used < P->timing_slots) ev = &P->timing_events[5 * P->timing_used++];
  if (ev) LAUNCH(hipEventRecord(ev[0], s));
  LAUNCH(launch_r2c(P, x, spec, adjoint, adjoint && fix ? 1 : 0, s));
  if (ev) LAUNCH(hipEventRecord(ev[1], s));
  LAUNCH(launch_accumulate(P, spec, bout, s));
  if (ev) LAUNCH(hipEventRecord(ev[2], s));
  LAUNCH(launch_c2r(P, bout, y, adjoint, s));
  if (ev) LAUNCH(hipEventRecord(ev[3], s));
  if (fix) LAUNCH(launch_pole_fix(P, x, y, adjoint, s));
  if (ev) LAUNCH(hipEventRecord(ev[4], s));
  return ARKCOS_OK;
}

}  // namespace arkcos

using namespace arkcos;

extern "C" {

void arkcos_default_options(arkcos_options_t* o) {
  if (!o) return;
  o->oversample = 0;
  o->kgen = 0;
  o->fix_pole_pixels = 1;
  o->band_tol = -1.0;
  o->mode = 0;
  o->own_grid = 0;
  o->kernel_eval = 0;
  o->table_nodes = 0;
  for (int32_t& r : o->reserved) r = 0;
}

arkcos_status_t arkcos_plan(const arkcos_geometry_t* geom, const arkcos_profile_t* profile,
                            double support_radius_rad, arkcos_dtype_t dtype,
                            const arkcos_options_t* opts, arkcos_plan_t* out) {
  g_last_error.clear();
  try {
    return build_plan(geom, profile, support_radius_rad, dtype, opts, out);
  } catch (const std::bad_alloc&) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(ARKCOS_ERR_INTERNAL, "unexpected exception in plan creation");
  }
}

arkcos_status_t arkcos_plan_for_error(const arkcos_geometry_t* geom, const arkcos_profile_t* profile,
                                      const double* cl, int32_t lmax, double target_sigma2,
                                      arkcos_dtype_t dtype, const arkcos_options_t* opts,
                                      arkcos_plan_t* out, double* radius_rad) {
  g_last_error.clear();
  if (!out) return fail(ARKCOS_ERR_INVALID_VALUE, "null output handle");
  double R = 0.0;
  arkcos_status_t st = arkcos_choose_radius(profile, cl, lmax, target_sigma2, &R);
  if (st != ARKCOS_OK) return st;
  if (!(R > 0.0))
    return fail(ARKCOS_ERR_NOT_SUPPORTED, "the truncation-error target holds without any kernel support (R = 0)");
  st = arkcos_plan(geom, profile, R, dtype, opts, out);
  if (st == ARKCOS_OK && radius_rad) *radius_rad = R;
  return st;
}

arkcos_status_t arkcos_plan_destroy(arkcos_plan_t plan) {
  if (!plan) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != plan->device) (void)hipSetDevice(plan->device);
  for (void* a : plan->allocations) (void)hipFree(a);
  for (hipEvent_t e : plan->timing_events) (void)hipEventDestroy(e);
  if (cur != plan->device) (void)hipSetDevice(cur);
  delete plan;
  return ARKCOS_OK;
}

arkcos_status_t arkcos_plan_get_info(arkcos_plan_t P, arkcos_plan_info_t* info) {
  if (!P || !info) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  std::memset(info, 0, sizeof(*info));
  info->npix = P->npix;
  info->nrings = P->nrings;
  for (const auto& U : P->h_units) info->n_pairs += (int64_t)(U.pend - U.pbeg) * (U.im >= 0 ? 2 : 1);
  info->n_table_pairs = P->n_table_pairs;
  info->spectrum_modes = P->spec_total;
  info->output_modes = P->out_total;
  info->pair_modes = P->pair_modes;
  info->taps = P->coef_total;
  info->table_entries = P->table_total;
  info->oversample = P->oversample;
  info->dtype = P->dtype;
  info->n_knots = (int32_t)P->knots.size();
  info->workspace_bytes = workspace_bytes(P);
  info->plan_bytes = P->plan_bytes;
  for (const auto& pr : P->h_pairs)
    if (pr.band >= 0 && pr.kind >= 0 && pr.kind < 4) ++info->pairs_by_kind[pr.kind];
  info->acc_seg_units = P->acc_units;
  info->acc_group = P->acc_tiles;
  info->acc_window = P->acc_shape.max_window;
  info->acc_tuned = P->acc_tuned;
  info->support_radius_rad = P->radius;
  info->table_fft_rows = P->n_tfft[0] + P->n_tfft[1] + P->n_tfft[2];
  info->grad_fft_rows = P->n_gfft[0] + P->n_gfft[1] + P->n_gfft[2];
  info->acc_units_per_wave = P->acc_upw;
  return ARKCOS_OK;
}

arkcos_status_t arkcos_workspace_size(arkcos_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  *bytes = workspace_bytes(plan);
  return ARKCOS_OK;
}

arkcos_status_t arkcos_convolve(arkcos_plan_t plan, const void* x, void* y, void* ws, hipStream_t stream) {
  if (!plan) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan");
  arkcos_status_t st = check_maps(plan, x, y, ws);
  if (st != ARKCOS_OK) return st;
  return run_pipeline(plan, x, y, ws, 0, stream);
}

arkcos_status_t arkcos_convolve_adjoint(arkcos_plan_t plan, const void* r, void* xbar, void* ws,
                                        hipStream_t stream) {
  if (!plan) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan");
  arkcos_status_t st = check_maps(plan, r, xbar, ws);
  if (st != ARKCOS_OK) return st;
  return run_pipeline(plan, r, xbar, ws, 1, stream);
}

arkcos_status_t arkcos_kernel_grad(arkcos_plan_t plan, const void* x, const void* r, double* grad,
                                   void* ws, uint32_t flags, hipStream_t stream) {
  if (!plan) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan");
  if (plan->prof_kind != 1) return fail(ARKCOS_ERR_NOT_SUPPORTED, "knot gradient needs a spline profile");
  if (plan->opts.kernel_eval != 0)
    return fail(ARKCOS_ERR_NOT_SUPPORTED, "knot gradient needs the exact kernel evaluation (kernel_eval 0)");
  if (!grad) return fail(ARKCOS_ERR_INVALID_VALUE, "null gradient pointer");
  if (!x || !r || !ws) return fail(ARKCOS_ERR_INVALID_VALUE, "null map or workspace pointer");
  const size_t bytes = (size_t)plan->npix * elem_size(plan);
  const size_t wsb = workspace_bytes(plan);
  if (overlaps(x, bytes, ws, wsb) || overlaps(r, bytes, ws, wsb) ||
      overlaps(grad, plan->knots.size() * sizeof(double), ws, wsb))
    return fail(ARKCOS_ERR_INVALID_VALUE, "workspace overlaps an argument");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(ARKCOS_ERR_INVALID_VALUE, "workspace must be 256-byte aligned");
  arkcos_status_t st = check_device(plan);
  if (st != ARKCOS_OK) return st;
  return run_kernel_grad(plan, x, r, grad, ws, flags, stream);
}

arkcos_status_t arkcos_set_knots(arkcos_plan_t plan, const double* knot_values) {
  if (!plan || !knot_values) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (plan->prof_kind != 1) return fail(ARKCOS_ERR_NOT_SUPPORTED, "plan has no spline profile");
  arkcos_status_t st = check_device(plan);
  if (st != ARKCOS_OK) return st;
  // every call already enqueued (on any stream) finishes with the old knots
  LAUNCH(hipDeviceSynchronize());
  LAUNCH(hipMemcpy(plan->d_knots, knot_values, plan->knots.size() * sizeof(double), hipMemcpyHostToDevice));
  LAUNCH(update_knots(plan, plan->d_knots, nullptr));
  LAUNCH(hipStreamSynchronize(nullptr));
  return ARKCOS_OK;
}

arkcos_status_t arkcos_set_knots_async(arkcos_plan_t plan, const double* knot_values, hipStream_t stream) {
  if (!plan || !knot_values) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (plan->prof_kind != 1) return fail(ARKCOS_ERR_NOT_SUPPORTED, "plan has no spline profile");
  arkcos_status_t st = check_device(plan);
  if (st != ARKCOS_OK) return st;
  LAUNCH(update_knots(plan, knot_values, stream));
  return ARKCOS_OK;
}

arkcos_status_t arkcos_plan_timing(arkcos_plan_t plan, int32_t max_calls) {
  if (!plan || max_calls < 0) return fail(ARKCOS_ERR_INVALID_VALUE, "bad argument");
  for (hipEvent_t e : plan->timing_events) (void)hipEventDestroy(e);
  plan->timing_events.clear();
  plan->timing_slots = plan->timing_used = 0;
  if (max_calls == 0) return ARKCOS_OK;
  plan->timing_events.resize(5 * (size_t)max_calls);
  for (auto& e : plan->timing_events)
    if (hipEventCreate(&e) != hipSuccess) return fail(ARKCOS_ERR_DEVICE, "hipEventCreate failed");
  plan->timing_slots = max_calls;
  return ARKCOS_OK;
}

arkcos_status_t arkcos_stage_times(arkcos_plan_t plan, double* ms, int64_t* calls) {
  if (!plan || !ms || !calls) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  for (int32_t c = 0; c < plan->timing_used; ++c) {
    hipEvent_t* ev = &plan->timing_events[5 * c];
    if (hipEventSynchronize(ev[4]) != hipSuccess) return fail(ARKCOS_ERR_DEVICE, "hipEventSynchronize failed");
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess)
        return fail(ARKCOS_ERR_DEVICE, "hipEventElapsedTime failed");
      ms[k] += t;
    }
  }
  *calls = plan->timing_used;
  plan->timing_used = 0;
  return ARKCOS_OK;
}

const char* arkcos_status_string(arkcos_status_t s) {
  switch (s) {
    case ARKCOS_OK: return "ARKCOS_OK";
    case ARKCOS_ERR_INVALID_VALUE: return "ARKCOS_ERR_INVALID_VALUE";
    case ARKCOS_ERR_NOT_SUPPORTED: return "ARKCOS_ERR_NOT_SUPPORTED";
    case ARKCOS_ERR_OUT_OF_MEMORY: return "ARKCOS_ERR_OUT_OF_MEMORY";
    case ARKCOS_ERR_DEVICE: return "ARKCOS_ERR_DEVICE";
    case ARKCOS_ERR_INTERNAL: return "ARKCOS_ERR_INTERNAL";
  }
  return "ARKCOS_UNKNOWN_STATUS";
}

const char* arkcos_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
