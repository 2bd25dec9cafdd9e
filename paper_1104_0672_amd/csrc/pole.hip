// The first and last HEALPix ring (4 pixels each) recomputed by the direct
// sum y_p = sum_q K(theta_pq) x_q w_q (paper Sect. 4.2), in FP64 with the
// haversine distance.  In the transposed map the same 8 rows become 8
// columns: xbar_q += w_q sum_{p in poles} K(theta_pq) r_p.
#include "arkcos_internal.h"
#include "device_common.h"

namespace arkcos {

struct PoleArgs {
  const int32_t* n;
  const int64_t* start;
  const int32_t* phase_den;
  const double* theta;
  const double* sint;
  const double* w;
  int32_t nrings;
  int32_t kind;     // profile
  double inv2s2, radius, h, theta_max;
  int32_t nk;
  const double* knots;
  const double* mom;
};

__device__ __forceinline__ double pole_profile(const PoleArgs& P, double t) {
  if (t > P.radius) return 0.0;
  if (P.kind == 0) return exp(-t * t * P.inv2s2);
  if (t > P.theta_max + kSupportTol) return 0.0;
  int a = (int)floor(t / P.h);
  a = a < 0 ? 0 : (a > P.nk - 2 ? P.nk - 2 : a);
  double u = t / P.h - a, v = 1.0 - u, h2 = P.h * P.h / 6.0;
  return v * P.knots[a] + u * P.knots[a + 1] +
         h2 * ((v * v * v - v) * P.mom[a] + (u * u * u - u) * P.mom[a + 1]);
}

// Longitude of pixel k of a ring, in units of pi: (2k + s) / N with s = 1 for
// rings offset by pi / N (all HEALPix polar rings and the shifted equatorial
// rings, where phase_den = N), s = 0 otherwise.
__device__ __forceinline__ double pixel_distance(const PoleArgs& P, int ia, int ka, int ib, int kb) {
  int64_t na = P.n[ia], nb = P.n[ib];
  int64_t sa = P.phase_den[ia] ? 1 : 0, sb = P.phase_den[ib] ? 1 : 0;
  // (phi_a - phi_b) / (2 pi) = ((2ka + sa) nb - (2kb + sb) na) / (2 na nb)
  int64_t num = (2 * (int64_t)ka + sa) * nb - (2 * (int64_t)kb + sb) * na;
  double half_dphi = sinpi((double)num / (double)(2 * na * nb));
  double a = sin(0.5 * (P.theta[ia] - P.theta[ib]));
  double hav = a * a + P.sint[ia] * P.sint[ib] * half_dphi * half_dphi;
  double r = sqrt(hav);
  return 2.0 * asin(r < 1.0 ? r : 1.0);
}

// The direct sum for pole pixel b (0..3: first ring, 4..7: last ring) with
// the whole block; `rings` lists the rings within R of either pole ring.
// The rings of the list (kPoleRings at a time) and their pixel counts are
// staged in LDS, so the candidate pixels of all rings are spread over the
// threads at once.  Returns the block's sum on every thread.
constexpr int kPoleRings = 256;

template <typename R>
__device__ double pole_pixel_sum(const PoleArgs& P, const int32_t* __restrict__ rings, int nlist, int b,
                                 const R* __restrict__ x) {
  __shared__ int32_t rj[kPoleRings], rfirst[kPoleRings + 1];
  __shared__ double red[kBlock];
  const int ip = b < 4 ? 0 : P.nrings - 1, kp = b & 3;
  double acc = 0.0;
  for (int l0 = 0; l0 < nlist; l0 += kPoleRings) {
    const int cnt = min(kPoleRings, nlist - l0);
    // pixel counts of the rings in reach (0 for the others), then their prefix sums
    if (threadIdx.x < cnt) {
      const int j = rings[l0 + threadIdx.x];
      rj[threadIdx.x] = j;
      rfirst[threadIdx.x + 1] = fabs(P.theta[j] - P.theta[ip]) > P.radius ? 0 : P.n[j];
    }
    if (threadIdx.x == 0) rfirst[0] = 0;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int t = 0; t < cnt; ++t) rfirst[t + 1] += rfirst[t];
    __syncthreads();
    const int total = rfirst[cnt];
    int t = 0;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
      while (rfirst[t + 1] <= q) ++t;
      const int j = rj[t], k = q - rfirst[t];
      const double d = pixel_distance(P, ip, kp, j, k);
      acc += pole_profile(P, d) * P.w[j] * (double)x[P.start[j] + k];
    }
    __syncthreads();
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  return red[0];
}

// Forward: one block per pole pixel (blockIdx.x < 8).
template <typename R>
__global__ void __launch_bounds__(kBlock) pole_forward_kernel(PoleArgs P, const int32_t* __restrict__ rings,
                                                              int32_t nlist, const R* __restrict__ x,
                                                              R* __restrict__ y) {
  const int b = blockIdx.x;
  const double v = pole_pixel_sum<R>(P, rings, nlist, b, x);
  if (threadIdx.x == 0) y[P.start[b < 4 ? 0 : P.nrings - 1] + (b & 3)] = (R)v;
}

// Transpose: one block per ring j within the support of either pole ring.
template <typename R>
__global__ void __launch_bounds__(kBlock) pole_adjoint_kernel(PoleArgs P, const int32_t* __restrict__ rings,
                                                              const R* __restrict__ r, R* __restrict__ xbar) {
  const int j = rings[blockIdx.x];
  const int nj = P.n[j];
  for (int k = threadIdx.x; k < nj; k += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < 8; ++b) {
      const int ip = b < 4 ? 0 : P.nrings - 1, kp = b & 3;
      if (fabs(P.theta[j] - P.theta[ip]) > P.radius) continue;
      double t = pixel_distance(P, ip, kp, j, k);
      acc += pole_profile(P, t) * (double)r[P.start[ip] + kp];
    }
    int64_t q = P.start[j] + k;
    xbar[q] = (R)((double)xbar[q] + P.w[j] * acc);
  }
}

PoleArgs make_pole_args(arkcos_plan_s* P) {
  PoleArgs a{};
  a.n = P->rt.n;
  a.start = P->rt.start;
  a.phase_den = P->rt.phase_den;
  a.theta = P->d_theta;
  a.sint = P->d_sin;
  a.w = P->rt.w;
  a.nrings = (int32_t)P->nrings;
  a.kind = P->prof_kind;
  double sigma = P->fwhm / sqrt(8.0 * log(2.0));
  a.inv2s2 = P->prof_kind == 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
  a.radius = P->radius + kSupportTol;
  a.nk = (int32_t)P->knots.size();
  a.theta_max = P->theta_max;
  a.h = a.nk > 1 ? P->theta_max / (a.nk - 1) : 0.0;
  a.knots = P->d_knots;
  a.mom = P->d_spline_mom;
  return a;
}

hipError_t launch_pole_fix(arkcos_plan_s* P, const void* x, void* y, int32_t adjoint, hipStream_t s) {
  PoleArgs a = make_pole_args(P);
  int32_t count = 0;
  int32_t* list = pole_ring_list(P, &count);
  if (count == 0) return hipSuccess;
  if (!adjoint) {
    if (P->dtype == ARKCOS_F32)
      pole_forward_kernel<float><<<8, kBlock, 0, s>>>(a, list, count, (const float*)x, (float*)y);
    else
      pole_forward_kernel<double><<<8, kBlock, 0, s>>>(a, list, count, (const double*)x, (double*)y);
  } else {
    if (P->dtype == ARKCOS_F32)
      pole_adjoint_kernel<float><<<count, kBlock, 0, s>>>(a, list, (const float*)x, (float*)y);
    else
      pole_adjoint_kernel<double><<<count, kBlock, 0, s>>>(a, list, (const double*)x, (double*)y);
  }
  return hipGetLastError();
}

// Batched pole rows: entry (map, k) with k < 8 (forward: pole pixel) or k an
// index into the map's pole-ring list (transpose).
struct PoleMap {
  PoleArgs a;
  const int32_t* rings;
  int32_t nlist;
  int32_t pad;
};

template <typename R>
__global__ void __launch_bounds__(kBlock) pole_batch_kernel(const PoleMap* __restrict__ maps,
                                                            const int2* __restrict__ entries, int32_t adjoint,
                                                            const R* const* __restrict__ xs, R* const* __restrict__ ys) {
  const int2 e = entries[blockIdx.x];
  const PoleMap pm = maps[e.x];
  const PoleArgs& P = pm.a;
  const R* x = xs[e.x];
  R* y = ys[e.x];
  if (!adjoint) {
    const int b = e.y;
    const double v = pole_pixel_sum<R>(P, pm.rings, pm.nlist, b, x);
    if (threadIdx.x == 0) y[P.start[b < 4 ? 0 : P.nrings - 1] + (b & 3)] = (R)v;
  } else {
    const int j = pm.rings[e.y];
    const int nj = P.n[j];
    for (int k = threadIdx.x; k < nj; k += blockDim.x) {
      double acc = 0.0;
      for (int b = 0; b < 8; ++b) {
        const int ip = b < 4 ? 0 : P.nrings - 1, kp = b & 3;
        if (fabs(P.theta[j] - P.theta[ip]) > P.radius) continue;
        acc += pole_profile(P, pixel_distance(P, ip, kp, j, k)) * (double)x[P.start[ip] + kp];
      }
      const int64_t q = P.start[j] + k;
      y[q] = (R)((double)y[q] + P.w[j] * acc);
    }
  }
}

size_t pole_map_size() { return sizeof(PoleMap); }

void fill_pole_map(arkcos_plan_s* P, void* out) {
  PoleMap pm{};
  pm.a = make_pole_args(P);
  pm.rings = pole_ring_list(P, &pm.nlist);
  *reinterpret_cast<PoleMap*>(out) = pm;
}

hipError_t launch_pole_batch(arkcos_dtype_t dt, const void* maps, const int2* entries, int32_t count, int32_t adjoint,
                             const void* xs, const void* ys, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (dt == ARKCOS_F32)
    pole_batch_kernel<float><<<count, kBlock, 0, s>>>((const PoleMap*)maps, entries, adjoint,
                                                      (const float* const*)xs, (float* const*)ys);
  else
    pole_batch_kernel<double><<<count, kBlock, 0, s>>>((const PoleMap*)maps, entries, adjoint,
                                                       (const double* const*)xs, (double* const*)ys);
  return hipGetLastError();
}

}  // namespace arkcos
