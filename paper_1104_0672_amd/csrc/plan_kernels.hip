// Plan-time kernels: the kernel rows of every ring pair (step b of the
// hybrid method, paper Sect. 4.1), their bands, the optional K_ij(m) tables,
// and the Bluestein filters of the ring FFTs.
//
// The angular distance between a pixel of output ring i (at longitude 0) and
// a longitude nu on input ring j is evaluated in FP64 haversine form,
//   hav = sin^2((theta_i - theta_j)/2) + sin(theta_i) sin(theta_j) sin^2(nu/2),
//   theta = 2 asin(sqrt(hav)),
// which equals the paper's alpha^2 = 2(1 - cos alpha) parametrisation
// (eq. "kernel_angle") without its cancellation at small angles.
#include "arkcos_internal.h"
#include "device_common.h"

namespace arkcos {

struct ProfileDev {
  int32_t kind;      // 0 Gaussian, 1 spline
  double inv2s2;     // 1 / (2 sigma^2)
  double radius;     // support radius + tolerance
  int32_t nk;
  double h, theta_max;
  const double* knots;
  const double* mom;
  // the biased linear table of Sect. 4.1 (kernel_eval = 1): T[k] =
  // K(2 asin(sqrt(u_k) / 2)) at u_k = k du, k < tn, du = u(radius) / (tn - 1)
  const double* utab;
  int32_t tn;
  double du, umax;
};

__device__ __forceinline__ double profile_eval(const ProfileDev& P, double t) {
  if (t > P.radius) return 0.0;
  if (P.kind == 0) return exp(-t * t * P.inv2s2);
  if (t > P.theta_max + kSupportTol) return 0.0;
  int a = (int)floor(t / P.h);
  a = a < 0 ? 0 : (a > P.nk - 2 ? P.nk - 2 : a);
  double u = t / P.h - a, v = 1.0 - u, h2 = P.h * P.h / 6.0;
  return v * P.knots[a] + u * P.knots[a + 1] +
         h2 * ((v * v * v - v) * P.mom[a] + (u * u * u - u) * P.mom[a + 1]);
}

// Haversine of the distance between (theta_i, 0) and (theta_j, nu) with
// nu = pi * num / den: hav = sin^2(theta / 2).
__device__ __forceinline__ double ring_hav(double ti, double tj, double si, double sj, int64_t num, int64_t den) {
  double a = sin(0.5 * (ti - tj));
  double b = sinpi(0.5 * (double)num / (double)den);
  return a * a + si * sj * b * b;
}

// K at the sample of haversine hav: from the exact distance
// theta = 2 asin(sqrt(hav)), or, with the table of Sect. 4.1, by linear
// interpolation in the squared chord u = 2 (1 - cos theta) = 4 hav.
__device__ __forceinline__ double kernel_at(const ProfileDev& P, double hav) {
  if (P.utab) {
    const double u = 4.0 * hav;
    if (u > P.umax) return 0.0;
    const double x = u / P.du;
    int k = (int)floor(x);
    k = k < 0 ? 0 : (k > P.tn - 2 ? P.tn - 2 : k);
    const double f = x - (double)k;
    return fma(f, P.utab[k + 1] - P.utab[k], P.utab[k]);
  }
  const double r = sqrt(hav);
  return profile_eval(P, 2.0 * asin(r < 1.0 ? r : 1.0));
}

// Fills the table of the biased kernel evaluation (kernel_eval = 1).
__global__ void __launch_bounds__(kBlock) utable_kernel(ProfileDev prof, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= prof.tn) return;
  // the last node sits at the support radius itself
  const double r = 0.5 * sqrt((double)k * prof.du);
  out[k] = profile_eval(prof, k == prof.tn - 1 ? prof.radius : 2.0 * asin(r < 1.0 ? r : 1.0));
}

// Node d of pair q: nu_d / pi = 2 (d + s/2) / (p L) = (2d + s) / (p L).
// Every sample of the pair's window is written (at coef_off[q]); abs_sum
// (optional) receives the sum of their magnitudes.
template <typename R>
__global__ void __launch_bounds__(kBlock) kernel_rows_kernel(
    const PairDev* __restrict__ pairs, const int32_t* __restrict__ pair_i,
    const int32_t* __restrict__ pair_shift, const int64_t* __restrict__ coef_off,
    const int32_t* __restrict__ ncoef_window, const double* __restrict__ theta,
    const double* __restrict__ sint, const double* __restrict__ w, int64_t L, ProfileDev prof,
    double* __restrict__ coef64, R* __restrict__ coef, double* __restrict__ abs_sum) {
  const int q = blockIdx.x;
  PairDev pr = pairs[q];
  pr.off = coef_off[q];
  pr.ncoef = ncoef_window[q];
  const int i = pair_i[q], j = pr.j, s = pair_shift[q];
  const int64_t pl = (int64_t)pr.grid;
  const double ti = theta[i], tj = theta[j], si = sint[i], sj = sint[j];
  double part = 0.0;
  for (int d = threadIdx.x; d < pr.ncoef; d += blockDim.x) {
    double g = w[j] * kernel_at(prof, ring_hav(ti, tj, si, sj, 2 * (int64_t)d + s, pl));
    double c = 2.0;
    if (s == 0 && (d == 0 || 2 * (int64_t)d == pl)) c = 1.0;
    double a = c * g / (double)pl;
    coef64[pr.off + d] = a;
    coef[pr.off + d] = (R)a;
    part += fabs(a);
  }
  if (!abs_sum) return;
  __shared__ double red[kBlock];
  red[threadIdx.x] = part;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) abs_sum[q] = red[0];
}

// K_ij(m) in FP64 from the kernel samples:
//   centred grid:  K(m) = sum_d a_d cos(d x),        x = 2 pi m / (p L)
//   shifted grid:  K(m) = sum_d a_d cos((2d+1) y),   y = pi m / L
// with the half weight of the grid's Nyquist mode m = p L / 2.  The centred
// sum uses Reinsch's modification of the Clenshaw recurrence, which carries
// the differences b_k -/+ b_k+1 and the exactly computed 1 -/+ cos x, so its
// rounding error does not grow with the number of samples near x = 0 and
// x = pi (where the plain recurrence loses ~n^2 eps, enough to fake a wide
// band for full-ring pairs).
__device__ __forceinline__ double k_of_m_fp64(const double* __restrict__ a, int n, int m, int shift,
                                              int64_t pl, int nyq) {
  double k;
  if (shift) {
    const double cx = cospi(2.0 * (double)m / (double)pl), cy = cospi((double)m / (double)pl);
    double al = 2.0 * cx, b1 = 0.0, b2 = 0.0;
    for (int d = n - 1; d >= 0; --d) {
      double b0 = fma(al, b1, a[d] - b2);
      b2 = b1;
      b1 = b0;
    }
    k = (b1 - b2) * cy;
  } else {
    const double hx = (double)m / (double)pl;      // x / (2 pi)
    const double sh = sinpi(hx), ch = cospi(hx);  // sin(x/2), cos(x/2)
    double b = 0.0, dd = 0.0;
    if (ch * ch >= 0.5) {                          // cos x >= 0: d_k = b_k - b_k+1
      const double lam = -4.0 * sh * sh;           // 2 cos x - 2
      for (int d = n - 1; d >= 0; --d) {
        dd = fma(lam, b, dd + a[d]);
        b = b + dd;
      }
      k = dd - 0.5 * lam * (b - dd);               // S = d_0 - (lam/2) b_1
    } else {                                       // cos x < 0: d_k = b_k + b_k+1
      const double lam = 4.0 * ch * ch;            // 2 cos x + 2
      for (int d = n - 1; d >= 0; --d) {
        dd = fma(lam, b, a[d] - dd);
        b = dd - b;
      }
      k = dd - 0.5 * lam * (dd - b);               // S = d_0 - (lam/2) b_1
    }
  }
  return m == nyq ? 0.5 * k : k;
}

__global__ void __launch_bounds__(kBlock) band_kernel(
    const PairDev* __restrict__ pairs, const int32_t* __restrict__ pair_shift,
    const double* __restrict__ coef64, int64_t L, double thr, int32_t* __restrict__ band_out) {
  const int q = blockIdx.x;
  const PairDev pr = pairs[q];
  const int64_t pl = (int64_t)pr.grid;
  int best = -1;
  for (int m = threadIdx.x; m <= pr.nyq; m += blockDim.x) {
    double k = k_of_m_fp64(coef64 + pr.off, pr.ncoef, m, pair_shift[q], pl, pr.nyq);
    if (fabs(k) > thr) best = m;
  }
  __shared__ int red[kBlock];
  red[threadIdx.x] = best;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) band_out[q] = red[0];
}

// Tables: K_ij(m) for m <= band of the pairs listed in `list` (their coef64
// offsets are read from `coef_off`, their table offsets from pairs[].off),
// zero from band + 1 to the end of the last mode tile.
template <typename R>
__global__ void __launch_bounds__(kBlock) table_kernel(
    const PairDev* __restrict__ pairs, const int32_t* __restrict__ pair_shift,
    const int32_t* __restrict__ list, const int64_t* __restrict__ coef_off,
    const double* __restrict__ coef64, int64_t L, R* __restrict__ table) {
  const int t = blockIdx.x;
  const int q = list[t];
  const PairDev pr = pairs[q];
  const int64_t pl = (int64_t)pr.grid;
  const int end = table_span(pr.band);
  for (int m = threadIdx.x; m < end; m += blockDim.x)
    table[pr.off + m] =
        m <= pr.band ? (R)k_of_m_fp64(coef64 + coef_off[t], pr.ncoef, m, pair_shift[q], pl, pr.nyq) : R(0);
}

// Tables of the FFT rows (spline plans): K(m) = h(m) sum_{d < n} a_d cos(2 pi m d / G)
// for m <= band (h = 1/2 at the Nyquist mode), zero to the end of the last
// tile.  With S = G / (2 P), the samples split into S real sub-sequences
// x_q = a_{S q + s} of 2 P points, and
//   K(m) = Re sum_s exp(-2 pi i s m / G) X_s(m mod 2P),
// X_s the forward 2P-point transform of x (one packed P-point LDS FFT).  One
// block per row; each thread keeps its modes over the passes, so the
// table's partial sums need no synchronisation.
template <typename R, int NT>
__global__ void __launch_bounds__(NT) table_fft_kernel(const PairDev* __restrict__ pairs,
                                                       const RowFft* __restrict__ rows,
                                                       const int64_t* __restrict__ coef_off,
                                                       const double* __restrict__ coef64,
                                                       const cx_t<R>* __restrict__ tw, int64_t TN,
                                                       R* __restrict__ table) {
  using C = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const RowFft row = rows[blockIdx.x];
  const int q = row.pair, Pn = row.P;
  const PairDev pr = pairs[q];
  const int64_t G = pr.grid;
  const int S = (int)(G / (2 * (int64_t)Pn));
  const int nc = pr.ncoef, band = pr.band;
  const double* a = coef64 + coef_off[q];
  R* T = table + pr.off;
  const int64_t kstep = TN / (2 * (int64_t)Pn), gstep = TN / G;
  for (int s = 0; s < S; ++s) {
    for (int l = threadIdx.x; l < Pn; l += NT) {
      const int64_t d0 = (int64_t)S * (2 * l) + s, d1 = d0 + S;
      buf[lidx(l)] = cmake<C>(d0 < nc ? (R)a[d0] : R(0), d1 < nc ? (R)a[d1] : R(0));
    }
    __syncthreads();
    lds_fft<R, false, NT>(buf, Pn, tw, (int)TN);
    for (int m = threadIdx.x; m <= band; m += NT) {
      const int k = m & (2 * Pn - 1);
      const C X = real_from_packed<R>(buf, Pn, k, tw[k * kstep]);
      const C ph = tw[(((int64_t)s * m) & (G - 1)) * gstep];  // exp(-2 pi i s m / G)
      const R v = ph.x * X.x - ph.y * X.y;
      T[m] = s == 0 ? v : T[m] + v;
    }
    __syncthreads();  // buf is rewritten by the next pass
  }
  const int end = table_span(band);
  for (int m = threadIdx.x; m < end; m += NT) {
    if (m > band) T[m] = R(0);
    else if (m == pr.nyq) T[m] *= R(0.5);
  }
}

template <typename R, int NT>
static hipError_t table_fft_launch(arkcos_plan_s* P, const RowFft* rows, int32_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  int32_t pmax = NT * 16;
  const size_t lds = (size_t)lds_elems(pmax) * sizeof(cx_t<R>);
  hipError_t e = hipFuncSetAttribute((const void*)table_fft_kernel<R, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  table_fft_kernel<R, NT><<<count, NT, lds, s>>>(P->d_pairs, rows, P->d_coef_off, P->d_coef64,
                                                 (const cx_t<R>*)P->d_twiddle, P->twiddle_n, (R*)P->d_table);
  return hipGetLastError();
}

hipError_t launch_table_fft(arkcos_plan_s* P, hipStream_t s) {
  const RowFft* r0 = P->d_tfft;
  const RowFft* r1 = r0 + P->n_tfft[0];
  const RowFft* r2 = r1 + P->n_tfft[1];
  hipError_t e;
  if (P->dtype == ARKCOS_F32) {
    e = table_fft_launch<float, 256>(P, r0, P->n_tfft[0], s);
    if (e == hipSuccess) e = table_fft_launch<float, 512>(P, r1, P->n_tfft[1], s);
    if (e == hipSuccess) e = table_fft_launch<float, 1024>(P, r2, P->n_tfft[2], s);
  } else {
    e = table_fft_launch<double, 256>(P, r0, P->n_tfft[0], s);
    if (e == hipSuccess) e = table_fft_launch<double, 512>(P, r1, P->n_tfft[1], s);
  }
  return e;
}

// Bluestein filter of length n: FFT_M of b_l = exp(+i pi l^2 / n) placed at l
// and M - l for 0 <= l < n, followed by the chirp exp(-i pi l^2 / n), l < n,
// and the ring's half-angle phases w_r = exp(-i pi r / (2 n)), r <= n / 2
// (the ring has N = 2 n pixels).
template <typename R, int NT>
__global__ void __launch_bounds__(NT) bluestein_filter_kernel(
    const int32_t* __restrict__ rings, const int32_t* __restrict__ ring_n,
    const int32_t* __restrict__ fft_m, const int64_t* __restrict__ bl_off,
    const cx_t<R>* __restrict__ tw, int TN, cx_t<R>* __restrict__ out) {
  using C = cx_t<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  C* buf = reinterpret_cast<C*>(smem);
  const int ring = rings[blockIdx.x];
  const int n = ring_n[ring] / 2, M = fft_m[ring];
  for (int l = threadIdx.x; l < M; l += blockDim.x) {
    int src = -1;
    if (l < n) src = l;
    else if (M - l < n) src = M - l;
    buf[lidx(l)] = src >= 0 ? cconj(chirp<R>(src, n)) : cmake<C>(R(0), R(0));
  }
  __syncthreads();
  lds_fft<R, false, NT>(buf, M, tw, TN);
  C* o = out + bl_off[ring];
  for (int l = threadIdx.x; l < M; l += blockDim.x) o[l] = buf[lidx(l)];
  for (int l = threadIdx.x; l < n; l += blockDim.x) o[M + l] = chirp<R>(l, n);
  for (int r = threadIdx.x; r <= n / 2; r += blockDim.x) o[M + n + r] = cconj(expipi<R>(r, 2 * n));
}

// Clamped-spline moments of the knot values src (n of them, spacing h),
// solved on the device by the tridiagonal (Thomas) recurrence; the knots are
// copied to knots first (src may equal knots).  One thread: n <= 64.
__global__ void spline_update_kernel(const double* __restrict__ src, int n, double h, double* knots, double* mom) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double c[64], diag[64], rhs[64];
  for (int k = 0; k < n; ++k) c[k] = src[k];
  for (int k = 0; k < n; ++k) knots[k] = c[k];
  const double s6 = 6.0 / (h * h);
  for (int k = 0; k < n; ++k) {
    if (k == 0) { diag[k] = 2; rhs[k] = s6 * (c[1] - c[0]); }
    else if (k == n - 1) { diag[k] = 2; rhs[k] = -s6 * (c[n - 1] - c[n - 2]); }
    else { diag[k] = 4; rhs[k] = s6 * (c[k + 1] - 2 * c[k] + c[k - 1]); }
  }
  // sub- and super-diagonals are 1 everywhere they exist
  for (int k = 1; k < n; ++k) {
    const double f = 1.0 / diag[k - 1];
    diag[k] -= f;
    rhs[k] -= f * rhs[k - 1];
  }
  double next = rhs[n - 1] / diag[n - 1];
  mom[n - 1] = next;
  for (int k = n - 2; k >= 0; --k) {
    next = (rhs[k] - next) / diag[k];
    mom[k] = next;
  }
}

hipError_t launch_spline_update(arkcos_plan_s* P, const double* d_src, hipStream_t s) {
  const int n = (int)P->knots.size();
  spline_update_kernel<<<1, 64, 0, s>>>(d_src, n, P->theta_max / (n - 1), P->d_knots, P->d_spline_mom);
  return hipGetLastError();
}

static ProfileDev make_profile(arkcos_plan_s* P) {
  ProfileDev pd{};
  pd.kind = P->prof_kind;
  double sigma = P->fwhm / sqrt(8.0 * log(2.0));
  pd.inv2s2 = P->prof_kind == 0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
  pd.radius = P->radius + kSupportTol;
  pd.nk = (int32_t)P->knots.size();
  pd.theta_max = P->theta_max;
  pd.h = pd.nk > 1 ? P->theta_max / (pd.nk - 1) : 0.0;
  pd.knots = P->d_knots;
  pd.mom = P->d_spline_mom;
  if (P->d_utable) {
    pd.utab = P->d_utable;
    pd.tn = P->utable_n;
    const double sh = sin(0.5 * pd.radius);
    pd.umax = 4.0 * sh * sh;
    pd.du = pd.umax / (double)(pd.tn - 1);
  }
  return pd;
}

hipError_t launch_kernel_rows(arkcos_plan_s* P, double* abs_sum, hipStream_t s) {
  if (P->n_pairs == 0) return hipSuccess;
  ProfileDev pd = make_profile(P);
  if (P->d_utable) {
    // the table from the current profile first (same stream)
    ProfileDev tp = pd;
    tp.utab = nullptr;
    utable_kernel<<<(unsigned)((pd.tn + kBlock - 1) / kBlock), kBlock, 0, s>>>(tp, P->d_utable);
  }
  if (P->dtype == ARKCOS_F32)
    kernel_rows_kernel<float><<<(unsigned)P->n_pairs, kBlock, 0, s>>>(
        P->d_pairs, P->d_pair_i, P->d_pair_shift, P->d_coef_off, P->d_ncoef_window, P->d_theta, P->d_sin,
        P->rt.w, P->L, pd, P->d_coef64, (float*)P->d_coef, abs_sum);
  else
    kernel_rows_kernel<double><<<(unsigned)P->n_pairs, kBlock, 0, s>>>(
        P->d_pairs, P->d_pair_i, P->d_pair_shift, P->d_coef_off, P->d_ncoef_window, P->d_theta, P->d_sin,
        P->rt.w, P->L, pd, P->d_coef64, (double*)P->d_coef, abs_sum);
  return hipGetLastError();
}

hipError_t launch_band(arkcos_plan_s* P, double thr, int32_t* band_out, hipStream_t s) {
  if (P->n_pairs == 0) return hipSuccess;
  band_kernel<<<(unsigned)P->n_pairs, kBlock, 0, s>>>(P->d_pairs, P->d_pair_shift, P->d_coef64,
                                                       P->L, thr, band_out);
  return hipGetLastError();
}

hipError_t launch_table_list(arkcos_plan_s* P, const int32_t* d_list, const int64_t* d_coef_off,
                             int32_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (P->dtype == ARKCOS_F32)
    table_kernel<float><<<count, kBlock, 0, s>>>(P->d_pairs, P->d_pair_shift, d_list, d_coef_off,
                                                P->d_coef64, P->L, (float*)P->d_table);
  else
    table_kernel<double><<<count, kBlock, 0, s>>>(P->d_pairs, P->d_pair_shift, d_list, d_coef_off,
                                                 P->d_coef64, P->L, (double*)P->d_table);
  return hipGetLastError();
}

hipError_t launch_bluestein_filters(arkcos_plan_s* P, const int32_t* d_ring_list, int32_t count,
                                    hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int lds = (int)((size_t)lds_elems(P->max_bl_m) * (P->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2)));
  const int nt = fft_threads(P->dtype, P->max_bl_m);
  hipError_t e;
  if (P->dtype == ARKCOS_F32 && nt == 1024) {
    e = hipFuncSetAttribute((const void*)bluestein_filter_kernel<float, 1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    bluestein_filter_kernel<float, 1024><<<count, 1024, lds, s>>>(
        d_ring_list, P->rt.n, P->rt.fft_m, P->rt.bl_off, (const float2*)P->d_twiddle, P->twiddle_n,
        (float2*)P->d_bl);
  } else if (P->dtype == ARKCOS_F32 && nt == 512) {
    e = hipFuncSetAttribute((const void*)bluestein_filter_kernel<float, 512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    bluestein_filter_kernel<float, 512><<<count, 512, lds, s>>>(
        d_ring_list, P->rt.n, P->rt.fft_m, P->rt.bl_off, (const float2*)P->d_twiddle, P->twiddle_n,
        (float2*)P->d_bl);
  } else if (P->dtype == ARKCOS_F32) {
    e = hipFuncSetAttribute((const void*)bluestein_filter_kernel<float, 256>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    bluestein_filter_kernel<float, 256><<<count, 256, lds, s>>>(
        d_ring_list, P->rt.n, P->rt.fft_m, P->rt.bl_off, (const float2*)P->d_twiddle, P->twiddle_n,
        (float2*)P->d_bl);
  } else if (nt == 512) {
    e = hipFuncSetAttribute((const void*)bluestein_filter_kernel<double, 512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    bluestein_filter_kernel<double, 512><<<count, 512, lds, s>>>(
        d_ring_list, P->rt.n, P->rt.fft_m, P->rt.bl_off, (const double2*)P->d_twiddle, P->twiddle_n,
        (double2*)P->d_bl);
  } else {
    e = hipFuncSetAttribute((const void*)bluestein_filter_kernel<double, 256>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    bluestein_filter_kernel<double, 256><<<count, 256, lds, s>>>(
        d_ring_list, P->rt.n, P->rt.fft_m, P->rt.bl_off, (const double2*)P->d_twiddle, P->twiddle_n,
        (double2*)P->d_bl);
  }
  return hipGetLastError();
}

}  // namespace arkcos
