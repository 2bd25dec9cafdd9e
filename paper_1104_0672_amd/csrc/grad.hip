// Gradient of L = 1/2 |C x - t|^2 with respect to the spline knot values c_k
// of the kernel profile, given r = C x - t.
//
// The ring pipeline computes y_ik = sum_{|m| <= M_i} B_i(m) e^{i m phi_ik} with
// B_i(m) = sum_j K_ij(m) A~_j(m) and K_ij(m) = h_ij(m) sum_d a_ijd cos(m nu_d)
// (h = 1/2 at the grid's Nyquist mode, 1 elsewhere; a_ijd = c_d w_j K(theta_ijd)
// / (p L), c_d the symmetric-node multiplicity).  Hence
//   <r, y> = sum_pairs sum_m eps_m h_ij(m) K~_ij(m) X_ij(m),
//   X_ij(m) = Re[conj(R~_i(m)) A~_j(m)],  eps_0 = 1, eps_m = 2 (m >= 1),
// where R~_i is the extended spectrum of r on output ring i, and
//   dL/dc_k = sum_pairs sum_d (c_d w_j / (p L)) phi_k(theta_ijd) Y_ij(d),
//   Y_ij(d) = sum_m eps_m h_ij(m) cos(m nu_d) X_ij(m)
// (a per-pair Fourier-space correlation reduced over m, then over the kernel
// samples).  phi_k is the cardinal clamped cubic spline: on knot interval a,
// with u = (theta - theta_a) / h,
//   phi_k = (1-u) [a = k] + u [a+1 = k] + h^2/6 ((1-u)^3-(1-u)) S_ak + h^2/6 (u^3-u) S_a+1,k
// (S: second-derivative moments of the basis splines).  Each unit (output
// ring and mirror) accumulates the four interval sums per knot interval in
// FP64; a final single-block pass adds the per-unit partials in a fixed order
// and maps them onto the knots, so the result is deterministic.  The pole
// rows recomputed by the direct sum contribute
//   sum_{p in poles} r_p sum_q phi_k(theta_pq) x_q w_q.
#include "arkcos_internal.h"
#include "device_common.h"

#include <string>

namespace arkcos {

struct GradArgs {
  const UnitDev* units;
  const PairDev* pairs;
  const int32_t* pair_shift;
  const int32_t* ncoef_window;
  const double* theta;
  const double* sint;
  const double* w;
  const int64_t* spec_off;
  const int64_t* out_off;
  const int32_t* n;
  const int64_t* start;
  const int32_t* phase_den;
  int32_t nrings;
  int64_t L;
  int32_t nk;
  double h, radius, theta_max;
  double* slots;         // [slot][4 * (nk - 1)]
  int64_t TN;            // length of the twiddle table
  int32_t zcache_bytes;  // LDS for a wide row's correlation
};

constexpr int kGradSpl = kGradPass / 64;  // wide rows: samples per lane in a pass
constexpr int kNarrowChunk = 16;           // narrow rows: samples summed per pass over the modes
constexpr int kGradRestart = 1024;  // wide rows: modes between exact restarts of the cosine recurrence
static_assert(64 * kGradSpl <= kBlock, "a pass's samples are scattered at once");

__device__ __forceinline__ double grad_distance(double ti, double tj, double si, double sj, int64_t num,
                                                int64_t den) {
  double a = sin(0.5 * (ti - tj));
  double b = sinpi(0.5 * (double)num / (double)den);
  double hav = a * a + si * sj * b * b;
  double r = sqrt(hav);
  return 2.0 * asin(r < 1.0 ? r : 1.0);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds weight * (basis pieces at distance t) into the interval sums U[a][0..3]
// (nothing beyond the support or the last knot).
__device__ __forceinline__ void interval_add(double* U, const GradArgs& g, double t, double weight) {
  if (t > g.radius || t > g.theta_max + kSupportTol) return;
  int a = (int)floor(t / g.h);
  a = a < 0 ? 0 : (a > g.nk - 2 ? g.nk - 2 : a);
  const double u = t / g.h - a, v = 1.0 - u, h2 = g.h * g.h / 6.0;
  U[4 * a + 0] += weight * v;
  U[4 * a + 1] += weight * u;
  U[4 * a + 2] += weight * h2 * (v * v * v - v);
  U[4 * a + 3] += weight * h2 * (u * u * u - u);
}

// Ordered scatter of up to blockDim samples: thread k provides the distance
// t_k and weight of its sample; thread 0 adds them into U in index order.
__device__ __forceinline__ void ordered_scatter(double* U, const GradArgs& g, double* st, double* sw, int count,
                                                double t, double wgt) {
  st[threadIdx.x] = t;
  sw[threadIdx.x] = wgt;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < count; ++k) interval_add(U, g, st[k], sw[k]);
  __syncthreads();
}

// The same for the samples of one kernel row (count <= kBlock): thread k
// provides sample d0 + k, whose distance does not decrease with k (it grows with the
// longitude offset), so the interval index is non-decreasing in k and each
// interval's samples are a contiguous run.  Thread (a, c) sums piece c over
// interval a's run in thread order and adds the sum into U: parallel, and
// still independent of timing.  Samples outside the support get index nk
// (past every interval), which keeps the order.
__device__ __forceinline__ void row_scatter(double* U, const GradArgs& g, int* sa, double* sp, int count, double t,
                                            double wgt) {
  const int tid = threadIdx.x;
  int a = g.nk;
  double pc[4] = {0.0, 0.0, 0.0, 0.0};
  if (tid < count && !(t > g.radius || t > g.theta_max + kSupportTol)) {
    a = (int)floor(t / g.h);
    a = a < 0 ? 0 : (a > g.nk - 2 ? g.nk - 2 : a);
    const double u = t / g.h - a, v = 1.0 - u, h2 = g.h * g.h / 6.0;
    pc[0] = wgt * v;
    pc[1] = wgt * u;
    pc[2] = wgt * h2 * (v * v * v - v);
    pc[3] = wgt * h2 * (u * u * u - u);
  }
  if (tid < count) {
    sa[tid] = a;
#pragma unroll
    for (int c = 0; c < 4; ++c) sp[c * kBlock + tid] = pc[c];
  }
  __syncthreads();
  for (int k = tid; k < 4 * (g.nk - 1); k += blockDim.x) {
    const int ia = k >> 2, c = k & 3;
    int lo = 0, hi = count;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sa[mid] < ia) lo = mid + 1;
      else hi = mid;
    }
    if (lo < count && sa[lo] == ia) {
      double sum = 0.0;
      for (int d = lo; d < count && sa[d] == ia; ++d) sum += sp[c * kBlock + d];
      U[k] += sum;
    }
  }
  __syncthreads();
}

// cos(pi k / pl) for integers k >= 0 on one kernel grid: read from the
// twiddle table (tw[k'] = exp(-2 pi i k' / TN)) when 2 pl divides its length,
// otherwise computed.  `table` is fixed per grid, so the loops below are
// compiled once for each case and the table reads carry no branches.
template <typename R> struct GridCos {
  const cx_t<R>* tw;
  int64_t pl, mask, stride;
  __device__ __forceinline__ R raw(int64_t k) const { return tw[(k & mask) * stride].x; }
  __device__ __forceinline__ double exact(int64_t k) const { return cospi((double)(k % (2 * pl)) / (double)pl); }
};
template <typename R>
__device__ __forceinline__ GridCos<R> grid_cos(const cx_t<R>* tw, int64_t pl, int64_t TN, bool& table) {
  table = TN % (2 * pl) == 0;
  return GridCos<R>{tw, pl, 2 * pl - 1, table ? TN / (2 * pl) : 0};
}

// One block per run of work items (a fixed, cost-balanced partition), its
// interval sums accumulated over the run in item order and written to the
// block's slot.  An item is either the narrow rows (at most kGradMaxCoef
// samples) of one unit, or a range of samples of one wide row.
//
// Narrow rows: threads over modes, per-thread sums for every sample, the
// cosines by the three-term recurrence in the sample index d.
//
// Wide rows: the correlation Z(m) = eps_m h(m) (X_ij(m) + X_i'j'(m)) of the
// pair over the item's mode chunk is staged in LDS once per item (in the
// plan's precision; the chunks' partial sums of a sample add up linearly in
// the interval sums), then the
// item's samples are taken 64 kGradSpl at a time, each lane holding
// kGradSpl samples and each wave one contiguous range of modes, so every
// mode's Z is one broadcast LDS read for a whole wave and needs no
// reduction across lanes; the waves' partial sums are added in wave order.
template <typename R>
__global__ void __launch_bounds__(kGradThreads) grad_items_kernel(GradArgs g, const GradItem* __restrict__ items,
                                                                  const int32_t* __restrict__ run,
                                                                  const cx_t<R>* __restrict__ aspec,
                                                                  const cx_t<R>* __restrict__ rspec,
                                                                  const cx_t<R>* __restrict__ tw) {
  using C = cx_t<R>;
  constexpr int NWV = kGradThreads / 64;
  extern __shared__ __align__(16) unsigned char gsm[];
  R* zc = reinterpret_cast<R*>(gsm);  // Z(m) of the current wide row
  __shared__ double U[4 * 63];
  __shared__ double Y[kGradMaxCoef];
  __shared__ double sp[4 * kBlock];
  __shared__ int sa[kBlock];
  // partial sums: a wide-row pass's per-wave sums, or a narrow row's
  // per-wave reductions (never in use at the same time)
  __shared__ double red[NWV * 64 * kGradSpl];
  double* part = red;
  static_assert(kGradMaxCoef <= 64 * kGradSpl, "narrow reductions fit the pass buffer");
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nint4 = 4 * (g.nk - 1);
  for (int e = tid; e < nint4; e += blockDim.x) U[e] = 0.0;
  __syncthreads();
  // per-thread sums acc[0..cnt) -> Y[y0..y0 + cnt) (every wave's sums, then
  // the waves in order), Y ready on return
  auto reduce = [&](auto& acc, int cnt, int y0) {
    constexpr int NA = sizeof(acc) / sizeof(acc[0]);
#pragma unroll
    for (int d = 0; d < NA; ++d) {
      if (d < cnt) {
        const double v = wave_sum(acc[d]);
        if (lane == 0) part[wv * kGradMaxCoef + d] = v;
      }
    }
    __syncthreads();
    if (tid < cnt) {
      double t = 0.0;
      for (int k = 0; k < NWV; ++k) t += part[k * kGradMaxCoef + tid];
      Y[y0 + tid] = t;
    }
    __syncthreads();
  };
  const int it0 = run[blockIdx.x], it1 = run[blockIdx.x + 1];
  for (int it = it0; it < it1; ++it) {
    const GradItem item = items[it];
    const UnitDev u = g.units[item.unit];
    const bool mirror = u.im >= 0;
    const int q0 = item.pair < 0 ? u.pbeg : item.pair, q1 = item.pair < 0 ? u.pend : item.pair + 1;
    for (int q = q0; q < q1; ++q) {
      const PairDev pr = g.pairs[q];
      const int nc = g.ncoef_window[q], s = g.pair_shift[q];
      if (pr.band < 0 || (item.pair < 0) != (nc <= kGradMaxCoef)) continue;
      const int j = pr.j, jm = g.nrings - 1 - j;
      const int64_t pl = (int64_t)pr.grid;
      const C* ai = aspec + g.spec_off[j];
      const C* ri = rspec + g.out_off[u.i];
      const C* am = aspec + g.spec_off[jm];
      const C* rm = mirror ? rspec + g.out_off[u.im] : ri;
      const double scale = g.w[j] / (double)pl;
      auto xcorr = [&](int m) -> double {  // eps_m h(m) (X_ij(m) + X_i'j'(m))
        const C a0 = ai[m], r0 = ri[m];
        double X = (double)r0.x * a0.x + (double)r0.y * a0.y;
        if (mirror) {
          const C a1 = am[m], r1 = rm[m];
          X += (double)r1.x * a1.x + (double)r1.y * a1.y;
        }
        double wm = m == 0 ? 1.0 : 2.0;
        if (m == pr.nyq) wm *= 0.5;
        return X * wm;
      };
      auto sample = [&](int d, double& t, double& cd) {
        t = grad_distance(g.theta[u.i], g.theta[j], g.sint[u.i], g.sint[j], 2 * (int64_t)d + s, pl);
        cd = (s == 0 && (d == 0 || 2 * (int64_t)d == pl)) ? 1.0 : 2.0;
      };
      bool table = false;
      const GridCos<R> gc = grid_cos<R>(tw, pl, g.TN, table);
      if (item.pair < 0) {
        // the samples in chunks of kNarrowChunk, each chunk's cosines started
        // from their exact values at its first two samples (a row's sums
        // for all 48 samples at once would hold 96 registers per thread,
        // and the kernel's wide-row passes would lose half their waves)
        for (int dc = 0; dc < nc; dc += kNarrowChunk) {
          double acc[kNarrowChunk];
#pragma unroll
          for (int d = 0; d < kNarrowChunk; ++d) acc[d] = 0.0;
          auto modes = [&](auto tab) {
            constexpr bool TAB = decltype(tab)::value;
            const int64_t e0 = 2 * (int64_t)dc + s, e1 = e0 + 2;
            for (int m = tid; m <= pr.band; m += blockDim.x) {
              // cos(m nu_d), nu_d = pi (2d + s) / pl, by the Chebyshev recurrence in d
              double c0, c1, step;
              if constexpr (TAB) {
                const R a = gc.raw((int64_t)m * e0), b = gc.raw((int64_t)m * e1), c = gc.raw(2 * (int64_t)m);
                c0 = a;
                c1 = b;
                step = 2.0 * (double)c;
              } else {
                c0 = gc.exact((int64_t)m * e0);
                c1 = gc.exact((int64_t)m * e1);
                step = 2.0 * gc.exact(2 * (int64_t)m);
              }
              const double X = xcorr(m);
#pragma unroll
              for (int d = 0; d < kNarrowChunk; ++d) {
                acc[d] = fma(X, c0, acc[d]);
                const double c2 = fma(step, c1, -c0);
                c0 = c1;
                c1 = c2;
              }
            }
          };
          if (table) modes(std::true_type{});
          else modes(std::false_type{});
          reduce(acc, min(kNarrowChunk, nc - dc), dc);
        }
        double t = 0.0, cd = 0.0, wgt = 0.0;
        if (tid < nc) {
          sample(tid, t, cd);
          wgt = cd * scale * Y[tid];
        }
        row_scatter(U, g, sa, sp, nc, t, wgt);
        continue;
      }
      // a wide row's mode chunk [m0, m1): stage Z(m) (or evaluate it on the
      // fly when it does not fit)
      const int band = __builtin_amdgcn_readfirstlane(pr.band);
      const int m0 = __builtin_amdgcn_readfirstlane(item.m0);
      const int m1 = __builtin_amdgcn_readfirstlane(min(item.m1, band + 1));
      const bool cached = (int64_t)(m1 - m0) * (int64_t)sizeof(R) <= (int64_t)g.zcache_bytes;
      if (cached) {
        for (int m = m0 + tid; m < m1; m += blockDim.x) zc[m - m0] = (R)xcorr(m);
        __syncthreads();
      }
      // passes of 64 x kGradSpl samples: lane l holds samples d + l + 64 k
      // (k < kGradSpl), wave w the w-th of NWV contiguous mode ranges; per
      // sample cos(m nu_d) runs by the recurrence in m, restarted from exact
      // values every kGradRestart modes; the NWV partial sums of a sample are
      // added in wave order
      const int nmode = m1 - m0;
      const int mlo = __builtin_amdgcn_readfirstlane(m0 + (int)((int64_t)nmode * wv / NWV));
      const int mhi = __builtin_amdgcn_readfirstlane(m0 + (int)((int64_t)nmode * (wv + 1) / NWV));
      const int dend = item.d0 + item.cnt;
      auto passes = [&](auto cached_tag) {
      constexpr bool CACHED = decltype(cached_tag)::value;
      for (int pd = item.d0; pd < dend; pd += 64 * kGradSpl) {
        double acc[kGradSpl], st[kGradSpl];
        int64_t kd[kGradSpl];  // nu_d = pi kd / pl
#pragma unroll
        for (int k = 0; k < kGradSpl; ++k) {
          acc[k] = 0.0;
          kd[k] = 2 * (int64_t)(pd + lane + 64 * k) + s;
          st[k] = 2.0 * cospi((double)(kd[k] % (2 * pl)) / (double)pl);
        }
        for (int mr = mlo; mr < mhi; mr += kGradRestart) {
          const int me = min(mr + kGradRestart, mhi);
          double c0[kGradSpl], c1[kGradSpl];
#pragma unroll
          for (int k = 0; k < kGradSpl; ++k) {
            c0[k] = cospi((double)(((int64_t)mr * kd[k]) % (2 * pl)) / (double)pl);
            c1[k] = cospi((double)(((int64_t)(mr + 1) * kd[k]) % (2 * pl)) / (double)pl);
          }
          int m = mr;
          // (rows whose Z(m) is not staged evaluate it one mode at a time:
          // eight on-the-fly correlations in flight would cost the whole
          // kernel registers and occupancy)
          for (; CACHED && m + 8 <= me; m += 8) {
            double z[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) z[e] = CACHED ? (double)zc[m - m0 + e] : xcorr(m + e);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
#pragma unroll
              for (int k = 0; k < kGradSpl; ++k) {
                acc[k] = fma(z[e], c0[k], acc[k]);
                const double c2 = fma(st[k], c1[k], -c0[k]);
                c0[k] = c1[k];
                c1[k] = c2;
              }
            }
          }
          for (; m < me; ++m) {
            const double z = CACHED ? (double)zc[m - m0] : xcorr(m);
#pragma unroll
            for (int k = 0; k < kGradSpl; ++k) {
              acc[k] = fma(z, c0[k], acc[k]);
              const double c2 = fma(st[k], c1[k], -c0[k]);
              c0[k] = c1[k];
              c1[k] = c2;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < kGradSpl; ++k) red[wv * 64 * kGradSpl + lane + 64 * k] = acc[k];
        __syncthreads();
        const int cnt = min(64 * kGradSpl, dend - pd);
        double t = 0.0, cd = 0.0, wgt = 0.0;
        if (tid < cnt) {
          double y = 0.0;
          for (int w = 0; w < NWV; ++w) y += red[w * 64 * kGradSpl + tid];
          sample(pd + tid, t, cd);
          wgt = cd * scale * y;
        }
        row_scatter(U, g, sa, sp, cnt, t, wgt);
      }
      };
      if (cached) passes(std::true_type{});
      else passes(std::false_type{});
      __syncthreads();  // zc is rewritten by the next row
    }
  }
  double* out = g.slots + (size_t)blockIdx.x * nint4;
  for (int e = tid; e < nint4; e += blockDim.x) out[e] = U[e];
}

// Direct-sum pole rows: one block per pole pixel p, slot slot0 + b.
template <typename R>
__global__ void __launch_bounds__(kBlock) grad_pole_kernel(GradArgs g, const int32_t* __restrict__ rings,
                                                           int32_t nlist, const R* __restrict__ x,
                                                           const R* __restrict__ r, int32_t slot0) {
  __shared__ double U[4 * 63];
  __shared__ double st[kBlock];
  __shared__ double sw[kBlock];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int nint4 = 4 * (g.nk - 1);
  for (int e = tid; e < nint4; e += blockDim.x) U[e] = 0.0;
  __syncthreads();
  const int ip = b < 4 ? 0 : g.nrings - 1, kp = b & 3;
  const double rp = (double)r[g.start[ip] + kp];
  for (int li = 0; li < nlist; ++li) {
    const int jr = rings[li];
    if (fabs(g.theta[jr] - g.theta[ip]) > g.radius) continue;
    const int nj = g.n[jr];
    for (int k0 = 0; k0 < nj; k0 += blockDim.x) {
      const int k = k0 + tid;
      double t = 1e300, wgt = 0.0;
      if (k < nj) {
        const int64_t na = g.n[ip], nb = nj;
        const int64_t sa = g.phase_den[ip] ? 1 : 0, sb = g.phase_den[jr] ? 1 : 0;
        const int64_t num = (2 * (int64_t)kp + sa) * nb - (2 * (int64_t)k + sb) * na;
        const double hd = sinpi((double)num / (double)(2 * na * nb));
        const double a = sin(0.5 * (g.theta[ip] - g.theta[jr]));
        const double hav = a * a + g.sint[ip] * g.sint[jr] * hd * hd;
        const double rr = sqrt(hav);
        t = 2.0 * asin(rr < 1.0 ? rr : 1.0);
        wgt = rp * (double)x[g.start[jr] + k] * g.w[jr];
      }
      ordered_scatter(U, g, st, sw, min((int)blockDim.x, nj - k0), t, wgt);
    }
  }
  double* out = g.slots + (size_t)(slot0 + b) * nint4;
  for (int e = tid; e < nint4; e += blockDim.x) out[e] = U[e];
}

// Sum of the slots in a fixed order, then the map onto the knots.
// The slots' interval sums: block e adds column e (thread t the slots t,
// t + kBlock, ...), then the threads' sums in a fixed tree.
__global__ void __launch_bounds__(kBlock) grad_sum_kernel(const double* __restrict__ slots, int32_t nslots,
                                                          int32_t nint4, double* __restrict__ sums) {
  static_assert((kBlock & (kBlock - 1)) == 0, "tree reduction over a power-of-two block");
  __shared__ double part[kBlock];
  const int e = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nslots; k += kBlock) s += slots[(size_t)k * nint4 + e];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[e] = part[0];
}

__global__ void __launch_bounds__(kBlock) grad_final_kernel(const double* __restrict__ sums, int32_t nk,
                                                            const double* __restrict__ basis_mom,
                                                            double* __restrict__ grad) {
  __shared__ double Us[4 * 63];
  const int nint4 = 4 * (nk - 1);
  for (int e = threadIdx.x; e < nint4; e += blockDim.x) Us[e] = sums[e];
  __syncthreads();
  for (int k = threadIdx.x; k < nk; k += blockDim.x) {
    double gk = 0.0;
    if (k <= nk - 2) gk += Us[4 * k + 0];
    if (k >= 1) gk += Us[4 * (k - 1) + 1];
    for (int a = 0; a <= nk - 2; ++a)
      gk += Us[4 * a + 2] * basis_mom[a * nk + k] + Us[4 * a + 3] * basis_mom[(a + 1) * nk + k];
    grad[k] = gk;
  }
}

arkcos_status_t run_kernel_grad(arkcos_plan_s* P, const void* x, const void* r, double* grad, void* ws,
                                uint32_t flags, hipStream_t s) {
  void *spec, *bout;
  workspace_split(P, ws, &spec, &bout);
  double* slots = grad_slots(P, ws);
  const bool fix = P->geom.kind == 1 && P->opts.fix_pole_pixels;
  hipError_t e = hipSuccess;
  if (!(flags & 1u)) e = launch_r2c_layout(P, x, spec, false, 0, s);
  if (e == hipSuccess) e = launch_r2c_layout(P, r, bout, true, fix ? 1 : 0, s);
  if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("ring transform: ") + hipGetErrorString(e));
  GradArgs g{};
  g.units = P->d_units;
  g.pairs = P->d_pairs;
  g.pair_shift = P->d_pair_shift;
  g.ncoef_window = P->d_ncoef_window;
  g.theta = P->d_theta;
  g.sint = P->d_sin;
  g.w = P->rt.w;
  g.spec_off = P->rt.spec_off;
  g.out_off = P->rt.out_off;
  g.n = P->rt.n;
  g.start = P->rt.start;
  g.phase_den = P->rt.phase_den;
  g.nrings = (int32_t)P->nrings;
  g.L = P->L;
  g.nk = (int32_t)P->knots.size();
  g.h = P->theta_max / (g.nk - 1);
  g.radius = P->radius + kSupportTol;
  g.theta_max = P->theta_max;
  g.slots = slots;
  g.TN = P->twiddle_n;
  g.zcache_bytes = P->grad_zcache_bytes;
  const int32_t nruns = P->n_grad_runs;
  const size_t lds = (size_t)P->grad_zcache_bytes;
  if (P->dtype == ARKCOS_F32) {
    e = hipFuncSetAttribute((const void*)grad_items_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e == hipSuccess)
      grad_items_kernel<float><<<nruns, kGradThreads, lds, s>>>(g, P->d_grad_items, P->d_grad_run,
                                                                (const float2*)spec, (const float2*)bout,
                                                                (const float2*)P->d_twiddle);
  } else {
    e = hipFuncSetAttribute((const void*)grad_items_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e == hipSuccess)
      grad_items_kernel<double><<<nruns, kGradThreads, lds, s>>>(g, P->d_grad_items, P->d_grad_run,
                                                                 (const double2*)spec, (const double2*)bout,
                                                                 (const double2*)P->d_twiddle);
  }
  if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("gradient kernels: ") + hipGetErrorString(e));
  int32_t nslots = nruns;
  if (fix) {
    int32_t count = 0;
    int32_t* list = pole_ring_list(P, &count);
    if (P->dtype == ARKCOS_F32)
      grad_pole_kernel<float><<<8, kBlock, 0, s>>>(g, list, count, (const float*)x, (const float*)r, nruns);
    else
      grad_pole_kernel<double><<<8, kBlock, 0, s>>>(g, list, count, (const double*)x, (const double*)r, nruns);
    nslots += 8;
  }
  // (the workspace holds n_grad_runs + 8 slots and then the sums)
  double* sums = slots + (size_t)(nruns + 8) * (size_t)(4 * (g.nk - 1));
  grad_sum_kernel<<<(unsigned)(4 * (g.nk - 1)), kBlock, 0, s>>>(slots, nslots, 4 * (g.nk - 1), sums);
  grad_final_kernel<<<1, kBlock, 0, s>>>(sums, g.nk, P->d_basis_mom, grad);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("gradient kernels: ") + hipGetErrorString(e));
  return ARKCOS_OK;
}

}  // namespace arkcos
