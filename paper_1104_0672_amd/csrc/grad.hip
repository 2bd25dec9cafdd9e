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

// X_ij(m) + X_i'j'(m), X = Re[conj(R~_i(m)) A~_j(m)], for output ring i
// (mirror i') and input ring j (mirror j'); a mirror ring has the pixel
// count and offset of its ring.
template <typename R> struct PairX {
  using C = cx_t<R>;
  const C *ai, *ri, *am, *rm;
  uint32_t Ni, Nj;
  float invi, invj;
  bool shi, shj, mirror;
  __device__ __forceinline__ PairX(const GradArgs& g, const C* aspec, const C* rspec, const UnitDev& u, int j) {
    const int jm = g.nrings - 1 - j;
    ai = aspec + g.spec_off[j];
    am = aspec + g.spec_off[jm];
    ri = rspec + g.out_off[u.i];
    mirror = u.im >= 0;
    rm = mirror ? rspec + g.out_off[u.im] : ri;
    Ni = (uint32_t)g.n[u.i];
    Nj = (uint32_t)g.n[j];
    shi = g.phase_den[u.i] != 0;
    shj = g.phase_den[j] != 0;
    invi = 1.0f / (float)Ni;
    invj = 1.0f / (float)Nj;
  }
  // in precision T (the row FFTs take it in the plan's precision)
  template <typename T> __device__ __forceinline__ T eval(uint32_t m) const {
    const ExtIdx ej = ext_index(Nj, invj, shj, m), ei = ext_index(Ni, invi, shi, m);
    const C a0 = ext_at(ai, ej), r0 = ext_at(ri, ei);
    T X = (T)r0.x * (T)a0.x + (T)r0.y * (T)a0.y;
    if (mirror) {
      const C a1 = ext_at(am, ej), r1 = ext_at(rm, ei);
      X += (T)r1.x * (T)a1.x + (T)r1.y * (T)a1.y;
    }
    return X;
  }
  __device__ __forceinline__ double operator()(uint32_t m) const { return eval<double>(m); }
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
      const PairX<R> px(g, aspec, rspec, u, j);
      const double scale = g.w[j] / (double)pl;
      auto xcorr = [&](int m) -> double {  // eps_m h(m) (X_ij(m) + X_i'j'(m))
        const double X = px((uint32_t)m);
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
#pragma unroll 4  // four modes' loads in flight (1 % of the gradient)
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

// Interval sums held by one wavefront: lane l keeps entries l + 64 j (j < 4)
// of the 4 (nk - 1) <= 252 sums in registers.  wave_interval_add adds the
// pieces of 64 consecutive samples (lane k: sample k, invalid lanes give
// nothing): their interval indices do not decrease with the lane, so a
// segmented scan over lanes of equal index leaves each interval's total in
// its last lane, and the (few) totals are added into the owning lanes one
// interval at a time.  The order of every addition is fixed.
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void wave_interval_add(double (&Ur)[4], const GradArgs& g, bool valid, double t,
                                                  double wgt) {
  const int lane = threadIdx.x & 63;
  int a = g.nk;  // past every interval: outside the support or no sample
  double pc[4] = {0.0, 0.0, 0.0, 0.0};
  if (valid && !(t > g.radius || t > g.theta_max + kSupportTol)) {
    a = (int)floor(t / g.h);
    a = a < 0 ? 0 : (a > g.nk - 2 ? g.nk - 2 : a);
    const double u = t / g.h - a, v = 1.0 - u, h2 = g.h * g.h / 6.0;
    pc[0] = wgt * v;
    pc[1] = wgt * u;
    pc[2] = wgt * h2 * (v * v * v - v);
    pc[3] = wgt * h2 * (u * u * u - u);
  }
  if (__ballot(a < g.nk) == 0) return;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int au = __shfl_up(a, off, 64);
    double up[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) up[c] = __shfl_up(pc[c], off, 64);
    if (lane >= off && au == a) {
#pragma unroll
      for (int c = 0; c < 4; ++c) pc[c] += up[c];
    }
  }
  const int an = __shfl_down(a, 1, 64);
  uint64_t ends = __ballot(a < g.nk && (lane == 63 || an != a));
  while (ends) {
    const int e = __builtin_ctzll(ends);
    ends &= ends - 1;
    const int ae = __builtin_amdgcn_readlane(a, e);
    const double s0 = readlane_f64(pc[0], e), s1 = readlane_f64(pc[1], e);
    const double s2 = readlane_f64(pc[2], e), s3 = readlane_f64(pc[3], e);
    const int k0 = 4 * ae, j = k0 >> 6;  // entries k0 .. k0 + 3: lanes (k0 & 63) + c of register j
    if ((lane >> 2) == ((k0 & 63) >> 2)) {
      const int c = lane & 3;
      const double v = c == 0 ? s0 : (c == 1 ? s1 : (c == 2 ? s2 : s3));
      if (j == 0) Ur[0] += v;
      else if (j == 1) Ur[1] += v;
      else if (j == 2) Ur[2] += v;
      else Ur[3] += v;
    }
  }
}

// The LDS FFT as a call: inlined into the row kernel, the compiler's
// schedule of it holds about twice the registers (a 1024-thread block then
// spills).
template <typename R, bool INV, int NT>
__device__ __noinline__ void lds_fft_outlined(cx_t<R>* buf, int M, const cx_t<R>* __restrict__ tw, int TN) {
  lds_fft<R, INV, NT>(buf, M, tw, TN);
}

// Wide rows by FFT: Y(d) = sum_{m <= band, m < G} Z(m) cos(2 pi m d / G) with
// Z(m) = eps_m h(m) (X_ij(m) + X_i'j'(m)) on a power-of-two grid G, in one of
// two forms (RowFft::half).  The S-pass form: with S = G / (2 P), the modes
// split into S real sub-sequences z_q = Z(S q + s) of 2 P points, and
//   Y(d) = Re sum_s exp(2 pi i s d / G) Y_s(d mod 2P),
// Y_s the inverse 2P-point transform of z (one packed P-point LDS FFT).  The
// half-length form (P = G / 4, one pass) is described where it is taken.  One
// block per row writes Y(d), d < nc, to the row's place in the chunk's buffer
// (thread k owns the samples k + NT i in every pass).
template <typename R, int NT>
__global__ void __launch_bounds__(NT) grad_row_fft_kernel(GradArgs g, const RowFft* __restrict__ rows,
                                                          const int64_t* __restrict__ yoff,
                                                          const cx_t<R>* __restrict__ aspec,
                                                          const cx_t<R>* __restrict__ rspec,
                                                          const cx_t<R>* __restrict__ tw, R* __restrict__ Y) {
  using C = cx_t<R>;
  extern __shared__ __align__(16) unsigned char gsm[];
  C* buf = reinterpret_cast<C*>(gsm);
  const int tid = threadIdx.x;
  const RowFft row = rows[blockIdx.x];
  const UnitDev u = g.units[row.unit];
  const bool mirror = u.im >= 0;
  const int q = row.pair, Pn = row.P;
  const PairDev pr = g.pairs[q];
  const int64_t G = pr.grid;
  const int S = (int)(G / (2 * (int64_t)Pn));
  const int nc = g.ncoef_window[q], band = pr.band;
  const int j = pr.j;
  const PairX<R> px(g, aspec, rspec, u, j);
  R* Yr = Y + yoff[blockIdx.x];
  auto xcorr = [&](int64_t m) -> R {  // eps_m h(m) (X_ij(m) + X_i'j'(m)), zero past the band
    if (m > band) return R(0);
    const R X = px.template eval<R>((uint32_t)m);
    R wm = m == 0 ? R(1) : R(2);
    if (m == pr.nyq) wm *= R(0.5);
    return X * wm;
  };
  const int64_t kstep = g.TN / (2 * (int64_t)Pn), gstep = g.TN / G;
  if (row.half) {
    // The half-length cosine sum (N = G / 2, Pn = N / 2).  The modes m < G
    // fold onto 0..N (cos(2 pi m d / G) is even about N):
    //   f_0 = 2 Z(0), f_N = 2 Z(N), f_m = Z(m) + Z(G - m) (0 < m < N),
    //   Y(d) = f_0 / 2 + (-1)^d f_N / 2 + sum_{0 < m < N} f_m cos(pi m d / N).
    // With y_j = (f_j + f_{N-j}) / 2 - sin(pi j / N) (f_j - f_{N-j}) (j < N)
    // and X the N-point inverse transform of y (one packed Pn-point FFT),
    //   Y(2k) = Re X(k),   Y(2k + 1) = Y(1) + sum_{0 < k' <= k} Im X(k'),
    //   Y(1) = (f_0 - f_N) / 2 + sum_{0 < m < N} f_m cos(pi m / N)
    // (summed while y is built): the sine-weighted differences cancel in
    // Re X and leave the first differences of the odd samples in Im X.  Half
    // the transform of the S-pass form; the odd samples by a block scan in a
    // fixed order.
    constexpr int NW = NT / 64;
    __shared__ R wsum[NW];
    const int lane = tid & 63, wv = tid >> 6, N = 2 * Pn;
    R* br = reinterpret_cast<R*>(buf);
    auto put = [&](int jj, R v) { br[2 * lidx(jj >> 1) + (jj & 1)] = v; };
    R f1 = R(0);
    for (int jj = tid; jj <= Pn; jj += NT) {
      if (jj == 0) {
        const R z0 = xcorr(0), zn = xcorr(N);
        put(0, z0 + zn);
        f1 += z0 - zn;
      } else if (jj == Pn) {
        put(Pn, xcorr(Pn) + xcorr(G - Pn));  // sin = 1, cos = 0
      } else {
        const C t = tw[(int64_t)jj * gstep];  // exp(-i pi jj / N)
        const R fa = xcorr(jj) + xcorr(G - jj), fb = xcorr(N - jj) + xcorr(N + jj);
        const R h = R(0.5) * (fa + fb), dl = -t.y * (fa - fb);
        put(jj, h - dl);
        put(N - jj, h + dl);
        f1 += t.x * (fa - fb);
      }
    }
    for (int o = 32; o > 0; o >>= 1) f1 += __shfl_xor(f1, o, 64);
    if (lane == 0) wsum[wv] = f1;
    __syncthreads();
    R carry = R(0);  // Y(1)
    for (int w = 0; w < NW; ++w) carry += wsum[w];
    lds_fft_outlined<R, true, NT>(buf, Pn, tw, (int)g.TN);  // its barriers also order the wsum reads
    const int ke = (nc + 1) / 2, ko = nc / 2;  // even and odd samples below nc
    for (int k0 = 0; k0 < ke; k0 += NT) {
      const int k = k0 + tid;
      C X = cmake<C>(R(0), R(0));
      if (k < ke) X = real_from_packed<R>(buf, Pn, k, cconj(tw[(int64_t)k * kstep]));
      R v = (k >= 1 && k < ko) ? X.y : R(0);
      for (int o = 1; o < 64; o <<= 1) {
        const R u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
      }
      if (lane == 63) wsum[wv] = v;
      __syncthreads();
      R pre = R(0), tot = R(0);
      for (int w = 0; w < NW; ++w) {
        const R sw = wsum[w];
        if (w < wv) pre += sw;
        tot += sw;
      }
      if (k < ke) Yr[2 * k] = X.x;
      if (k < ko) Yr[2 * k + 1] = carry + pre + v;
      carry += tot;
      __syncthreads();  // wsum is rewritten by the next round
    }
    return;
  }
  for (int s = 0; s < S; ++s) {
    for (int l = tid; l < Pn; l += NT) {
      const int64_t m0 = (int64_t)S * (2 * l) + s;
      buf[lidx(l)] = cmake<C>(xcorr(m0), xcorr(m0 + S));
    }
    __syncthreads();
    lds_fft_outlined<R, true, NT>(buf, Pn, tw, (int)g.TN);
    for (int d = tid; d < nc; d += NT) {
      const int k = d & (2 * Pn - 1);
      const C X = real_from_packed<R>(buf, Pn, k, cconj(tw[k * kstep]));
      const C ph = cconj(tw[(((int64_t)s * d) & (G - 1)) * gstep]);  // exp(2 pi i s d / G)
      const R v = ph.x * X.x - ph.y * X.y;
      Yr[d] = s == 0 ? v : Yr[d] + v;
    }
    __syncthreads();  // buf is rewritten by the next pass
  }
}

template <typename R, int NT>
static hipError_t grad_row_fft_launch(const GradArgs& g, const RowFft* rows, const int64_t* yoff, int32_t count,
                                      const void* spec, const void* bout, const void* twd, void* Y, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t lds = (size_t)lds_elems(16 * NT) * sizeof(cx_t<R>);
  hipError_t e = hipFuncSetAttribute((const void*)grad_row_fft_kernel<R, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  grad_row_fft_kernel<R, NT><<<count, NT, lds, s>>>(g, rows, yoff, (const cx_t<R>*)spec, (const cx_t<R>*)bout,
                                                    (const cx_t<R>*)twd, (R*)Y);
  return hipGetLastError();
}

// The FFT rows' Y(d) into the interval sums: persistent blocks take the
// rows b, b + grid, ... of a chunk in order; wave w of a block takes the
// samples 64 (4 k + w) .. + 63 (k = 0, 1, ...) of a row into its register
// sums; at the end the waves' sums are added in wave order and written to
// (first chunk) or added into (later chunks) the block's slot.
template <typename R>
__global__ void __launch_bounds__(kBlock) grad_row_scatter_kernel(GradArgs g, const RowFft* __restrict__ rows,
                                                                  int32_t nrows, const int64_t* __restrict__ yoff,
                                                                  const R* __restrict__ Y, int32_t slot0,
                                                                  int32_t accumulate) {
  constexpr int NW = kBlock / 64;
  __shared__ double part[NW * 256];
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  double Ur[4] = {0.0, 0.0, 0.0, 0.0};
  for (int ri = blockIdx.x; ri < nrows; ri += gridDim.x) {
    const RowFft row = rows[ri];
    const UnitDev u = g.units[row.unit];
    const int q = row.pair;
    const PairDev pr = g.pairs[q];
    const int64_t G = pr.grid;
    const int nc = g.ncoef_window[q], j = pr.j;
    const double scale = g.w[j] / (double)G;
    const double thi = g.theta[u.i], thj = g.theta[j], si = g.sint[u.i], sj = g.sint[j];
    const R* Yr = Y + yoff[ri];
    for (int d0 = 64 * wv; d0 < nc; d0 += 64 * NW) {
      const int d = d0 + lane;
      double t = 0.0, wgt = 0.0;
      if (d < nc) {
        t = grad_distance(thi, thj, si, sj, 2 * (int64_t)d, G);
        const double cd = (d == 0 || 2 * (int64_t)d == G) ? 1.0 : 2.0;
        wgt = cd * scale * (double)Yr[d];
      }
      wave_interval_add(Ur, g, d < nc, t, wgt);
    }
  }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) part[wv * 256 + lane + 64 * jj] = Ur[jj];
  __syncthreads();
  const int nint4 = 4 * (g.nk - 1);
  double* out = g.slots + (size_t)(slot0 + blockIdx.x) * nint4;
  for (int e = tid; e < nint4; e += kBlock) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += part[w * 256 + e];
    out[e] = accumulate ? out[e] + v : v;
  }
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
  // the wide rows taken by FFTs, a chunk at a time: Y(d) of the chunk's rows
  // (one launch per block size), then their interval sums into the slots
  // after the runs'
  if (P->n_gfft_slots > 0) {
    void* Y = grad_y(P, ws);
    const int32_t cls_end[3] = {P->n_gfft[0], P->n_gfft[0] + P->n_gfft[1],
                                P->n_gfft[0] + P->n_gfft[1] + P->n_gfft[2]};
    for (size_t c = 0; c + 1 < P->h_gfft_chunk.size() && e == hipSuccess; ++c) {
      const int32_t r0 = P->h_gfft_chunk[c], r1 = P->h_gfft_chunk[c + 1];
      auto part = [&](int k, int32_t& b) {  // rows of block-size class k in [r0, r1)
        const int32_t lo = std::max(r0, k == 0 ? 0 : cls_end[k - 1]), hi = std::min(r1, cls_end[k]);
        b = lo;
        return hi - lo;
      };
      int32_t b0 = 0, b1 = 0, b2 = 0;
      const int32_t n0 = part(0, b0), n1 = part(1, b1), n2 = part(2, b2);
      const RowFft* rows = P->d_gfft;
      const int64_t* yo = P->d_gfft_yoff;
      if (P->dtype == ARKCOS_F32) {
        e = grad_row_fft_launch<float, 256>(g, rows + b0, yo + b0, n0, spec, bout, P->d_twiddle, Y, s);
        if (e == hipSuccess)
          e = grad_row_fft_launch<float, 512>(g, rows + b1, yo + b1, n1, spec, bout, P->d_twiddle, Y, s);
        if (e == hipSuccess)
          e = grad_row_fft_launch<float, 1024>(g, rows + b2, yo + b2, n2, spec, bout, P->d_twiddle, Y, s);
        if (e == hipSuccess) {
          grad_row_scatter_kernel<float><<<P->n_gfft_slots, kBlock, 0, s>>>(g, rows + r0, r1 - r0, yo + r0,
                                                                             (const float*)Y, nruns, c > 0);
          e = hipGetLastError();
        }
      } else {
        e = grad_row_fft_launch<double, 256>(g, rows + b0, yo + b0, n0, spec, bout, P->d_twiddle, Y, s);
        if (e == hipSuccess)
          e = grad_row_fft_launch<double, 512>(g, rows + b1, yo + b1, n1, spec, bout, P->d_twiddle, Y, s);
        if (e == hipSuccess) {
          grad_row_scatter_kernel<double><<<P->n_gfft_slots, kBlock, 0, s>>>(g, rows + r0, r1 - r0, yo + r0,
                                                                              (const double*)Y, nruns, c > 0);
          e = hipGetLastError();
        }
      }
    }
    if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("gradient kernels: ") + hipGetErrorString(e));
  }
  const int32_t nmain = nruns + P->n_gfft_slots;
  int32_t nslots = nmain;
  if (fix) {
    int32_t count = 0;
    int32_t* list = pole_ring_list(P, &count);
    if (P->dtype == ARKCOS_F32)
      grad_pole_kernel<float><<<8, kBlock, 0, s>>>(g, list, count, (const float*)x, (const float*)r, nmain);
    else
      grad_pole_kernel<double><<<8, kBlock, 0, s>>>(g, list, count, (const double*)x, (const double*)r, nmain);
    nslots += 8;
  }
  // (the workspace holds n_grad_runs + n_gfft_slots + 8 slots and then the sums)
  double* sums = slots + (size_t)(nmain + 8) * (size_t)(4 * (g.nk - 1));
  grad_sum_kernel<<<(unsigned)(4 * (g.nk - 1)), kBlock, 0, s>>>(slots, nslots, 4 * (g.nk - 1), sums);
  grad_final_kernel<<<1, kBlock, 0, s>>>(sums, g.nk, P->d_basis_mom, grad);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("gradient kernels: ") + hipGetErrorString(e));
  return ARKCOS_OK;
}

}  // namespace arkcos
