// Step (c) of the hybrid method (paper Sect. 4.1): for every output ring i
//   B_i(m) = sum_{j in support(i)} K_ij(m) A~_j(m)
// with K_ij(m) produced on the fly from the FP64-derived kernel samples of
// the pair by the Clenshaw recurrence (step b), or read from a precomputed
// table for wide pairs.  A work item is one output ring together with its
// north/south mirror (same K_ij(m) for the mirrored pair, as in the paper's
// ring-reduction kernel that treats both hemispheres at once) and a tile of
// kModeTile consecutive modes; each thread owns one mode, so spectrum loads
// and B stores are coalesced and no atomics are needed: the sum over j runs
// in a fixed order, so results are deterministic.
#include "arkcos_internal.h"
#include "device_common.h"

#include <algorithm>

namespace arkcos {

template <typename R> struct AccArgs {
  const UnitDev* units;
  const PairDev* pairs;
  const WorkItem* items;
  const BandDev* bands;
  const int64_t* spec_off;
  const int32_t* spec_len;
  const int64_t* out_off;
  const R* coef;
  const R* table;
  const int32_t* ring_n;
  int32_t nrings;
  int32_t L;
  int32_t p;
};

// cos(pi * num / den) and sin(pi * num / den) for the mode angles.
template <typename R> __device__ __forceinline__ cx_t<R> cispi_frac(int num, int den) {
  int t = (int)((uint32_t)num % (2u * (uint32_t)den));
  return expipi<R>(t, den);
}

// Per-thread constants of the two kernel grids a unit's pairs use at mode m:
// the output ring's own length N_i (equal-length pairs) and the fine grid
// p L (all other pairs).
template <typename R> struct ModeAngles {
  int32_t fine;    // p L
  R c1, cp;        // cos(2 pi m / N_i), cos(2 pi m / (p L))
  R s1h, c1h;      // sin, cos of pi m / N_i      (half angle; shifted grid)
  R sph, cph;      // sin, cos of pi m / (p L)    (half angle)
};

// K(m) of one pair from its kernel samples (step b).  Sample rows are stored
// zero-padded to whole chunks of 8; the recurrence runs over chunks of 4
// (one uniform load each), i.e. over ceil(n / 4) * 4 samples.
template <typename R>
__device__ __forceinline__ R pair_k(int kind, int grid, int ncoef, int nyq, int band, int64_t off,
                                    const R* __restrict__ coef, const R* __restrict__ table,
                                    const ModeAngles<R>& A, int m) {
  R k;
  const int n4 = (ncoef + 3) & ~3;
  if (kind == KG_TABLE) {
    k = m <= band ? table[off + m] : R(0);
  } else if (kind == KG_REINSCH) {
    // centred grid, Reinsch's form: stable for longer rows near x = 0 and pi
    const R* cf = coef + off;
    const bool own = grid != A.fine;
    const R sh = own ? A.s1h : A.sph, ch = own ? A.c1h : A.cph;
    R b = R(0), dd = R(0);
    if (ch * ch >= R(0.5)) {
      const R lam = R(-4) * sh * sh;
      for (int c = n4 - 4; c >= 0; c -= 4) {
        R cc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) cc[e] = cf[c + e];
#pragma unroll
        for (int e = 3; e >= 0; --e) {
          dd = fma(lam, b, dd + cc[e]);
          b = b + dd;
        }
      }
      k = dd - R(0.5) * lam * (b - dd);
    } else {
      const R lam = R(4) * ch * ch;
      for (int c = n4 - 4; c >= 0; c -= 4) {
        R cc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) cc[e] = cf[c + e];
#pragma unroll
        for (int e = 3; e >= 0; --e) {
          dd = fma(lam, b, cc[e] - dd);
          b = dd - b;
        }
      }
      k = dd - R(0.5) * lam * (dd - b);
    }
    if (m == nyq) k *= R(0.5);
  } else {
    const R* cf = coef + off;
    const R cx = grid != A.fine ? A.c1 : A.cp;
    const R al = R(2) * cx;
    R b1 = R(0), b2 = R(0);
    for (int c = n4 - 4; c >= 0; c -= 4) {
      R cc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) cc[e] = cf[c + e];
#pragma unroll
      for (int e = 3; e >= 0; --e) {
        R b0 = fma(al, b1, cc[e] - b2);
        b2 = b1;
        b1 = b0;
      }
    }
    k = kind == KG_SHIFTED ? (b1 - b2) * A.c1h : b1 - b2 * cx;
    if (m == nyq) k *= R(0.5);
  }
  return k;
}

template <typename R> struct AccLds { static constexpr int kRings = 48; };
template <> struct AccLds<double> { static constexpr int kRings = 24; };

// One work item: a band of up to kBandUnits consecutive units and kAccTile
// modes.  The block first stages A~_j(m) (and the mirror ring's spectrum) of
// every input ring in the band's window into LDS, one coalesced row per ring;
// then wavefront w accumulates unit u0 + w over its pairs, lane = mode, with
// all pair data wave-uniform.
// One work item (band of units, kAccTile modes) with the block's waves; the
// band table is the caller's (a plan's own bands, or a batch's).  Every wave
// of the block must call it; it synchronises the block.
template <typename R>
__device__ __forceinline__ void accumulate_item(const AccArgs<R>& a, const BandDev& bd, int m0,
                                                const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout,
                                                cx_t<R>* sa) {
  using C = cx_t<R>;
  constexpr int CH = AccLds<R>::kRings;  // input rings staged at a time
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int m = m0 + lane;
  const bool active = w < bd.nu;
  UnitDev u{};
  if (active) u = a.units[bd.u0 + w];
  const bool busy = active && m0 <= u.band;
  const bool mirror = u.im >= 0;
  const int pl = a.p * a.L;
  const int Ni = active ? a.ring_n[u.i] : a.L;
  ModeAngles<R> ang;
  {
    const C e1 = cispi_frac<R>(2 * m, Ni), ep = cispi_frac<R>(2 * m, pl);
    const C h1 = cispi_frac<R>(m, Ni), hp = cispi_frac<R>(m, pl);
    ang.fine = pl;
    ang.c1 = e1.x; ang.cp = ep.x;
    ang.c1h = h1.x; ang.s1h = h1.y;
    ang.cph = hp.x; ang.sph = hp.y;
  }
  C acc0 = cmake<C>(R(0), R(0)), acc1 = acc0;
  // the unit's pair descriptors, one pair per lane (64 at a time), read back
  // with readlane as wave-uniform values
  const int npair = u.pend - u.pbeg;
  int qi = 0, base = -64;
  int vj = 0, vband = -1, vkind = 0, vp = 1, vnc = 0, vnyq = 0, voff_lo = 0, voff_hi = 0;
  const int win = bd.jhi - bd.jlo + 1;
  for (int c0 = 0; c0 < win; c0 += CH) {
    const int c1 = min(win, c0 + CH);
    for (int r = w; r < 2 * (c1 - c0); r += nwaves) {
      int j = bd.jlo + c0 + (r >> 1);
      if (r & 1) j = a.nrings - 1 - j;
      C v = cmake<C>(R(0), R(0));
      if (m < a.spec_len[j]) v = spec[a.spec_off[j] + m];
      sa[r * kAccTile + lane] = v;
    }
    __syncthreads();
    if (busy) {
      for (; qi < npair; ++qi) {
        if (qi - base >= 64) {
          base = qi;
          if (base + lane < npair) {
            const PairDev mine = a.pairs[u.pbeg + base + lane];
            vj = mine.j; vband = mine.band; vkind = mine.kind; vp = mine.grid;
            vnc = mine.ncoef; vnyq = mine.nyq;
            voff_lo = (int)(uint32_t)(uint64_t)mine.off;
            voff_hi = (int)(uint32_t)((uint64_t)mine.off >> 32);
          }
        }
        const int t = qi - base;
        const int j = __builtin_amdgcn_readlane(vj, t);
        if (j >= bd.jlo + c1) break;
        const int band = __builtin_amdgcn_readlane(vband, t);
        if (m0 > band) continue;
        const int kind = __builtin_amdgcn_readlane(vkind, t);
        const int pp = __builtin_amdgcn_readlane(vp, t);
        const int nc = __builtin_amdgcn_readlane(vnc, t);
        const int nyq = __builtin_amdgcn_readlane(vnyq, t);
        const int64_t off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(voff_hi, t) << 32) |
                                      (uint64_t)(uint32_t)__builtin_amdgcn_readlane(voff_lo, t));
        R k = pair_k<R>(kind, pp, nc, nyq, band, off, a.coef, a.table, ang, m);
        if (m > band) k = R(0);
        const int row = 2 * (j - bd.jlo - c0);
        const C s0 = sa[row * kAccTile + lane];
        acc0 = cmake<C>(fma(k, s0.x, acc0.x), fma(k, s0.y, acc0.y));
        if (mirror) {
          const C s1 = sa[(row + 1) * kAccTile + lane];
          acc1 = cmake<C>(fma(k, s1.x, acc1.x), fma(k, s1.y, acc1.y));
        }
      }
    }
    __syncthreads();
  }
  if (busy && m <= u.band) {
    bout[a.out_off[u.i] + m] = acc0;
    if (mirror) bout[a.out_off[u.im] + m] = acc1;
  }
}

template <typename R>
__global__ void __launch_bounds__(kAccThreads) accumulate_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec,
                                                                 cx_t<R>* __restrict__ bout) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WorkItem it = a.items[blockIdx.x];
  accumulate_item<R>(a, a.bands[it.unit], it.m0, spec, bout, reinterpret_cast<cx_t<R>*>(smem));
}

// Batched form: one persistent launch drains a queue of (map, band, first
// mode) items shared by many plans; every block exits once the queue counter
// passes the item count.
template <typename R>
__global__ void __launch_bounds__(kAccThreads) accumulate_batch_kernel(
    const AccArgs<R>* __restrict__ maps, const int64_t* __restrict__ spec_base,
    const int64_t* __restrict__ out_base, const BatchItem* __restrict__ items, int32_t n_items,
    int32_t* __restrict__ counter, const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int cur;
  for (;;) {
    __syncthreads();  // the previous item is done with `cur` and the LDS tiles
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const AccArgs<R> a = maps[bi.map];
    accumulate_item<R>(a, a.bands[bi.band], bi.m0, spec + spec_base[bi.map], bout + out_base[bi.map],
                       reinterpret_cast<cx_t<R>*>(smem));
  }
}

__global__ void reset_counter_kernel(int32_t* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

size_t acc_args_size() { return sizeof(AccArgs<float>); }

void fill_acc_args(arkcos_plan_s* P, const BandDev* bands, void* out) {
  if (P->dtype == ARKCOS_F32) {
    AccArgs<float> a{P->d_units, P->d_pairs, P->d_items, bands, P->rt.spec_off, P->rt.spec_len,
                     P->rt.out_off, (const float*)P->d_coef, (const float*)P->d_table, P->rt.n,
                     (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    *reinterpret_cast<AccArgs<float>*>(out) = a;
  } else {
    AccArgs<double> a{P->d_units, P->d_pairs, P->d_items, bands, P->rt.spec_off, P->rt.spec_len,
                      P->rt.out_off, (const double*)P->d_coef, (const double*)P->d_table, P->rt.n,
                      (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    *reinterpret_cast<AccArgs<double>*>(out) = a;
  }
}

size_t acc_lds_bytes(arkcos_dtype_t dt, int32_t max_window) {
  if (dt == ARKCOS_F32)
    return 2 * (size_t)std::min<int32_t>(max_window, AccLds<float>::kRings) * kAccTile * sizeof(float2);
  return 2 * (size_t)std::min<int32_t>(max_window, AccLds<double>::kRings) * kAccTile * sizeof(double2);
}

hipError_t launch_accumulate_batch(arkcos_dtype_t dt, const void* maps, const int64_t* spec_base,
                                   const int64_t* out_base, const BatchItem* items, int32_t n_items,
                                   int32_t* counter, const void* spec, void* bout, int32_t grid,
                                   int32_t units_per_band, size_t lds, hipStream_t s) {
  reset_counter_kernel<<<1, 64, 0, s>>>(counter);
  const int threads = 64 * units_per_band;
  if (dt == ARKCOS_F32) {
    hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_kernel<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    accumulate_batch_kernel<float><<<grid, threads, lds, s>>>((const AccArgs<float>*)maps, spec_base, out_base,
                                                              items, n_items, counter, (const float2*)spec,
                                                              (float2*)bout);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_kernel<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    accumulate_batch_kernel<double><<<grid, threads, lds, s>>>((const AccArgs<double>*)maps, spec_base, out_base,
                                                               items, n_items, counter, (const double2*)spec,
                                                               (double2*)bout);
  }
  return hipGetLastError();
}

static size_t acc_lds(const arkcos_plan_s* P) {
  if (P->dtype == ARKCOS_F32)
    return 2 * (size_t)std::min<int32_t>(P->max_window, AccLds<float>::kRings) * kAccTile * sizeof(float2);
  return 2 * (size_t)std::min<int32_t>(P->max_window, AccLds<double>::kRings) * kAccTile * sizeof(double2);
}

// Modes beyond a unit's band stay zero (B_i has out_len_i = band_i + 1 modes,
// so nothing is left unwritten).

hipError_t configure_accumulate(arkcos_plan_s* P) {
  const size_t lds = acc_lds(P);
  if (P->dtype == ARKCOS_F32)
    return hipFuncSetAttribute((const void*)accumulate_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipFuncSetAttribute((const void*)accumulate_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s) {
  if (P->h_items.empty()) return hipSuccess;
  if (P->dtype == ARKCOS_F32) {
    AccArgs<float> a{P->d_units, P->d_pairs, P->d_items, P->d_bands, P->rt.spec_off, P->rt.spec_len,
                     P->rt.out_off, (const float*)P->d_coef, (const float*)P->d_table, P->rt.n,
                     (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    accumulate_kernel<float><<<(unsigned)P->h_items.size(), kAccThreads,
                                acc_lds(P), s>>>(a, (const float2*)spec, (float2*)bout);
  } else {
    AccArgs<double> a{P->d_units, P->d_pairs, P->d_items, P->d_bands, P->rt.spec_off, P->rt.spec_len,
                      P->rt.out_off, (const double*)P->d_coef, (const double*)P->d_table, P->rt.n,
                      (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    accumulate_kernel<double><<<(unsigned)P->h_items.size(), kAccThreads,
                                 acc_lds(P), s>>>(a, (const double2*)spec, (double2*)bout);
  }
  return hipGetLastError();
}

}  // namespace arkcos
