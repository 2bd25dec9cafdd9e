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

namespace arkcos {

template <typename R> struct AccArgs {
  const UnitDev* units;
  const PairDev* pairs;
  const WorkItem* items;
  const int64_t* spec_off;
  const int64_t* out_off;
  const int32_t* out_len;
  const R* coef;
  const R* table;
  int32_t nrings;
  int32_t L;
  int32_t p;
};

// cos(pi * num / den) for the mode angles.
template <typename R> __device__ __forceinline__ R cospi_frac(int num, int den) {
  int64_t t = ((int64_t)num) % (2 * (int64_t)den);
  return expipi<R>((int)t, den).x;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) accumulate_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec,
                                                            cx_t<R>* __restrict__ bout) {
  using C = cx_t<R>;
  const WorkItem it = a.items[blockIdx.x];
  const UnitDev u = a.units[it.unit];
  const int m = it.m0 + threadIdx.x;
  const int L = a.L, pl = a.p * a.L;
  // cos of the mode angle on the three kernel grids
  const R c1 = cospi_frac<R>(2 * m, L);    // centred, p = 1:  cos(2 pi m / L)
  const R ch = cospi_frac<R>(m, L);        // shifted grid:    cos(pi m / L)
  const R cp = cospi_frac<R>(2 * m, pl);   // centred, p > 1:  cos(2 pi m / (p L))
  C acc0 = cmake<C>(R(0), R(0)), acc1 = acc0;
  const bool mirror = u.im >= 0;
  for (int q = u.pbeg; q < u.pend; ++q) {
    const PairDev pr = a.pairs[q];
    if (it.m0 > pr.band) continue;  // whole tile above the pair's band
    R k;
    if (pr.kind == KG_TABLE) {
      k = m <= pr.band ? a.table[pr.off + m] : R(0);
    } else {
      const R* cf = a.coef + pr.off;
      const R cx = pr.kind == KG_SHIFTED ? c1 : (pr.p == 1 ? c1 : cp);
      const R al = R(2) * cx;
      R b1 = R(0), b2 = R(0);
      for (int d = pr.ncoef - 1; d >= 0; --d) {
        R b0 = fma(al, b1, cf[d] - b2);
        b2 = b1;
        b1 = b0;
      }
      k = pr.kind == KG_SHIFTED ? (b1 - b2) * ch : b1 - b2 * cx;
      if (m == pr.nyq) k *= R(0.5);
    }
    if (m <= pr.band) {
      const C s0 = spec[a.spec_off[pr.j] + m];
      acc0 = cmake<C>(fma(k, s0.x, acc0.x), fma(k, s0.y, acc0.y));
      if (mirror) {
        const C s1 = spec[a.spec_off[a.nrings - 1 - pr.j] + m];
        acc1 = cmake<C>(fma(k, s1.x, acc1.x), fma(k, s1.y, acc1.y));
      }
    }
  }
  if (m <= u.band) {
    bout[a.out_off[u.i] + m] = acc0;
    if (mirror) bout[a.out_off[u.im] + m] = acc1;
  }
}

// Modes beyond a unit's band stay zero (B_i has out_len_i = band_i + 1 modes,
// so nothing is left unwritten).

hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s) {
  if (P->h_items.empty()) return hipSuccess;
  if (P->dtype == ARKCOS_F32) {
    AccArgs<float> a{P->d_units, P->d_pairs, P->d_items, P->rt.spec_off, P->rt.out_off,
                     P->rt.out_len, (const float*)P->d_coef, (const float*)P->d_table,
                     (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    accumulate_kernel<float><<<(unsigned)P->h_items.size(), kBlock, 0, s>>>(
        a, (const float2*)spec, (float2*)bout);
  } else {
    AccArgs<double> a{P->d_units, P->d_pairs, P->d_items, P->rt.spec_off, P->rt.out_off,
                      P->rt.out_len, (const double*)P->d_coef, (const double*)P->d_table,
                      (int32_t)P->nrings, (int32_t)P->L, P->oversample};
    accumulate_kernel<double><<<(unsigned)P->h_items.size(), kBlock, 0, s>>>(
        a, (const double2*)spec, (double2*)bout);
  }
  return hipGetLastError();
}

}  // namespace arkcos
