// Step (c) of the hybrid method (paper Sect. 4.1): for every output ring i
//   B_i(m) = sum_{j in support(i)} K_ij(m) A~_j(m)
// with K_ij(m) (step b) read from the plan's precomputed tables or produced
// on the fly from the FP64-derived kernel samples of the pair by a
// Chebyshev recurrence.  An output unit is a ring together with its
// north/south mirror (the mirrored pair has the same K_ij(m), as in the
// paper's ring-reduction kernel that treats both hemispheres at once).
//
// Sweep: a work item owns one tile of kSweepTile modes (one per lane) and a
// segment of consecutive units, which it sweeps G units at a time (one
// wavefront per unit).  The input rings inside the support of the current
// units sit in an LDS ring buffer (slot j mod cap: the spectrum tile of ring
// j and of its mirror); moving to the next group only loads the rings that
// enter the support, so a spectrum tile is read about once per segment, not
// once per unit.  The rows of the next group are loaded into registers while
// the current group is summed.  Each unit sums its pairs in list order
// (table pairs first, their loads issued in batches, then the recurrence
// pairs), one lane per mode, with no atomics: the result does not depend on
// the segment or group size, and it is deterministic.
#include "arkcos_internal.h"
#include "device_common.h"

#include <algorithm>

namespace arkcos {

template <typename R> struct AccArgs {
  const UnitDev* units;
  const PairDev* pairs;
  const WorkItem* items;
  const SegDev* segs;
  const int64_t* spec_off;
  const int32_t* spec_len;
  const int64_t* out_off;
  const R* coef;
  const R* table;
  const int32_t* ring_n;
  const cx_t<R>* tw;   // exp(-2 pi i k / TN)
  int32_t TN;
  int32_t nrings;
  int32_t L;
  int32_t p;
  int32_t cap;         // ring slots of the LDS window
};

// (cos, sin) of pi m / den: from the twiddle table when 2 den divides its
// length, otherwise computed.
template <typename R>
__device__ __forceinline__ cx_t<R> half_angle(int m, int den, const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  if ((den & (den - 1)) == 0 && 2 * den <= TN) {
    const C t = gload(tw + (m & (2 * den - 1)) * (TN / (2 * den)));
    return cmake<C>(t.x, -t.y);
  }
  const int r = (int)((uint32_t)m % (2u * (uint32_t)den));
  return expipi<R>(r, den);
}

// Per-mode constants of the two kernel grids a unit's pairs use at mode m
// (the output ring's own length N_i for equal-length pairs, the fine grid
// p L for the others), computed once per tile.
template <typename R> struct ModeConst {
  R al_own, al_fine;    // 2 cos(2 pi m / G): Clenshaw's multiplier
  R c1h;                // cos(pi m / N_i): the shifted own grid's factor
  R lam_own, lam_fine;  // Reinsch's multiplier (-4 sin^2 or 4 cos^2 of pi m / G)
  R sg_own, sg_fine;    // Reinsch's form: +1 near x = 1, -1 near x = -1
};

template <typename R>
__device__ __forceinline__ ModeConst<R> mode_const(int m, int Ni, int pl, const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  const C h1 = half_angle<R>(m, Ni, tw, TN), hp = half_angle<R>(m, pl, tw, TN);
  ModeConst<R> k;
  // cos 2t = (cos t - sin t)(cos t + sin t)
  k.al_own = R(2) * (h1.x - h1.y) * (h1.x + h1.y);
  k.al_fine = R(2) * (hp.x - hp.y) * (hp.x + hp.y);
  k.c1h = h1.x;
  const bool po = h1.x * h1.x >= R(0.5), pf = hp.x * hp.x >= R(0.5);
  k.lam_own = po ? R(-4) * h1.y * h1.y : R(4) * h1.x * h1.x;
  k.lam_fine = pf ? R(-4) * hp.y * hp.y : R(4) * hp.x * hp.x;
  k.sg_own = po ? R(1) : R(-1);
  k.sg_fine = pf ? R(1) : R(-1);
  return k;
}

// A pair's descriptor with wave-uniform fields: meta = kind << 24 | own
// grid << 26.
struct PairU {
  uint32_t meta;
  int32_t band, ncoef;
  uint32_t off;
};

__device__ __forceinline__ int pl_kind(uint32_t meta) { return (int)((meta >> 24) & 3); }
__device__ __forceinline__ bool pl_own(uint32_t meta) { return (meta >> 26) & 1; }

// Runs STEP over a row of n8 (a multiple of 8) kernel samples from the top
// down, in chunks of 8 read with wave-uniform (scalar) loads; the rows start
// on whole chunks (the sample array is allocated aligned), so a chunk is one
// aligned load.  Rows of one chunk, the common case, take no loop.
template <typename R, typename STEP>
__device__ __forceinline__ void recur_row(int n8, const R* __restrict__ cf, STEP step) {
  auto chunk = [&](int c) {
    const R* p = static_cast<const R*>(__builtin_assume_aligned(cf + c, 8 * sizeof(R)));
    R cc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) cc[t] = p[t];
#pragma unroll
    for (int t = 7; t >= 0; --t) step(cc[t]);
  };
  if (n8 == 8) {
    chunk(0);
    return;
  }
  for (int c = n8 - 8; c >= 0; c -= 8) chunk(c);
}

template <typename R, int MPL, bool OWN>
__device__ __forceinline__ void clenshaw_row(int n8, const R* __restrict__ cf, const ModeConst<R> (&A)[MPL],
                                             R (&b1)[MPL], R (&b2)[MPL]) {
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    b1[e] = R(0);
    b2[e] = R(0);
  }
  recur_row<R>(n8, cf, [&](R c) {
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      const R b0 = fma(OWN ? A[e].al_own : A[e].al_fine, b1[e], c - b2[e]);
      b2[e] = b1[e];
      b1[e] = b0;
    }
  });
}

template <typename R, int MPL, bool OWN>
__device__ __forceinline__ void reinsch_row(int n8, const R* __restrict__ cf, const ModeConst<R> (&A)[MPL],
                                            R (&k)[MPL]) {
  R b[MPL], dd[MPL];
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    b[e] = R(0);
    dd[e] = R(0);
  }
  recur_row<R>(n8, cf, [&](R c) {
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      const R lam = OWN ? A[e].lam_own : A[e].lam_fine, sg = OWN ? A[e].sg_own : A[e].sg_fine;
      dd[e] = fma(lam, b[e], fma(sg, dd[e], c));
      b[e] = fma(sg, b[e], dd[e]);
    }
  });
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    const R lam = OWN ? A[e].lam_own : A[e].lam_fine, sg = OWN ? A[e].sg_own : A[e].sg_fine;
    k[e] = dd[e] - sg * R(0.5) * lam * (b[e] - dd[e]);
  }
}

// K_ij(m) of an on-the-fly pair d at this lane's modes m0 + lane + 64 e
// (step b): Clenshaw's recurrence for rows of up to kClenshawMaxCoef samples,
// Reinsch's modified form for longer rows; every branch is wave-uniform.
template <typename R, int MPL>
__device__ __forceinline__ void pair_k(const PairU& d, const R* __restrict__ coef, const ModeConst<R> (&A)[MPL],
                                       int m0, int lane, int ny_own, int ny_fine, R (&k)[MPL]) {
  const int kind = pl_kind(d.meta);
  const bool own = pl_own(d.meta);
  const int n8 = (d.ncoef + 7) & ~7;
  const R* cf = coef + d.off;
  if (kind == KG_REINSCH) {
    if (own) reinsch_row<R, MPL, true>(n8, cf, A, k);
    else reinsch_row<R, MPL, false>(n8, cf, A, k);
  } else {
    // (a shifted grid is always the output ring's own; with p = 1 the own
    // grid of an equatorial ring is also the fine grid, so `own` may be
    // false for it, with the same angles)
    R b1[MPL], b2[MPL];
    if (kind == KG_SHIFTED) {
      clenshaw_row<R, MPL, true>(n8, cf, A, b1, b2);
#pragma unroll
      for (int e = 0; e < MPL; ++e) k[e] = (b1[e] - b2[e]) * A[e].c1h;
    } else if (own) {
      clenshaw_row<R, MPL, true>(n8, cf, A, b1, b2);
#pragma unroll
      for (int e = 0; e < MPL; ++e) k[e] = b1[e] - b2[e] * (R(0.5) * A[e].al_own);
    } else {
      clenshaw_row<R, MPL, false>(n8, cf, A, b1, b2);
#pragma unroll
      for (int e = 0; e < MPL; ++e) k[e] = b1[e] - b2[e] * (R(0.5) * A[e].al_fine);
    }
  }
  // half weight at the grid's Nyquist mode, nothing beyond the pair's band
  const int ny = own ? ny_own : ny_fine;
  if (ny >= m0 && ny < m0 + 64 * MPL) {
#pragma unroll
    for (int e = 0; e < MPL; ++e)
      if (m0 + 64 * e + lane == ny) k[e] *= R(0.5);
  }
  if (d.band < m0 + 64 * MPL - 1) {
#pragma unroll
    for (int e = 0; e < MPL; ++e)
      if (m0 + 64 * e + lane > d.band) k[e] = R(0);
  }
}


constexpr int kTableBatch = 32;   // table pairs whose loads are issued together
constexpr int kPrefetchRows = 4;  // next-group spectrum rows held in registers per wave

// Input-ring window of the segment in LDS: slot s holds the tile of ring j
// (row 0) and of its mirror nr - 1 - j (row 1) for j = s mod cap.
template <typename R>
__device__ __forceinline__ cx_t<R>* win_row(cx_t<R>* win, int cap, int j, int half) {
  return win + ((j % cap) * 2 + half) * kSweepTile;
}

// One work item: units [seg.u0, seg.u0 + seg.nu) over the modes
// [tile kSweepTile, (tile + 1) kSweepTile).  Every wave of the block must
// call this; it synchronises the block.  WIN = false (supports too wide for
// the LDS window, cap = 0): the spectra are read from memory at each pair.
template <typename R, int G, bool TAB_ONLY, bool WIN>
__device__ __forceinline__ void sweep_item(const AccArgs<R>& a, const SegDev seg, const int tile,
                                           const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout,
                                           cx_t<R>* win) {
  using C = cx_t<R>;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m0 = tile * kSweepTile, m = m0 + lane;
  const int uend = seg.u0 + seg.nu;
  const int cap = a.cap, nr = a.nrings;
  // the spectrum row of ring j (half 0) or of its mirror (half 1), this lane's mode
  auto row_value = [&](int j, int half) -> C {
    const int ring = half ? nr - 1 - j : j;
    const int64_t off = __builtin_amdgcn_readfirstlane(gload(a.spec_off + ring));
    const int len = __builtin_amdgcn_readfirstlane(gload(a.spec_len + ring));
    return m < len ? gload(spec + off + m) : cmake<C>(R(0), R(0));
  };
  // rows of rings [jl, jh] straight into the window, wave by wave
  auto load_rows = [&](int jl, int jh, int first_row) {
    const int nrow = 2 * (jh - jl + 1);
    for (int r = first_row + w; r < nrow; r += G) {
      const int j = jl + (r >> 1);
      win_row<R>(win, cap, j, r & 1)[lane] = row_value(j, r & 1);
    }
  };
  auto unit_hi = [&](int u) { return __builtin_amdgcn_readfirstlane(gload(&a.units[u].jhi)); };

  int hi = WIN ? unit_hi(min(seg.u0 + G, uend) - 1) : 0;
  if (WIN) load_rows(seg.jlo, hi, 0);
  for (int u = seg.u0; u < uend; u += G) {
    if (WIN) __syncthreads();  // the window holds every ring of this group's supports
    // the next group's new rows: the first kPrefetchRows G into registers now
    const bool more = WIN && u + G < uend;
    const int nhi = more ? unit_hi(min(u + 2 * G, uend) - 1) : hi;
    C pf[kPrefetchRows];
#pragma unroll
    for (int k = 0; k < kPrefetchRows; ++k) {
      const int r = w + G * k;
      if (r < 2 * (nhi - hi)) pf[k] = row_value(hi + 1 + (r >> 1), r & 1);
    }
    const int uu = u + w;
    if (uu < uend) {
      const UnitDev* U = a.units + uu;
      const int band = __builtin_amdgcn_readfirstlane(gload(&U->band));
      if (m0 <= band) {
        const int i = __builtin_amdgcn_readfirstlane(gload(&U->i));
        const int im = __builtin_amdgcn_readfirstlane(gload(&U->im));
        const int pbeg = __builtin_amdgcn_readfirstlane(gload(&U->pbeg));
        const int pend = __builtin_amdgcn_readfirstlane(gload(&U->pend));
        const bool mirror = im >= 0;
        C acc0 = cmake<C>(R(0), R(0)), acc1 = acc0;
        auto add = [&](int j, R k) {
          const C v0 = WIN ? win_row<R>(win, cap, j, 0)[lane] : row_value(j, 0);
          acc0 = cmake<C>(fma(k, v0.x, acc0.x), fma(k, v0.y, acc0.y));
          if (mirror) {
            const C v1 = WIN ? win_row<R>(win, cap, j, 1)[lane] : row_value(j, 1);
            acc1 = cmake<C>(fma(k, v1.x, acc1.x), fma(k, v1.y, acc1.y));
          }
        };
        // table pairs, kTableBatch at a time with all their loads in flight
        for (int qb = pbeg; qb < pend; qb += kTableBatch) {
          R kv[kTableBatch];
          int jj[kTableBatch];
          uint32_t live = 0;
#pragma unroll
          for (int x = 0; x < kTableBatch; ++x) {
            const int q = qb + x;
            jj[x] = 0;
            if (q < pend) {
              const PairDev* pr = a.pairs + q;
              const int kind = __builtin_amdgcn_readfirstlane(gload(&pr->kind));
              const int pb = __builtin_amdgcn_readfirstlane(gload(&pr->band));
              if ((TAB_ONLY || kind == KG_TABLE) && pb >= m0) {
                const uint32_t off = __builtin_amdgcn_readfirstlane((uint32_t)gload(&pr->off));
                jj[x] = __builtin_amdgcn_readfirstlane(gload(&pr->j));
                kv[x] = gload(a.table + off + m);
                live |= 1u << x;
              }
            }
          }
#pragma unroll
          for (int x = 0; x < kTableBatch; ++x)
            if ((live >> x) & 1u) add(jj[x], kv[x]);
        }
        if (!TAB_ONLY) {
          // pairs whose K_ij(m) comes from the recurrence
          const int pl = a.p * a.L;
          const int Ni = __builtin_amdgcn_readfirstlane(gload(a.ring_n + i));
          ModeConst<R> mc[1];
          mc[0] = mode_const<R>(m, Ni, pl, a.tw, a.TN);
          for (int q = pbeg; q < pend; ++q) {
            const PairDev* pr = a.pairs + q;
            const int kind = __builtin_amdgcn_readfirstlane(gload(&pr->kind));
            const int pb = __builtin_amdgcn_readfirstlane(gload(&pr->band));
            if (kind == KG_TABLE || pb < m0) continue;
            PairU d;
            const int grid = __builtin_amdgcn_readfirstlane(gload(&pr->grid));
            d.meta = ((uint32_t)kind << 24) | ((grid != pl ? 1u : 0u) << 26);
            d.band = pb;
            d.ncoef = __builtin_amdgcn_readfirstlane(gload(&pr->ncoef));
            d.off = __builtin_amdgcn_readfirstlane((uint32_t)gload(&pr->off));
            R k[1];
            pair_k<R, 1>(d, a.coef, mc, m0, lane, Ni / 2, pl / 2, k);
            add(__builtin_amdgcn_readfirstlane(gload(&pr->j)), k[0]);
          }
        }
        if (m <= band) {
          gstore(bout + gload(a.out_off + i) + m, acc0);
          if (mirror) gstore(bout + gload(a.out_off + im) + m, acc1);
        }
      }
    }
    if (more) {
      // the next group's rows: the prefetched ones, then any beyond them
      // (their slots held rings below this group's supports: nobody reads them)
#pragma unroll
      for (int k = 0; k < kPrefetchRows; ++k) {
        const int r = w + G * k;
        if (r < 2 * (nhi - hi)) win_row<R>(win, cap, hi + 1 + (r >> 1), r & 1)[lane] = pf[k];
      }
      if (2 * (nhi - hi) > kPrefetchRows * G) load_rows(hi + 1, nhi, kPrefetchRows * G);
      hi = nhi;
    }
  }
}

// A segment descriptor read with wave-uniform (scalar) values.
__device__ __forceinline__ SegDev load_seg(const SegDev* g) {
  SegDev s;
  s.u0 = __builtin_amdgcn_readfirstlane(gload(&g->u0));
  s.nu = __builtin_amdgcn_readfirstlane(gload(&g->nu));
  s.jlo = __builtin_amdgcn_readfirstlane(gload(&g->jlo));
  s.band = __builtin_amdgcn_readfirstlane(gload(&g->band));
  return s;
}

template <typename R, int G, bool TAB_ONLY, bool WIN>
__global__ void __launch_bounds__(64 * G) accumulate_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec,
                                                            cx_t<R>* __restrict__ bout) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WorkItem it = a.items[blockIdx.x];
  sweep_item<R, G, TAB_ONLY, WIN>(a, load_seg(a.segs + it.band), it.t0, spec, bout,
                                  reinterpret_cast<cx_t<R>*>(smem));
}

// Batched form: one persistent launch drains a queue of (map, segment, tile)
// items shared by many plans; every block exits once the queue counter
// passes the item count.
template <typename R, int G, bool TAB_ONLY, bool WIN>
__global__ void __launch_bounds__(64 * G) accumulate_batch_kernel(
    const AccArgs<R>* __restrict__ maps, const int64_t* __restrict__ spec_base,
    const int64_t* __restrict__ out_base, const BatchItem* __restrict__ items, int32_t n_items,
    int32_t* __restrict__ counter, const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int cur;
  for (;;) {
    __syncthreads();  // the previous item is done with `cur` and the window
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(cur);
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const AccArgs<R> a = maps[bi.map];
    sweep_item<R, G, TAB_ONLY, WIN>(a, load_seg(a.segs + bi.band), bi.t0, spec + spec_base[bi.map],
                                    bout + out_base[bi.map], reinterpret_cast<cx_t<R>*>(smem));
  }
}

__global__ void reset_counter_kernel(int32_t* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

size_t acc_args_size() { return sizeof(AccArgs<float>); }

template <typename R>
static AccArgs<R> make_acc_args(const arkcos_plan_s* P, const SegDev* segs, const WorkItem* items, int32_t cap) {
  return AccArgs<R>{P->d_units, P->d_pairs, items, segs, P->rt.spec_off, P->rt.spec_len,
                    P->rt.out_off, (const R*)P->d_coef, (const R*)P->d_table, P->rt.n,
                    (const cx_t<R>*)P->d_twiddle, P->twiddle_n, (int32_t)P->nrings, (int32_t)P->L, P->oversample,
                    cap};
}

void fill_acc_args(arkcos_plan_s* P, const SegDev* segs, int32_t cap, void* out) {
  if (P->dtype == ARKCOS_F32)
    *reinterpret_cast<AccArgs<float>*>(out) = make_acc_args<float>(P, segs, nullptr, cap);
  else
    *reinterpret_cast<AccArgs<double>*>(out) = make_acc_args<double>(P, segs, nullptr, cap);
}

// LDS of one block: cap slots of two rows of kSweepTile complex values.
size_t acc_lds_bytes(arkcos_dtype_t dt, int32_t cap) {
  return (size_t)std::max(cap, 1) * 2 * kSweepTile * (dt == ARKCOS_F32 ? sizeof(float2) : sizeof(double2));
}

template <typename K> static hipError_t allow_acc_lds(K* k, size_t bytes) {
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R, int G, bool TAB_ONLY, bool WIN>
static hipError_t batch_launch(const void* maps, const int64_t* spec_base, const int64_t* out_base,
                               const BatchItem* items, int32_t n_items, int32_t* counter, const void* spec,
                               void* bout, int32_t grid, size_t lds, hipStream_t s) {
  hipError_t e = allow_acc_lds(accumulate_batch_kernel<R, G, TAB_ONLY, WIN>, lds);
  if (e != hipSuccess) return e;
  accumulate_batch_kernel<R, G, TAB_ONLY, WIN><<<grid, 64 * G, lds, s>>>(
      (const AccArgs<R>*)maps, spec_base, out_base, items, n_items, counter, (const cx_t<R>*)spec, (cx_t<R>*)bout);
  return hipGetLastError();
}

template <typename R, bool TAB_ONLY>
static hipError_t batch_launch_g(int32_t group, int32_t cap, const void* maps, const int64_t* spec_base,
                                 const int64_t* out_base, const BatchItem* items, int32_t n_items, int32_t* counter,
                                 const void* spec, void* bout, int32_t grid, size_t lds, hipStream_t s) {
  if (cap == 0)
    return batch_launch<R, 4, TAB_ONLY, false>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid,
                                               0, s);
  return group == 4 ? batch_launch<R, 4, TAB_ONLY, true>(maps, spec_base, out_base, items, n_items, counter, spec,
                                                         bout, grid, lds, s)
                    : batch_launch<R, 8, TAB_ONLY, true>(maps, spec_base, out_base, items, n_items, counter, spec,
                                                         bout, grid, lds, s);
}

// cap: the largest window of the batch's maps, or 0 when some map reads its
// spectra from memory (then every map does, with groups of 4).
hipError_t launch_accumulate_batch(arkcos_dtype_t dt, const void* maps, const int64_t* spec_base,
                                   const int64_t* out_base, const BatchItem* items, int32_t n_items,
                                   int32_t* counter, const void* spec, void* bout, int32_t grid, int32_t group,
                                   bool all_tables, int32_t cap, hipStream_t s) {
  reset_counter_kernel<<<1, 64, 0, s>>>(counter);
  const size_t lds = acc_lds_bytes(dt, cap);
  if (dt == ARKCOS_F32)
    return all_tables ? batch_launch_g<float, true>(group, cap, maps, spec_base, out_base, items, n_items, counter,
                                                    spec, bout, grid, lds, s)
                      : batch_launch_g<float, false>(group, cap, maps, spec_base, out_base, items, n_items, counter,
                                                     spec, bout, grid, lds, s);
  return all_tables ? batch_launch_g<double, true>(group, cap, maps, spec_base, out_base, items, n_items, counter,
                                                   spec, bout, grid, lds, s)
                    : batch_launch_g<double, false>(group, cap, maps, spec_base, out_base, items, n_items, counter,
                                                    spec, bout, grid, lds, s);
}

// Modes beyond a unit's band stay unwritten: B_i has out_len_i = band_i + 1
// modes.

template <typename R, int G, bool TAB_ONLY, bool WIN>
static hipError_t launch_one(const arkcos_plan_s* P, const AccConfig& c, const void* spec, void* bout, hipStream_t s) {
  const size_t lds = WIN ? acc_lds_bytes(P->dtype, c.cap) : 0;
  hipError_t e = allow_acc_lds(accumulate_kernel<R, G, TAB_ONLY, WIN>, lds);
  if (e != hipSuccess) return e;
  accumulate_kernel<R, G, TAB_ONLY, WIN><<<(unsigned)c.n_items, 64 * G, lds, s>>>(
      make_acc_args<R>(P, c.d_segs, c.d_items, c.cap), (const cx_t<R>*)spec, (cx_t<R>*)bout);
  return hipGetLastError();
}

template <typename R, bool TAB_ONLY>
static hipError_t launch_tab(const arkcos_plan_s* P, const AccConfig& c, const void* spec, void* bout,
                             hipStream_t s) {
  if (c.cap == 0) return launch_one<R, 4, TAB_ONLY, false>(P, c, spec, bout, s);
  return c.group == 4 ? launch_one<R, 4, TAB_ONLY, true>(P, c, spec, bout, s)
                      : launch_one<R, 8, TAB_ONLY, true>(P, c, spec, bout, s);
}

hipError_t launch_accumulate_config(const arkcos_plan_s* P, const AccConfig& c, const void* spec, void* bout,
                                    hipStream_t s) {
  if (c.n_items == 0) return hipSuccess;
  if (P->dtype == ARKCOS_F32)
    return P->all_tables ? launch_tab<float, true>(P, c, spec, bout, s) : launch_tab<float, false>(P, c, spec, bout, s);
  return P->all_tables ? launch_tab<double, true>(P, c, spec, bout, s) : launch_tab<double, false>(P, c, spec, bout, s);
}

hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s) {
  return launch_accumulate_config(P, P->acc, spec, bout, s);
}

}  // namespace arkcos
