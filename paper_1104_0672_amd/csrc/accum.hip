// Step (c) of the hybrid method (paper Sect. 4.1): for every output ring i
//   B_i(m) = sum_{j in support(i)} K_ij(m) A~_j(m)
// with K_ij(m) produced on the fly from the FP64-derived kernel samples of
// the pair by a Chebyshev recurrence (step b), or read from a precomputed
// table for wide pairs.  An output unit is a ring together with its
// north/south mirror (the mirrored pair has the same K_ij(m), as in the
// paper's ring-reduction kernel that treats both hemispheres at once).  A
// work item is a band of consecutive units (one wavefront each) and a run of
// mode tiles; a lane owns kModesPerLane modes of a tile, so spectrum loads
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
  const cx_t<R>* tw;   // exp(-2 pi i k / TN)
  int32_t TN;
  int32_t nrings;
  int32_t L;
  int32_t p;
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

// Per-mode constants of the two kernel grids a unit's pairs use at mode m:
// the output ring's own length N_i (equal-length pairs) and the fine grid
// p L (all other pairs).
template <typename R> struct ModeAngles {
  R c1, cp;        // cos(2 pi m / N_i), cos(2 pi m / (p L))
  R s1h, c1h;      // sin, cos of pi m / N_i      (half angle; shifted grid)
  R sph, cph;      // sin, cos of pi m / (p L)    (half angle)
};

template <typename R>
__device__ __forceinline__ ModeAngles<R> mode_angles(int m, int Ni, int pl, const cx_t<R>* __restrict__ tw, int TN) {
  using C = cx_t<R>;
  const C h1 = half_angle<R>(m, Ni, tw, TN), hp = half_angle<R>(m, pl, tw, TN);
  ModeAngles<R> a;
  a.c1h = h1.x; a.s1h = h1.y;
  a.cph = hp.x; a.sph = hp.y;
  a.c1 = (h1.x - h1.y) * (h1.x + h1.y);  // cos 2t = (cos t - sin t)(cos t + sin t)
  a.cp = (hp.x - hp.y) * (hp.x + hp.y);
  return a;
}

constexpr int kModesPerLane = kAccTile / 64;
constexpr int kPrefetchCoef = 16;  // kernel samples of the next pair held in registers

// A pair as staged in LDS for one work item.
struct PairLds {
  uint32_t meta;   // row (j - jlo) | kind << 24 | own grid << 26
  int32_t band;
  int32_t ncoef;
  uint32_t off;    // coefficient or table offset
};

__device__ __forceinline__ int pl_row(const PairLds& d) { return (int)(d.meta & 0xffffff); }
__device__ __forceinline__ int pl_kind(const PairLds& d) { return (int)((d.meta >> 24) & 3); }
__device__ __forceinline__ bool pl_own(const PairLds& d) { return (d.meta >> 26) & 1; }

// Loads the kernel samples of pair d that its evaluation needs first: the
// top kPrefetchCoef samples of its row, or the row and what follows it for
// rows of at most 8 (the sample array is padded so this stays in bounds).
// All lanes read the same addresses; rows are zero-padded to whole chunks
// of 8.
template <typename R>
__device__ __forceinline__ void prefetch_coef(const PairLds& d, const R* __restrict__ coef, R (&buf)[kPrefetchCoef]) {
  const int n8 = (d.ncoef + 7) & ~7;
  const R* cf = coef + d.off + max(n8 - kPrefetchCoef, 0);
#pragma unroll
  for (int t = 0; t < kPrefetchCoef; ++t) buf[t] = gload(cf + t);
}

// One step of the Clenshaw recurrence b_d = 2x b_{d+1} - b_{d+2} + a_d for
// every mode of the lane.
template <typename R, int MPL>
__device__ __forceinline__ void clenshaw_step(R c, const R (&al)[MPL], R (&b1)[MPL], R (&b2)[MPL]) {
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    const R b0 = fma(al[e], b1[e], c - b2[e]);
    b2[e] = b1[e];
    b1[e] = b0;
  }
}

// One step of Reinsch's modified recurrence (stable near x = +-1) in the form
// sigma = +1 (x > 0) or -1 (x < 0).
template <typename R, int MPL>
__device__ __forceinline__ void reinsch_step(R c, const R (&lam)[MPL], const R (&sg)[MPL], R (&b)[MPL],
                                             R (&dd)[MPL]) {
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    dd[e] = fma(lam[e], b[e], fma(sg[e], dd[e], c));
    b[e] = fma(sg[e], b[e], dd[e]);
  }
}

// Runs STEP over the kernel samples of a row of n8 (a multiple of 8)
// samples from the top down: the top 16 (or 8) from the prefetched
// registers, the rest from memory in chunks of 8, each loaded one chunk
// ahead.
template <typename R, typename STEP>
__device__ __forceinline__ void recur_row(int n8, const R* __restrict__ cf, const R (&buf)[kPrefetchCoef], STEP step) {
  if (n8 <= 8) {
#pragma unroll
    for (int t = 7; t >= 0; --t) step(buf[t]);
    return;
  }
  R nx[8];
  if (n8 > 16) {
#pragma unroll
    for (int t = 0; t < 8; ++t) nx[t] = gload(cf + n8 - 24 + t);
  }
#pragma unroll
  for (int t = 15; t >= 0; --t) step(buf[t]);
  for (int c = n8 - 24; c >= 0; c -= 8) {
    R cc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) cc[t] = nx[t];
    if (c >= 8) {
#pragma unroll
      for (int t = 0; t < 8; ++t) nx[t] = gload(cf + c - 8 + t);
    }
#pragma unroll
    for (int t = 7; t >= 0; --t) step(cc[t]);
  }
}

// K_ij(m) of an on-the-fly pair d at this lane's modes m[e] (step b), from
// the prefetched registers and, for long rows, the rest of the row.
template <typename R, int MPL>
__device__ __forceinline__ void pair_k(const PairLds& d, const R* __restrict__ coef, const R (&buf)[kPrefetchCoef],
                                       const ModeAngles<R> (&A)[MPL], const int (&m)[MPL], int ny_own, int ny_fine,
                                       R (&k)[MPL]) {
  const int kind = pl_kind(d);
  const bool own = pl_own(d);
  const int ny = own ? ny_own : ny_fine;
  const int n8 = (d.ncoef + 7) & ~7;
  const R* cf = coef + d.off;
  if (kind == KG_REINSCH) {
    R lam[MPL], sg[MPL], b[MPL], dd[MPL];
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      const R sh = own ? A[e].s1h : A[e].sph, ch = own ? A[e].c1h : A[e].cph;
      const bool pos = ch * ch >= R(0.5);
      lam[e] = pos ? R(-4) * sh * sh : R(4) * ch * ch;
      sg[e] = pos ? R(1) : R(-1);
      b[e] = R(0);
      dd[e] = R(0);
    }
    recur_row<R>(n8, cf, buf, [&](R c) { reinsch_step<R, MPL>(c, lam, sg, b, dd); });
#pragma unroll
    for (int e = 0; e < MPL; ++e) k[e] = dd[e] - sg[e] * R(0.5) * lam[e] * (b[e] - dd[e]);
  } else {
    R al[MPL], b1[MPL], b2[MPL];
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      al[e] = R(2) * (own ? A[e].c1 : A[e].cp);
      b1[e] = R(0);
      b2[e] = R(0);
    }
    recur_row<R>(n8, cf, buf, [&](R c) { clenshaw_step<R, MPL>(c, al, b1, b2); });
#pragma unroll
    for (int e = 0; e < MPL; ++e)
      k[e] = kind == KG_SHIFTED ? (b1[e] - b2[e]) * A[e].c1h : b1[e] - b2[e] * (R(0.5) * al[e]);
  }
#pragma unroll
  for (int e = 0; e < MPL; ++e) {
    if (m[e] == ny) k[e] *= R(0.5);
    if (m[e] > d.band) k[e] = R(0);
  }
}

template <typename R> struct AccLds { static constexpr int kRings = 22; };
template <> struct AccLds<double> { static constexpr int kRings = 11; };

// Spectrum row of one staged input ring: offset and length in the workspace.
struct RowRef {
  int64_t off;
  int32_t len, pad;
};

// Byte offsets of the row table and the pair descriptors in the LDS of an
// accumulation block (the staged spectra come first).
struct AccLayout {
  int32_t rows_off, pairs_off;
};

constexpr int kTableGroup = 8;  // table pairs whose values are loaded together

// One work item: the units of band bd (one wavefront each) over the tiles
// [t0, t0 + nt) of kAccTile modes; lane l holds modes m0 + l + 64 e.  The
// band's pair descriptors are staged into LDS once, each unit's list split
// (in input-ring order) into table pairs and on-the-fly pairs.  The input
// rings of the window are staged in chunks of CH rings (a ring and its
// mirror per row pair), the spectra of the next (tile, chunk) stage loaded
// into registers while the current stage is accumulated.  Per stage a wave
// first streams its table pairs, kTableGroup at a time with all their loads
// issued together, then evaluates its on-the-fly pairs with the next pair's
// kernel samples in flight.  Every wave of the block must call this; it
// synchronises the block.
template <typename R, int NW>
__device__ __forceinline__ void accumulate_band(const AccArgs<R>& a, const BandDev& bd, const int t0, const int nt,
                                                const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout,
                                                unsigned char* smem, const AccLayout lay) {
  using C = cx_t<R>;
  constexpr int CH = AccLds<R>::kRings;        // input rings staged at a time
  constexpr int RPW = (2 * CH + NW - 1) / NW;  // staged rows per wave
  constexpr int MPL = kModesPerLane;
  C* sa = reinterpret_cast<C*>(smem);
  RowRef* rows = reinterpret_cast<RowRef*>(smem + lay.rows_off);
  PairLds* dsc = reinterpret_cast<PairLds*>(smem + lay.pairs_off);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int win = max(bd.jhi - bd.jlo + 1, 0);
  const int nch = max((win + CH - 1) / CH, 1);
  const int pl = a.p * a.L;
  for (int r = threadIdx.x; r < 2 * win; r += NW * 64) {
    int j = bd.jlo + (r >> 1);
    if (r & 1) j = a.nrings - 1 - j;
    rows[r].off = gload(a.spec_off + j);
    rows[r].len = gload(a.spec_len + j);
  }
  const bool active = w < bd.nu;
  UnitDev u{};
  if (active) {
    u.i = gload(&a.units[bd.u0 + w].i);
    u.im = gload(&a.units[bd.u0 + w].im);
    u.pbeg = gload(&a.units[bd.u0 + w].pbeg);
    u.pend = gload(&a.units[bd.u0 + w].pend);
    u.band = gload(&a.units[bd.u0 + w].band);
  }
  const bool mirror = u.im >= 0;
  const int npair = active ? u.pend - u.pbeg : 0;
  PairLds* mine = dsc + (active ? u.pbeg - bd.pbeg : 0);
  // this unit's descriptors: table pairs first, then the others, each in order
  int ntab = 0;
  {
    int nt_seen = 0;
    for (int b = 0; b < npair; b += 64) {
      const int q = b + lane;
      const bool valid = q < npair;
      const bool tab = valid && gload(&a.pairs[u.pbeg + q].kind) == KG_TABLE;
      const uint64_t tm = __ballot(tab);
      ntab += __popcll(tm);
    }
    for (int b = 0; b < npair; b += 64) {
      const int q = b + lane;
      const bool valid = q < npair;
      PairDev pr{};
      if (valid) {
        const PairDev* g = a.pairs + u.pbeg + q;
        pr.j = gload(&g->j);
        pr.kind = gload(&g->kind);
        pr.band = gload(&g->band);
        pr.ncoef = gload(&g->ncoef);
        pr.grid = gload(&g->grid);
        pr.off = gload(&g->off);
      }
      const bool tab = valid && pr.kind == KG_TABLE;
      const uint64_t tm = __ballot(tab), vm = __ballot(valid);
      const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
      const int tb = __popcll(tm & below);
      const int ob = __popcll(vm & ~tm & below);
      if (valid) {
        PairLds d;
        d.meta = (uint32_t)(pr.j - bd.jlo) | ((uint32_t)pr.kind << 24) | ((pr.grid != pl ? 1u : 0u) << 26);
        d.band = pr.band;
        d.ncoef = pr.ncoef;
        d.off = (uint32_t)pr.off;
        mine[tab ? nt_seen + tb : ntab + (b - nt_seen) + ob] = d;
      }
      nt_seen += __popcll(tm);
    }
  }
  const int Ni = active ? gload(a.ring_n + u.i) : a.L;
  const int ny_own = Ni / 2, ny_fine = pl / 2;
  __syncthreads();  // row table and descriptors ready

  const int nst = nt * nch;
  C pre[RPW][MPL];
  auto issue = [&](int s) {
    const int t = s / nch, c = s - t * nch;
    const int m = (t0 + t) * kAccTile + lane;
    const int cs = c * CH, nrow = 2 * (min(win, cs + CH) - cs);
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
#pragma unroll
      for (int e = 0; e < MPL; ++e) pre[k][e] = cmake<C>(R(0), R(0));
      if (r < nrow) {
        const RowRef rr = rows[2 * cs + r];
#pragma unroll
        for (int e = 0; e < MPL; ++e)
          if (m + 64 * e < rr.len) pre[k][e] = gload(spec + rr.off + m + 64 * e);
      }
    }
  };
  issue(0);
  C acc0[MPL], acc1[MPL];
  ModeAngles<R> ang[MPL];
  int mm[MPL];
  int qt = 0, qo = 0, phase = 0;
  PairLds dA{}, dB{};
  R bA[kPrefetchCoef], bB[kPrefetchCoef];
  int m0 = 0, c0 = 0, c1 = 0;
  auto accumulate_pair = [&](int row, const R (&k)[MPL]) {
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      const C s0 = sa[row * kAccTile + 64 * e + lane];
      acc0[e] = cmake<C>(fma(k[e], s0.x, acc0[e].x), fma(k[e], s0.y, acc0[e].y));
    }
    if (mirror) {
#pragma unroll
      for (int e = 0; e < MPL; ++e) {
        const C s1 = sa[(row + 1) * kAccTile + 64 * e + lane];
        acc1[e] = cmake<C>(fma(k[e], s1.x, acc1[e].x), fma(k[e], s1.y, acc1[e].y));
      }
    }
  };
  // evaluates the current on-the-fly pair (cur, cb) and prefetches the next
  // one into (nx, nb); false at the end of the list or of the staged chunk
  auto step = [&](const PairLds& cur, const R (&cb)[kPrefetchCoef], PairLds& nx, R (&nb)[kPrefetchCoef]) {
    if (qo >= npair || pl_row(cur) >= c1) return false;
    if (qo + 1 < npair) {
      nx = mine[qo + 1];
      nx.meta = __builtin_amdgcn_readfirstlane(nx.meta);
      nx.ncoef = __builtin_amdgcn_readfirstlane(nx.ncoef);
      nx.band = __builtin_amdgcn_readfirstlane(nx.band);
      prefetch_coef<R>(nx, a.coef, nb);
    }
    if (m0 <= cur.band) {
      R k[MPL];
      pair_k<R, MPL>(cur, a.coef, cb, ang, mm, ny_own, ny_fine, k);
      accumulate_pair(2 * (pl_row(cur) - c0), k);
    }
    ++qo;
    return true;
  };
  for (int s = 0; s < nst; ++s) {
    const int t = s / nch, c = s - t * nch;
    m0 = (t0 + t) * kAccTile;
    c0 = c * CH;
    c1 = min(win, c0 + CH);
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
      if (r < 2 * (c1 - c0)) {
#pragma unroll
        for (int e = 0; e < MPL; ++e) sa[r * kAccTile + 64 * e + lane] = pre[k][e];
      }
    }
    __syncthreads();
    if (s + 1 < nst) issue(s + 1);
    const bool busy = active && m0 <= u.band;
    if (c == 0) {
#pragma unroll
      for (int e = 0; e < MPL; ++e) {
        acc0[e] = cmake<C>(R(0), R(0));
        acc1[e] = acc0[e];
        mm[e] = m0 + 64 * e + lane;
        if (busy) ang[e] = mode_angles<R>(mm[e], Ni, pl, a.tw, a.TN);
      }
      qt = 0;
      qo = ntab;
      phase = 0;
    }
    if (busy) {
      // table pairs of this chunk, kTableGroup at a time
      while (qt < ntab) {
        R kv[kTableGroup][MPL];
        int rw[kTableGroup];
        int g = 0;
#pragma unroll
        for (int x = 0; x < kTableGroup; ++x) {
          rw[x] = -1;
          if (qt + x < ntab && g == x) {
            PairLds d = mine[qt + x];
            d.meta = __builtin_amdgcn_readfirstlane(d.meta);
            if (pl_row(d) < c1) {
              rw[x] = 2 * (pl_row(d) - c0);
              g = x + 1;
#pragma unroll
              for (int e = 0; e < MPL; ++e) kv[x][e] = mm[e] <= d.band ? gload(a.table + d.off + mm[e]) : R(0);
            }
          }
        }
        if (g == 0) break;
#pragma unroll
        for (int x = 0; x < kTableGroup; ++x)
          if (x < g) accumulate_pair(rw[x], kv[x]);
        qt += g;
      }
      // on-the-fly pairs of this chunk
      if (qo < npair && phase == 0 && (c == 0 || qo == ntab)) {
        dA = mine[qo];
        dA.meta = __builtin_amdgcn_readfirstlane(dA.meta);
        dA.ncoef = __builtin_amdgcn_readfirstlane(dA.ncoef);
        dA.band = __builtin_amdgcn_readfirstlane(dA.band);
        prefetch_coef<R>(dA, a.coef, bA);
      }
      // the two prefetch buffers alternate; each call site names its own
      // buffers so that they stay in registers
      bool more = true;
      if (phase == 1) {
        more = step(dB, bB, dA, bA);
        if (more) phase = 0;
      }
      while (more) {
        if (!step(dA, bA, dB, bB)) break;
        if (!step(dB, bB, dA, bA)) {
          phase = 1;
          break;
        }
      }
      if (c == nch - 1) {
#pragma unroll
        for (int e = 0; e < MPL; ++e)
          if (mm[e] <= u.band) {
            gstore(bout + gload(a.out_off + u.i) + mm[e], acc0[e]);
            if (mirror) gstore(bout + gload(a.out_off + u.im) + mm[e], acc1[e]);
          }
      }
    }
    __syncthreads();
  }
}

// A band descriptor read with wave-uniform (scalar) values.
__device__ __forceinline__ BandDev load_band(const BandDev* g) {
  BandDev b;
  b.u0 = __builtin_amdgcn_readfirstlane(gload(&g->u0));
  b.nu = __builtin_amdgcn_readfirstlane(gload(&g->nu));
  b.jlo = __builtin_amdgcn_readfirstlane(gload(&g->jlo));
  b.jhi = __builtin_amdgcn_readfirstlane(gload(&g->jhi));
  b.band = __builtin_amdgcn_readfirstlane(gload(&g->band));
  b.pbeg = __builtin_amdgcn_readfirstlane(gload(&g->pbeg));
  b.npair = __builtin_amdgcn_readfirstlane(gload(&g->npair));
  b.pad = 0;
  return b;
}

template <typename R>
__global__ void __launch_bounds__(kAccThreads) accumulate_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec,
                                                                 cx_t<R>* __restrict__ bout, AccLayout lay) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WorkItem it = a.items[blockIdx.x];
  accumulate_band<R, kBandUnits>(a, a.bands[it.band], it.t0, it.nt, spec, bout, smem, lay);
}

// Batched form: one persistent launch drains a queue of (map, band, tiles)
// items shared by many plans; every block exits once the queue counter
// passes the item count.
template <typename R, int NW>
__global__ void __launch_bounds__(64 * NW) accumulate_batch_kernel(
    const AccArgs<R>* __restrict__ maps, const int64_t* __restrict__ spec_base,
    const int64_t* __restrict__ out_base, const BatchItem* __restrict__ items, int32_t n_items,
    int32_t* __restrict__ counter, const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout, AccLayout lay) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int cur;
  for (;;) {
    __syncthreads();  // the previous item is done with `cur` and the LDS tiles
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(cur);
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    const AccArgs<R> a = maps[bi.map];
    accumulate_band<R, NW>(a, load_band(a.bands + bi.band), bi.t0, bi.nt, spec + spec_base[bi.map],
                           bout + out_base[bi.map], smem, lay);
  }
}

__global__ void reset_counter_kernel(int32_t* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

size_t acc_args_size() { return sizeof(AccArgs<float>); }

template <typename R> static AccArgs<R> make_acc_args(const arkcos_plan_s* P, const BandDev* bands) {
  return AccArgs<R>{P->d_units, P->d_pairs, P->d_items, bands, P->rt.spec_off, P->rt.spec_len,
                    P->rt.out_off, (const R*)P->d_coef, (const R*)P->d_table, P->rt.n,
                    (const cx_t<R>*)P->d_twiddle, P->twiddle_n, (int32_t)P->nrings, (int32_t)P->L, P->oversample};
}

void fill_acc_args(arkcos_plan_s* P, const BandDev* bands, void* out) {
  if (P->dtype == ARKCOS_F32)
    *reinterpret_cast<AccArgs<float>*>(out) = make_acc_args<float>(P, bands);
  else
    *reinterpret_cast<AccArgs<double>*>(out) = make_acc_args<double>(P, bands);
}

// LDS of one accumulation block: the staged spectra (2 CH rows of kAccTile
// complex values, CH = min(window, kRings)), the row table of the whole
// window, the band's pair descriptors.
static AccLayout acc_layout(arkcos_dtype_t dt, const AccShape& sh) {
  const int32_t win = std::max(sh.max_window, 1);
  size_t tile;
  if (dt == ARKCOS_F32)
    tile = 2 * (size_t)std::min<int32_t>(win, AccLds<float>::kRings) * kAccTile * sizeof(float2);
  else
    tile = 2 * (size_t)std::min<int32_t>(win, AccLds<double>::kRings) * kAccTile * sizeof(double2);
  AccLayout l;
  l.rows_off = (int32_t)tile;
  l.pairs_off = (int32_t)(tile + 2 * (size_t)win * sizeof(RowRef));
  return l;
}

size_t acc_lds_bytes(arkcos_dtype_t dt, const AccShape& sh) {
  return (size_t)acc_layout(dt, sh).pairs_off + (size_t)std::max(sh.max_band_pairs, 1) * sizeof(PairLds);
}

template <typename R, int NW>
static hipError_t batch_launch(const void* maps, const int64_t* spec_base, const int64_t* out_base,
                               const BatchItem* items, int32_t n_items, int32_t* counter, const void* spec,
                               void* bout, int32_t grid, size_t lds, AccLayout lay, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_kernel<R, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  accumulate_batch_kernel<R, NW><<<grid, 64 * NW, lds, s>>>((const AccArgs<R>*)maps, spec_base, out_base, items,
                                                            n_items, counter, (const cx_t<R>*)spec, (cx_t<R>*)bout,
                                                            lay);
  return hipGetLastError();
}

hipError_t launch_accumulate_batch(arkcos_dtype_t dt, const void* maps, const int64_t* spec_base,
                                   const int64_t* out_base, const BatchItem* items, int32_t n_items,
                                   int32_t* counter, const void* spec, void* bout, int32_t grid,
                                   int32_t units_per_band, const AccShape& shape, hipStream_t s) {
  reset_counter_kernel<<<1, 64, 0, s>>>(counter);
  const size_t lds = acc_lds_bytes(dt, shape);
  const AccLayout lay = acc_layout(dt, shape);
  if (dt == ARKCOS_F32)
    return units_per_band == 4
               ? batch_launch<float, 4>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid, lds,
                                        lay, s)
               : batch_launch<float, 8>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid, lds,
                                        lay, s);
  return units_per_band == 4
             ? batch_launch<double, 4>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid, lds,
                                       lay, s)
             : batch_launch<double, 8>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid, lds,
                                       lay, s);
}

// Modes beyond a unit's band stay zero (B_i has out_len_i = band_i + 1 modes,
// so nothing is left unwritten).

hipError_t configure_accumulate(arkcos_plan_s* P) {
  const size_t lds = acc_lds_bytes(P->dtype, P->acc_shape);
  if (P->dtype == ARKCOS_F32)
    return hipFuncSetAttribute((const void*)accumulate_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipFuncSetAttribute((const void*)accumulate_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s) {
  if (P->h_items.empty()) return hipSuccess;
  const size_t lds = acc_lds_bytes(P->dtype, P->acc_shape);
  const AccLayout lay = acc_layout(P->dtype, P->acc_shape);
  if (P->dtype == ARKCOS_F32)
    accumulate_kernel<float><<<(unsigned)P->h_items.size(), kAccThreads, lds, s>>>(
        make_acc_args<float>(P, P->d_bands), (const float2*)spec, (float2*)bout, lay);
  else
    accumulate_kernel<double><<<(unsigned)P->h_items.size(), kAccThreads, lds, s>>>(
        make_acc_args<double>(P, P->d_bands), (const double2*)spec, (double2*)bout, lay);
  return hipGetLastError();
}

}  // namespace arkcos
