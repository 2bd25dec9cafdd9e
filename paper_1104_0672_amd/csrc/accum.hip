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

constexpr int kModesPerLane = kAccTile / 64;
constexpr int kTableGroup = 2;     // table pairs whose values are loaded together

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

// A pair as staged in LDS for one work item.
struct PairLds {
  uint32_t meta;   // row (j - jlo) | kind << 24 | own grid << 26
  int32_t band;
  int32_t ncoef;
  uint32_t off;    // coefficient or table offset
};

__device__ __forceinline__ int pl_row(uint32_t meta) { return (int)(meta & 0xffffff); }
__device__ __forceinline__ int pl_kind(uint32_t meta) { return (int)((meta >> 24) & 3); }
__device__ __forceinline__ bool pl_own(uint32_t meta) { return (meta >> 26) & 1; }

// A pair's descriptor with wave-uniform fields.
struct PairU {
  uint32_t meta;
  int32_t band, ncoef;
  uint32_t off;
};

__device__ __forceinline__ PairU uniform_pair(const PairLds& d) {
  PairU p;
  p.meta = __builtin_amdgcn_readfirstlane(d.meta);
  p.band = __builtin_amdgcn_readfirstlane(d.band);
  p.ncoef = __builtin_amdgcn_readfirstlane(d.ncoef);
  p.off = __builtin_amdgcn_readfirstlane(d.off);
  return p;
}

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

template <typename R> struct AccLds { static constexpr int kRings = 8; };
template <> struct AccLds<double> { static constexpr int kRings = 4; };

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

// One work item: the units of band bd (one wavefront each) over the tiles
// [t0, t0 + nt) of kAccTile modes; lane l holds modes m0 + l + 64 e.  The
// band's pair descriptors are staged into LDS once, each unit's list split
// (in input-ring order) into table pairs and on-the-fly pairs.  The input
// rings of the window are staged in chunks of CH rings (a ring and its
// mirror per row pair), the spectra of the next (tile, chunk) stage loaded
// into registers while the current stage is accumulated.  Per stage a wave
// first streams its table pairs, kTableGroup at a time with all their loads
// issued together, then evaluates its on-the-fly pairs, the next pair's
// kernel samples loaded while the current one is evaluated.  Every wave of
// the block must call this; it synchronises the block.
template <typename R, int NW, bool TAB_ONLY = false>
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
  // chunks are fixed ranges of CH input rings [cbase + c CH, cbase + (c + 1) CH),
  // the same for every band layout, so that the order of the sum over a
  // unit's pairs (by chunk, then tables before the rest, each by ring) does
  // not depend on how units are grouped into bands
  const int cbase = win > 0 ? bd.jlo / CH * CH : 0;
  const int nch = win > 0 ? (bd.jhi + 1 - cbase + CH - 1) / CH : 1;
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
    for (int b = 0; b < npair; b += 64) {
      const int q = b + lane;
      const bool tab = q < npair && gload(&a.pairs[u.pbeg + q].kind) == KG_TABLE;
      ntab += __popcll(__ballot(tab));
    }
    int nt_seen = 0;
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
    const int cs = cbase + c * CH;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
      const int j = cs + (r >> 1);
#pragma unroll
      for (int e = 0; e < MPL; ++e) pre[k][e] = cmake<C>(R(0), R(0));
      if (r < 2 * CH && j >= bd.jlo && j <= bd.jhi) {
        const RowRef rr = rows[2 * (j - bd.jlo) + (r & 1)];
#pragma unroll
        for (int e = 0; e < MPL; ++e)
          if (m + 64 * e < rr.len) pre[k][e] = gload(spec + rr.off + m + 64 * e);
      }
    }
  };
  issue(0);
  C acc0[MPL], acc1[MPL];
  ModeConst<R> mc[MPL];
  int qt = 0, qo = 0;
  PairU cur{};
  int m0 = 0, c0 = 0, c1 = 0;  // c0, c1: the staged chunk's rings, relative to jlo
  auto accumulate_pair = [&](int row, const R (&k)[MPL]) {
    const C* s0 = sa + row * kAccTile + lane;
#pragma unroll
    for (int e = 0; e < MPL; ++e) {
      const C v = s0[64 * e];
      acc0[e] = cmake<C>(fma(k[e], v.x, acc0[e].x), fma(k[e], v.y, acc0[e].y));
    }
    if (mirror) {
#pragma unroll
      for (int e = 0; e < MPL; ++e) {
        const C v = s0[kAccTile + 64 * e];
        acc1[e] = cmake<C>(fma(k[e], v.x, acc1[e].x), fma(k[e], v.y, acc1[e].y));
      }
    }
  };
  for (int s = 0; s < nst; ++s) {
    const int t = s / nch, c = s - t * nch;
    m0 = (t0 + t) * kAccTile;
    c0 = cbase + c * CH - bd.jlo;
    c1 = c0 + CH;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
      if (r < 2 * CH) {
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
        if (busy && !TAB_ONLY) mc[e] = mode_const<R>(m0 + 64 * e + lane, Ni, pl, a.tw, a.TN);
      }
      qt = 0;
      qo = ntab;
      if (!TAB_ONLY && busy && qo < npair) cur = uniform_pair(mine[qo]);
    }
    // Up to G table pairs of the staged chunk from descriptor qt on: the
    // descriptors are read together (the descriptor area has CH spare
    // entries, so reads past a unit's last pair stay inside it), then the
    // tile of every pair whose band reaches it is loaded without bounds
    // checks (tables are zero-padded to whole tiles) and with no register
    // cleared in between, so that the loads overlap each other and the
    // spectrum prefetch; then they are accumulated.  Returns the pairs used.
    auto table_group = [&](auto gsize) -> int {
      constexpr int G = decltype(gsize)::value;
      PairU d[G];
#pragma unroll
      for (int x = 0; x < G; ++x) d[x] = uniform_pair(mine[qt + x]);
      int g = 0;
      uint32_t live = 0;
#pragma unroll
      for (int x = 0; x < G; ++x)
        if (g == x && qt + x < ntab && pl_row(d[x].meta) < c1) {
          g = x + 1;
          if (d[x].band >= m0) live |= 1u << x;
        }
      R kv[G][MPL];
#pragma unroll
      for (int x = 0; x < G; ++x)
        if ((live >> x) & 1u) {
          const R* tb = a.table + d[x].off + m0;
#pragma unroll
          for (int e = 0; e < MPL; ++e) kv[x][e] = gload(tb + 64 * e + lane);
        }
#pragma unroll
      for (int x = 0; x < G; ++x)
        if ((live >> x) & 1u) accumulate_pair(2 * (pl_row(d[x].meta) - c0), kv[x]);
      qt += g;
      return g;
    };
    if (busy && TAB_ONLY) {
      // every pair has a table: a unit has at most CH pairs in a chunk
      table_group(std::integral_constant<int, CH>{});
    } else if (busy) {
      while (qt < ntab)
        if (table_group(std::integral_constant<int, kTableGroup>{}) == 0) break;
      // on-the-fly pairs of this chunk
      while (qo < npair && pl_row(cur.meta) < c1) {
        const PairU d = cur;
        if (qo + 1 < npair) cur = uniform_pair(mine[qo + 1]);
        if (m0 <= d.band) {
          R k[MPL];
          pair_k<R, MPL>(d, a.coef, mc, m0, lane, ny_own, ny_fine, k);
          accumulate_pair(2 * (pl_row(d.meta) - c0), k);
        }
        ++qo;
      }
    }
    if (busy && c == nch - 1) {
      const int64_t o0 = gload(a.out_off + u.i);
      const int64_t o1 = mirror ? gload(a.out_off + u.im) : 0;
#pragma unroll
      for (int e = 0; e < MPL; ++e) {
        const int m = m0 + 64 * e + lane;
        if (m <= u.band) {
          gstore(bout + o0 + m, acc0[e]);
          if (mirror) gstore(bout + o1 + m, acc1[e]);
        }
      }
    }
    __syncthreads();
  }
}

// Table-only plans, U units per wavefront: the band holds U NW units and
// wave w takes the units w + NW x (x < U), so the window of input rings a
// band stages (its units' supports, some 36 rings wider than the band at
// nside 2048 / 5') serves U times as many units per block.  Per stage a wave
// streams the table tiles of its first unit's pairs in the staged chunk, then
// those of its next, each exactly as the one-unit form does (the same order
// of the sum over a unit's pairs).  Every wave must call this; it
// synchronises the block.
template <typename R, int NW, int U, int CHR = AccLds<R>::kRings>
__device__ __forceinline__ void accumulate_band_tabu(const AccArgs<R>& a, const BandDev& bd, const int t0,
                                                     const int nt, const cx_t<R>* __restrict__ spec,
                                                     cx_t<R>* __restrict__ bout, unsigned char* smem,
                                                     const AccLayout lay) {
  using C = cx_t<R>;
  constexpr int CH = CHR;
  constexpr int RPW = (2 * CH + NW - 1) / NW;
  constexpr int MPL = kModesPerLane;
  C* sa = reinterpret_cast<C*>(smem);
  RowRef* rows = reinterpret_cast<RowRef*>(smem + lay.rows_off);
  PairLds* dsc = reinterpret_cast<PairLds*>(smem + lay.pairs_off);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int win = max(bd.jhi - bd.jlo + 1, 0);
  const int cbase = win > 0 ? bd.jlo / CH * CH : 0;
  const int nch = win > 0 ? (bd.jhi + 1 - cbase + CH - 1) / CH : 1;
  for (int r = threadIdx.x; r < 2 * win; r += NW * 64) {
    int j = bd.jlo + (r >> 1);
    if (r & 1) j = a.nrings - 1 - j;
    rows[r].off = gload(a.spec_off + j);
    rows[r].len = gload(a.spec_len + j);
  }
  UnitDev u[U];
  bool act[U], mirror[U];
  int npair[U];
  PairLds* mine[U];
#pragma unroll
  for (int x = 0; x < U; ++x) {
    const int ux = w + NW * x;
    act[x] = ux < bd.nu;
    u[x] = UnitDev{};
    if (act[x]) {
      u[x].i = gload(&a.units[bd.u0 + ux].i);
      u[x].im = gload(&a.units[bd.u0 + ux].im);
      u[x].pbeg = gload(&a.units[bd.u0 + ux].pbeg);
      u[x].pend = gload(&a.units[bd.u0 + ux].pend);
      u[x].band = gload(&a.units[bd.u0 + ux].band);
    }
    mirror[x] = u[x].im >= 0;
    npair[x] = act[x] ? u[x].pend - u[x].pbeg : 0;
    mine[x] = dsc + (act[x] ? u[x].pbeg - bd.pbeg : 0);
    // every pair has a table: the descriptors in input-ring order
    for (int b = 0; b < npair[x]; b += 64) {
      const int q = b + lane;
      if (q < npair[x]) {
        const PairDev* g = a.pairs + u[x].pbeg + q;
        PairLds d;
        d.meta = (uint32_t)(gload(&g->j) - bd.jlo) | ((uint32_t)KG_TABLE << 24);
        d.band = gload(&g->band);
        d.ncoef = 0;
        d.off = (uint32_t)gload(&g->off);
        mine[x][q] = d;
      }
    }
  }
  __syncthreads();  // row table and descriptors ready

  const int nst = nt * nch;
  C pre[RPW][MPL];
  auto issue = [&](int s) {
    const int t = s / nch, c = s - t * nch;
    const int m = (t0 + t) * kAccTile + lane;
    const int cs = cbase + c * CH;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
      const int j = cs + (r >> 1);
#pragma unroll
      for (int e = 0; e < MPL; ++e) pre[k][e] = cmake<C>(R(0), R(0));
      if (r < 2 * CH && j >= bd.jlo && j <= bd.jhi) {
        const RowRef rr = rows[2 * (j - bd.jlo) + (r & 1)];
#pragma unroll
        for (int e = 0; e < MPL; ++e)
          if (m + 64 * e < rr.len) pre[k][e] = gload(spec + rr.off + m + 64 * e);
      }
    }
  };
  issue(0);
  C acc0[U][MPL], acc1[U][MPL];
  int qt[U];
#pragma unroll
  for (int x = 0; x < U; ++x) qt[x] = 0;
  for (int s = 0; s < nst; ++s) {
    const int t = s / nch, c = s - t * nch;
    const int m0 = (t0 + t) * kAccTile;
    const int c0 = cbase + c * CH - bd.jlo, c1 = c0 + CH;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = w + NW * k;
      if (r < 2 * CH) {
#pragma unroll
        for (int e = 0; e < MPL; ++e) sa[r * kAccTile + 64 * e + lane] = pre[k][e];
      }
    }
    __syncthreads();
    if (s + 1 < nst) issue(s + 1);
#pragma unroll
    for (int x = 0; x < U; ++x) {
      const bool busy = act[x] && m0 <= u[x].band;
      if (c == 0) {
#pragma unroll
        for (int e = 0; e < MPL; ++e) {
          acc0[x][e] = cmake<C>(R(0), R(0));
          acc1[x][e] = acc0[x][e];
        }
        qt[x] = 0;
      }
      // this unit's pairs in the staged chunk, in groups of up to GS: the
      // group's descriptors read together (the area has 8 spare entries),
      // then every live tile loaded, then accumulated
      constexpr int GS = CH < 8 ? CH : 8;
      for (int grp = 0; busy && grp < CH / GS; ++grp) {
        PairU d[GS];
#pragma unroll
        for (int y = 0; y < GS; ++y) d[y] = uniform_pair(mine[x][qt[x] + y]);
        // the group's pairs in the chunk (a prefix: pairs are in input-ring
        // order) and those whose band reaches the tile, by one ballot each
        // over lanes 0 .. GS-1 instead of a scalar test per pair
        bool in_chunk = false, reach = false;
        if (lane < GS && qt[x] + lane < npair[x]) {
          const PairLds dl = mine[x][qt[x] + lane];
          in_chunk = pl_row(dl.meta) < c1;
          reach = in_chunk && dl.band >= m0;
        }
        const int g = __builtin_amdgcn_readfirstlane(__popcll(__ballot(in_chunk)));
        const uint32_t live = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)__ballot(reach));
        R kv[GS][MPL];
#pragma unroll
        for (int y = 0; y < GS; ++y)
          if ((live >> y) & 1u) {
            const R* tb = a.table + d[y].off + m0;
#pragma unroll
            for (int e = 0; e < MPL; ++e) kv[y][e] = gload(tb + 64 * e + lane);
          }
#pragma unroll
        for (int y = 0; y < GS; ++y)
          if ((live >> y) & 1u) {
            const C* s0 = sa + 2 * (pl_row(d[y].meta) - c0) * kAccTile + lane;
#pragma unroll
            for (int e = 0; e < MPL; ++e) {
              const C v = s0[64 * e];
              acc0[x][e] = cmake<C>(fma(kv[y][e], v.x, acc0[x][e].x), fma(kv[y][e], v.y, acc0[x][e].y));
            }
            if (mirror[x]) {
#pragma unroll
              for (int e = 0; e < MPL; ++e) {
                const C v = s0[kAccTile + 64 * e];
                acc1[x][e] = cmake<C>(fma(kv[y][e], v.x, acc1[x][e].x), fma(kv[y][e], v.y, acc1[x][e].y));
              }
            }
          }
        qt[x] += g;
        if (g < GS) break;
      }
      if (busy && c == nch - 1) {
        const int64_t o0 = gload(a.out_off + u[x].i);
        const int64_t o1 = mirror[x] ? gload(a.out_off + u[x].im) : 0;
#pragma unroll
        for (int e = 0; e < MPL; ++e) {
          const int m = m0 + 64 * e + lane;
          if (m <= u[x].band) {
            gstore(bout + o0 + m, acc0[x][e]);
            if (mirror[x]) gstore(bout + o1 + m, acc1[x][e]);
          }
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

// TAB_ONLY: every pair of the plan has a table of K_ij(m) (no recurrence
// code, fewer registers, more waves: the FP32 form is held to 80 VGPRs, so
// that three blocks share a CU instead of two).
template <typename R, int NW, bool TAB_ONLY>
__global__ void __launch_bounds__(64 * NW)
    __attribute__((amdgpu_waves_per_eu((TAB_ONLY && sizeof(R) == 4) ? 6 : 1))) accumulate_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec,
                                                                 cx_t<R>* __restrict__ bout, AccLayout lay) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WorkItem it = a.items[blockIdx.x];
  accumulate_band<R, NW, TAB_ONLY>(a, a.bands[it.band], it.t0, it.nt, spec, bout, smem, lay);
}

// Table-only plans with U units per wavefront (bands of U NW units), CHR
// input rings staged at a time.
template <typename R, int NW, int U, int CHR = AccLds<R>::kRings>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4)))
    accumulate_u_kernel(AccArgs<R> a, const cx_t<R>* __restrict__ spec, cx_t<R>* __restrict__ bout, AccLayout lay) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WorkItem it = a.items[blockIdx.x];
  accumulate_band_tabu<R, NW, U, CHR>(a, a.bands[it.band], it.t0, it.nt, spec, bout, smem, lay);
}

// Batched form: one persistent launch drains a queue of (map, band, tiles)
// items shared by many plans; every block exits once the queue counter
// passes the item count.
template <typename R, int NW, bool TAB_ONLY>
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
    accumulate_band<R, NW, TAB_ONLY>(a, load_band(a.bands + bi.band), bi.t0, bi.nt, spec + spec_base[bi.map],
                                     bout + out_base[bi.map], smem, lay);
  }
}

// The batched form with U units per wavefront (table-only batches).
template <typename R, int NW, int U, int CHR = AccLds<R>::kRings>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) accumulate_batch_u_kernel(
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
    accumulate_band_tabu<R, NW, U, CHR>(a, load_band(a.bands + bi.band), bi.t0, bi.nt, spec + spec_base[bi.map],
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

void fill_acc_args(arkcos_plan_s* P, const BandDev* bands, void* out, const int64_t* spec_off,
                   const int32_t* spec_len) {
  if (P->dtype == ARKCOS_F32) {
    AccArgs<float> a = make_acc_args<float>(P, bands);
    if (spec_off) a.spec_off = spec_off;
    if (spec_len) a.spec_len = spec_len;
    *reinterpret_cast<AccArgs<float>*>(out) = a;
  } else {
    AccArgs<double> a = make_acc_args<double>(P, bands);
    if (spec_off) a.spec_off = spec_off;
    if (spec_len) a.spec_len = spec_len;
    *reinterpret_cast<AccArgs<double>*>(out) = a;
  }
}

// LDS of one accumulation block: the staged spectra (2 CH rows of kAccTile
// complex values), the row table of the whole window, the band's pair
// descriptors.
static AccLayout acc_layout(arkcos_dtype_t dt, const AccShape& sh, int32_t staged_rings = 0) {
  const int32_t win = std::max(sh.max_window, 1);
  size_t tile;
  if (dt == ARKCOS_F32)
    tile = 2 * (size_t)(staged_rings ? staged_rings : AccLds<float>::kRings) * kAccTile * sizeof(float2);
  else
    tile = 2 * (size_t)(staged_rings ? staged_rings : AccLds<double>::kRings) * kAccTile * sizeof(double2);
  AccLayout l;
  l.rows_off = (int32_t)tile;
  l.pairs_off = (int32_t)(tile + 2 * (size_t)win * sizeof(RowRef));
  return l;
}

size_t acc_lds_bytes(arkcos_dtype_t dt, const AccShape& sh, int32_t staged_rings) {
  // 8 spare descriptors: a group of table pairs reads up to 8 descriptors at once
  return (size_t)acc_layout(dt, sh, staged_rings).pairs_off +
         (size_t)(std::max(sh.max_band_pairs, 1) + 8) * sizeof(PairLds);
}

template <typename R, int NW, bool TAB_ONLY>
static hipError_t batch_launch(const void* maps, const int64_t* spec_base, const int64_t* out_base,
                               const BatchItem* items, int32_t n_items, int32_t* counter, const void* spec,
                               void* bout, int32_t grid, size_t lds, AccLayout lay, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_kernel<R, NW, TAB_ONLY>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  accumulate_batch_kernel<R, NW, TAB_ONLY><<<grid, 64 * NW, lds, s>>>(
      (const AccArgs<R>*)maps, spec_base, out_base, items, n_items, counter, (const cx_t<R>*)spec, (cx_t<R>*)bout,
      lay);
  return hipGetLastError();
}

template <typename R, bool TAB_ONLY>
static hipError_t batch_launch_nw(int32_t units_per_band, const void* maps, const int64_t* spec_base,
                                  const int64_t* out_base, const BatchItem* items, int32_t n_items, int32_t* counter,
                                  const void* spec, void* bout, int32_t grid, size_t lds, AccLayout lay,
                                  hipStream_t s) {
  if (units_per_band == 16)
    return batch_launch<R, 16, TAB_ONLY>(maps, spec_base, out_base, items, n_items, counter, spec, bout, grid, lds,
                                         lay, s);
  return units_per_band == 4 ? batch_launch<R, 4, TAB_ONLY>(maps, spec_base, out_base, items, n_items, counter, spec,
                                                            bout, grid, lds, lay, s)
                             : batch_launch<R, 8, TAB_ONLY>(maps, spec_base, out_base, items, n_items, counter, spec,
                                                            bout, grid, lds, lay, s);
}

hipError_t launch_accumulate_batch(arkcos_dtype_t dt, const void* maps, const int64_t* spec_base,
                                   const int64_t* out_base, const BatchItem* items, int32_t n_items,
                                   int32_t* counter, const void* spec, void* bout, int32_t grid,
                                   int32_t units_per_band, bool all_tables, const AccShape& shape, hipStream_t s,
                                   int32_t units_per_wave, int32_t staged_rings) {
  reset_counter_kernel<<<1, 64, 0, s>>>(counter);
  const size_t lds = acc_lds_bytes(dt, shape);
  const AccLayout lay = acc_layout(dt, shape);
  if (dt == ARKCOS_F32 && all_tables && units_per_wave == 2 && units_per_band == 16 && staged_rings == 16) {
    const size_t lds16 = acc_lds_bytes(dt, shape, 16);
    hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_u_kernel<float, 8, 2, 16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds16);
    if (e != hipSuccess) return e;
    accumulate_batch_u_kernel<float, 8, 2, 16><<<grid, 512, lds16, s>>>(
        (const AccArgs<float>*)maps, spec_base, out_base, items, n_items, counter, (const float2*)spec, (float2*)bout,
        acc_layout(dt, shape, 16));
    return hipGetLastError();
  }
  if (dt == ARKCOS_F32 && all_tables && units_per_wave == 2 && units_per_band == 16) {
    hipError_t e = hipFuncSetAttribute((const void*)accumulate_batch_u_kernel<float, 8, 2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    accumulate_batch_u_kernel<float, 8, 2><<<grid, 512, lds, s>>>((const AccArgs<float>*)maps, spec_base, out_base,
                                                                  items, n_items, counter, (const float2*)spec,
                                                                  (float2*)bout, lay);
    return hipGetLastError();
  }
  if (dt == ARKCOS_F32)
    return all_tables ? batch_launch_nw<float, true>(units_per_band, maps, spec_base, out_base, items, n_items,
                                                     counter, spec, bout, grid, lds, lay, s)
                      : batch_launch_nw<float, false>(units_per_band, maps, spec_base, out_base, items, n_items,
                                                      counter, spec, bout, grid, lds, lay, s);
  return all_tables ? batch_launch_nw<double, true>(units_per_band, maps, spec_base, out_base, items, n_items,
                                                    counter, spec, bout, grid, lds, lay, s)
                    : batch_launch_nw<double, false>(units_per_band, maps, spec_base, out_base, items, n_items,
                                                     counter, spec, bout, grid, lds, lay, s);
}

// Modes beyond a unit's band stay zero (B_i has out_len_i = band_i + 1 modes,
// so nothing is left unwritten).

template <typename K> static hipError_t allow_acc_lds(K* k, size_t bytes) {
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t configure_accumulate_shape(const arkcos_plan_s* P, const AccShape& shape) {
  const size_t lds = acc_lds_bytes(P->dtype, shape);
  hipError_t e;
  if (P->dtype == ARKCOS_F32) {
    e = allow_acc_lds(accumulate_kernel<float, 8, false>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<float, 8, true>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<float, 16, false>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<float, 16, true>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_u_kernel<float, 8, 2>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_u_kernel<float, 8, 3>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_u_kernel<float, 8, 2, 16>, acc_lds_bytes(P->dtype, shape, 16));
  } else {
    e = allow_acc_lds(accumulate_kernel<double, 8, false>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<double, 8, true>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<double, 16, false>, lds);
    if (e == hipSuccess) e = allow_acc_lds(accumulate_kernel<double, 16, true>, lds);
  }
  return e;
}

hipError_t configure_accumulate(arkcos_plan_s* P) { return configure_accumulate_shape(P, P->acc_shape); }

template <typename R, int NW>
static void launch_nw(const arkcos_plan_s* P, const AccArgs<R>& a, unsigned grid, size_t lds, AccLayout lay,
                      const void* spec, void* bout, hipStream_t s) {
  auto k = P->all_tables ? accumulate_kernel<R, NW, true> : accumulate_kernel<R, NW, false>;
  k<<<grid, 64 * NW, lds, s>>>(a, (const cx_t<R>*)spec, (cx_t<R>*)bout, lay);
}

// One launch of the plan's accumulation with the given bands, items and
// shape (the plan's own, or a candidate timed at plan creation).
hipError_t launch_accumulate_shape(const arkcos_plan_s* P, const BandDev* bands, const WorkItem* items,
                                   int32_t n_items, int32_t units, const AccShape& shape, const void* spec,
                                   void* bout, hipStream_t s, int32_t units_per_wave, int32_t staged_rings) {
  if (n_items == 0) return hipSuccess;
  const size_t lds = acc_lds_bytes(P->dtype, shape);
  const AccLayout lay = acc_layout(P->dtype, shape);
  if (P->dtype == ARKCOS_F32) {
    AccArgs<float> a = make_acc_args<float>(P, bands);
    a.items = items;
    if (units_per_wave == 2 && staged_rings == 16 && P->all_tables && units == 16) {
      accumulate_u_kernel<float, 8, 2, 16><<<(unsigned)n_items, 512, acc_lds_bytes(P->dtype, shape, 16), s>>>(
          a, (const float2*)spec, (float2*)bout, acc_layout(P->dtype, shape, 16));
    } else if (units_per_wave > 1 && P->all_tables && units == 8 * units_per_wave) {
      if (units_per_wave == 2)
        accumulate_u_kernel<float, 8, 2><<<(unsigned)n_items, 512, lds, s>>>(a, (const float2*)spec, (float2*)bout, lay);
      else
        accumulate_u_kernel<float, 8, 3><<<(unsigned)n_items, 512, lds, s>>>(a, (const float2*)spec, (float2*)bout, lay);
    } else if (units == 16) {
      launch_nw<float, 16>(P, a, (unsigned)n_items, lds, lay, spec, bout, s);
    }
    else launch_nw<float, 8>(P, a, (unsigned)n_items, lds, lay, spec, bout, s);
  } else {
    AccArgs<double> a = make_acc_args<double>(P, bands);
    a.items = items;
    if (units == 16) launch_nw<double, 16>(P, a, (unsigned)n_items, lds, lay, spec, bout, s);
    else launch_nw<double, 8>(P, a, (unsigned)n_items, lds, lay, spec, bout, s);
  }
  return hipGetLastError();
}

hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s) {
  return launch_accumulate_shape(P, P->d_bands, P->d_items, (int32_t)P->h_items.size(), P->acc_units, P->acc_shape,
                                 spec, bout, s, P->acc_upw, P->acc_ch);
}

}  // namespace arkcos
