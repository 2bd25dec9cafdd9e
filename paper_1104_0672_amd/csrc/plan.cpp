// Host side of plan creation: ring geometry, ring pairs inside the kernel
// support, kernel-sample windows, bands, tables, FFT strategies and the
// device-memory layout of spectra and output coefficients.
//
// Geometry (paper Sect. 4.1; HEALPix after Gorski et al. 2005): rings
// r = 1 .. 4 nside - 1; polar rings hold 4r pixels offset by pi/(4r) at
// z = 1 - r^2/(3 nside^2); equatorial rings hold 4 nside pixels at
// z = 4/3 - 2r/(3 nside), offset by pi/(4 nside) when r - nside is even; the
// south cap mirrors the north.  ECP rings are at theta_i = (i + 1/2) pi / n_theta
// with n_phi unshifted pixels and band areas as weights.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>

#include "arkcos_internal.h"
#include "device_common.h"

namespace arkcos {

namespace {

struct Status {
  arkcos_status_t st = ARKCOS_OK;
  std::string msg;
};

template <typename T> hipError_t dev_alloc(arkcos_plan_s* P, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) return e;
  P->allocations.push_back(p);
  P->plan_bytes += count * sizeof(T);
  *ptr = static_cast<T*>(p);
  return hipSuccess;
}

template <typename T> hipError_t upload(arkcos_plan_s* P, T** ptr, const std::vector<T>& v) {
  hipError_t e = dev_alloc(P, ptr, v.size());
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpy(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(_e == hipErrorOutOfMemory ? ARKCOS_ERR_OUT_OF_MEMORY : ARKCOS_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                     \
  } while (0)

// P of the FFT path for the kernel row of pair q with nc samples (spline
// plans; 0: the direct sums).  The row's grid G must be a power of two of at
// least kFftRowMinGrid longitudes dividing the twiddle table's length, its
// nodes centred, and the FFTs (S = G /
// (2 P) sub-transforms of P points, P at most 16384 in FP32 and 8192 in FP64,
// the largest that one workgroup's LDS holds) cheaper than the sums over
// samples x modes.
int64_t fft_row_max_points(const arkcos_plan_s* P) { return P->dtype == ARKCOS_F32 ? 16384 : 8192; }

int32_t fft_row_points(const arkcos_plan_s* P, int64_t q, int64_t nc) {
  const PairDev& pr = P->h_pairs[q];
  if (P->prof_kind != 1 || P->h_pair_shift[q] || pr.band < 0 || nc <= kGradMaxCoef) return 0;
  const int64_t G = pr.grid;
  if (!is_pow2(G) || G < kFftRowMinGrid || P->twiddle_n % G != 0) return 0;
  const int64_t pcap = fft_row_max_points(P);
  const int64_t Pn = std::min<int64_t>(G / 2, pcap);
  const int64_t S = G / (2 * Pn);
  const double direct = (double)nc * (double)(pr.band + 1);
  const double fft = 4.0 * (double)S * (double)Pn * std::log2((double)Pn) + 2.0 * (double)G;
  return direct > fft ? (int32_t)Pn : 0;
}

// Rows grouped by block size (fft_row_threads), biggest first within each.
static void group_fft_rows(std::vector<RowFft>& rows, int32_t counts[3]) {
  auto cls = [](int32_t Pn) { return Pn <= 4096 ? 0 : (Pn <= 8192 ? 1 : 2); };
  std::stable_sort(rows.begin(), rows.end(), [&](const RowFft& a, const RowFft& b) {
    return cls(a.P) != cls(b.P) ? cls(a.P) < cls(b.P) : a.P > b.P;
  });
  for (int c = 0; c < 3; ++c) counts[c] = 0;
  for (const RowFft& r : rows) ++counts[cls(r.P)];
}

// Uploads the spline knots and their moments (spline plans only).
arkcos_status_t upload_knots(arkcos_plan_s* P) {
  if (P->prof_kind != 1) return ARKCOS_OK;
  std::vector<double> mom;
  spline_moments(P->knots, P->theta_max / (P->knots.size() - 1), mom);
  HIPCHK(hipMemcpy(P->d_knots, P->knots.data(), P->knots.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(P->d_spline_mom, mom.data(), mom.size() * sizeof(double), hipMemcpyHostToDevice));
  return ARKCOS_OK;
}

// Work items of the knot gradient (spline plans): per unit its narrow rows,
// and every wide row cut into mode chunks whose correlation fits
// kGradZBytes of LDS, each chunk into sample ranges of about kGradItemWork
// samples x modes; then the items cut into runs of equal estimated cost, one
// run per gradient block, eight times as many runs as resident blocks so that
// the estimate's errors even out (a block that drew cheap runs takes more).
// Depends only on the pairs' windows and bands, which knot updates keep.
arkcos_status_t build_grad_items(arkcos_plan_s* P) {
  std::vector<GradItem> items;
  std::vector<double> cost;
  std::vector<RowFft> fft_rows;
  int64_t zmax = 0;
  // (ARKCOS_GRAD_HALF=0 keeps every FFT row on the S-pass form, so that
  // tests compare the two)
  const char* he = getenv("ARKCOS_GRAD_HALF");
  const bool half_off = he && *he == '0';
  const int64_t rsz = P->dtype == ARKCOS_F32 ? 4 : 8;
  const int64_t chunk = kGradZBytes / rsz;
  for (int64_t u = 0; u < P->n_units; ++u) {
    const UnitDev& U = P->h_units[u];
    double narrow = 0.0;
    for (int32_t q = U.pbeg; q < U.pend; ++q) {
      const PairDev& pr = P->h_pairs[q];
      const int64_t nc = P->h_ncoef_window[q];
      if (pr.band >= 0 && nc <= kGradMaxCoef) narrow += (double)kGradMaxCoef * (pr.band + 1) + 1000.0;
    }
    if (narrow > 0.0) {
      items.push_back(GradItem{(int32_t)u, -1, 0, 0, 0, 0});
      cost.push_back(narrow);
    }
    for (int32_t q = U.pbeg; q < U.pend; ++q) {
      const PairDev& pr = P->h_pairs[q];
      const int64_t nc = P->h_ncoef_window[q];
      if (pr.band < 0 || nc <= kGradMaxCoef) continue;
      if (const int32_t Pn = fft_row_points(P, q, nc); Pn > 0) {
        // the half-length cosine sum (one pass of G / 4 points) wherever it
        // fits one workgroup, else S passes of Pn points.  Its odd samples
        // are a running sum of first differences, whose rounding errors add
        // up along the row: FP32 rows take it only up to kHalfMaxSamplesF32
        // samples (within about six times the S-pass rounding there).
        const int64_t G = pr.grid;
        const bool short_enough = P->dtype == ARKCOS_F64 || nc <= kHalfMaxSamplesF32;
        if (!half_off && short_enough && G / 4 <= fft_row_max_points(P) && nc <= G / 2 + 1)
          fft_rows.push_back(RowFft{(int32_t)u, q, (int32_t)(G / 4), 1});
        else
          fft_rows.push_back(RowFft{(int32_t)u, q, Pn, 0});
        continue;
      }
      const int64_t nm = pr.band + 1;
      for (int64_t m0 = 0; m0 < nm; m0 += chunk) {
        const int64_t len = std::min(chunk, nm - m0);
        zmax = std::max<int64_t>(zmax, len);
        int64_t per = (int64_t)(kGradItemWork / (double)len) / kGradPass * kGradPass;
        per = std::max<int64_t>(per, kGradPass);
        for (int64_t d0 = 0; d0 < nc; d0 += per) {
          const int64_t cnt = std::min(per, nc - d0);
          items.push_back(GradItem{(int32_t)u, q, (int32_t)d0, (int32_t)cnt, (int32_t)m0, (int32_t)(m0 + len)});
          cost.push_back((double)(cnt + 8) * len + 4000.0);
        }
      }
    }
  }
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device));
  const int64_t nruns =
      std::max<int64_t>(1, std::min<int64_t>((int64_t)items.size(), 8 * kGradBlocksPerCU * (int64_t)cus));
  double total = 0.0;
  for (double c : cost) total += c;
  std::vector<int32_t> run(nruns + 1, (int32_t)items.size());
  run[0] = 0;
  double acc = 0.0;
  int64_t r = 1;
  for (size_t k = 0; k < items.size() && r < nruns; ++k) {
    acc += cost[k];
    while (r < nruns && acc >= total * (double)r / (double)nruns) run[r++] = (int32_t)(k + 1);
  }
  P->h_grad_items = items;
  P->n_grad_runs = (int32_t)nruns;
  // FFT rows: Y(d) of each row at an offset in its chunk's buffer (chunks
  // of at most kGradYBytes), and the persistent blocks of the interval sums,
  // each with its own slot
  group_fft_rows(fft_rows, P->n_gfft);
  {
    // (ARKCOS_GRAD_CHUNK_BYTES sets a smaller chunk budget, so that tests
    // reach the chunked path on small plans)
    int64_t budget = kGradYBytes;
    if (const char* e = getenv("ARKCOS_GRAD_CHUNK_BYTES"); e && *e) budget = std::max<int64_t>(atoll(e), 1);
    std::vector<int64_t> yoff(fft_rows.size());
    P->h_gfft_chunk.assign(1, 0);
    P->grad_y_elems = 0;
    int64_t used = 0;
    for (size_t k = 0; k < fft_rows.size(); ++k) {
      const int64_t nc = P->h_ncoef_window[fft_rows[k].pair];
      if (used > 0 && (used + nc) * rsz > budget) {
        P->h_gfft_chunk.push_back((int32_t)k);
        used = 0;
      }
      yoff[k] = used;
      used += nc;
      P->grad_y_elems = std::max(P->grad_y_elems, used);
    }
    P->h_gfft_chunk.push_back((int32_t)fft_rows.size());
    HIPCHK(upload(P, &P->d_gfft_yoff, yoff));
  }
  P->n_gfft_slots = std::min<int32_t>((int32_t)fft_rows.size(), 4 * cus);
  HIPCHK(upload(P, &P->d_gfft, fft_rows));
  // a wide-row item's correlation (one mode chunk) is staged in LDS
  P->grad_zcache_bytes = (int32_t)((std::max<int64_t>(zmax, 1) * rsz + 15) / 16 * 16);
  HIPCHK(upload(P, &P->d_grad_items, items));
  HIPCHK(upload(P, &P->d_grad_run, run));
  return ARKCOS_OK;
}

// Kernel samples, bands and tables from the profile, at plan creation.
// Spline plans keep every kernel sample of a pair's window and every mode
// up to the grid's Nyquist mode (no band truncation), so that the layout
// fixed here holds for any later knot values (update_knots).
arkcos_status_t build_kernel_tables(arkcos_plan_s* P) {
  const bool spline = P->prof_kind == 1;
  hipStream_t s = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  struct Guard { hipStream_t s; ~Guard() { hipStreamDestroy(s); } } guard{s};

  const int64_t np = P->n_pairs;
  double* d_abs = nullptr;
  int32_t* d_band = nullptr;
  std::vector<double> abs_sum(np);
  std::vector<int32_t> band(np);
  if (np > 0) {
    HIPCHK(hipMalloc(&d_abs, np * sizeof(double)));
    HIPCHK(hipMalloc(&d_band, np * sizeof(int32_t)));
  }
  struct Free { void* a; void* b; ~Free() { if (a) hipFree(a); if (b) hipFree(b); } } fr{d_abs, d_band};

  // kernel samples over each pair's full window, indexed by coefficient
  // offsets: until the table choices below, a pair's off is its sample
  // offset (the band kernel reads the samples through it)
  for (int64_t q = 0; q < np; ++q) P->h_pairs[q].off = P->h_coef_off[q];
  HIPCHK(hipMemcpy(P->d_pairs, P->h_pairs.data(), np * sizeof(PairDev), hipMemcpyHostToDevice));
  HIPCHK(launch_kernel_rows(P, d_abs, s));
  HIPCHK(hipStreamSynchronize(s));
  if (np > 0) HIPCHK(hipMemcpy(abs_sum.data(), d_abs, np * sizeof(double), hipMemcpyDeviceToHost));

  double scale = 0.0;
  for (double v : abs_sum) scale = std::max(scale, v);
  // drop trailing samples whose magnitudes sum to at most a tenth of the band
  // tolerance: |K_ij(m)| then changes by less than 0.1 band_tol times the
  // largest kernel-row magnitude at every m, so the row is not cut off with a
  // step that would widen its spectrum
  if (np > 0 && !spline) {
    std::vector<double> c64(P->coef_total);
    HIPCHK(hipMemcpy(c64.data(), P->d_coef64, P->coef_total * sizeof(double), hipMemcpyDeviceToHost));
    const double cut = 0.1 * P->band_tol * scale;
    for (int64_t q = 0; q < np; ++q) {
      int32_t n = P->h_ncoef_window[q];
      const double* a = c64.data() + P->h_coef_off[q];
      double dropped = 0.0;
      while (n > 1 && dropped + fabs(a[n - 1]) <= cut) dropped += fabs(a[--n]);
      P->h_pairs[q].ncoef = n;
    }
    HIPCHK(hipMemcpy(P->d_pairs, P->h_pairs.data(), np * sizeof(PairDev), hipMemcpyHostToDevice));
  }
  if (P->band_tol > 0 && np > 0 && !spline) {
    HIPCHK(launch_band(P, P->band_tol * scale, d_band, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(band.data(), d_band, np * sizeof(int32_t), hipMemcpyDeviceToHost));
  } else {
    for (int64_t q = 0; q < np; ++q) band[q] = (spline || abs_sum[q] > 0) ? P->h_pairs[q].nyq : -1;
  }
  if (P->opts.mode == 1) {
    // the plain mode of Sect. 4.1: input spectra zero-padded past N_j / 2
    // and output coefficients truncated at N_i / 2, i.e. a pair contributes
    // only its modes m <= min(N_i, N_j) / 2 (both rings of a mirrored pair
    // have the lengths of the northern one)
    for (int64_t q = 0; q < np; ++q) {
      const int32_t top = (int32_t)(std::min(P->h_n[P->h_pair_i[q]], P->h_n[P->h_pairs[q].j]) / 2);
      band[q] = std::min(band[q], top);
    }
  }

  // A table pair reads the table of its transpose when that one exists:
  // K_ji(m) = K_ij(m) if rings i and j have equal pixel weights and the two
  // pairs have the same grid, shift and band (the kernel depends only on the
  // angular distance, and the grid is symmetric under a change of sign of
  // the longitude offset).  (j, i) is a pair of the unit of ring j or, for a
  // southern ring j, the mirror image (mirror j, mirror i) in the unit of
  // mirror j.  Halves the tables on HEALPix grids (and counts once towards
  // the automatic choice's budget).
  std::vector<int64_t> unit_of(P->nrings, -1);
  for (int64_t u = 0; u < P->n_units; ++u) unit_of[P->h_units[u].i] = u;
  auto transpose = [&](int64_t q) -> int64_t {
    const int64_t nr = P->nrings;
    int64_t i = P->h_pair_i[q], j = P->h_pairs[q].j;
    if (j > nr - 1 - j) {
      j = nr - 1 - j;
      i = nr - 1 - i;
    }
    const int64_t u = unit_of[j];
    if (u < 0) return -1;
    const PairDev* b = P->h_pairs.data() + P->h_units[u].pbeg;
    const PairDev* e = P->h_pairs.data() + P->h_units[u].pend;
    const PairDev* f = std::lower_bound(b, e, (int32_t)i, [](const PairDev& x, int32_t v) { return x.j < v; });
    return (f != e && f->j == i) ? (int64_t)(f - P->h_pairs.data()) : -1;
  };
  auto compatible = [&](int64_t t, int64_t q) {
    const PairDev &o = P->h_pairs[t], &pr = P->h_pairs[q];
    return band[t] == band[q] && o.grid == pr.grid && o.nyq == pr.nyq && P->h_pair_shift[t] == P->h_pair_shift[q] &&
           P->h_w[P->h_pair_i[q]] == P->h_w[pr.j];
  };
  // table selection and offsets: automatic choice = tables for every pair if
  // they fit in kAutoTableBytes (the accumulation then only streams them), or
  // if the rows too wide for the recurrence, whose tables are built anyway,
  // already hold at least kAutoTableShare of them; otherwise tables only for
  // those wide rows
  bool all_auto = false;
  if (P->opts.kgen == 0) {
    int64_t entries = 0, wide = 0;
    for (int64_t q = 0; q < np; ++q) {
      if (band[q] < 0) continue;
      const int64_t t = transpose(q);
      if (!(t >= 0 && t < q && compatible(t, q))) {
        entries += table_span(band[q]);
        if (P->h_pairs[q].ncoef > kOtfMaxCoef) wide += table_span(band[q]);
      }
    }
    all_auto = entries * (int64_t)(P->dtype == ARKCOS_F32 ? 4 : 8) <= kAutoTableBytes ||
               (double)wide >= kAutoTableShare * (double)entries;
  }
  int64_t table_total = 0, ntab = 0;
  std::vector<int32_t> tab_list;
  std::vector<int64_t> tab_coef;
  std::vector<RowFft> tab_fft;  // wide spline rows whose tables come from FFTs
  P->h_tab_owner.assign(np, -1);
  for (int64_t q = 0; q < np; ++q) {
    PairDev& pr = P->h_pairs[q];
    pr.band = band[q];
    bool table = false;
    if (pr.band >= 0) {
      if (P->opts.kgen == 2 || all_auto) table = true;
      else if (P->opts.kgen == 0) table = pr.ncoef > kOtfMaxCoef;
    }
    if (table) {
      P->h_tab_owner[q] = q;
      const int64_t t = transpose(q);
      if (t >= 0 && t < q && P->h_pairs[t].kind == KG_TABLE && compatible(t, q))
        P->h_tab_owner[q] = P->h_tab_owner[t];
    }
    if (table && P->h_tab_owner[q] != q) {
      pr.kind = KG_TABLE;
      pr.off = P->h_pairs[P->h_tab_owner[q]].off;
      ++ntab;
    } else if (table) {
      pr.kind = KG_TABLE;
      pr.off = table_total;
      table_total += table_span(pr.band);
      if (const int32_t Pn = fft_row_points(P, q, pr.ncoef); Pn > 0) {
        tab_fft.push_back(RowFft{-1, (int32_t)q, Pn, 0});
      } else {
        tab_list.push_back((int32_t)q);
        tab_coef.push_back(P->h_coef_off[q]);
      }
      ++ntab;
    } else {
      pr.kind = P->h_pair_shift[q] ? KG_SHIFTED : (pr.ncoef > kClenshawMaxCoef ? KG_REINSCH : KG_CENTRED);
      pr.off = P->h_coef_off[q];
    }
  }
  // the accumulation addresses samples and tables with 32-bit offsets
  if (table_total >= (int64_t(1) << 32) ||
      (P->coef_total + 16) * (int64_t)(P->dtype == ARKCOS_F32 ? 4 : 8) >= (int64_t(1) << 31))
    return fail(ARKCOS_ERR_NOT_SUPPORTED, "kernel samples beyond 2 GiB or tables beyond 2^32 elements");
  P->n_table_pairs = ntab;
  P->table_total = table_total;
  {
    bool all = true;
    for (int64_t q = 0; q < np && all; ++q)
      if (P->h_pairs[q].band >= 0 && P->h_pairs[q].kind != KG_TABLE) all = false;
    P->all_tables = all && ntab > 0;
  }
  const size_t rsz = P->dtype == ARKCOS_F32 ? sizeof(float) : sizeof(double);
  {
    void* t = nullptr;
    HIPCHK(hipMalloc(&t, std::max<int64_t>(table_total, 1) * rsz));
    P->allocations.push_back(t);
    P->plan_bytes += std::max<int64_t>(table_total, 1) * rsz;
    P->d_table = t;
  }
  HIPCHK(hipMemcpy(P->d_pairs, P->h_pairs.data(), np * sizeof(PairDev), hipMemcpyHostToDevice));
  // the pairs whose tables are computed (shared ones once), kept for knot updates
  P->n_tab_list = (int32_t)tab_list.size();
  HIPCHK(upload(P, &P->d_tab_list, tab_list));
  HIPCHK(upload(P, &P->d_tab_coef, tab_coef));
  group_fft_rows(tab_fft, P->n_tfft);
  HIPCHK(upload(P, &P->d_tfft, tab_fft));
  HIPCHK(launch_table_list(P, P->d_tab_list, P->d_tab_coef, P->n_tab_list, s));
  HIPCHK(launch_table_fft(P, s));
  HIPCHK(hipStreamSynchronize(s));
  return ARKCOS_OK;
}

// New spline knots (device array of n_knots doubles) applied on stream s:
// moments, kernel samples and K_ij(m) tables recomputed in place with the
// layout of plan creation.  Enqueues kernels only (no allocation, no host
// synchronisation), so it can be captured in a graph.
hipError_t update_knots(arkcos_plan_s* P, const double* d_src, hipStream_t s) {
  hipError_t e = launch_spline_update(P, d_src, s);
  if (e != hipSuccess) return e;
  e = launch_kernel_rows(P, nullptr, s);
  if (e != hipSuccess) return e;
  e = launch_table_list(P, P->d_tab_list, P->d_tab_coef, P->n_tab_list, s);
  if (e != hipSuccess) return e;
  return launch_table_fft(P, s);
}

// Bands of units_per_band units and their items (mode tiles in runs of
// tiles), heaviest first so that a launch does not end on a long item.
static void make_bands_items(const arkcos_plan_s* P, int32_t units, int32_t tiles, std::vector<BandDev>& bands,
                             AccShape* shape, std::vector<WorkItem>& items) {
  build_bands(P, units, bands, shape);
  std::vector<WorkItem> its;
  std::vector<double> cost;
  accumulation_items(P, bands, tiles, its, cost);
  std::vector<size_t> ord(its.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  items.clear();
  for (size_t k : ord) items.push_back(its[k]);
}

// The accumulation's band shape: units per band (8 or 16 wavefronts per
// block; wider bands re-read the window's spectra less often but hold fewer
// waves per CU) and mode tiles per item.  Plans of a million pixels or more
// time every candidate on a scratch workspace (the kernel's control flow
// does not depend on the data) and keep the fastest; smaller plans take 8
// units and 4 tiles.  ARKCOS_ACC_SHAPE="U,T[,W[,C]]" forces a choice.  The result
// does not depend on the shape: every unit sums its pairs in the same order.
arkcos_status_t choose_accumulation_shape(arkcos_plan_s* P) {
  struct Cand {
    int32_t units, tiles, upw;  // units per band, mode tiles per item, units per wavefront
    int32_t ch = 0;             // input rings staged at a time (0: the default)
  };
  std::vector<Cand> cand;
  if (const char* e = getenv("ARKCOS_ACC_SHAPE"); e && *e) {
    int u = 0, t = 0, w = 1, ch = 0;
    const int got = sscanf(e, "%d,%d,%d,%d", &u, &t, &w, &ch);
    const bool per_wave = got >= 3 && w >= 2 && w <= 3 && u == 8 * w && P->all_tables && P->dtype == ARKCOS_F32;
    if (got >= 2 && (u == 8 || u == 16 || per_wave) && t >= 1 && t <= 16)
      cand.push_back({u, t, per_wave ? w : 1, (per_wave && w == 2 && got == 4 && ch == 16) ? 16 : 0});
  }
  if (cand.empty()) {
    // (16-unit bands only in FP32: the FP64 recurrence form would spill;
    // two units per wavefront only for table-only FP32 plans)
    if (P->npix >= (int64_t(1) << 20) && P->dtype == ARKCOS_F32) {
      cand = {{8, 4, 1}, {16, 4, 1}, {8, 2, 1}, {16, 2, 1}, {8, 8, 1}, {16, 8, 1}};
      if (P->all_tables)
        cand.insert(cand.end(), {{16, 4, 2}, {16, 2, 2}, {24, 2, 3}, {16, 4, 2, 16}, {16, 2, 2, 16}});
    } else if (P->npix >= (int64_t(1) << 20)) {
      cand = {{8, 4, 1}, {8, 2, 1}, {8, 8, 1}};
    } else {
      cand = {{kBandUnits, kTilesPerItem, 1}};
    }
  }
  P->acc_tuned = 0;
  if (cand.size() == 1) {
    P->acc_units = cand[0].units;
    P->acc_tiles = cand[0].tiles;
    P->acc_upw = cand[0].upw;
    P->acc_ch = cand[0].ch;
    make_bands_items(P, P->acc_units, P->acc_tiles, P->h_bands, &P->acc_shape, P->h_items);
    return ARKCOS_OK;
  }
  void *ws = nullptr, *d_b = nullptr, *d_i = nullptr;
  struct Free {
    void** a[3];
    ~Free() { for (void** p : a) if (*p) hipFree(*p); }
  } fr{{&ws, &d_b, &d_i}};
  const size_t wsb = workspace_bytes(P);
  HIPCHK(hipMalloc(&ws, wsb));
  HIPCHK(hipMemset(ws, 0, wsb));
  void *spec = nullptr, *bout = nullptr;
  workspace_split(P, ws, &spec, &bout);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() { hipEventDestroy(a); hipEventDestroy(b); }
  } ev{e0, e1};
  float best = 1e30f;
  size_t best_k = 0;
  for (size_t k = 0; k < cand.size(); ++k) {
    std::vector<BandDev> bands;
    std::vector<WorkItem> items;
    AccShape sh;
    make_bands_items(P, cand[k].units, cand[k].tiles, bands, &sh, items);
    if (d_b) HIPCHK(hipFree(d_b));
    if (d_i) HIPCHK(hipFree(d_i));
    d_b = d_i = nullptr;
    HIPCHK(hipMalloc(&d_b, std::max<size_t>(bands.size(), 1) * sizeof(BandDev)));
    HIPCHK(hipMalloc(&d_i, std::max<size_t>(items.size(), 1) * sizeof(WorkItem)));
    if (!bands.empty()) HIPCHK(hipMemcpy(d_b, bands.data(), bands.size() * sizeof(BandDev), hipMemcpyHostToDevice));
    if (!items.empty()) HIPCHK(hipMemcpy(d_i, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    HIPCHK(configure_accumulate_shape(P, sh));
    const int32_t ni = (int32_t)items.size();
    HIPCHK(launch_accumulate_shape(P, (BandDev*)d_b, (WorkItem*)d_i, ni, cand[k].units, sh, spec, bout, nullptr,
                                   cand[k].upw, cand[k].ch));
    HIPCHK(hipEventRecord(e0, nullptr));
    for (int r = 0; r < 3; ++r)
      HIPCHK(launch_accumulate_shape(P, (BandDev*)d_b, (WorkItem*)d_i, ni, cand[k].units, sh, spec, bout, nullptr,
                                     cand[k].upw, cand[k].ch));
    HIPCHK(hipEventRecord(e1, nullptr));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (const char* e = getenv("ARKCOS_ACC_TIMES"); e && *e == '1')
      fprintf(stderr, "arkcos plan: accumulation candidate %d units, %d tiles, %d per wave, %d rings staged: %.4f ms\n",
              cand[k].units, cand[k].tiles, cand[k].upw, cand[k].ch, ms / 3.0f);
    if (ms < best) {
      best = ms;
      best_k = k;
    }
  }
  P->acc_units = cand[best_k].units;
  P->acc_tiles = cand[best_k].tiles;
  P->acc_upw = cand[best_k].upw;
  P->acc_ch = cand[best_k].ch;
  P->acc_tuned = 1;
  make_bands_items(P, P->acc_units, P->acc_tiles, P->h_bands, &P->acc_shape, P->h_items);
  return ARKCOS_OK;
}

arkcos_status_t build_plan(const arkcos_geometry_t* g, const arkcos_profile_t* prof, double R,
                           arkcos_dtype_t dtype, const arkcos_options_t* o, arkcos_plan_s** out) {
  // ---------------------------------------------------------- validation
  if (!g || !prof || !out) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (dtype != ARKCOS_F32 && dtype != ARKCOS_F64) return fail(ARKCOS_ERR_INVALID_VALUE, "bad dtype");
  if (!(R > 0) || !(R < M_PI)) return fail(ARKCOS_ERR_INVALID_VALUE, "support radius must be in (0, pi)");
  arkcos_options_t opts;
  arkcos_default_options(&opts);
  if (o) opts = *o;
  if (opts.oversample != 0 && !(is_pow2(opts.oversample) && opts.oversample <= 16))
    return fail(ARKCOS_ERR_INVALID_VALUE, "oversample must be 0, 1, 2, 4, 8 or 16");
  if (opts.kgen < 0 || opts.kgen > 2) return fail(ARKCOS_ERR_INVALID_VALUE, "kgen must be 0, 1 or 2");
  if (opts.mode < 0 || opts.mode > 1) return fail(ARKCOS_ERR_INVALID_VALUE, "mode must be 0 or 1");
  if (opts.own_grid < 0 || opts.own_grid > 1) return fail(ARKCOS_ERR_INVALID_VALUE, "own_grid must be 0 or 1");
  if (opts.kernel_eval < 0 || opts.kernel_eval > 1)
    return fail(ARKCOS_ERR_INVALID_VALUE, "kernel_eval must be 0 or 1");
  if (opts.table_nodes != 0 && (opts.table_nodes < 2 || opts.table_nodes > (1 << 24)))
    return fail(ARKCOS_ERR_INVALID_VALUE, "table_nodes must be 0 or in 2 .. 2^24");
  for (int32_t r : opts.reserved)
    if (r != 0) return fail(ARKCOS_ERR_INVALID_VALUE, "reserved option fields must be 0");
  if (g->kind == 0) {
    if (g->n_theta < 1 || g->n_phi < 4 || (g->n_phi & 1) || g->n_theta > (1 << 20) || g->n_phi > (1 << 20))
      return fail(ARKCOS_ERR_INVALID_VALUE, "ECP needs n_theta >= 1 and an even n_phi >= 4");
  } else if (g->kind == 1) {
    if (g->nside < 1 || g->nside > 8192) return fail(ARKCOS_ERR_INVALID_VALUE, "nside must be in 1 .. 8192");
  } else {
    return fail(ARKCOS_ERR_INVALID_VALUE, "geometry kind must be 0 (ECP) or 1 (HEALPix)");
  }
  if (prof->kind == 0) {
    if (!(prof->fwhm_rad > 0)) return fail(ARKCOS_ERR_INVALID_VALUE, "Gaussian FWHM must be > 0");
  } else if (prof->kind == 1) {
    if (prof->n_knots < 3 || prof->n_knots > 64 || !(prof->theta_max_rad > 0) || !prof->knot_values)
      return fail(ARKCOS_ERR_INVALID_VALUE, "spline needs 3..64 knots, theta_max > 0 and knot values");
  } else {
    return fail(ARKCOS_ERR_INVALID_VALUE, "profile kind must be 0 (Gaussian) or 1 (spline)");
  }

  auto* P = new arkcos_plan_s();
  struct Owner {
    arkcos_plan_s* p;
    ~Owner() {
      if (p) {
        for (void* a : p->allocations) hipFree(a);
        delete p;
      }
    }
  } owner{P};
  HIPCHK(hipGetDevice(&P->device));
  P->dtype = dtype;
  P->geom = *g;
  P->prof_kind = prof->kind;
  P->fwhm = prof->fwhm_rad;
  P->theta_max = prof->theta_max_rad;
  if (prof->kind == 1) P->knots.assign(prof->knot_values, prof->knot_values + prof->n_knots);
  P->radius = R;
  P->opts = opts;
  P->band_tol = opts.band_tol >= 0 ? opts.band_tol : (dtype == ARKCOS_F32 ? 1e-9 : 0.0);

  // ------------------------------------------------------------ geometry
  int64_t nr, npix, L;
  if (g->kind == 1) {
    const int64_t ns = g->nside;
    nr = 4 * ns - 1;
    npix = 12 * ns * ns;
    L = 4 * ns;
  } else {
    nr = g->n_theta;
    npix = g->n_theta * g->n_phi;
    L = g->n_phi;
  }
  P->nrings = nr;
  P->npix = npix;
  P->L = L;
  P->h_theta.resize(nr); P->h_sin.resize(nr); P->h_cos.resize(nr); P->h_w.resize(nr);
  P->h_n.resize(nr); P->h_phase_den.resize(nr); P->h_start.resize(nr);
  if (g->kind == 1) {
    const int64_t ns = g->nside;
    const double area = 4.0 * M_PI / (double)npix;
    for (int64_t k = 0; k < nr; ++k) {
      const int64_t r = k + 1;
      double th;
      if (r < ns) {
        th = 2.0 * asin(r / (sqrt(6.0) * ns));
        P->h_n[k] = (int32_t)(4 * r);
        P->h_phase_den[k] = (int32_t)(4 * r);
        P->h_start[k] = 2 * r * (r - 1);
      } else if (r <= 3 * ns) {
        th = acos(4.0 / 3.0 - 2.0 * r / (3.0 * ns));
        P->h_n[k] = (int32_t)(4 * ns);
        P->h_phase_den[k] = ((r - ns) % 2 == 0) ? (int32_t)(4 * ns) : 0;
        P->h_start[k] = 2 * ns * (ns - 1) + 4 * ns * (r - ns);
      } else {
        const int64_t sr = 4 * ns - r;
        th = M_PI - 2.0 * asin(sr / (sqrt(6.0) * ns));
        P->h_n[k] = (int32_t)(4 * sr);
        P->h_phase_den[k] = (int32_t)(4 * sr);
        P->h_start[k] = npix - 2 * sr * (sr + 1);
      }
      P->h_theta[k] = th;
      P->h_w[k] = area;
    }
  } else {
    const int64_t nt = g->n_theta, nphi = g->n_phi;
    for (int64_t i = 0; i < nt; ++i) {
      double a = M_PI * i / nt, b = M_PI * (i + 1) / nt;
      P->h_theta[i] = M_PI * (i + 0.5) / nt;
      P->h_w[i] = (2.0 * M_PI / nphi) * 2.0 * sin(0.5 * (a + b)) * sin(0.5 * (b - a));
      P->h_n[i] = (int32_t)nphi;
      P->h_phase_den[i] = 0;
      P->h_start[i] = i * nphi;
    }
  }
  for (int64_t k = 0; k < nr; ++k) {
    // the ring transforms take every longitude offset to be pi / N
    if (P->h_phase_den[k] != 0 && P->h_phase_den[k] != P->h_n[k])
      return fail(ARKCOS_ERR_INTERNAL, "ring offset other than pi / N");
    P->h_sin[k] = sin(P->h_theta[k]);
    P->h_cos[k] = cos(P->h_theta[k]);
  }

  // ------------------------------------------------------- oversampling
  int32_t p = opts.oversample;
  if (g->kind == 0) {
    p = 1;  // every ECP ring pair is aligned and exact
  } else if (p == 0) {
    const double pix = sqrt(4.0 * M_PI / (double)npix);
    double width = prof->kind == 0 ? prof->fwhm_rad : 2.0 * prof->theta_max_rad / (prof->n_knots - 1);
    int64_t need = (int64_t)ceil(4.3 * pix / width);
    p = (int32_t)std::min<int64_t>(16, std::max<int64_t>(1, next_pow2(need)));
  }
  P->oversample = p;

  // ------------------------------------------------------ units, pairs
  const int64_t nunits = (nr + 1) / 2;
  const double rt = R + kSupportTol;
  const double hav_r = sin(0.5 * rt) * sin(0.5 * rt);
  P->h_units.resize(nunits);
  for (int64_t u = 0; u < nunits; ++u) {
    const int64_t i = u, im = nr - 1 - u;
    UnitDev& U = P->h_units[u];
    U.i = (int32_t)i;
    U.im = im != i ? (int32_t)im : -1;
    U.pbeg = (int32_t)P->h_pairs.size();
    for (int64_t j = 0; j < nr; ++j) {
      const double dth = P->h_theta[i] - P->h_theta[j];
      if (fabs(dth) > rt) continue;
      PairDev pr{};
      pr.j = (int32_t)j;
      // rings of equal length (with offsets 0 or pi/N) are sampled at their
      // true pixel offsets on a grid of their own length: exact (Sect. 4.3;
      // the plain mode of Sect. 4.1 puts every pair on the p L grid).  With
      // own_grid = 1 only equatorial pairs (rings of L pixels) do so, as
      // Sect. 4.3 states it; a polar ring with itself or its mirror then
      // takes the p L grid like the other cap pairs.
      const bool aligned = opts.mode == 0 && P->h_n[i] == P->h_n[j] &&
                           (opts.own_grid == 0 || P->h_n[i] == L) &&
                           (P->h_phase_den[i] == 0 || P->h_phase_den[i] == P->h_n[i]) &&
                           (P->h_phase_den[j] == 0 || P->h_phase_den[j] == P->h_n[j]);
      int32_t shift = 0;
      int64_t G = (int64_t)p * L;
      if (aligned) {
        G = P->h_n[i];
        shift = ((P->h_phase_den[i] != 0) != (P->h_phase_den[j] != 0)) ? 1 : 0;
      }
      pr.grid = (int32_t)G;
      pr.nyq = (int32_t)(G / 2);
      // kernel-sample window from hav(R) >= sin^2(dtheta/2) + sin_i sin_j sin^2(nu/2)
      const double sa = sin(0.5 * dth);
      const double den = P->h_sin[i] * P->h_sin[j];
      const double qv = den > 0 ? (hav_r - sa * sa) / den : 2.0;
      const int64_t pl = G;
      const double hstep = 2.0 * M_PI / (double)pl;
      int64_t ncoef;
      if (qv >= 1.0) {
        ncoef = shift ? pl / 2 : pl / 2 + 1;
      } else {
        const double numax = 2.0 * asin(sqrt(std::max(qv, 0.0)));
        if (shift)
          ncoef = std::min<int64_t>(pl / 2, (int64_t)floor(numax / hstep - 0.5) + 2);
        else
          ncoef = std::min<int64_t>(pl / 2 + 1, (int64_t)floor(numax / hstep) + 2);
        ncoef = std::max<int64_t>(ncoef, 1);
      }
      pr.ncoef = (int32_t)ncoef;
      P->h_ncoef_window.push_back((int32_t)ncoef);
      P->h_coef_off.push_back(P->coef_total);
      P->coef_total += (ncoef + 7) / 8 * 8;  // rows padded with zeros to whole 8-sample chunks
      P->h_pairs.push_back(pr);
      P->h_pair_i.push_back((int32_t)i);
      P->h_pair_shift.push_back(shift);
    }
    U.pend = (int32_t)P->h_pairs.size();
    P->max_units_pairs = std::max(P->max_units_pairs, U.pend - U.pbeg);
  }
  P->n_units = nunits;
  P->n_pairs = (int64_t)P->h_pairs.size();

  // ------------------------------------------------------ FFT strategies
  // LDS FFTs of up to 16384 (FP32) or 8192 (FP64) complex points: 135 KB
  // of the CU's 160 KB, one 1024- or 512-thread block per ring (nside 4096
  // in FP32, 2048 in FP64)
  const int64_t maxM = dtype == ARKCOS_F32 ? 16384 : 8192;
  const size_t csz = dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  const size_t rsz = dtype == ARKCOS_F32 ? sizeof(float) : sizeof(double);
  std::vector<int32_t> fft_kind(nr), fft_m(nr);
  std::vector<int64_t> bl_off(nr, 0);
  std::map<int32_t, int64_t> bl_of_len;
  std::vector<int32_t> bl_rings;
  std::vector<size_t> ring_lds(nr, 0);
  int64_t twn = 4;
  size_t lds = 0;
  // Rings whose half length has no prime factor above 7 take the
  // mixed-radix transform when they fill launches of their own: at least
  // kMixedMinRings of them share a launch class (LDS bucket), or every
  // non-power-of-two ring of the plan qualifies (ECP grids, HEALPix belts of
  // such a length).  Scattered lengths (HEALPix polar rings: two rings per
  // length) stay with Bluestein, whose launches they share; in classes of
  // their own they ran as small, tail-bound launches (nside 2048 forward
  // 0.81 -> 0.89 ms).
  auto smooth7 = [](int64_t v) {
    for (int64_t f : {2, 3, 5, 7})
      while (v % f == 0) v /= f;
    return v == 1;
  };
  auto mixed_ok = [&](int64_t N) {
    const int64_t n = N / 2;
    return N > kDirectMax && !is_pow2(n) && smooth7(n) && n <= maxM;
  };
  auto lds_bucket = [&](int64_t n) {
    size_t b = 32768;
    while (b < (size_t)lds_elems((int)n) * csz) b <<= 1;
    return b;
  };
  std::map<size_t, int64_t> mixed_per_bucket;
  int64_t n_mixed_ok = 0, n_not_pow2 = 0;
  for (int64_t k = 0; k < nr; ++k) {
    const int64_t N = P->h_n[k];
    if (N > kDirectMax && !is_pow2(N / 2)) ++n_not_pow2;
    if (mixed_ok(N)) {
      ++mixed_per_bucket[lds_bucket(N / 2)];
      ++n_mixed_ok;
    }
  }
  constexpr int64_t kMixedMinRings = 1024;
  const bool all_mixed = n_mixed_ok == n_not_pow2;
  for (int64_t k = 0; k < nr; ++k) {
    const int64_t N = P->h_n[k];
    if (N <= kDirectMax) {
      fft_kind[k] = FFT_DIRECT;
      fft_m[k] = 0;
      ring_lds[k] = (size_t)(lds_elems((int)(N / 2)) + N) * csz + N * rsz;
      lds = std::max(lds, ring_lds[k]);
      continue;
    }
    const int64_t n = N / 2;
    if (mixed_ok(N) && (all_mixed || mixed_per_bucket[lds_bucket(n)] >= kMixedMinRings)) {
      // a mixed-radix transform of the ring's own length (no Bluestein)
      fft_kind[k] = FFT_MIXED;
      fft_m[k] = (int32_t)n;
      ring_lds[k] = (size_t)lds_elems((int)n) * csz;
      lds = std::max(lds, ring_lds[k]);
    } else if (is_pow2(n)) {
      if (n > maxM) return fail(ARKCOS_ERR_NOT_SUPPORTED, "ring FFT longer than the LDS limit");
      fft_kind[k] = FFT_POW2;
      fft_m[k] = (int32_t)n;
      twn = std::max(twn, 2 * N);  // w_r = exp(-i pi r / N) read from the table
      ring_lds[k] = (size_t)lds_elems((int)n) * csz;
      lds = std::max(lds, ring_lds[k]);
    } else {
      const int64_t M = next_pow2(2 * n - 1);
      if (M > maxM) return fail(ARKCOS_ERR_NOT_SUPPORTED, "Bluestein FFT longer than the LDS limit");
      fft_kind[k] = FFT_BLUESTEIN;
      fft_m[k] = (int32_t)M;
      twn = std::max(twn, M);
      ring_lds[k] = (size_t)lds_elems((int)M) * csz;
      lds = std::max(lds, ring_lds[k]);
      auto it = bl_of_len.find((int32_t)N);
      if (it == bl_of_len.end()) {
        bl_of_len[(int32_t)N] = P->bl_total;
        bl_off[k] = P->bl_total;
        P->bl_total += M + n + n / 2 + 1;  // filter, chirp, half-angle phases
        bl_rings.push_back((int32_t)k);
        P->max_bl_m = std::max<int32_t>(P->max_bl_m, (int32_t)M);
      } else {
        bl_off[k] = it->second;
      }
    }
  }
  // the accumulation reads exp(i pi m / (p L)) from the table as well
  if (is_pow2((int64_t)P->oversample * L)) twn = std::max<int64_t>(twn, 2 * (int64_t)P->oversample * L);
  // a short ring's fold shares its period sums through 4 kFoldThreads values of LDS
  for (int64_t k = 0; k < nr; ++k) ring_lds[k] = std::max(ring_lds[k], (size_t)4 * kFoldThreads * csz);
  lds = std::max(lds, (size_t)4 * kFoldThreads * csz);
  P->twiddle_n = (int32_t)twn;
  P->max_fft_lds = (int32_t)((lds + 15) / 16 * 16);
  P->h_ring_lds.resize(nr);
  P->h_fft_len = fft_m;
  P->h_fft_kind = fft_kind;
  for (int64_t k = 0; k < nr; ++k) P->h_ring_lds[k] = (int32_t)((ring_lds[k] + 15) / 16 * 16);
  {
    // launch classes by LDS size: power-of-two buckets from 32 KiB, so that
    // the many small rings share one launch; within a class the longest
    // rings come first.  Workgroups go to the 8 XCDs round-robin, so each
    // run of 8 northern rings is followed by their 8 mirrors: a ring and its
    // mirror then run on the same XCD and share its L2 copy of their
    // Bluestein filter.
    // Rings whose FFT length has a compile-time kernel (ct_fft_length) get a
    // class of their own per length.
    std::map<size_t, std::vector<std::pair<int32_t, int32_t>>> pairs_of;
    std::vector<int64_t> order((nr + 1) / 2);
    for (int64_t k = 0; k < (int64_t)order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return P->h_n[x] > P->h_n[y]; });
    std::map<int32_t, int64_t> per_len;
    for (int64_t k = 0; k < nr; ++k) ++per_len[fft_m[k]];
    for (int64_t k : order) {
      size_t b = 32768;
      while (b < ring_lds[k]) b <<= 1;
      const int32_t ct = ct_fft_length(dtype, fft_m[k], per_len[fft_m[k]]);
      if (ct > 0) b = (size_t(1) << 40) + (size_t)ct;
      if (fft_kind[k] == FFT_MIXED) b |= size_t(1) << 39;  // mixed-radix rings: classes of their own
      pairs_of[b].push_back({(int32_t)k, nr - 1 - k != k ? (int32_t)(nr - 1 - k) : -1});
    }
    std::map<size_t, std::vector<int32_t>> cls;
    for (auto& [b, prs] : pairs_of) {
      std::vector<int32_t>& lst = cls[b];
      for (size_t c = 0; c < prs.size(); c += 8) {
        const size_t e = std::min(prs.size(), c + 8);
        for (size_t a = c; a < e; ++a) lst.push_back(prs[a].first);
        for (size_t a = c; a < e; ++a)
          if (prs[a].second >= 0) lst.push_back(prs[a].second);
      }
    }
    for (auto it = cls.rbegin(); it != cls.rend(); ++it) {
      FftClass c;
      c.count = (int32_t)it->second.size();
      size_t mx = 0;
      int32_t len = 0, lo = INT32_MAX;
      for (int32_t k : it->second) {
        mx = std::max(mx, ring_lds[k]);
        len = std::max(len, fft_m[k]);
        lo = std::min(lo, fft_m[k]);
      }
      c.lds = (int32_t)((mx + 15) / 16 * 16);
      c.mf = (lo == len) ? ct_fft_length(dtype, len, per_len[len]) : 0;
      if (it->first & (size_t(1) << 39)) c.mf = -1;
      c.threads = c.mf > 0 ? c.mf / 16 : fft_threads(dtype, len);
      HIPCHK(upload(P, &c.d_rings, it->second));
      P->fft_classes.push_back(c);
    }
  }

  // ------------------------------------------------------ device tables
  HIPCHK(upload(P, &P->rt.n, P->h_n));
  HIPCHK(upload(P, &P->rt.start, P->h_start));
  HIPCHK(upload(P, &P->rt.phase_den, P->h_phase_den));
  HIPCHK(upload(P, &P->rt.fft_kind, fft_kind));
  HIPCHK(upload(P, &P->rt.fft_m, fft_m));
  HIPCHK(upload(P, &P->rt.bl_off, bl_off));
  HIPCHK(upload(P, &P->rt.w, P->h_w));
  HIPCHK(upload(P, &P->d_theta, P->h_theta));
  HIPCHK(upload(P, &P->d_sin, P->h_sin));
  HIPCHK(upload(P, &P->d_pair_i, P->h_pair_i));
  HIPCHK(upload(P, &P->d_pair_shift, P->h_pair_shift));
  HIPCHK(upload(P, &P->d_coef_off, P->h_coef_off));
  HIPCHK(upload(P, &P->d_ncoef_window, P->h_ncoef_window));
  if (prof->kind == 1) {
    // moments of the basis splines (the spline through e_k), S[a][k]
    const int nk = (int)P->knots.size();
    std::vector<double> S((size_t)nk * nk), e(nk, 0.0), mom;
    for (int k = 0; k < nk; ++k) {
      e[k] = 1.0;
      spline_moments(e, P->theta_max / (nk - 1), mom);
      for (int a = 0; a < nk; ++a) S[(size_t)a * nk + k] = mom[a];
      e[k] = 0.0;
    }
    HIPCHK(upload(P, &P->d_basis_mom, S));
  }
  HIPCHK(dev_alloc(P, &P->d_pairs, P->h_pairs.size()));
  HIPCHK(dev_alloc(P, &P->d_coef64, P->coef_total));
  HIPCHK(hipMemset(P->d_coef64, 0, std::max<int64_t>(P->coef_total, 1) * sizeof(double)));
  {
    // padded by 16 zeros: the accumulation prefetches 16 samples per pair
    void* c = nullptr;
    HIPCHK(hipMalloc(&c, (P->coef_total + 16) * rsz));
    HIPCHK(hipMemset(c, 0, (P->coef_total + 16) * rsz));
    P->allocations.push_back(c);
    P->plan_bytes += (P->coef_total + 16) * rsz;
    P->d_coef = c;
  }
  HIPCHK(dev_alloc(P, &P->d_knots, std::max<size_t>(P->knots.size(), 1)));
  if (opts.kernel_eval == 1) {
    // the biased linear table of Sect. 4.1 (filled with the kernel samples)
    P->utable_n = opts.table_nodes > 0 ? opts.table_nodes : 65536;
    HIPCHK(dev_alloc(P, &P->d_utable, (size_t)P->utable_n));
  }
  HIPCHK(dev_alloc(P, &P->d_spline_mom, std::max<size_t>(P->knots.size(), 1)));
  {
    arkcos_status_t st = upload_knots(P);
    if (st != ARKCOS_OK) return st;
  }

  // twiddles exp(-2 pi i k / twn), computed in FP64
  {
    std::vector<double> tw(2 * twn);
    for (int64_t k = 0; k < twn; ++k) {
      double a = -2.0 * M_PI * (double)k / (double)twn;
      tw[2 * k] = cos(a);
      tw[2 * k + 1] = sin(a);
    }
    void* d = nullptr;
    HIPCHK(hipMalloc(&d, twn * csz));
    P->allocations.push_back(d);
    P->plan_bytes += twn * csz;
    if (dtype == ARKCOS_F32) {
      std::vector<float> tf(tw.begin(), tw.end());
      HIPCHK(hipMemcpy(d, tf.data(), twn * csz, hipMemcpyHostToDevice));
    } else {
      HIPCHK(hipMemcpy(d, tw.data(), twn * csz, hipMemcpyHostToDevice));
    }
    P->d_twiddle = d;
  }
  {
    void* d = nullptr;
    HIPCHK(hipMalloc(&d, std::max<int64_t>(P->bl_total, 1) * csz));
    P->allocations.push_back(d);
    P->plan_bytes += std::max<int64_t>(P->bl_total, 1) * csz;
    P->d_bl = d;
  }
  HIPCHK(configure_fft_kernels(P));
  if (!bl_rings.empty()) {
    int32_t* d_list = nullptr;
    HIPCHK(hipMalloc(&d_list, bl_rings.size() * sizeof(int32_t)));
    struct F { void* a; ~F() { hipFree(a); } } f{d_list};
    HIPCHK(hipMemcpy(d_list, bl_rings.data(), bl_rings.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(launch_bluestein_filters(P, d_list, (int32_t)bl_rings.size(), nullptr));
    HIPCHK(hipDeviceSynchronize());
  }

  // ------------------------------------------- kernel samples and bands
  {
    arkcos_status_t st = build_kernel_tables(P);
    if (st != ARKCOS_OK) return st;
  }
  if (const char* e = getenv("ARKCOS_PLAN_STATS"); e && *e == '1') {
    // (pair, mode) products per kernel-generation kind and row length
    std::map<std::pair<int, int>, int64_t> h;
    for (int64_t q = 0; q < P->n_pairs; ++q) {
      const PairDev& pr = P->h_pairs[q];
      if (pr.band < 0) continue;
      const int row = pr.kind == KG_TABLE ? 0 : (pr.ncoef + 7) / 8 * 8;
      h[{pr.kind, row}] += (int64_t)(pr.band + 1);
    }
    for (auto& kv : h)
      fprintf(stderr, "arkcos plan: kind %d row %d: %lld unit-pair modes\n", kv.first.first, kv.first.second,
              (long long)kv.second);
    // the knot gradient's per-pair correlation: window samples x modes
    double sm_narrow = 0.0, sm_wide = 0.0;
    int64_t n_narrow = 0, n_wide = 0, max_nc = 0;
    for (int64_t q = 0; q < P->n_pairs; ++q) {
      const PairDev& pr = P->h_pairs[q];
      if (pr.band < 0) continue;
      const int64_t nc = P->h_ncoef_window[q];
      max_nc = std::max(max_nc, nc);
      if (nc <= kGradMaxCoef) sm_narrow += (double)nc * (pr.band + 1), ++n_narrow;
      else sm_wide += (double)nc * (pr.band + 1), ++n_wide;
    }
    fprintf(stderr, "arkcos plan: gradient samples x modes: %lld narrow rows %.3g, %lld wide rows %.3g (max %lld samples)\n",
            (long long)n_narrow, sm_narrow, (long long)n_wide, sm_wide, (long long)max_nc);
  }
  if (P->prof_kind == 1) {
    arkcos_status_t st = build_grad_items(P);
    if (st != ARKCOS_OK) return st;
  }

  // ----------------------------------------- spectra / output layout
  P->h_spec_len.assign(nr, 0);
  P->h_out_len.assign(nr, 0);
  P->pair_modes = 0;
  for (int64_t u = 0; u < nunits; ++u) {
    UnitDev& U = P->h_units[u];
    int32_t ub = -1;
    for (int32_t q = U.pbeg; q < U.pend; ++q) {
      const PairDev& pr = P->h_pairs[q];
      ub = std::max(ub, pr.band);
      if (pr.band < 0) continue;
      P->h_spec_len[pr.j] = std::max(P->h_spec_len[pr.j], pr.band + 1);
      P->pair_modes += (int64_t)(pr.band + 1) * (U.im >= 0 ? 2 : 1);
      if (U.im >= 0) {
        const int64_t jm = nr - 1 - pr.j;
        P->h_spec_len[jm] = std::max(P->h_spec_len[jm], pr.band + 1);
      }
    }
    U.band = ub;
    U.jlo = P->h_pairs[U.pbeg].j;
    U.jhi = P->h_pairs[U.pend - 1].j;
    P->h_out_len[U.i] = ub + 1;
    if (U.im >= 0) P->h_out_len[U.im] = ub + 1;
  }
  P->h_spec_off.assign(nr, 0);
  P->h_out_off.assign(nr, 0);
  for (int64_t k = 0; k < nr; ++k) {
    P->h_spec_off[k] = P->spec_total;
    P->spec_total += P->h_spec_len[k];
    P->h_out_off[k] = P->out_total;
    P->out_total += P->h_out_len[k];
  }
  HIPCHK(upload(P, &P->rt.spec_off, P->h_spec_off));
  HIPCHK(upload(P, &P->rt.spec_len, P->h_spec_len));
  HIPCHK(upload(P, &P->rt.out_off, P->h_out_off));
  HIPCHK(upload(P, &P->rt.out_len, P->h_out_len));
  HIPCHK(upload(P, &P->d_units, P->h_units));

  // bands of consecutive units, and work items: (band, first mode) tiles
  {
    arkcos_status_t st = choose_accumulation_shape(P);
    if (st != ARKCOS_OK) return st;
  }
  HIPCHK(upload(P, &P->d_items, P->h_items));
  HIPCHK(upload(P, &P->d_bands, P->h_bands));
  HIPCHK(configure_accumulate(P));

  // rings whose pixels can lie within R of a pole pixel (direct-sum columns)
  if (g->kind == 1) {
    std::vector<int32_t> lst;
    for (int64_t j = 0; j < nr; ++j)
      if (fabs(P->h_theta[j] - P->h_theta[0]) <= rt || fabs(P->h_theta[j] - P->h_theta[nr - 1]) <= rt)
        lst.push_back((int32_t)j);
    P->n_pole_rings = (int32_t)lst.size();
    HIPCHK(upload(P, &P->d_pole_rings, lst));
  }

  HIPCHK(hipDeviceSynchronize());
  *out = P;
  owner.p = nullptr;
  return ARKCOS_OK;
}

// Work items of the accumulation: each band's mode tiles in runs of
// tiles_per_item, with an estimate of their cost (recurrence length of the
// pairs still inside their band, summed over the tiles).
void accumulation_items(const arkcos_plan_s* P, const std::vector<BandDev>& bands, int32_t tiles_per_item,
                        std::vector<WorkItem>& items, std::vector<double>& cost) {
  items.clear();
  cost.clear();
  for (int32_t b = 0; b < (int32_t)bands.size(); ++b) {
    const BandDev& bd = bands[b];
    if (bd.band < 0) continue;
    const int32_t ntile = bd.band / kAccTile + 1;
    for (int32_t t0 = 0; t0 < ntile; t0 += tiles_per_item) {
      const int32_t nt = std::min(tiles_per_item, ntile - t0);
      double c = 0.0;
      for (int32_t u = bd.u0; u < bd.u0 + bd.nu; ++u) {
        const UnitDev& U = P->h_units[u];
        for (int32_t q = U.pbeg; q < U.pend; ++q) {
          const PairDev& pr = P->h_pairs[q];
          const int32_t live = std::min(nt, pr.band / kAccTile + 1 - t0);
          if (live <= 0) continue;
          c += live * (pr.kind == KG_TABLE ? 3.0 : (double)((pr.ncoef + 3) / 4 * 4) + 4.0);
        }
      }
      items.push_back(WorkItem{b, t0, nt, 0});
      cost.push_back(c + 8.0 * nt);
    }
  }
}

// Groups consecutive units into bands of units_per_band, with the input-ring
// window of each band and the largest window.
void build_bands(const arkcos_plan_s* P, int32_t units_per_band, std::vector<BandDev>& bands, AccShape* shape) {
  bands.clear();
  *shape = AccShape{};
  const int64_t nunits = P->n_units, nr = P->nrings;
  for (int64_t u0 = 0; u0 < nunits; u0 += units_per_band) {
    BandDev B{};
    B.u0 = (int32_t)u0;
    B.nu = (int32_t)std::min<int64_t>(units_per_band, nunits - u0);
    B.jlo = (int32_t)nr;
    B.jhi = -1;
    B.band = -1;
    B.pbeg = P->h_units[u0].pbeg;
    B.npair = P->h_units[u0 + B.nu - 1].pend - B.pbeg;
    for (int64_t u = u0; u < u0 + B.nu; ++u) {
      const UnitDev& U = P->h_units[u];
      if (U.pend > U.pbeg) {
        B.jlo = std::min(B.jlo, P->h_pairs[U.pbeg].j);
        B.jhi = std::max(B.jhi, P->h_pairs[U.pend - 1].j);
      }
      B.band = std::max(B.band, U.band);
    }
    if (B.jhi >= B.jlo) shape->max_window = std::max(shape->max_window, B.jhi - B.jlo + 1);
    shape->max_band_pairs = std::max(shape->max_band_pairs, B.npair);
    bands.push_back(B);
  }
}

int32_t* pole_ring_list(arkcos_plan_s* P, int32_t* count) {
  *count = P->n_pole_rings;
  return P->d_pole_rings;
}

// Workspace: extended input spectra | output-ring coefficients | (spline
// plans) per-unit gradient partials, each 256-byte aligned.
static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

static size_t grad_slot_bytes(const arkcos_plan_s* P) {
  if (P->prof_kind != 1) return 0;
  // one slot per run and per FFT-row block, eight for the pole rows, one for their sum
  return al256((size_t)(P->n_grad_runs + P->n_gfft_slots + 9) * 4 * (P->knots.size() - 1) * sizeof(double));
}

// the FFT rows' Y(d) (one chunk at a time), after the slots
static size_t grad_y_bytes(const arkcos_plan_s* P) {
  if (P->prof_kind != 1 || P->grad_y_elems == 0) return 0;
  return al256((size_t)P->grad_y_elems * (P->dtype == ARKCOS_F32 ? sizeof(float) : sizeof(double)));
}

size_t workspace_bytes(const arkcos_plan_s* P) {
  const size_t csz = P->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  return al256(std::max<int64_t>(P->spec_total, 1) * csz) + al256(std::max<int64_t>(P->out_total, 1) * csz) +
         grad_slot_bytes(P) + grad_y_bytes(P);
}

void* grad_y(const arkcos_plan_s* P, void* ws) {
  return reinterpret_cast<char*>(grad_slots(P, ws)) + grad_slot_bytes(P);
}

double* grad_slots(const arkcos_plan_s* P, void* ws) {
  const size_t csz = P->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  return reinterpret_cast<double*>(static_cast<char*>(ws) + al256(std::max<int64_t>(P->spec_total, 1) * csz) +
                                   al256(std::max<int64_t>(P->out_total, 1) * csz));
}

}  // namespace arkcos
