// Batched form: many maps of uneven size, each with its own plan (its own
// geometry and kernel profile), convolved by one pass of batched ring
// transforms, one persistent accumulation launch over a shared work queue,
// and one pass of batched inverse transforms.
//
// Shared-input form: one map convolved with many kernels on one geometry
// (e.g. the symmetric components an asymmetric beam is split into, paper
// Sect. 5).  The input's extended spectra are computed once, in the union of
// the plans' spectrum layouts (every ring as long as the longest any plan
// needs), and every plan's accumulation reads them from there; the
// accumulation and the inverse transforms run batched over the kernels.
//
// The queue holds (map, band of output rings, mode tiles) items of every
// map, ordered by decreasing estimated cost so the persistent workgroups end
// together.  The band size (output rings per item) and the number of
// persistent workgroups are chosen by timing the accumulation on a subset of
// the maps (up to four maps of each ring count).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "arkcos_internal.h"
#include "device_common.h"

using namespace arkcos;

namespace {

struct ClassDev {
  int2* entries = nullptr;
  int32_t count = 0;
  int32_t lds = 0;
  int32_t threads = 256;
  int32_t mf = 0;  // the compile-time FFT length of every ring of the class, if they share one
};

}  // namespace

struct arkcos_batch_s {
  int device = 0;
  arkcos_dtype_t dtype = ARKCOS_F32;
  int32_t n = 0;
  std::vector<arkcos_plan_s*> plans;
  int32_t units_per_band = kBandUnits, grid = 0, tuned = 0;
  int32_t units_per_wave = 1;  // 2: table-only FP32 batches, bands of 16 units in 8-wave blocks
  int32_t staged_rings = 0;    // input rings the accumulation stages at a time (0: the default)
  bool all_tables = false;  // every plan reads all its K_ij(m) from tables
  AccShape acc_shape;
  int64_t spec_total = 0, out_total = 0, npix_total = 0;
  std::vector<int64_t> h_spec_base, h_out_base;
  // device
  int64_t* d_spec_base = nullptr;
  int64_t* d_out_base = nullptr;
  void* d_acc_args = nullptr;            // AccArgs per map
  arkcos::BatchItem* d_items = nullptr;
  int32_t n_items = 0;
  void* d_rargs[4] = {nullptr, nullptr, nullptr, nullptr};  // R2C fwd, R2C adj, C2R fwd, C2R adj
  std::vector<ClassDev> classes;
  // shared-input form: the R2C classes of the one input map, and the union
  // spectrum layout every plan reads
  bool shared = false;
  std::vector<ClassDev> in_classes;
  int64_t* d_union_off = nullptr;
  int32_t* d_union_len = nullptr;
  void* d_pole_maps = nullptr;
  int2* d_pole_fwd = nullptr;
  int2* d_pole_adj = nullptr;
  int32_t n_pole_fwd = 0, n_pole_adj = 0;
  std::vector<void*> allocations;
  std::vector<hipEvent_t> timing_events;
  int32_t timing_slots = 0, timing_used = 0;
};

namespace {

#define BCHK(expr)                                                                          \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(_e == hipErrorOutOfMemory ? ARKCOS_ERR_OUT_OF_MEMORY : ARKCOS_ERR_DEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                       \
  } while (0)

template <typename T> hipError_t balloc(arkcos_batch_s* B, T** p, size_t count) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  B->allocations.push_back(v);
  *p = static_cast<T*>(v);
  return hipSuccess;
}

template <typename T> hipError_t bupload(arkcos_batch_s* B, T** p, const std::vector<T>& v) {
  hipError_t e = balloc(B, p, v.size());
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Queue of one batch configuration: per-map bands on the device, the AccArgs
// pointing at them, and the items sorted by decreasing estimated cost.
struct Queue {
  std::vector<BandDev*> d_bands;
  std::vector<char> acc_args;
  std::vector<BatchItem> items;
  AccShape shape;
};

hipError_t build_queue(arkcos_batch_s* B, const std::vector<int32_t>& maps, int32_t upb, Queue& Q,
                       std::vector<void*>& owned) {
  const size_t asz = acc_args_size();
  Q.acc_args.assign(asz * maps.size(), 0);
  std::vector<std::pair<double, BatchItem>> costed;
  for (size_t mi = 0; mi < maps.size(); ++mi) {
    arkcos_plan_s* P = B->plans[maps[mi]];
    std::vector<BandDev> bands;
    AccShape sh;
    build_bands(P, upb, bands, &sh);
    Q.shape.max_window = std::max(Q.shape.max_window, sh.max_window);
    Q.shape.max_band_pairs = std::max(Q.shape.max_band_pairs, sh.max_band_pairs);
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(bands.size(), 1) * sizeof(BandDev));
    if (e != hipSuccess) return e;
    owned.push_back(d);
    e = hipMemcpy(d, bands.data(), bands.size() * sizeof(BandDev), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    Q.d_bands.push_back((BandDev*)d);
    fill_acc_args(P, (const BandDev*)d, Q.acc_args.data() + asz * mi, B->d_union_off, B->d_union_len);
    std::vector<WorkItem> its;
    std::vector<double> cost;
    accumulation_items(P, bands, kTilesPerItem, its, cost);
    for (size_t k = 0; k < its.size(); ++k)
      costed.push_back({cost[k], BatchItem{(int32_t)mi, its[k].band, its[k].t0, its[k].nt}});
  }
  std::stable_sort(costed.begin(), costed.end(),
                   [](const std::pair<double, BatchItem>& a, const std::pair<double, BatchItem>& b) {
                     return a.first > b.first;
                   });
  Q.items.clear();
  for (auto& c : costed) Q.items.push_back(c.second);
  return hipSuccess;
}

std::string tune_key(const arkcos_batch_s* B) {
  std::ostringstream k;
  k << "dt" << (int)B->dtype << "_n" << B->n << "_t" << (B->all_tables ? 1 : 0) << (B->shared ? "_s" : "");
  uint64_t h = 1469598103934665603ull;
  for (auto* P : B->plans) {
    const int64_t v[3] = {P->npix, P->pair_modes, P->coef_total};
    for (int64_t x : v) {
      h ^= (uint64_t)x;
      h *= 1099511628211ull;
    }
  }
  k << "_" << std::hex << h;
  return k.str();
}

// Cache lines: key, units per band, blocks per CU, units per wavefront,
// staged rings.
bool read_cache(const std::string& key, int32_t* upb, int32_t* bpc, int32_t* upw, int32_t* ch) {
  const char* path = getenv("ARKCOS_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k;
    int32_t a = 0, b = 0, c = 0, d = 0;
    if ((in >> k >> a >> b >> c >> d) && k == key) {
      *upb = a;
      *bpc = b;
      *upw = c;
      *ch = d;
      return true;
    }
  }
  return false;
}

void write_cache(const std::string& key, int32_t upb, int32_t bpc, int32_t upw, int32_t ch) {
  const char* path = getenv("ARKCOS_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << upb << " " << bpc << " " << upw << " " << ch << "\n";
}

// Times the accumulation of one queue on the subset's workspace (zero
// spectra); returns milliseconds per launch.
hipError_t time_queue(arkcos_batch_s* B, const Queue& Q, const std::vector<int64_t>& sb,
                      const std::vector<int64_t>& ob, void* spec, void* bout, int32_t* counter, int32_t upb,
                      int32_t grid, float* ms, int32_t upw, int32_t ch) {
  void *dargs = nullptr, *ditems = nullptr, *dsb = nullptr, *dob = nullptr;
  hipError_t e = hipMalloc(&dargs, Q.acc_args.size());
  if (e == hipSuccess) e = hipMalloc(&ditems, std::max<size_t>(Q.items.size(), 1) * sizeof(BatchItem));
  if (e == hipSuccess) e = hipMalloc(&dsb, sb.size() * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&dob, ob.size() * sizeof(int64_t));
  if (e == hipSuccess) e = hipMemcpy(dargs, Q.acc_args.data(), Q.acc_args.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ditems, Q.items.data(), Q.items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dsb, sb.data(), sb.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dob, ob.data(), ob.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int reps = 3;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    if (r == 1) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess)
      e = launch_accumulate_batch(B->dtype, dargs, (const int64_t*)dsb, (const int64_t*)dob, (const BatchItem*)ditems,
                                  (int32_t)Q.items.size(), counter, spec, bout, grid, upb, B->all_tables, Q.shape,
                                  nullptr, upw, ch);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  *ms = t / reps;
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(dargs);
  hipFree(ditems);
  hipFree(dsb);
  hipFree(dob);
  return e;
}

arkcos_status_t autotune(arkcos_batch_s* B, int32_t* upb_out, int32_t* bpc_out, int32_t* upw_out,
                         int32_t* ch_out) {
  // subset: up to four maps per ring count
  std::map<int64_t, int> seen;
  std::vector<int32_t> sub;
  for (int32_t i = 0; i < B->n; ++i)
    if (seen[B->plans[i]->nrings]++ < 4) sub.push_back(i);
  std::vector<int64_t> sb, ob;
  int64_t st = 0, ot = 0;
  for (int32_t i : sub) {
    sb.push_back(B->shared ? 0 : st);
    ob.push_back(ot);
    st += B->shared ? 0 : B->plans[i]->spec_total;
    ot += B->plans[i]->out_total;
  }
  if (B->shared) st = B->spec_total;  // every plan reads the one union layout
  const size_t csz = B->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  void *spec = nullptr, *bout = nullptr, *ctr = nullptr;
  BCHK(hipMalloc(&spec, std::max<int64_t>(st, 1) * csz));
  struct F { void* a; ~F() { hipFree(a); } } f1{spec};
  BCHK(hipMalloc(&bout, std::max<int64_t>(ot, 1) * csz));
  F f2{bout};
  BCHK(hipMalloc(&ctr, 256));
  F f3{ctr};
  BCHK(hipMemset(spec, 0, std::max<int64_t>(st, 1) * csz));
  int cus = 0;
  BCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
  float best = 1e30f;
  int32_t bu = kBandUnits, bb = 2, bw = 1, bc = 0;
  // (units per band, units per wavefront, staged rings): two units per
  // wavefront only for table-only FP32 batches
  struct Shape {
    int32_t upb, upw, ch;
  };
  std::vector<Shape> shapes = {{4, 1, 0}, {8, 1, 0}, {16, 1, 0}};
  // (staging 16 rings at a time, {16, 2, 16}, measured no faster on the 256-map
  // batch and slower on ten kernels over one input map: not a candidate)
  if (B->all_tables && B->dtype == ARKCOS_F32) shapes.push_back({16, 2, 0});
  for (const Shape& sh : shapes) {
    const int32_t upb = sh.upb;
    Queue Q;
    std::vector<void*> owned;
    hipError_t e = build_queue(B, sub, upb, Q, owned);
    for (int32_t bpc : {1, 2, 4}) {
      float ms = 0.f;
      if (e == hipSuccess)
        e = time_queue(B, Q, sb, ob, spec, bout, (int32_t*)ctr, upb, cus * bpc, &ms, sh.upw, sh.ch);
      if (e == hipSuccess && ms < best) {
        best = ms;
        bu = upb;
        bb = bpc;
        bw = sh.upw;
        bc = sh.ch;
      }
    }
    for (void* p : owned) hipFree(p);
    if (e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  }
  *upb_out = bu;
  *bpc_out = bb;
  *upw_out = bw;
  *ch_out = bc;
  return ARKCOS_OK;
}

// Rings of the given (map, ring) entries grouped into ring-transform
// classes: rings of similar LDS needs share a launch, and rings of a length
// with a compile-time transform get a class of their own.
hipError_t make_classes(arkcos_batch_s* B, const std::vector<int2>& entries, std::vector<ClassDev>& out) {
  std::map<int64_t, std::vector<int2>> cls;
  std::map<int32_t, int64_t> per_len;
  for (const int2& e : entries) ++per_len[B->plans[e.x]->h_fft_len[e.y]];
  for (const int2& e : entries) {
    arkcos_plan_s* P = B->plans[e.x];
    int64_t b = 32768;  // small rings of every map share one launch
    while (b < P->h_ring_lds[e.y]) b <<= 1;
    // a compile-time FFT length: one class per length
    const int32_t ct = ct_fft_length(B->dtype, P->h_fft_len[e.y], per_len[P->h_fft_len[e.y]]);
    if (ct > 0) b = (int64_t(1) << 40) + ct;
    if (P->h_fft_kind[e.y] == FFT_MIXED) b |= int64_t(1) << 39;  // mixed-radix rings: classes of their own
    cls[b].push_back(e);
  }
  for (auto it = cls.rbegin(); it != cls.rend(); ++it) {
    ClassDev c;
    c.count = (int32_t)it->second.size();
    int32_t mx = 0, len = 0, lo = INT32_MAX;
    for (const int2& e : it->second) {
      mx = std::max(mx, B->plans[e.x]->h_ring_lds[e.y]);
      len = std::max(len, B->plans[e.x]->h_fft_len[e.y]);
      lo = std::min(lo, B->plans[e.x]->h_fft_len[e.y]);
    }
    c.lds = mx;
    // one compile-time FFT length for the whole class: compile-time transforms
    c.mf = (lo == len) ? ct_fft_length(B->dtype, len, per_len[len]) : 0;
    if (it->first & (int64_t(1) << 39)) c.mf = -1;
    c.threads = c.mf > 0 ? c.mf / 16 : fft_threads(B->dtype, len);
    hipError_t e = bupload(B, &c.entries, it->second);
    if (e != hipSuccess) return e;
    out.push_back(c);
  }
  return hipSuccess;
}

arkcos_status_t build_batch(int32_t n, const arkcos_plan_t* plans, bool shared, arkcos_batch_t* out) {
  if (n < 1 || !plans || !out) return fail(ARKCOS_ERR_INVALID_VALUE, "need n >= 1 plans and an output handle");
  int dev = -1;
  BCHK(hipGetDevice(&dev));
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(ARKCOS_ERR_INVALID_VALUE, "null plan in batch");
    if (plans[i]->device != dev) return fail(ARKCOS_ERR_INVALID_VALUE, "plans live on another device");
    if (plans[i]->dtype != plans[0]->dtype) return fail(ARKCOS_ERR_INVALID_VALUE, "plans of mixed dtype");
    if (shared) {
      const arkcos_geometry_t &a = plans[i]->geom, &b = plans[0]->geom;
      if (a.kind != b.kind || (a.kind == 1 ? a.nside != b.nside : (a.n_theta != b.n_theta || a.n_phi != b.n_phi)))
        return fail(ARKCOS_ERR_INVALID_VALUE, "a shared-input batch needs plans of one geometry");
      if (plans[i]->opts.fix_pole_pixels != plans[0]->opts.fix_pole_pixels)
        return fail(ARKCOS_ERR_INVALID_VALUE, "a shared-input batch needs one fix_pole_pixels setting");
    }
  }
  auto* B = new arkcos_batch_s();
  struct Owner {
    arkcos_batch_s* b;
    ~Owner() {
      if (b) {
        for (void* a : b->allocations) hipFree(a);
        delete b;
      }
    }
  } owner{B};
  B->device = dev;
  B->n = n;
  B->dtype = plans[0]->dtype;
  B->plans.assign(plans, plans + n);
  B->shared = shared;
  B->all_tables = true;
  for (auto* P : B->plans) {
    B->all_tables = B->all_tables && P->all_tables;
    B->h_spec_base.push_back(shared ? 0 : B->spec_total);
    B->h_out_base.push_back(B->out_total);
    B->spec_total += shared ? 0 : P->spec_total;
    B->out_total += P->out_total;
    B->npix_total += P->npix;
  }
  if (shared) {
    // union spectrum layout: each ring as long as the longest any plan reads
    const int64_t nr = B->plans[0]->nrings;
    std::vector<int32_t> len(nr, 0);
    std::vector<int64_t> off(nr, 0);
    for (auto* P : B->plans)
      for (int64_t k = 0; k < nr; ++k) len[k] = std::max(len[k], P->h_spec_len[k]);
    for (int64_t k = 0; k < nr; ++k) {
      off[k] = B->spec_total;
      B->spec_total += len[k];
    }
    BCHK(bupload(B, &B->d_union_off, off));
    BCHK(bupload(B, &B->d_union_len, len));
  }
  BCHK(bupload(B, &B->d_spec_base, B->h_spec_base));
  BCHK(bupload(B, &B->d_out_base, B->h_out_base));

  // ring-transform arguments (forward/transpose, both layouts) and classes
  const size_t rsz = ring_args_size();
  for (int v = 0; v < 4; ++v) {
    std::vector<char> h(rsz * n);
    for (int32_t i = 0; i < n; ++i) {
      arkcos_plan_s* P = B->plans[i];
      const bool fix = P->geom.kind == 1 && P->opts.fix_pole_pixels;
      const bool outl = v >= 2, adj = (v & 1) != 0;
      if (shared && !outl)  // the one input map, in the union layout
        fill_ring_args(B->plans[0], false, adj ? 1 : 0, (adj && fix) ? 1 : 0, h.data() + rsz * i, B->d_union_off,
                       B->d_union_len);
      else
        fill_ring_args(P, outl, adj ? 1 : 0, (!outl && adj && fix) ? 1 : 0, h.data() + rsz * i);
    }
    void* d = nullptr;
    BCHK(hipMalloc(&d, h.size()));
    B->allocations.push_back(d);
    BCHK(hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice));
    B->d_rargs[v] = d;
  }
  {
    std::vector<int2> all_rings, in_rings;
    for (int32_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < B->plans[i]->nrings; ++k) all_rings.push_back(make_int2(i, (int)k));
    BCHK(make_classes(B, all_rings, B->classes));
    if (shared) {
      for (int64_t k = 0; k < B->plans[0]->nrings; ++k) in_rings.push_back(make_int2(0, (int)k));
      BCHK(make_classes(B, in_rings, B->in_classes));
    }
  }
  // pole rows
  {
    const size_t psz = pole_map_size();
    std::vector<char> h(psz * n);
    std::vector<int2> fwd, adj;
    for (int32_t i = 0; i < n; ++i) {
      arkcos_plan_s* P = B->plans[i];
      fill_pole_map(P, h.data() + psz * i);
      if (P->geom.kind == 1 && P->opts.fix_pole_pixels && P->n_pole_rings > 0) {
        for (int b = 0; b < 8; ++b) fwd.push_back(make_int2(i, b));
        for (int k = 0; k < P->n_pole_rings; ++k) adj.push_back(make_int2(i, k));
      }
    }
    void* d = nullptr;
    BCHK(hipMalloc(&d, h.size()));
    B->allocations.push_back(d);
    BCHK(hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice));
    B->d_pole_maps = d;
    BCHK(bupload(B, &B->d_pole_fwd, fwd));
    BCHK(bupload(B, &B->d_pole_adj, adj));
    B->n_pole_fwd = (int32_t)fwd.size();
    B->n_pole_adj = (int32_t)adj.size();
  }

  // band size and grid: cached, else measured
  int32_t upb = kBandUnits, bpc = 2, upw = 1, ch = 0;
  const std::string key = tune_key(B);
  if (read_cache(key, &upb, &bpc, &upw, &ch) && (ch == 0 || ch == 16) &&
      (upw == 1 || (upw == 2 && upb == 16 && B->all_tables && B->dtype == ARKCOS_F32))) {
    B->tuned = 2;
  } else {
    arkcos_status_t st = autotune(B, &upb, &bpc, &upw, &ch);
    if (st != ARKCOS_OK) return st;
    write_cache(key, upb, bpc, upw, ch);
    B->tuned = 1;
  }
  B->units_per_wave = upw;
  B->staged_rings = upw == 2 ? ch : 0;
  int cus = 0;
  BCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  B->units_per_band = upb;
  B->grid = cus * bpc;
  std::vector<int32_t> all(n);
  for (int32_t i = 0; i < n; ++i) all[i] = i;
  Queue Q;
  std::vector<void*> owned;
  hipError_t e = build_queue(B, all, upb, Q, owned);
  for (void* p : owned) B->allocations.push_back(p);
  BCHK(e);
  B->acc_shape = Q.shape;
  void* d = nullptr;
  BCHK(hipMalloc(&d, Q.acc_args.size()));
  B->allocations.push_back(d);
  BCHK(hipMemcpy(d, Q.acc_args.data(), Q.acc_args.size(), hipMemcpyHostToDevice));
  B->d_acc_args = d;
  BCHK(bupload(B, &B->d_items, Q.items));
  B->n_items = (int32_t)Q.items.size();
  BCHK(hipDeviceSynchronize());
  *out = B;
  owner.b = nullptr;
  return ARKCOS_OK;
}

// Workspace: queue counter (256 bytes) | the call's map pointers (x then y,
// n each) | spectra | output coefficients, each part 256-byte aligned.
size_t ptr_table_bytes(const arkcos_batch_s* B) { return ((size_t)2 * B->n * sizeof(void*) + 255) / 256 * 256; }

size_t batch_ws_bytes(const arkcos_batch_s* B) {
  const size_t csz = B->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  return 256 + ptr_table_bytes(B) + al(std::max<int64_t>(B->spec_total, 1) * csz) +
         al(std::max<int64_t>(B->out_total, 1) * csz);
}

// Map pointers of one call, passed by value to a kernel that writes them into
// the call's region of the workspace (so every call, eager or captured in a
// graph, reads its own pointers; nothing is uploaded from the host).
constexpr int kPtrChunk = 64;
struct PtrChunk {
  const void* p[kPtrChunk];
};

__global__ void fill_ptrs_kernel(PtrChunk c, int32_t count, const void** __restrict__ dst) {
  if ((int32_t)threadIdx.x < count) gstore(dst + threadIdx.x, c.p[threadIdx.x]);
}

hipError_t write_ptrs(const void* const* src, int32_t n, const void** dst, hipStream_t s) {
  for (int32_t b = 0; b < n; b += kPtrChunk) {
    PtrChunk c{};
    const int32_t cnt = std::min(kPtrChunk, n - b);
    for (int32_t k = 0; k < cnt; ++k) c.p[k] = src[b + k];
    fill_ptrs_kernel<<<1, kPtrChunk, 0, s>>>(c, cnt, dst + b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

#define BLAUNCH(expr)                                                                              \
  do {                                                                                             \
    hipError_t _e = (expr);                                                                        \
    if (_e != hipSuccess) return fail(ARKCOS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// x: n input pointers (a shared-input batch: n copies of its one input).
arkcos_status_t run_batch(arkcos_batch_s* B, const void* const* x, void* const* y, int32_t adjoint, void* ws,
                          hipStream_t s) {
  if (!x || !y || !ws) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (B->shared && adjoint) return fail(ARKCOS_ERR_NOT_SUPPORTED, "a shared-input batch runs the forward map only");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(ARKCOS_ERR_INVALID_VALUE, "workspace must be 256-byte aligned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != B->device)
    return fail(ARKCOS_ERR_INVALID_VALUE, "batch was created on another device");
  const size_t esz = B->dtype == ARKCOS_F32 ? sizeof(float) : sizeof(double);
  for (int32_t i = 0; i < B->n; ++i) {
    if (!x[i] || !y[i]) return fail(ARKCOS_ERR_INVALID_VALUE, "null map pointer");
    const size_t bi = (size_t)B->plans[i]->npix * esz;
    for (int32_t k = 0; k < B->n; ++k) {
      const size_t bk = (size_t)B->plans[k]->npix * esz;
      auto px = reinterpret_cast<uintptr_t>(x[i]), py = reinterpret_cast<uintptr_t>(y[k]);
      if (px < py + bk && py < px + bi) return fail(ARKCOS_ERR_INVALID_VALUE, "an input map overlaps an output map");
    }
  }
  const size_t csz = B->dtype == ARKCOS_F32 ? sizeof(float2) : sizeof(double2);
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  char* base = static_cast<char*>(ws);
  int32_t* counter = reinterpret_cast<int32_t*>(base);
  const void** d_xs = reinterpret_cast<const void**>(base + 256);
  const void** d_ys = d_xs + B->n;
  void* spec = base + 256 + ptr_table_bytes(B);
  void* bout = static_cast<char*>(spec) + al(std::max<int64_t>(B->spec_total, 1) * csz);
  hipEvent_t* ev = nullptr;
  if (B->timing_used < B->timing_slots) ev = &B->timing_events[5 * B->timing_used++];
  if (ev) BLAUNCH(hipEventRecord(ev[0], s));
  BLAUNCH(write_ptrs(x, B->n, d_xs, s));
  BLAUNCH(write_ptrs(y, B->n, d_ys, s));
  for (const ClassDev& c : (B->shared ? B->in_classes : B->classes))
    BLAUNCH(launch_ring_batch(B->dtype, false, B->d_rargs[adjoint ? 1 : 0], c.entries, c.count, c.lds, c.threads, c.mf, d_xs, spec,
                              B->d_spec_base, s));
  if (ev) BLAUNCH(hipEventRecord(ev[1], s));
  BLAUNCH(launch_accumulate_batch(B->dtype, B->d_acc_args, B->d_spec_base, B->d_out_base, B->d_items, B->n_items,
                                  counter, spec, bout, B->grid, B->units_per_band, B->all_tables, B->acc_shape, s,
                                  B->units_per_wave, B->staged_rings));
  if (ev) BLAUNCH(hipEventRecord(ev[2], s));
  for (const ClassDev& c : B->classes)
    BLAUNCH(launch_ring_batch(B->dtype, true, B->d_rargs[adjoint ? 3 : 2], c.entries, c.count, c.lds, c.threads, c.mf, d_ys, bout,
                              B->d_out_base, s));
  if (ev) BLAUNCH(hipEventRecord(ev[3], s));
  if (!adjoint)
    BLAUNCH(launch_pole_batch(B->dtype, B->d_pole_maps, B->d_pole_fwd, B->n_pole_fwd, 0, d_xs, d_ys, s));
  else
    BLAUNCH(launch_pole_batch(B->dtype, B->d_pole_maps, B->d_pole_adj, B->n_pole_adj, 1, d_xs, d_ys, s));
  if (ev) BLAUNCH(hipEventRecord(ev[4], s));
  return ARKCOS_OK;
}

}  // namespace

extern "C" {

arkcos_status_t arkcos_batch_plan(int32_t n, const arkcos_plan_t* plans, arkcos_batch_t* out) {
  try {
    return build_batch(n, plans, false, out);
  } catch (const std::bad_alloc&) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(ARKCOS_ERR_INTERNAL, "unexpected exception in batch creation");
  }
}

arkcos_status_t arkcos_batch_plan_shared_input(int32_t n, const arkcos_plan_t* plans, arkcos_batch_t* out) {
  try {
    return build_batch(n, plans, true, out);
  } catch (const std::bad_alloc&) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(ARKCOS_ERR_INTERNAL, "unexpected exception in batch creation");
  }
}

arkcos_status_t arkcos_batch_convolve_shared(arkcos_batch_t B, const void* x, void* const* y, void* ws,
                                             hipStream_t stream) {
  if (!B) return fail(ARKCOS_ERR_INVALID_VALUE, "null batch");
  if (!B->shared) return fail(ARKCOS_ERR_INVALID_VALUE, "batch was not created with arkcos_batch_plan_shared_input");
  if (!x) return fail(ARKCOS_ERR_INVALID_VALUE, "null input map");
  try {
    std::vector<const void*> xs(B->n, x);
    return run_batch(B, xs.data(), y, 0, ws, stream);
  } catch (const std::bad_alloc&) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(ARKCOS_ERR_INTERNAL, "unexpected exception in batch call");
  }
}

arkcos_status_t arkcos_batch_get_info(arkcos_batch_t B, arkcos_batch_info_t* info) {
  if (!B || !info) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  std::memset(info, 0, sizeof(*info));
  info->n_maps = B->n;
  info->seg_units = B->units_per_band;
  info->group = B->units_per_band / B->units_per_wave;
  info->units_per_wave = B->units_per_wave;
  info->grid = B->grid;
  info->tuned = B->tuned;
  info->n_items = B->n_items;
  info->npix_total = B->npix_total;
  info->workspace_bytes = batch_ws_bytes(B);
  return ARKCOS_OK;
}

arkcos_status_t arkcos_batch_workspace_size(arkcos_batch_t B, size_t* bytes) {
  if (!B || !bytes) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  *bytes = batch_ws_bytes(B);
  return ARKCOS_OK;
}

arkcos_status_t arkcos_batch_convolve(arkcos_batch_t B, const void* const* x, void* const* y, int32_t adjoint,
                                      void* ws, hipStream_t stream) {
  if (!B) return fail(ARKCOS_ERR_INVALID_VALUE, "null batch");
  if (B->shared) return fail(ARKCOS_ERR_INVALID_VALUE, "a shared-input batch is called with arkcos_batch_convolve_shared");
  if (adjoint != 0 && adjoint != 1) return fail(ARKCOS_ERR_INVALID_VALUE, "adjoint must be 0 or 1");
  try {
    return run_batch(B, x, y, adjoint, ws, stream);
  } catch (...) {
    return fail(ARKCOS_ERR_INTERNAL, "unexpected exception in batch call");
  }
}

arkcos_status_t arkcos_batch_timing(arkcos_batch_t B, int32_t max_calls) {
  if (!B || max_calls < 0) return fail(ARKCOS_ERR_INVALID_VALUE, "bad argument");
  for (hipEvent_t e : B->timing_events) (void)hipEventDestroy(e);
  B->timing_events.clear();
  B->timing_slots = B->timing_used = 0;
  if (max_calls == 0) return ARKCOS_OK;
  B->timing_events.resize(5 * (size_t)max_calls);
  for (auto& e : B->timing_events)
    if (hipEventCreate(&e) != hipSuccess) return fail(ARKCOS_ERR_DEVICE, "hipEventCreate failed");
  B->timing_slots = max_calls;
  return ARKCOS_OK;
}

arkcos_status_t arkcos_batch_stage_times(arkcos_batch_t B, double* ms, int64_t* calls) {
  if (!B || !ms || !calls) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  for (int32_t c = 0; c < B->timing_used; ++c) {
    hipEvent_t* ev = &B->timing_events[5 * c];
    if (hipEventSynchronize(ev[4]) != hipSuccess) return fail(ARKCOS_ERR_DEVICE, "hipEventSynchronize failed");
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess)
        return fail(ARKCOS_ERR_DEVICE, "hipEventElapsedTime failed");
      ms[k] += t;
    }
  }
  *calls = B->timing_used;
  B->timing_used = 0;
  return ARKCOS_OK;
}

arkcos_status_t arkcos_batch_destroy(arkcos_batch_t B) {
  if (!B) return fail(ARKCOS_ERR_INVALID_VALUE, "null batch");
  for (void* a : B->allocations) (void)hipFree(a);
  for (hipEvent_t e : B->timing_events) (void)hipEventDestroy(e);
  delete B;
  return ARKCOS_OK;
}

}  // extern "C"
