// Internal structures shared by the host plan builder, the C ABI and the HIP
// kernels of the ARKCoS library.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "arkcos.h"

namespace arkcos {

constexpr double kSupportTol = 1e-9;   // pairs with theta <= R + 1e-9 are inside
constexpr int kBlock = 256;            // threads per block for every kernel
constexpr int kModeTile = 256;         // modes per accumulation work item
constexpr int kDirectMax = 64;         // rings up to this length use a plain DFT
constexpr int kOtfMaxCoef = 48;        // wider kernel rows use a K_ij(m) table (auto mode)
constexpr int kClenshawMaxCoef = 16;   // longer centred rows use Reinsch's recurrence
constexpr int kBandUnits = 8;          // output units (ring + mirror) per accumulation work item
constexpr int kAccTile = 256;          // modes per accumulation tile (four per lane)
constexpr int kAccThreads = 64 * kBandUnits;  // one wavefront per unit

// FFT strategy of one ring length.
// FFT_MIXED: n = 2^a 3^b 5^c 7^d, not a power of two: mixed-radix passes.
enum FftKind : int32_t { FFT_DIRECT = 0, FFT_POW2 = 1, FFT_BLUESTEIN = 2, FFT_MIXED = 3 };

// K_ij(m) source of one ring pair.
//  KG_CENTRED  : nodes 2 pi d / G, recurrence on cos(m nu)
//  KG_SHIFTED  : nodes 2 pi (d + 1/2) / G (equal-length rings offset by pi/G)
//  KG_TABLE    : precomputed K_ij(m), m <= band
//  KG_REINSCH  : centred nodes, Reinsch's form of the recurrence (longer rows)
enum PairKind : int32_t { KG_CENTRED = 0, KG_SHIFTED = 1, KG_TABLE = 2, KG_REINSCH = 3 };

// Per-ring table, device side (struct of arrays).
struct RingTables {
  int32_t* n = nullptr;          // pixels in the ring
  int64_t* start = nullptr;      // first pixel (RING order)
  int32_t* phase_den = nullptr;  // longitude offset phi0 = pi / phase_den (0: none)
  int32_t* fft_kind = nullptr;
  int32_t* fft_m = nullptr;      // pow2: n/2; Bluestein: convolution length M
  int64_t* bl_off = nullptr;     // Bluestein filter offset (complex elements)
  int64_t* spec_off = nullptr;   // extended spectrum offset (complex elements)
  int32_t* spec_len = nullptr;   // extended spectrum length (modes 0 .. len-1)
  int64_t* out_off = nullptr;    // B_i offset (complex elements)
  int32_t* out_len = nullptr;    // B_i length
  double* w = nullptr;           // pixel area of the ring
};

// One ring pair (i, j) of a north output ring i; its mirror pair (i', j')
// with i' = nr-1-i, j' = nr-1-j uses the same K_ij(m).
struct PairDev {
  int32_t j;         // input ring
  int32_t kind;      // PairKind
  int32_t band;      // K_ij(m) = 0 for m > band
  int32_t nyq;       // p L / 2: this mode carries half weight
  int32_t ncoef;     // recurrence coefficients (KG_CENTRED / KG_SHIFTED)
  int32_t grid;      // longitudes of the kernel grid (ring length, or oversample * L)
  int64_t off;       // coefficient offset (recurrence) or table offset
};

// An output unit: a north ring i and its mirror (or -1 for the self-mirror ring).
struct UnitDev {
  int32_t i, im;
  int32_t pbeg, pend;   // pairs [pbeg, pend)
  int32_t band;         // max band over the unit's pairs
  int32_t jlo, jhi;     // input rings of its first and last pair
  int32_t pad;
};

// One work item of the knot gradient: the narrow rows (at most
// kGradMaxCoef samples) of unit `unit` (pair = -1), or the samples
// [d0, d0 + cnt) of the wide row `pair` of that unit over its modes [m0, m1).
struct GradItem {
  int32_t unit, pair, d0, cnt, m0, m1;
};
constexpr int kGradMaxCoef = 48;      // rows up to this length: one item per unit, threads over modes
constexpr int kGradPass = 256;        // samples of a wide row per pass over its modes
constexpr int kGradThreads = 256;     // threads per gradient block
constexpr double kGradItemWork = 16777216.0;  // samples x modes of a wide-row item
constexpr int kGradZBytes = 32768;    // LDS for a wide-row item's correlation: its modes come in chunks of this
constexpr int kGradBlocksPerCU = 3;   // gradient blocks resident per CU (LDS and registers)

// A wide kernel row (more than kGradMaxCoef samples, centred nodes) on a
// power-of-two grid of G longitudes, taken by FFTs instead of sums over
// samples x modes (spline plans: the knot gradient's correlation Y(d) and the
// K_ij(m) tables): S = G / (2 P) real sub-sequences of 2 P points (every
// S-th mode or sample), each one LDS FFT of P complex points.
struct RowFft {
  int32_t unit, pair, P;
  int32_t half;  // gradient rows: 1 for the half-length cosine sum (P = G / 4, one pass)
};
constexpr int64_t kFftRowMinGrid = 512;  // smaller grids: the direct sums
constexpr int64_t kHalfMaxSamplesF32 = 1024;  // FP32 gradient rows of the half-length cosine sum: samples
constexpr int64_t kGradYBytes = int64_t(256) << 20;  // Y buffer of the FFT rows: chunks of at most this
// P of the FFT path for pair q with nc samples, or 0 for the direct sums
int32_t fft_row_points(const arkcos_plan_s* P, int64_t q, int64_t nc);
// the largest P of an FFT row (one workgroup's LDS)
int64_t fft_row_max_points(const arkcos_plan_s* P);
// block size (threads) of an FFT row of P points: 16 points per thread
constexpr int fft_row_threads(int32_t P) { return P <= 4096 ? 256 : (P <= 8192 ? 512 : 1024); }

// One accumulation work item: band `band`, mode tiles [t0, t0 + nt) of
// kAccTile modes each.
struct WorkItem {
  int32_t band, t0, nt, pad;
};

// One queue entry of the batched accumulation: the same for plan `map`.
struct BatchItem {
  int32_t map, band, t0, nt;
};

constexpr int kTilesPerItem = 4;     // mode tiles per accumulation work item
constexpr int kFoldThreads = 256;    // threads sharing the period sums of a short ring's fold (C2R)
// entries of a pair's K_ij(m) table: modes 0..band, zero-padded to whole
// mode tiles so that a tile is read without bounds checks
__host__ __device__ constexpr int32_t table_span(int32_t band) { return (band / kAccTile + 1) * kAccTile; }
constexpr int64_t kAutoTableBytes = int64_t(1) << 30;  // automatic choice: tables for every pair up to this size,
constexpr double kAutoTableShare = 0.8;  // or when the wide rows' tables are at least this share of all

// A band of up to kBandUnits consecutive units: the input rings they need.
struct BandDev {
  int32_t u0, nu;       // units [u0, u0 + nu)
  int32_t jlo, jhi;     // input rings [jlo, jhi]
  int32_t band;         // max band over the units
  int32_t pbeg, npair;  // the units' pairs [pbeg, pbeg + npair) (contiguous)
  int32_t pad;
};

// What sizes the LDS of an accumulation block: the widest input-ring window
// and the most pairs of any band.
struct AccShape {
  int32_t max_window = 0;
  int32_t max_band_pairs = 0;
};


// Rings whose FFTs share one launch: similar LDS needs, so small rings are
// not held to the occupancy of the largest.
struct FftClass {
  int32_t* d_rings = nullptr;
  int32_t count = 0;
  int32_t lds = 0;
  int32_t threads = 256;  // block size: 512 when an FFT is longer than 4096 points
  int32_t mf = 0;         // the FFT length of every ring of the class, if they share one;
                          // -1: a class of mixed-radix rings (FFT_MIXED)
};

}  // namespace arkcos

struct arkcos_plan_s {
  int device = 0;
  arkcos_dtype_t dtype = ARKCOS_F32;
  arkcos_geometry_t geom{};
  int32_t prof_kind = 0;
  double fwhm = 0, theta_max = 0, radius = 0;
  std::vector<double> knots;
  arkcos_options_t opts{};
  int32_t oversample = 1;
  double band_tol = 0;

  int64_t npix = 0, nrings = 0, L = 0;
  int64_t n_units = 0, n_pairs = 0, n_table_pairs = 0;
  int64_t spec_total = 0, out_total = 0, coef_total = 0, table_total = 0, bl_total = 0;
  int64_t pair_modes = 0;
  int32_t max_fft_lds = 0;     // bytes of LDS the ring FFT kernels need
  int32_t max_bl_m = 0;
  int32_t twiddle_n = 0;       // length of the twiddle table (largest power-of-two FFT)
  int32_t max_units_pairs = 0;
  int32_t max_coef_per_unit = 0;

  // host copies
  std::vector<double> h_theta, h_sin, h_cos, h_w;
  std::vector<int32_t> h_n, h_phase_den;
  std::vector<int64_t> h_start;
  std::vector<arkcos::UnitDev> h_units;
  std::vector<arkcos::PairDev> h_pairs;
  std::vector<int32_t> h_pair_i;         // output ring of each pair
  std::vector<int32_t> h_pair_shift;     // half-shift flag per pair
  std::vector<int64_t> h_tab_owner;      // pair whose table a table pair reads (itself, or its transpose)
  std::vector<int64_t> h_coef_off;       // recurrence-coefficient offset per pair
  std::vector<int32_t> h_ncoef_window;   // kernel samples inside each pair's window
  std::vector<arkcos::FftClass> fft_classes;
  std::vector<int32_t> h_ring_lds;       // LDS bytes of each ring's transform
  std::vector<int32_t> h_fft_len;        // its complex FFT length (0: plain DFT)
  std::vector<int32_t> h_fft_kind;       // its FftKind
  std::vector<int32_t> h_spec_len, h_out_len;
  std::vector<int64_t> h_spec_off, h_out_off;

  // device
  arkcos::RingTables rt;
  arkcos::UnitDev* d_units = nullptr;
  arkcos::PairDev* d_pairs = nullptr;
  std::vector<arkcos::WorkItem> h_items;
  arkcos::WorkItem* d_items = nullptr;
  arkcos::BandDev* d_bands = nullptr;
  arkcos::AccShape acc_shape;  // LDS needs of the accumulation bands
  int32_t acc_units = arkcos::kBandUnits;      // units per band (wavefronts per block): 8 or 16
  int32_t acc_tiles = arkcos::kTilesPerItem;   // mode tiles per work item
  int32_t acc_tuned = 0;                       // 1: band shape chosen by timing at plan creation
  int32_t acc_upw = 1;                         // units per wavefront (2: 16-unit bands in 8-wave blocks)
  int32_t acc_ch = 0;                          // input rings staged at a time (0: the dtype's default)
  std::vector<arkcos::BandDev> h_bands;
  bool all_tables = false;     // every pair reads K_ij(m) from a table
  void* d_coef = nullptr;       // recurrence coefficients, plan dtype
  double* d_coef64 = nullptr;   // the same in FP64 (plan-time table building, gradient)
  void* d_table = nullptr;      // K_ij(m) tables, plan dtype
  void* d_bl = nullptr;         // Bluestein filters, complex plan dtype
  void* d_twiddle = nullptr;    // exp(-2 pi i k / twiddle_n), complex plan dtype
  double* d_theta = nullptr;    // ring colatitudes
  double* d_sin = nullptr;
  double* d_cos = nullptr;
  double* d_knots = nullptr;    // spline knot values
  int32_t* d_tab_list = nullptr;  // pairs whose K_ij(m) tables are computed (shared ones once)
  int64_t* d_tab_coef = nullptr;  // their kernel-sample offsets
  int32_t n_tab_list = 0;
  double* d_utable = nullptr;   // kernel_eval = 1: K at nodes uniform in the squared chord
  int32_t utable_n = 0;
  double* d_spline_mom = nullptr;   // spline moments of the current knots
  int32_t* d_pair_i = nullptr;
  int32_t* d_pair_shift = nullptr;
  int64_t* d_coef_off = nullptr;    // recurrence-coefficient offset of every pair
  int32_t* d_ncoef_window = nullptr;  // kernel samples inside each pair's window
  double* d_basis_mom = nullptr;    // spline basis moments S[a][k], n_knots^2
  std::vector<arkcos::GradItem> h_grad_items;  // knot-gradient work items, in unit / pair / sample order
  // wide rows by FFT (spline plans), grouped by block size [256, 512, 1024]:
  // gradient rows (with the offset of each row's Y(d) in its chunk's buffer,
  // the chunk boundaries, and the blocks and slots of the interval sums),
  // and table rows
  arkcos::RowFft* d_gfft = nullptr;
  int64_t* d_gfft_yoff = nullptr;
  std::vector<int32_t> h_gfft_chunk;  // rows [chunk[c], chunk[c + 1]) share the Y buffer in turn
  int64_t grad_y_elems = 0;           // Y buffer: the largest chunk's samples
  int32_t n_gfft[3] = {0, 0, 0}, n_gfft_slots = 0;
  arkcos::RowFft* d_tfft = nullptr;
  int32_t n_tfft[3] = {0, 0, 0};
  arkcos::GradItem* d_grad_items = nullptr;
  int32_t* d_grad_run = nullptr;    // n_grad_runs + 1 item offsets: the items of each gradient block
  int32_t n_grad_runs = 0;
  int32_t grad_zcache_bytes = 0;    // LDS of a gradient block for a wide row's correlation
  int32_t* d_pole_rings = nullptr;  // rings within reach of a pole pixel
  int32_t n_pole_rings = 0;
  size_t plan_bytes = 0;

  std::vector<void*> allocations;

  // stage timing (profiling aid): 5 events per recorded call
  std::vector<hipEvent_t> timing_events;
  int32_t timing_slots = 0, timing_used = 0;
};

namespace arkcos {

void set_error(const std::string& msg);
arkcos_status_t fail(arkcos_status_t st, const std::string& msg);

// Kernel launchers (defined next to their kernels).
hipError_t launch_kernel_rows(arkcos_plan_s* P, double* coef_abs_sum, hipStream_t s);
// new spline knots (device, n_knots doubles) and their clamped-spline moments
hipError_t launch_spline_update(arkcos_plan_s* P, const double* d_src, hipStream_t s);
hipError_t launch_band(arkcos_plan_s* P, double threshold, int32_t* band_out, hipStream_t s);
hipError_t launch_table_list(arkcos_plan_s* P, const int32_t* d_list, const int64_t* d_coef_off,
                             int32_t count, hipStream_t s);
// the K_ij(m) tables of the FFT table rows (spline plans)
hipError_t launch_table_fft(arkcos_plan_s* P, hipStream_t s);
hipError_t configure_fft_kernels(arkcos_plan_s* P);
// batched form
size_t acc_args_size();
// spec_off / spec_len (device, may be null): a spectrum layout to read instead
// of the plan's own (a shared-input batch's union layout, which holds at
// least every mode the plan's pairs read).
void fill_acc_args(arkcos_plan_s* P, const BandDev* bands, void* out, const int64_t* spec_off = nullptr,
                   const int32_t* spec_len = nullptr);
size_t acc_lds_bytes(arkcos_dtype_t dt, const AccShape& shape, int32_t staged_rings = 0);
hipError_t launch_accumulate_batch(arkcos_dtype_t dt, const void* maps, const int64_t* spec_base,
                                   const int64_t* out_base, const BatchItem* items, int32_t n_items,
                                   int32_t* counter, const void* spec, void* bout, int32_t grid,
                                   int32_t units_per_band, bool all_tables, const AccShape& shape, hipStream_t s,
                                   int32_t units_per_wave = 1, int32_t staged_rings = 0);
hipError_t configure_accumulate(arkcos_plan_s* P);
hipError_t configure_accumulate_shape(const arkcos_plan_s* P, const AccShape& shape);
hipError_t launch_accumulate_shape(const arkcos_plan_s* P, const BandDev* bands, const WorkItem* items,
                                   int32_t n_items, int32_t units, const AccShape& shape, const void* spec,
                                   void* bout, hipStream_t s, int32_t units_per_wave = 1, int32_t staged_rings = 0);
size_t ring_args_size();
void fill_ring_args(arkcos_plan_s* P, bool out_side, int32_t adjoint, int32_t zero_pole, void* out,
                    const int64_t* off = nullptr, const int32_t* len = nullptr);
hipError_t launch_ring_batch(arkcos_dtype_t dt, bool inverse, const void* args, const void* entries, int32_t count,
                             int32_t lds, int32_t threads, int32_t mf, const void* maps, void* ws,
                             const int64_t* base, hipStream_t s);
int fft_threads(arkcos_dtype_t dt, int32_t fft_len);
// FFT lengths with compile-time ring kernels (16 points per thread): the
// length itself if fft_len is one of them for the dtype, else 0.  The
// 1024- and 2048-point kernels (64 and 128 threads) pay off only in launches
// of many rings: they are used when `rings` (the rings of that length in
// the launch set) reaches kCtMinRings.
constexpr int64_t kCtMinRings = 8192;
int32_t ct_fft_length(arkcos_dtype_t dt, int32_t fft_len, int64_t rings);

// Clamped cubic spline moments (second derivatives at the knots) for
// equispaced knots with spacing h; end slopes zero.
void spline_moments(const std::vector<double>& c, double h, std::vector<double>& M);
size_t pole_map_size();
void fill_pole_map(arkcos_plan_s* P, void* out);
hipError_t launch_pole_batch(arkcos_dtype_t dt, const void* maps, const int2* entries, int32_t count, int32_t adjoint,
                             const void* xs, const void* ys, hipStream_t s);
void build_bands(const arkcos_plan_s* P, int32_t units_per_band, std::vector<BandDev>& bands, AccShape* shape);
void accumulation_items(const arkcos_plan_s* P, const std::vector<BandDev>& bands, int32_t tiles_per_item,
                        std::vector<WorkItem>& items,
                        std::vector<double>& cost);
int32_t* pole_ring_list(arkcos_plan_s* P, int32_t* count);
void workspace_split(const arkcos_plan_s* P, void* ws, void** spec, void** bout);
double* grad_slots(const arkcos_plan_s* P, void* ws);
void* grad_y(const arkcos_plan_s* P, void* ws);  // Y(d) buffer of the FFT rows
hipError_t launch_r2c_layout(arkcos_plan_s* P, const void* x, void* spec, bool out_layout, int32_t zero_pole,
                             hipStream_t s);
size_t workspace_bytes(const arkcos_plan_s* P);
hipError_t launch_bluestein_filters(arkcos_plan_s* P, const int32_t* d_ring_list, int32_t count,
                                    hipStream_t s);
hipError_t launch_r2c(arkcos_plan_s* P, const void* x, void* spec, int32_t adjoint,
                      int32_t zero_pole_rings, hipStream_t s);
hipError_t launch_accumulate(arkcos_plan_s* P, const void* spec, void* bout, hipStream_t s);
hipError_t launch_c2r(arkcos_plan_s* P, const void* bout, void* y, int32_t adjoint, hipStream_t s);
hipError_t launch_pole_fix(arkcos_plan_s* P, const void* x, void* y, int32_t adjoint, hipStream_t s);

}  // namespace arkcos
