/*
 * arkcos.h -- C ABI of the MI355X (gfx950) implementation of the hybrid
 * Fourier/direct-space convolution of an isolatitude-ring sphere map with a
 * compact radial kernel (Elsner & Wandelt 2011, "ARKCoS").
 *
 * The operation (paper Sect. 2, eq. "def", discretised as in Sect. 3.1,
 * eq. "direct", with pixel areas w_q as quadrature weights):
 *
 *     y_p = sum_{q : theta_pq <= R} K(theta_pq) x_q w_q
 *
 * computed by the hybrid algorithm of Sect. 4.1 with the artifact suppression
 * of Sect. 4.3:
 *   (a) a real FFT of every input ring, phase-shifted to absolute longitude
 *       (eq. "fftrot") and periodically extended past the ring's Nyquist mode;
 *   (b) for every output ring i and input ring j inside the support, the
 *       azimuthal Fourier coefficients K_ij(m) of the kernel sampled at the
 *       angular distance theta(i, j, dphi) (eq. "kernel_angle"; the distance
 *       is evaluated in FP64 haversine form);
 *   (c) B_i(m) = sum_j K_ij(m) A_j(m);
 *   (d) reverse phase shift, aliasing of super-Nyquist modes onto the ring's
 *       own modes, inverse real FFT per output ring; on HEALPix the 8 pixels
 *       of the first and last ring are then recomputed by the direct sum
 *       (Sect. 4.2).
 * Equatorial HEALPix rings of equal length are paired without the phase
 * shift, with the kernel sampled at the true pixel offsets (Sect. 4.3); this
 * makes them exact.  Pairs involving a polar ring sample the kernel on
 * `oversample * 4 nside` longitudes instead of 4 nside.
 * The option `mode = 1` selects the paper's plain algorithm of Sect. 4.1
 * instead: every pair on the `oversample * 4 nside` grid, each ring's
 * spectrum zero-padded past its Nyquist mode in (a), and in (d) only the
 * output ring's modes |m| <= N_i / 2 kept (truncation instead of aliasing).
 *
 * Conventions shared by every entry point:
 *   - Maps are device buffers in RING order: HEALPix with npix = 12 nside^2,
 *     or ECP with npix = n_theta * n_phi (ring-major, theta_i = (i+1/2) pi /
 *     n_theta, phi_k = 2 pi k / n_phi).  The element type is the plan's dtype
 *     (float or double).  The caller owns every map, workspace and gradient
 *     buffer.
 *   - A plan owns only read-only device tables created by arkcos_plan on the
 *     device that is current at that call; every later call must run with the
 *     same device current.
 *   - Calls taking a stream only enqueue work on it and never synchronise the
 *     host; they allocate nothing.  Two calls that may overlap in time need
 *     separate workspaces.
 *   - Errors are returned as status codes; no call aborts or throws.  Host-side
 *     argument checks run before any work is enqueued; a non-OK status means
 *     nothing was enqueued.  arkcos_last_error() gives a message for the
 *     calling thread.
 */
#ifndef ARKCOS_H
#define ARKCOS_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arkcos_plan_s* arkcos_plan_t;
typedef struct arkcos_batch_s* arkcos_batch_t;

typedef enum {
  ARKCOS_OK = 0,
  ARKCOS_ERR_INVALID_VALUE = 1, /* bad argument: null pointer, size, aliasing */
  ARKCOS_ERR_NOT_SUPPORTED = 2, /* valid but outside what the library handles */
  ARKCOS_ERR_OUT_OF_MEMORY = 3, /* device allocation failed (plan creation) */
  ARKCOS_ERR_DEVICE = 4,        /* a HIP runtime call or launch failed */
  ARKCOS_ERR_INTERNAL = 5
} arkcos_status_t;

typedef enum { ARKCOS_F32 = 0, ARKCOS_F64 = 1 } arkcos_dtype_t;

/* Pixelisation (paper Sect. 4.1 for HEALPix; any isolatitude-ring grid with
 * equal ring lengths works as ECP). */
typedef struct {
  int32_t kind;     /* 0 = ECP, 1 = HEALPix (RING order) */
  int64_t nside;    /* HEALPix: 1 .. 8192 */
  int64_t n_theta;  /* ECP: number of rings */
  int64_t n_phi;    /* ECP: pixels per ring, even */
} arkcos_geometry_t;

/* Radial kernel profile K(theta), truncated at the support radius (Sect. 4). */
typedef struct {
  int32_t kind;             /* 0 = Gaussian exp(-theta^2 / 2 sigma^2), sigma = FWHM / sqrt(8 ln 2);
                               1 = clamped cubic spline through knot values at
                                   theta_k = k theta_max / (n_knots - 1), zero beyond theta_max */
  double fwhm_rad;          /* Gaussian */
  int32_t n_knots;          /* spline: 3 .. 64 */
  double theta_max_rad;     /* spline */
  const double* knot_values;/* spline: host array of n_knots values, copied by arkcos_plan */
} arkcos_profile_t;

typedef struct {
  int32_t oversample;       /* kernel grid refinement p for pairs involving a polar
                               ring: 1, 2, 4, 8 or 16; 0 = choose from the kernel's
                               width (p = next power of two >= 4.3 pixel / FWHM) */
  int32_t kgen;             /* how K_ij(m) is produced per call: 0 = automatic
                               (precomputed tables for every pair if they take at
                               most 1 GiB or if the wide pairs' tables, needed in
                               any case, hold at least 80 % of the entries,
                               otherwise the recurrence from the kernel samples
                               for narrow pairs and tables for wide ones),
                               1 = recurrence for every pair (wide rows still use
                               tables), 2 = precomputed table for every pair */
  int32_t fix_pole_pixels;  /* HEALPix: recompute the 8 pixels of the first and last
                               ring by the direct sum (default 1) */
  double band_tol;          /* Gaussian plans: modes with |K_ij(m)| below band_tol
                               times the largest kernel-row magnitude are dropped;
                               < 0 = default (1e-9 for F32, 0 for F64).  Spline
                               plans keep every mode up to each grid's Nyquist mode
                               and every kernel sample of a pair's window, so that
                               any later knot values fit the plan's layout */
  int32_t mode;             /* 0 = with the artifact suppression of Sect. 4.3
                               (default); 1 = the plain algorithm of Sect. 4.1
                               (zero-padded spectra, truncated output modes, no
                               pair on its own grid), for comparisons of the
                               two; on ECP grids both give the same result */
  int32_t own_grid;         /* mode 0: which ring pairs skip the phase shift and
                               sample the kernel at the true pixel offsets on a grid
                               of their own length (exact, like the direct sum).
                               0 = every pair of equal-length rings: the equatorial
                               pairs plus a polar ring with itself and with its
                               mirror (an extension of Sect. 4.3; default);
                               1 = equatorial pairs only, the scheme as Sect. 4.3
                               states it (with oversample = 1 the paper's method) */
  int32_t kernel_eval;      /* how the plan evaluates K at each kernel sample:
                               0 = K(theta) in FP64 from the haversine distance
                               (default); 1 = linear interpolation in the squared
                               chord u = 2(1 - cos theta) from a table of
                               K(2 asin(sqrt(u)/2)) (the biased table of Sect. 4.1,
                               eq. "kernel_angle"), nodes uniform in u over [0, u(R)] */
  int32_t table_nodes;      /* kernel_eval 1: nodes of that table, 2 .. 2^24;
                               0 = 65536 */
  int32_t reserved[4];      /* must be 0 */
} arkcos_options_t;

/* Summary of a plan (sizes, chosen parameters), for callers and tooling. */
typedef struct {
  int64_t npix, nrings, n_pairs, n_table_pairs;
  int64_t spectrum_modes;   /* complex coefficients held for the input rings */
  int64_t output_modes;     /* complex coefficients accumulated for the output rings */
  int64_t pair_modes;       /* sum over ring pairs of the modes accumulated */
  int64_t taps;             /* kernel samples held for the recurrence */
  int64_t table_entries;    /* precomputed K_ij(m) values (each pair's table
                               zero-padded to a multiple of 256 modes) */
  int32_t oversample, dtype, n_knots;
  int32_t reserved;
  size_t workspace_bytes, plan_bytes;
  int64_t pairs_by_kind[4]; /* ring pairs (north units) by how K_ij(m) is produced:
                               [0] Clenshaw recurrence on the centred grid,
                               [1] Clenshaw on the half-shifted own grid,
                               [2] precomputed table, [3] Reinsch's recurrence */
  int32_t acc_seg_units;    /* accumulation: output units (rings with their mirrors) per work
                               item, one wavefront each: 8 or 16 */
  int32_t acc_group;        /* mode tiles (256 modes each) per work item */
  int32_t acc_window;       /* widest input-ring window of a work item's units */
  int32_t acc_tuned;        /* 1: shape chosen by timing at plan creation, 0: fixed */
  double support_radius_rad; /* R of the plan (given, or chosen by arkcos_plan_for_error) */
  int32_t table_fft_rows;   /* spline plans: K_ij(m) tables computed by FFTs of the
                               kernel samples (wide rows on power-of-two grids) */
  int32_t grad_fft_rows;    /* spline plans: kernel rows whose knot-gradient
                               correlation is transformed by FFTs */
  int32_t acc_units_per_wave; /* accumulation: output units per wavefront (1; 2 or 3
                               for FP32 plans whose pairs all have tables, with
                               acc_seg_units = 8 x this) */
  int32_t reserved2;        /* 0 */
} arkcos_plan_info_t;

/* Fill *opts with the defaults (oversample 0, kgen 0, fix_pole_pixels 1,
 * band_tol -1, mode 0, own_grid 0, kernel_eval 0, table_nodes 0). */
void arkcos_default_options(arkcos_options_t* opts);

/* Build a plan on the current device: ring and pair tables, the FP64 kernel
 * samples of every ring pair (step b), bands and optional K_ij(m) tables.
 * support_radius_rad: R in (0, pi).  opts may be NULL (defaults).  Blocks the
 * host until the device tables are ready.  *out is set only on success.
 * Environment (tuning and test switches; none changes a result beyond
 * rounding): ARKCOS_ACC_SHAPE="U,T[,W[,C]]" fixes the accumulation's shape
 * (units per band, mode tiles per item, units per wavefront, staged rings)
 * instead of timing the candidates, ARKCOS_ACC_TIMES=1 prints the candidates'
 * times, ARKCOS_GRAD_CHUNK_BYTES sets the knot gradient's Y-buffer chunk,
 * ARKCOS_GRAD_HALF=0 keeps every FFT row of the knot gradient on the S-pass
 * form, ARKCOS_PLAN_STATS=1 prints the plan's (pair, mode) counts. */
arkcos_status_t arkcos_plan(const arkcos_geometry_t* geom, const arkcos_profile_t* profile,
                            double support_radius_rad, arkcos_dtype_t dtype,
                            const arkcos_options_t* opts, arkcos_plan_t* out);

/* arkcos_plan with the support radius chosen from a bound on the truncation
 * error instead of given (paper Sect. 4: the error of cutting the kernel at
 * R, sigma^2(R) below, is what fixes R).  R is the radius
 * arkcos_choose_radius(profile, cl, lmax, target_sigma2) returns: the
 * smallest radius whose truncation variance for the power spectrum cl[0..lmax]
 * (host array) is at most target_sigma2.  The plan is then built exactly as
 * arkcos_plan(geom, profile, R, dtype, opts) builds it.  radius_rad (host,
 * may be NULL) receives R.  Errors: those of the two calls; and
 * ARKCOS_ERR_NOT_SUPPORTED when the target holds without any support (R = 0),
 * since an empty kernel needs no plan.  Blocks the host like arkcos_plan. */
arkcos_status_t arkcos_plan_for_error(const arkcos_geometry_t* geom, const arkcos_profile_t* profile,
                                      const double* cl, int32_t lmax, double target_sigma2,
                                      arkcos_dtype_t dtype, const arkcos_options_t* opts,
                                      arkcos_plan_t* out, double* radius_rad);

arkcos_status_t arkcos_plan_destroy(arkcos_plan_t plan);
arkcos_status_t arkcos_plan_get_info(arkcos_plan_t plan, arkcos_plan_info_t* info);

/* Bytes of device workspace a convolve / adjoint / kernel_grad call needs
 * (256-byte aligned base required). */
arkcos_status_t arkcos_workspace_size(arkcos_plan_t plan, size_t* bytes);

/* y = C x (steps a-d).  x, y: device, npix elements of the plan's dtype; they
 * must not overlap.  ws: device workspace of arkcos_workspace_size bytes.  On
 * return of the enqueued work the workspace holds the extended spectra of x,
 * which arkcos_kernel_grad can reuse. */
arkcos_status_t arkcos_convolve(arkcos_plan_t plan, const void* x, void* y, void* ws,
                                hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): y = C x exactly as
 * arkcos_convolve computes it (same kernels, same order, the same bits), with
 * the workspace taken from a fixed device array inside the library
 * (arkcos_noalloc_scratch_bytes() bytes, 64 MiB, per device, held until the
 * process ends) instead of a caller's buffer.  No allocation of any kind.
 * Plans whose arkcos_workspace_size exceeds the array are rejected with
 * ARKCOS_ERR_NOT_SUPPORTED before any work is enqueued.  Every call on one
 * device shares that device's array: calls that may overlap in time on one
 * device race (serialise them, e.g. on one stream).  x, y as for
 * arkcos_convolve. */
arkcos_status_t arkcos_convolve_noalloc(arkcos_plan_t plan, const void* x, void* y, hipStream_t stream);
size_t arkcos_noalloc_scratch_bytes(void);

/* xbar = C^T r, the exact transpose of arkcos_convolve as a linear map: the
 * same ring pipeline with the roles of the ring pairs swapped, K_ji and the
 * pixel weights, i.e. xbar = w * C(r / w); the direct-sum pole rows transpose
 * into direct-sum columns.  On HEALPix (equal weights) the ring part equals
 * the forward map. */
arkcos_status_t arkcos_convolve_adjoint(arkcos_plan_t plan, const void* r, void* xbar, void* ws,
                                        hipStream_t stream);

/* Gradient of L = 1/2 |C x - t|^2 with respect to the spline knot values,
 * given r = C x - t:  g_k = <r, (dC/dc_k) x>, a per-ring-pair Fourier-space
 * correlation of the spectra of r and x reduced over modes and kernel samples
 * in FP64.  grad: device, n_knots doubles, overwritten.  Spline plans with
 * kernel_eval 0 only (ARKCOS_ERR_NOT_SUPPORTED otherwise).
 * flags bit 0: the workspace still holds the spectra of x from the last
 * arkcos_convolve(x) on it (skips their recomputation). */
arkcos_status_t arkcos_kernel_grad(arkcos_plan_t plan, const void* x, const void* r,
                                   double* grad, void* ws, uint32_t flags, hipStream_t stream);

/* Replace the spline knot values (host array of n_knots doubles) and rebuild
 * the kernel samples and K_ij(m) tables in place, with the plan's layout
 * (ring pairs, sample windows, bands, table choices are fixed at plan
 * creation and hold for any knot values).  Waits for all work on the device
 * first and returns once the new tables are ready. */
arkcos_status_t arkcos_set_knots(arkcos_plan_t plan, const double* knot_values);

/* The same with the knot values in device memory (n_knots doubles), enqueued
 * on `stream`: a few kernels, no allocation and no host synchronisation, so
 * it can be captured in a graph.  Calls on other streams that use the plan
 * must be ordered against it by the caller. */
arkcos_status_t arkcos_set_knots_async(arkcos_plan_t plan, const double* knot_values, hipStream_t stream);

/* ---- batched form: many maps of uneven size, each with its own plan ---- */

typedef struct {
  int32_t n_maps;
  int32_t seg_units;        /* output units (rings with mirrors) per work item, autotuned */
  int32_t group;            /* wavefronts per workgroup of the accumulation, autotuned */
  int32_t grid;             /* workgroups of the persistent accumulation launch, autotuned */
  int32_t tuned;            /* 1: measured now, 2: read from the autotune cache */
  int32_t units_per_wave;   /* output units per wavefront (1, or 2 for table-only FP32
                               batches: group = seg_units / 2) */
  int64_t n_items;          /* work items in the queue */
  int64_t npix_total;
  size_t workspace_bytes;
} arkcos_batch_info_t;

/* Group n plans (same dtype, same device) into one batch: one work queue of
 * (map, segment of output rings, mode tile) items over all maps, ordered
 * heaviest first.  The segment length, the rings summed at a time and the
 * persistent grid are chosen by an autotuner that times the accumulation on
 * a representative subset of the maps (results cached in the file named by
 * ARKCOS_AUTOTUNE_CACHE, if set).  Blocks the host.  The plans must outlive
 * the batch. */
arkcos_status_t arkcos_batch_plan(int32_t n, const arkcos_plan_t* plans, arkcos_batch_t* out);
arkcos_status_t arkcos_batch_get_info(arkcos_batch_t batch, arkcos_batch_info_t* info);
arkcos_status_t arkcos_batch_workspace_size(arkcos_batch_t batch, size_t* bytes);
/* Forward (adjoint = 0) or transpose (adjoint = 1) of every map i:
 * y[i] = C_i x[i].  x, y: host arrays of n device pointers (maps as for
 * arkcos_convolve; no x[i] may overlap any y[k]).  ws: arkcos_batch_workspace_size
 * bytes, 256-byte aligned.  Ring transforms run batched over all rings of all
 * maps; one persistent launch performs step (c) for every map.  The call's
 * map pointers are written into its workspace by kernels on the stream, so
 * the call only enqueues kernels, allocates nothing, never waits on the host
 * and can be captured in a hipGraph (several calls with different maps, e.g.
 * a forward and a transpose, in one graph). */
arkcos_status_t arkcos_batch_convolve(arkcos_batch_t batch, const void* const* x, void* const* y,
                                      int32_t adjoint, void* ws, hipStream_t stream);
/* Shared-input form: one map convolved with n kernels on one geometry,
 * y[i] = C_i x.  This is how an asymmetric beam is applied when it is split
 * into a few symmetric kernels (paper Sect. 5, on the ASYMFAST approach):
 * the input's extended spectra (step a) are computed once and every kernel's
 * ring-pair accumulation (steps b, c) reads them; the accumulation runs as
 * one persistent launch over all kernels and the inverse transforms (step d)
 * batched over them.  The plans must share dtype, device, geometry and
 * fix_pole_pixels (kernels, radii, oversampling and the other options may
 * differ).  Each y[i] equals arkcos_convolve of plan i on x bit for bit.
 * Created like arkcos_batch_plan (autotuned, blocks the host); its workspace
 * holds one set of input spectra.  The batch is used with
 * arkcos_batch_convolve_shared only (arkcos_batch_convolve rejects it).
 * x: device, the one input map; y: host array of n device pointers; no y[i]
 * may overlap x.  Forward only: the transpose of the stacked map is the sum
 * of the per-kernel transposes, available through an ordinary batch. */
arkcos_status_t arkcos_batch_plan_shared_input(int32_t n, const arkcos_plan_t* plans, arkcos_batch_t* out);
arkcos_status_t arkcos_batch_convolve_shared(arkcos_batch_t batch, const void* x, void* const* y, void* ws,
                                             hipStream_t stream);
/* Stage timing of batch calls, as arkcos_plan_timing / arkcos_stage_times
 * (stage 1 is the persistent accumulation launch). */
arkcos_status_t arkcos_batch_timing(arkcos_batch_t batch, int32_t max_calls);
arkcos_status_t arkcos_batch_stage_times(arkcos_batch_t batch, double* ms, int64_t* calls);
arkcos_status_t arkcos_batch_destroy(arkcos_batch_t batch);

/* ---- profiling aid ---- */

/* Stage timing: with max_calls > 0, the next max_calls convolve / adjoint
 * calls on this plan record HIP events on their own stream around each of
 * their kernels: stage 0 ring R2C (step a), 1 ring-pair accumulation (steps b
 * and c), 2 fold + C2R (step d), 3 pole-ring direct sum.  The events are
 * created here (this call allocates); max_calls = 0 releases them.  Must not
 * overlap with calls using the plan. */
arkcos_status_t arkcos_plan_timing(arkcos_plan_t plan, int32_t max_calls);
/* Milliseconds per stage summed over the calls recorded since the last
 * arkcos_plan_timing / arkcos_stage_times (ms: 4 doubles), and their count.
 * Waits for the recorded events; then starts a new recording window. */
arkcos_status_t arkcos_stage_times(arkcos_plan_t plan, double* ms, int64_t* calls);

/* ---------------------------------------------------------------------------
 * Support radius from the truncation error (paper Sect. 4).  Host-only: these
 * two calls touch no device and may run without a GPU.
 *
 * Cutting the kernel at radius R changes its Legendre coefficients
 * (K_l = 2 pi int_{-1}^{1} K(z) P_l(z) dz, Sect. 2) by
 *     dK_l(R) = -2 pi int_R^pi K(theta) P_l(cos theta) sin theta dtheta,
 * and for a signal with angular power spectrum C_l the convolved map then
 * has an error of variance
 *     sigma^2(R) = sum_{l=0}^{lmax} (2l + 1) / (4 pi) dK_l(R)^2 C_l.
 * The Gaussian is taken as zero beyond 40 sigma, the spline beyond
 * theta_max.  Quadrature: 16-point Gauss-Legendre panels in theta with at
 * least eight nodes per period of P_lmax.
 *
 * arkcos_truncation_variance: profile as for arkcos_plan; radius_rad in
 * [0, pi]; cl: host array of lmax + 1 values (lmax 0 .. 1e6); *sigma2
 * receives sigma^2(R); dk: optional host array of lmax + 1 values that
 * receives dK_l(R) (may be NULL).
 *
 * arkcos_choose_radius: the smallest radius, to 1e-12 of the support, whose
 * sigma^2 is at most target_sigma2, searched from the end of the support
 * inwards on 256 radii then refined by bisection (so the answer also holds
 * for kernels whose sigma^2 is not monotone in R); 0 if no radius exceeds
 * the target.  Errors: ARKCOS_ERR_INVALID_VALUE for bad arguments. */
arkcos_status_t arkcos_truncation_variance(const arkcos_profile_t* profile, double radius_rad, const double* cl,
                                           int32_t lmax, double* sigma2, double* dk);
arkcos_status_t arkcos_choose_radius(const arkcos_profile_t* profile, const double* cl, int32_t lmax,
                                     double target_sigma2, double* radius_rad);

const char* arkcos_status_string(arkcos_status_t status);
/* Message describing the last failure on the calling thread ("" if none). */
const char* arkcos_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ARKCOS_H */
