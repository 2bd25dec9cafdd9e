/*
 * FP64 brute-force oracle for radial-kernel convolution on isolatitude-ring
 * sphere grids.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the product path never does.  It
 * shares no code with the HIP library: geometry, kernel profiles and the
 * spline are written out again here from their definitions.
 *
 * What it computes (paper Sect. 2, eq. "def", discretised as in Sect. 3.1,
 * eq. "direct", with the pixel area w_q added as the quadrature weight):
 *
 *     y_p = sum_{q : theta_pq <= R} K(theta_pq) x_q w_q
 *
 * theta_pq = atan2(|n_p x n_q|, n_p . n_q) from 3-D unit vectors, which is
 * well conditioned at every angle.  A pair is inside the support when
 * theta_pq <= R + 1e-9 rad (the same tolerance the HIP path uses; it only
 * matters for exact ties, which the ECP grid has).
 *
 * Also:
 *   adjoint   xbar_q = w_q sum_p K(theta_pq) r_p           (explicit transpose)
 *   gradient  g_k    = sum_p r_p sum_q phi_k(theta_pq) x_q w_q
 *             for a spline kernel K = sum_k c_k phi_k (phi_k the cardinal
 *             clamped cubic spline through the unit vector e_k).
 * Every function can work on a subset of output pixels ("sampled mode").
 *
 * Grids:
 *   ECP      theta_i = (i + 1/2) pi / ntheta, phi_k = 2 pi k / nphi,
 *            w_i = (2 pi / nphi)(cos(i pi/ntheta) - cos((i+1) pi/ntheta)).
 *   HEALPix  RING order after Gorski et al. (2005): rings r = 1 .. 4 nside - 1;
 *            polar rings hold 4r pixels at phi = (k + 1/2) pi / (2r) and
 *            z = 1 - r^2 / (3 nside^2); equatorial rings hold 4 nside pixels
 *            at phi = (k + s/2) pi / (2 nside), s = (r - nside + 1) mod 2,
 *            z = 4/3 - 2r / (3 nside); the south cap mirrors the north.
 *            All pixels have area 4 pi / (12 nside^2).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SUPPORT_TOL 1e-9
#define SEARCH_MARGIN 1e-6

typedef struct {
  int64_t nrings, npix;
  double *theta, *phi0, *w;
  int64_t *n, *start;
} Grid;

typedef struct {
  int kind; /* 0 Gaussian, 1 spline */
  double sigma;
  int nk;
  double h, theta_max;
  const double *c; /* knot values */
  double *mom;     /* second-derivative moments of the spline through c */
  double *basis_mom; /* nk x nk: column k = moments of the spline through e_k */
  double radius;
} Profile;

/* ---------------------------------------------------------------- grids */

static int grid_build(int kind, int64_t nside, int64_t ntheta, int64_t nphi, Grid *g) {
  if (kind == 0) {
    if (ntheta < 1 || nphi < 1) return -1;
    g->nrings = ntheta;
    g->npix = ntheta * nphi;
  } else {
    if (nside < 1) return -1;
    g->nrings = 4 * nside - 1;
    g->npix = 12 * nside * nside;
  }
  int64_t nr = g->nrings;
  g->theta = malloc(sizeof(double) * nr);
  g->phi0 = malloc(sizeof(double) * nr);
  g->w = malloc(sizeof(double) * nr);
  g->n = malloc(sizeof(int64_t) * nr);
  g->start = malloc(sizeof(int64_t) * nr);
  if (kind == 0) {
    for (int64_t i = 0; i < nr; ++i) {
      double a = M_PI * i / ntheta, b = M_PI * (i + 1) / ntheta;
      g->theta[i] = M_PI * (i + 0.5) / ntheta;
      g->phi0[i] = 0.0;
      /* cos a - cos b = 2 sin((a+b)/2) sin((b-a)/2) */
      g->w[i] = (2.0 * M_PI / nphi) * 2.0 * sin(0.5 * (a + b)) * sin(0.5 * (b - a));
      g->n[i] = nphi;
      g->start[i] = i * nphi;
    }
  } else {
    double area = 4.0 * M_PI / (double)g->npix;
    for (int64_t k = 0; k < nr; ++k) {
      int64_t r = k + 1; /* ring number counted from the north pole */
      g->w[k] = area;
      if (r < nside) {
        g->theta[k] = 2.0 * asin(r / (sqrt(6.0) * nside));
        g->n[k] = 4 * r;
        g->phi0[k] = M_PI / (4.0 * r);
        g->start[k] = 2 * r * (r - 1);
      } else if (r <= 3 * nside) {
        double z = 4.0 / 3.0 - 2.0 * r / (3.0 * nside);
        g->theta[k] = acos(z);
        g->n[k] = 4 * nside;
        g->phi0[k] = ((r - nside + 1) % 2) * M_PI / (4.0 * nside);
        g->start[k] = 2 * nside * (nside - 1) + 4 * nside * (r - nside);
      } else {
        int64_t s = 4 * nside - r; /* ring number counted from the south pole */
        g->theta[k] = M_PI - 2.0 * asin(s / (sqrt(6.0) * nside));
        g->n[k] = 4 * s;
        g->phi0[k] = M_PI / (4.0 * s);
        g->start[k] = g->npix - 2 * s * (s + 1);
      }
    }
  }
  return 0;
}

static void grid_free(Grid *g) {
  free(g->theta); free(g->phi0); free(g->w); free(g->n); free(g->start);
}

static int64_t ring_of(const Grid *g, int64_t pix) {
  int64_t lo = 0, hi = g->nrings - 1;
  while (lo < hi) { /* last ring whose start <= pix */
    int64_t mid = (lo + hi + 1) / 2;
    if (g->start[mid] <= pix) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* ------------------------------------------------------------- profiles */

/* Clamped cubic spline on equispaced knots, in the moment form: on
 * [t_a, t_a+1] with u = (t - t_a)/h,
 *   S = (1-u) c_a + u c_a+1 + h^2/6 [((1-u)^3-(1-u)) M_a + (u^3-u) M_a+1],
 * interior rows  M_k-1 + 4 M_k + M_k+1 = 6 (c_k+1 - 2 c_k + c_k-1) / h^2,
 * clamped ends   2 M_0 + M_1 = 6 (c_1 - c_0) / h^2,
 *                M_n-2 + 2 M_n-1 = -6 (c_n-1 - c_n-2) / h^2. */
static void spline_moments(int n, double h, const double *c, double *M) {
  double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
  double *cc = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
  double s = 6.0 / (h * h);
  for (int k = 0; k < n; ++k) {
    if (k == 0) { a[k] = 0; b[k] = 2; cc[k] = 1; d[k] = s * (c[1] - c[0]); }
    else if (k == n - 1) { a[k] = 1; b[k] = 2; cc[k] = 0; d[k] = -s * (c[n - 1] - c[n - 2]); }
    else { a[k] = 1; b[k] = 4; cc[k] = 1; d[k] = s * (c[k + 1] - 2 * c[k] + c[k - 1]); }
  }
  /* Thomas algorithm */
  for (int k = 1; k < n; ++k) {
    double m = a[k] / b[k - 1];
    b[k] -= m * cc[k - 1];
    d[k] -= m * d[k - 1];
  }
  M[n - 1] = d[n - 1] / b[n - 1];
  for (int k = n - 2; k >= 0; --k) M[k] = (d[k] - cc[k] * M[k + 1]) / b[k];
  free(a); free(b); free(cc); free(d);
}

static int profile_build(int kind, double fwhm, int nk, double theta_max, const double *knots,
                         double radius, Profile *p) {
  memset(p, 0, sizeof(*p));
  p->kind = kind;
  p->radius = radius;
  if (kind == 0) {
    if (!(fwhm > 0)) return -1;
    p->sigma = fwhm / sqrt(8.0 * log(2.0));
    return 0;
  }
  if (nk < 3 || !(theta_max > 0) || !knots) return -1;
  p->nk = nk;
  p->theta_max = theta_max;
  p->h = theta_max / (nk - 1);
  p->c = knots;
  p->mom = malloc(sizeof(double) * nk);
  spline_moments(nk, p->h, knots, p->mom);
  p->basis_mom = malloc(sizeof(double) * nk * nk);
  double *e = calloc(nk, sizeof(double)), *m = malloc(sizeof(double) * nk);
  for (int k = 0; k < nk; ++k) {
    e[k] = 1.0;
    spline_moments(nk, p->h, e, m);
    for (int j = 0; j < nk; ++j) p->basis_mom[j * nk + k] = m[j];
    e[k] = 0.0;
  }
  free(e); free(m);
  return 0;
}

static void profile_free(Profile *p) { free(p->mom); free(p->basis_mom); }

static inline void spline_locate(const Profile *p, double t, int *a, double *u) {
  int ia = (int)floor(t / p->h);
  if (ia < 0) ia = 0;
  if (ia > p->nk - 2) ia = p->nk - 2;
  *a = ia;
  *u = t / p->h - ia;
}

/* K(t) including the truncation at the support radius. */
static inline double kernel_eval(const Profile *p, double t) {
  if (t > p->radius + SUPPORT_TOL) return 0.0;
  if (p->kind == 0) return exp(-t * t / (2.0 * p->sigma * p->sigma));
  if (t > p->theta_max + SUPPORT_TOL) return 0.0;
  int a; double u;
  spline_locate(p, t, &a, &u);
  double v = 1.0 - u, h2 = p->h * p->h / 6.0;
  return v * p->c[a] + u * p->c[a + 1] + h2 * ((v * v * v - v) * p->mom[a] + (u * u * u - u) * p->mom[a + 1]);
}

/* phi_k(t) for all k, added with weight s into acc[0..nk). */
static inline void basis_accumulate(const Profile *p, double t, double s, double *acc) {
  if (t > p->radius + SUPPORT_TOL || t > p->theta_max + SUPPORT_TOL) return;
  int a; double u;
  spline_locate(p, t, &a, &u);
  double v = 1.0 - u, h2 = p->h * p->h / 6.0;
  double ca = h2 * (v * v * v - v), cb = h2 * (u * u * u - u);
  const double *ma = p->basis_mom + (int64_t)a * p->nk, *mb = p->basis_mom + (int64_t)(a + 1) * p->nk;
  for (int k = 0; k < p->nk; ++k) acc[k] += s * (ca * ma[k] + cb * mb[k]);
  acc[a] += s * v;
  acc[a + 1] += s * u;
}

/* --------------------------------------------------------- neighbourhood */

typedef struct {
  double st, ct, sp, cp; /* sin/cos theta, sin/cos phi */
} Dir;

static inline Dir dir_of(double theta, double phi) {
  Dir d;
  d.st = sin(theta); d.ct = cos(theta); d.sp = sin(phi); d.cp = cos(phi);
  return d;
}

static inline double angle_between(Dir a, Dir b) {
  double ax = a.st * a.cp, ay = a.st * a.sp, az = a.ct;
  double bx = b.st * b.cp, by = b.st * b.sp, bz = b.ct;
  double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
  return atan2(sqrt(cx * cx + cy * cy + cz * cz), ax * bx + ay * by + az * bz);
}

/* Visit every pixel q within the support of the direction (theta_p, phi_p).
 * The candidate set is generous (rings within R + margin, a phi window widened
 * by one pixel on each side); the exact angle decides. */
#define FOR_EACH_NEIGHBOUR(G, PROF, THP, PHP, BODY)                                        \
  do {                                                                                     \
    double _R = (PROF)->radius;                                                            \
    Dir _dp = dir_of((THP), (PHP));                                                        \
    double _cR = cos(_R + SEARCH_MARGIN);                                                  \
    for (int64_t _j = 0; _j < (G)->nrings; ++_j) {                                         \
      double _thj = (G)->theta[_j];                                                        \
      if (fabs(_thj - (THP)) > _R + SEARCH_MARGIN) continue;                               \
      int64_t _nj = (G)->n[_j];                                                            \
      double _stj = sin(_thj), _ctj = cos(_thj);                                           \
      double _den = _dp.st * _stj;                                                         \
      int64_t _k0 = 0, _cnt = _nj;                                                         \
      if (_den > 1e-300) {                                                                 \
        double _c = (_cR - _dp.ct * _ctj) / _den;                                          \
        if (_c > -1.0) {                                                                   \
          double _dphi = acos(_c > 1.0 ? 1.0 : _c);                                        \
          double _dk = 2.0 * M_PI / _nj;                                                   \
          int64_t _lo = (int64_t)floor(((PHP) - _dphi - (G)->phi0[_j]) / _dk) - 1;         \
          int64_t _hi = (int64_t)ceil(((PHP) + _dphi - (G)->phi0[_j]) / _dk) + 1;          \
          if (_hi - _lo + 1 < _nj) { _k0 = _lo; _cnt = _hi - _lo + 1; }                    \
        }                                                                                  \
      }                                                                                    \
      for (int64_t _t = 0; _t < _cnt; ++_t) {                                              \
        int64_t _k = ((_k0 + _t) % _nj + _nj) % _nj;                                       \
        double _phq = (G)->phi0[_j] + 2.0 * M_PI * _k / _nj;                               \
        double _ang = angle_between(_dp, dir_of(_thj, _phq));                              \
        if (_ang > _R + SUPPORT_TOL) continue;                                             \
        int64_t q_index = (G)->start[_j] + _k;                                             \
        int64_t q_ring = _j;                                                               \
        double q_angle = _ang;                                                             \
        (void)q_ring;                                                                      \
        BODY                                                                               \
      }                                                                                    \
    }                                                                                      \
  } while (0)

static void pixel_dir(const Grid *g, int64_t pix, double *theta, double *phi, int64_t *ring) {
  int64_t i = ring_of(g, pix);
  *ring = i;
  *theta = g->theta[i];
  *phi = g->phi0[i] + 2.0 * M_PI * (pix - g->start[i]) / g->n[i];
}

/* ------------------------------------------------------------- exports */

int64_t oracle_npix(int kind, int64_t nside, int64_t ntheta, int64_t nphi) {
  return kind == 0 ? ntheta * nphi : 12 * nside * nside;
}

/* Ring table: theta, phi0, weight, pixel count and first pixel of each ring. */
int oracle_rings(int kind, int64_t nside, int64_t ntheta, int64_t nphi, double *theta,
                 double *phi0, double *w, int64_t *n, int64_t *start) {
  Grid g;
  if (grid_build(kind, nside, ntheta, nphi, &g)) return -1;
  memcpy(theta, g.theta, sizeof(double) * g.nrings);
  memcpy(phi0, g.phi0, sizeof(double) * g.nrings);
  memcpy(w, g.w, sizeof(double) * g.nrings);
  memcpy(n, g.n, sizeof(int64_t) * g.nrings);
  memcpy(start, g.start, sizeof(int64_t) * g.nrings);
  grid_free(&g);
  return 0;
}

/* K(theta) for a vector of angles (truncation included). */
int oracle_kernel(int pkind, double fwhm, int nk, double theta_max, const double *knots,
                  double radius, const double *t, double *out, int64_t n) {
  Profile p;
  if (profile_build(pkind, fwhm, nk, theta_max, knots, radius, &p)) return -1;
  for (int64_t i = 0; i < n; ++i) out[i] = kernel_eval(&p, t[i]);
  profile_free(&p);
  return 0;
}

/* phi_k(theta) for a vector of angles: out is n x nk, row-major. */
int oracle_basis(int nk, double theta_max, const double *knots, double radius, const double *t,
                 double *out, int64_t n) {
  Profile p;
  if (profile_build(1, 0.0, nk, theta_max, knots, radius, &p)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    memset(out + i * nk, 0, sizeof(double) * nk);
    basis_accumulate(&p, t[i], 1.0, out + i * nk);
  }
  profile_free(&p);
  return 0;
}

static int setup(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int pkind, double fwhm,
                 int nk, double theta_max, const double *knots, double radius, Grid *g,
                 Profile *p) {
  if (!(radius > 0) || radius >= M_PI) return -1;
  if (grid_build(kind, nside, ntheta, nphi, g)) return -1;
  if (profile_build(pkind, fwhm, nk, theta_max, knots, radius, p)) { grid_free(g); return -1; }
  return 0;
}

/* Forward direct sum.  If idx is NULL, y has npix entries; otherwise y[s] is
 * the output at pixel idx[s] for s < nidx. */
int oracle_convolve(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int pkind,
                    double fwhm, int nk, double theta_max, const double *knots, double radius,
                    const double *x, double *y, const int64_t *idx, int64_t nidx, int nthreads) {
  Grid g; Profile p;
  if (setup(kind, nside, ntheta, nphi, pkind, fwhm, nk, theta_max, knots, radius, &g, &p)) return -1;
  int64_t nout = idx ? nidx : g.npix;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < nout; ++s) {
    int64_t pix = idx ? idx[s] : s, ip;
    double th, ph;
    pixel_dir(&g, pix, &th, &ph, &ip);
    double acc = 0.0;
    FOR_EACH_NEIGHBOUR(&g, &p, th, ph, { acc += kernel_eval(&p, q_angle) * x[q_index] * g.w[q_ring]; });
    y[s] = acc;
  }
  grid_free(&g); profile_free(&p);
  return 0;
}

/* Explicit transpose: xbar_q = w_q sum_p K(theta_pq) r_p, for output pixels q. */
int oracle_adjoint(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int pkind,
                   double fwhm, int nk, double theta_max, const double *knots, double radius,
                   const double *r, double *xbar, const int64_t *idx, int64_t nidx, int nthreads) {
  Grid g; Profile p;
  if (setup(kind, nside, ntheta, nphi, pkind, fwhm, nk, theta_max, knots, radius, &g, &p)) return -1;
  int64_t nout = idx ? nidx : g.npix;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < nout; ++s) {
    int64_t qix = idx ? idx[s] : s, iq;
    double th, ph;
    pixel_dir(&g, qix, &th, &ph, &iq);
    double acc = 0.0;
    /* the neighbours visited here play the role of output pixels p */
    FOR_EACH_NEIGHBOUR(&g, &p, th, ph, { acc += kernel_eval(&p, q_angle) * r[q_index]; });
    xbar[s] = g.w[iq] * acc;
  }
  grid_free(&g); profile_free(&p);
  return 0;
}

/* Knot gradient of L = 1/2 |C x - t|^2 given r = C x - t:
 *   g_k = sum_p r_p sum_q phi_k(theta_pq) x_q w_q.
 * If idx is given, only output pixels p in idx contribute.  Per-thread partial
 * sums are combined in thread order, so the result is reproducible for a fixed
 * thread count. */
int oracle_knot_grad(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int nk,
                     double theta_max, const double *knots, double radius, const double *x,
                     const double *r, double *grad, const int64_t *idx, int64_t nidx,
                     int nthreads) {
  Grid g; Profile p;
  if (setup(kind, nside, ntheta, nphi, 1, 0.0, nk, theta_max, knots, radius, &g, &p)) return -1;
  int64_t nout = idx ? nidx : g.npix;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int nt = omp_get_max_threads();
  double *part = calloc((size_t)nt * nk, sizeof(double));
#pragma omp parallel
  {
    int tid = omp_get_thread_num();
    double *acc = part + (size_t)tid * nk;
    double *row = malloc(sizeof(double) * nk);
#pragma omp for schedule(static)
    for (int64_t s = 0; s < nout; ++s) {
      int64_t pix = idx ? idx[s] : s, ip;
      double th, ph;
      pixel_dir(&g, pix, &th, &ph, &ip);
      if (r[pix] == 0.0) continue;
      memset(row, 0, sizeof(double) * nk);
      FOR_EACH_NEIGHBOUR(&g, &p, th, ph, { basis_accumulate(&p, q_angle, x[q_index] * g.w[q_ring], row); });
      for (int k = 0; k < nk; ++k) acc[k] += r[pix] * row[k];
    }
    free(row);
  }
  for (int k = 0; k < nk; ++k) {
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += part[(size_t)t * nk + k];
    grad[k] = s;
  }
  free(part);
  grid_free(&g); profile_free(&p);
  return 0;
}

/* Number of support neighbours of each listed pixel (diagnostics, cost model). */
int oracle_neighbour_count(int kind, int64_t nside, int64_t ntheta, int64_t nphi, double radius,
                           const int64_t *idx, int64_t nidx, int64_t *count, double *min_gap) {
  Grid g; Profile p;
  if (setup(kind, nside, ntheta, nphi, 0, 1.0, 0, 0, NULL, radius + 1e-7, &g, &p)) return -1;
  double gap = 1e300;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : gap)
  for (int64_t s = 0; s < nidx; ++s) {
    int64_t ip;
    double th, ph;
    pixel_dir(&g, idx[s], &th, &ph, &ip);
    int64_t c = 0;
    /* p.radius was widened by 1e-7, so pairs just outside R are visited too:
       record how close any pair comes to the inclusion threshold R + 1e-9.
       Both sides compute angles in FP64 (errors ~1e-16 rad), so a gap well
       above that means every pair is classified the same way by both. */
    FOR_EACH_NEIGHBOUR(&g, &p, th, ph, {
      double d = fabs(q_angle - (radius + SUPPORT_TOL));
      if (d < gap) gap = d;
      if (q_angle <= radius + SUPPORT_TOL) ++c;
    });
    count[s] = c;
  }
  *min_gap = gap;
  grid_free(&g); profile_free(&p);
  return 0;
}
