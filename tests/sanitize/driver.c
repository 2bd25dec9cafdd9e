/* Host driver for the sanitizer build (AddressSanitizer + UndefinedBehavior
 * Sanitizer) of the oracle's direct sums and of the library's host-only
 * truncation-error calls.  Every entry point runs on tiny grids, on valid and
 * on invalid arguments; the sanitizers abort the process on any out-of-bounds
 * access, leak or undefined operation, so a zero exit status is the check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_npix(int kind, int64_t nside, int64_t ntheta, int64_t nphi);
int oracle_rings(int kind, int64_t nside, int64_t ntheta, int64_t nphi, double *theta, double *phi0, double *w,
                 int64_t *n, int64_t *start);
int oracle_kernel(int pkind, double fwhm, int nk, double theta_max, const double *knots, double radius,
                  const double *t, double *out, int64_t n);
int oracle_basis(int nk, double theta_max, const double *knots, double radius, const double *t, double *out,
                 int64_t n);
int oracle_convolve(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int pkind, double fwhm, int nk,
                    double theta_max, const double *knots, double radius, const double *x, double *y,
                    const int64_t *idx, int64_t nidx, int nthreads);
int oracle_adjoint(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int pkind, double fwhm, int nk,
                   double theta_max, const double *knots, double radius, const double *r, double *xbar,
                   const int64_t *idx, int64_t nidx, int nthreads);
int oracle_knot_grad(int kind, int64_t nside, int64_t ntheta, int64_t nphi, int nk, double theta_max,
                     const double *knots, double radius, const double *x, const double *r, double *grad,
                     const int64_t *idx, int64_t nidx, int nthreads);
int oracle_neighbour_count(int kind, int64_t nside, int64_t ntheta, int64_t nphi, double radius,
                           const int64_t *idx, int64_t nidx, int64_t *count, double *min_gap);

/* the library's host calls (truncation.cpp), C ABI of include/arkcos.h */
typedef struct {
  int32_t kind;
  double fwhm_rad;
  int32_t n_knots;
  double theta_max_rad;
  const double *knot_values;
} profile_t;
int arkcos_truncation_variance(const profile_t *p, double radius, const double *cl, int32_t lmax, double *s2,
                               double *dk);
int arkcos_choose_radius(const profile_t *p, const double *cl, int32_t lmax, double target, double *radius);

static int failures = 0;
#define EXPECT(c)                                              \
  do {                                                         \
    if (!(c)) {                                                \
      fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                              \
    }                                                          \
  } while (0)

int main(void) {
  double knots[12];
  for (int k = 0; k < 12; ++k) knots[k] = cos(0.3 * k) + 0.01 * k;
  /* geometries: HEALPix nside 1, 2, 4 and ECP 8 x 16 */
  const int64_t geo[4][4] = {{1, 1, 0, 0}, {1, 2, 0, 0}, {1, 4, 0, 0}, {0, 0, 8, 16}};
  for (int gi = 0; gi < 4; ++gi) {
    const int kind = (int)geo[gi][0];
    const int64_t nside = geo[gi][1], nt = geo[gi][2], np = geo[gi][3];
    const int64_t npix = oracle_npix(kind, nside, nt, np);
    const int64_t nr = kind == 1 ? 4 * nside - 1 : nt;
    double *th = malloc(sizeof(double) * nr), *ph = malloc(sizeof(double) * nr), *w = malloc(sizeof(double) * nr);
    int64_t *n = malloc(sizeof(int64_t) * nr), *st = malloc(sizeof(int64_t) * nr);
    EXPECT(oracle_rings(kind, nside, nt, np, th, ph, w, n, st) == 0);
    double *x = malloc(sizeof(double) * npix), *y = malloc(sizeof(double) * npix);
    double *r = malloc(sizeof(double) * npix), *g = malloc(sizeof(double) * 12);
    for (int64_t p = 0; p < npix; ++p) {
      x[p] = sin(0.7 * p);
      r[p] = cos(1.3 * p);
    }
    int64_t idx[3] = {0, npix / 2, npix - 1};
    int64_t cnt[3];
    double gap = 0.0;
    for (int pk = 0; pk < 2; ++pk) {
      for (int rad = 0; rad < 3; ++rad) {
        const double R = rad == 0 ? 0.3 : (rad == 1 ? 1.2 : 3.0);  /* up to nearly the whole sphere */
        EXPECT(oracle_convolve(kind, nside, nt, np, pk, 0.4, 12, R, knots, R, x, y, NULL, 0, 1) == 0);
        EXPECT(oracle_adjoint(kind, nside, nt, np, pk, 0.4, 12, R, knots, R, r, y, idx, 3, 1) == 0);
        EXPECT(oracle_neighbour_count(kind, nside, nt, np, R, idx, 3, cnt, &gap) == 0);
      }
    }
    EXPECT(oracle_knot_grad(kind, nside, nt, np, 12, 1.0, knots, 1.0, x, r, g, NULL, 0, 2) == 0);
    EXPECT(oracle_knot_grad(kind, nside, nt, np, 12, 1.0, knots, 1.0, x, r, g, idx, 3, 1) == 0);
    /* invalid arguments are refused */
    EXPECT(oracle_convolve(kind, nside, nt, np, 0, 0.4, 0, 0, NULL, 0.0, x, y, NULL, 0, 1) != 0);
    EXPECT(oracle_convolve(kind, nside, nt, np, 0, 0.4, 0, 0, NULL, 4.0, x, y, NULL, 0, 1) != 0);
    free(th); free(ph); free(w); free(n); free(st); free(x); free(y); free(r); free(g);
  }
  double t[5] = {0.0, 0.1, 0.5, 1.0, 2.0}, out[5 * 12];
  EXPECT(oracle_kernel(0, 0.4, 0, 0, NULL, 1.0, t, out, 5) == 0);
  EXPECT(oracle_kernel(1, 0.0, 12, 1.0, knots, 1.0, t, out, 5) == 0);
  EXPECT(oracle_basis(12, 1.0, knots, 1.0, t, out, 5) == 0);
  EXPECT(oracle_convolve(1, 0, 0, 0, 0, 0.4, 0, 0, NULL, 0.3, t, out, NULL, 0, 1) != 0); /* nside 0 */

  /* truncation error: valid, boundary and invalid arguments */
  double cl[41], dk[41], s2 = -1.0, R = -1.0;
  for (int l = 0; l <= 40; ++l) cl[l] = 1.0 / ((l + 1.0) * (l + 1.0));
  profile_t gp = {0, 0.05, 0, 0.0, NULL}, sp = {1, 0.0, 12, 0.2, knots}, bad = {1, 0.0, 2, 0.2, knots};
  EXPECT(arkcos_truncation_variance(&gp, 0.06, cl, 40, &s2, dk) == 0 && s2 >= 0.0);
  EXPECT(arkcos_truncation_variance(&sp, 0.0, cl, 40, &s2, NULL) == 0 && s2 > 0.0);
  EXPECT(arkcos_truncation_variance(&sp, M_PI, cl, 0, &s2, dk) == 0 && s2 == 0.0);
  EXPECT(arkcos_choose_radius(&gp, cl, 40, 1e-12, &R) == 0 && R > 0.0);
  EXPECT(arkcos_choose_radius(&sp, cl, 40, 1e9, &R) == 0 && R == 0.0);
  EXPECT(arkcos_truncation_variance(&gp, -0.1, cl, 40, &s2, dk) != 0);
  EXPECT(arkcos_truncation_variance(&gp, 0.1, cl, -1, &s2, dk) != 0);
  EXPECT(arkcos_truncation_variance(&bad, 0.1, cl, 40, &s2, dk) != 0);
  EXPECT(arkcos_truncation_variance(NULL, 0.1, cl, 40, &s2, dk) != 0);
  EXPECT(arkcos_choose_radius(&gp, NULL, 40, 1e-6, &R) != 0);
  EXPECT(arkcos_choose_radius(&gp, cl, 40, -1.0, &R) != 0);
  if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
  else printf("sanitizer driver: all calls clean\n");
  return failures ? 1 : 0;
}
