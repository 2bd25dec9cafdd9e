// Truncation error of the kernel's support radius (paper Sect. 4): cutting
// K at radius R changes its Legendre coefficients by
//   dK_l(R) = -2 pi int_R^pi K(theta) P_l(cos theta) sin theta dtheta
// (K_l = 2 pi int K(z) P_l(z) dz, Sect. 2), and a signal of angular power
// spectrum C_l then sees an error of variance
//   sigma^2(R) = sum_l (2l + 1) / (4 pi) dK_l(R)^2 C_l.
// Host code only: composite 16-point Gauss-Legendre quadrature in theta over
// the part of the kernel's support beyond R, P_l(cos theta) by the
// three-term recurrence.
#include "arkcos_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace arkcos {

// Clamped cubic spline moments (second derivatives at the knots) for
// equispaced knots with spacing h; end slopes zero (host code shared with
// the plan builder).
void spline_moments(const std::vector<double>& c, double h, std::vector<double>& M) {
  const int n = (int)c.size();
  std::vector<double> sub(n), diag(n), sup(n), rhs(n);
  const double s = 6.0 / (h * h);
  for (int k = 0; k < n; ++k) {
    if (k == 0) { sub[k] = 0; diag[k] = 2; sup[k] = 1; rhs[k] = s * (c[1] - c[0]); }
    else if (k == n - 1) { sub[k] = 1; diag[k] = 2; sup[k] = 0; rhs[k] = -s * (c[n - 1] - c[n - 2]); }
    else { sub[k] = 1; diag[k] = 4; sup[k] = 1; rhs[k] = s * (c[k + 1] - 2 * c[k] + c[k - 1]); }
  }
  for (int k = 1; k < n; ++k) {
    double f = sub[k] / diag[k - 1];
    diag[k] -= f * sup[k - 1];
    rhs[k] -= f * rhs[k - 1];
  }
  M.assign(n, 0.0);
  M[n - 1] = rhs[n - 1] / diag[n - 1];
  for (int k = n - 2; k >= 0; --k) M[k] = (rhs[k] - sup[k] * M[k + 1]) / diag[k];
}

namespace {

constexpr int kNodes = 16;

// 16-point Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on
// P_16 from the Chebyshev guesses).
struct GaussLegendre {
  double x[kNodes], w[kNodes];
  GaussLegendre() {
    for (int i = 0; i < kNodes; ++i) {
      double z = std::cos(M_PI * (i + 0.75) / (kNodes + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int l = 2; l <= kNodes; ++l) {
          const double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
          p0 = p1;
          p1 = p2;
        }
        dp = kNodes * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

struct Profile {
  int kind = 0;
  double inv2s2 = 0.0, sigma = 0.0;
  double theta_max = 0.0, h = 0.0;
  std::vector<double> c, M;

  double value(double t) const {
    if (kind == 0) return std::exp(-t * t * inv2s2);
    if (t >= theta_max) return 0.0;
    const int n = (int)c.size();
    const int a = std::min(n - 2, (int)(t / h));
    const double u = t / h - a, v = 1.0 - u;
    return v * c[a] + u * c[a + 1] + h * h / 6.0 * ((v * v * v - v) * M[a] + (u * u * u - u) * M[a + 1]);
  }
  // where the kernel is negligible (Gaussian: 40 sigma) or zero (spline)
  double end() const { return kind == 0 ? std::min(M_PI, 40.0 * sigma) : std::min(M_PI, theta_max); }
};

arkcos_status_t make_profile(const arkcos_profile_t* p, Profile& out) {
  if (!p) return fail(ARKCOS_ERR_INVALID_VALUE, "null profile");
  if (p->kind == 0) {
    if (!(p->fwhm_rad > 0)) return fail(ARKCOS_ERR_INVALID_VALUE, "Gaussian FWHM must be > 0");
    out.kind = 0;
    out.sigma = p->fwhm_rad / std::sqrt(8.0 * std::log(2.0));
    out.inv2s2 = 1.0 / (2.0 * out.sigma * out.sigma);
    return ARKCOS_OK;
  }
  if (p->kind == 1) {
    if (p->n_knots < 3 || p->n_knots > 64 || !(p->theta_max_rad > 0) || !p->knot_values)
      return fail(ARKCOS_ERR_INVALID_VALUE, "spline needs 3..64 knots, theta_max > 0 and knot values");
    out.kind = 1;
    out.theta_max = p->theta_max_rad;
    out.c.assign(p->knot_values, p->knot_values + p->n_knots);
    out.h = out.theta_max / (p->n_knots - 1);
    spline_moments(out.c, out.h, out.M);
    return ARKCOS_OK;
  }
  return fail(ARKCOS_ERR_INVALID_VALUE, "profile kind must be 0 (Gaussian) or 1 (spline)");
}

// dK_l(R) for l = 0..lmax.  The range [R, end] is cut at the spline's knots
// (a cubic on each piece), and each piece into panels with at least eight
// nodes per period 2 pi / l of P_l(cos theta) and, for the Gaussian, at
// most one sigma wide.
void tail_coefficients(const Profile& K, double R, int lmax, std::vector<double>& dk) {
  static const GaussLegendre gl;
  dk.assign(lmax + 1, 0.0);
  const double b = K.end();
  if (!(R < b)) return;
  std::vector<double> cuts{R};
  if (K.kind == 1)
    for (size_t a = 1; a + 1 < K.c.size(); ++a)
      if (a * K.h > R && a * K.h < b) cuts.push_back(a * K.h);
  cuts.push_back(b);
  for (size_t piece = 0; piece + 1 < cuts.size(); ++piece) {
    const double s0 = cuts[piece], s1 = cuts[piece + 1];
    int64_t panels = 1 + (int64_t)std::ceil((s1 - s0) * (lmax + 1) / (2.0 * M_PI) * 8.0 / kNodes);
    if (K.kind == 0) panels = std::max<int64_t>(panels, (int64_t)std::ceil((s1 - s0) / K.sigma));
    const double hw = 0.5 * (s1 - s0) / (double)panels;
    for (int64_t q = 0; q < panels; ++q) {
      const double mid = s0 + (2.0 * q + 1.0) * hw;
      for (int i = 0; i < kNodes; ++i) {
        const double t = mid + hw * gl.x[i];
        const double f = -2.0 * M_PI * hw * gl.w[i] * K.value(t) * std::sin(t);
        if (f == 0.0) continue;
        const double z = std::cos(t);
        double p0 = 1.0, p1 = z;
        dk[0] += f;
        if (lmax >= 1) dk[1] += f * z;
        for (int l = 1; l < lmax; ++l) {
          const double p2 = ((2.0 * l + 1.0) * z * p1 - l * p0) / (l + 1.0);
          p0 = p1;
          p1 = p2;
          dk[l + 1] += f * p2;
        }
      }
    }
  }
}

double variance(const Profile& K, double R, const double* cl, int lmax, std::vector<double>& dk) {
  tail_coefficients(K, R, lmax, dk);
  double s = 0.0;
  for (int l = 0; l <= lmax; ++l) s += (2.0 * l + 1.0) / (4.0 * M_PI) * dk[l] * dk[l] * cl[l];
  return s;
}

}  // namespace
}  // namespace arkcos

using namespace arkcos;

extern "C" {

arkcos_status_t arkcos_truncation_variance(const arkcos_profile_t* profile, double radius_rad, const double* cl,
                                           int32_t lmax, double* sigma2, double* dk) {
  if (!cl || !sigma2) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (lmax < 0 || lmax > 1000000) return fail(ARKCOS_ERR_INVALID_VALUE, "lmax must be in 0 .. 1000000");
  if (!(radius_rad >= 0.0) || radius_rad > M_PI) return fail(ARKCOS_ERR_INVALID_VALUE, "radius must be in [0, pi]");
  Profile K;
  arkcos_status_t st = make_profile(profile, K);
  if (st != ARKCOS_OK) return st;
  try {
    std::vector<double> d;
    *sigma2 = variance(K, radius_rad, cl, lmax, d);
    if (dk) std::copy(d.begin(), d.end(), dk);
  } catch (...) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  return ARKCOS_OK;
}

arkcos_status_t arkcos_choose_radius(const arkcos_profile_t* profile, const double* cl, int32_t lmax,
                                     double target_sigma2, double* radius_rad) {
  if (!cl || !radius_rad) return fail(ARKCOS_ERR_INVALID_VALUE, "null argument");
  if (lmax < 0 || lmax > 1000000) return fail(ARKCOS_ERR_INVALID_VALUE, "lmax must be in 0 .. 1000000");
  if (!(target_sigma2 >= 0.0)) return fail(ARKCOS_ERR_INVALID_VALUE, "target variance must be >= 0");
  Profile K;
  arkcos_status_t st = make_profile(profile, K);
  if (st != ARKCOS_OK) return st;
  try {
    std::vector<double> d;
    // scan from the end of the support inwards on a grid of kScan radii: the
    // largest grid radius whose variance exceeds the target, then bisection
    // between it and the next grid radius (the variance need not be monotone
    // for kernels that change sign, so the scan keeps the answer conservative)
    constexpr int kScan = 256;
    const double b = K.end();
    double hi = b;  // variance 0 at the end of the support
    double lo = -1.0;
    for (int k = kScan - 1; k >= 0; --k) {
      const double r = b * k / kScan;
      if (variance(K, r, cl, lmax, d) > target_sigma2) {
        lo = r;
        break;
      }
      hi = r;
    }
    if (lo < 0.0) {
      *radius_rad = 0.0;  // no truncation error above the target anywhere
      return ARKCOS_OK;
    }
    for (int it = 0; it < 60 && hi - lo > 1e-12 * b; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (variance(K, mid, cl, lmax, d) > target_sigma2) lo = mid;
      else hi = mid;
    }
    *radius_rad = hi;
  } catch (...) {
    return fail(ARKCOS_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  return ARKCOS_OK;
}

}  // extern "C"
