// Host-side analysis of the Couette-cell rheology: the cooperative-length fit of the local
// fluidity profile, eq. (predict) (the integrated form of eq. (fluidity) in a cell whose mean
// shear stress is uniform).  The profiles themselves come from the device (lb_profile,
// lb_profile_stats); this is a fit of a few hundred numbers and runs on the host.

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/lb.h"

namespace {

// Shape of eq. (predict), cosh((z - H/2)/zeta) / cosh(H/(2 zeta)), written with
// non-positive exponents only, (e^{(z-H)/zeta} + e^{-z/zeta}) / (1 + e^{-H/zeta}), so it
// neither overflows for small zeta nor loses the ends for 0 <= z <= H.
double shape(double z, double H, double zeta) {
  return (std::exp((z - H) / zeta) + std::exp(-z / zeta)) / (1.0 + std::exp(-H / zeta));
}

// For fixed zeta the model f = f_b (1 - g) + f_w g is linear in (f_b, f_w): solve the 2 x 2
// normal equations and return the sum of squared residuals (infinity if they are singular).
double solve_at(const double *z, const double *f, int n, double H, double zeta, double *fb, double *fw) {
  double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
  for (int i = 0; i < n; ++i) {
    const double g = shape(z[i], H, zeta), h = 1.0 - g;
    a11 += h * h;
    a12 += h * g;
    a22 += g * g;
    b1 += h * f[i];
    b2 += g * f[i];
  }
  const double det = a11 * a22 - a12 * a12;
  if (!(std::fabs(det) > 1e-14 * (a11 * a22 + 1e-300))) return INFINITY;
  *fb = (b1 * a22 - b2 * a12) / det;
  *fw = (a11 * b2 - a12 * b1) / det;
  double sse = 0;
  for (int i = 0; i < n; ++i) {
    const double g = shape(z[i], H, zeta);
    const double r = f[i] - (*fb * (1.0 - g) + *fw * g);
    sse += r * r;
  }
  return sse;
}

}  // namespace

extern "C" {

int lb_fit_cooperative_length(const double *z, const double *f, int32_t n, double H, double zeta_min,
                              double zeta_max, double out[4]) {
  if (!z || !f || !out || n < 3) return LB_EINVAL;
  if (!(H > 0.0) || !std::isfinite(H) || !(zeta_min > 0.0) || !(zeta_max > zeta_min) || !std::isfinite(zeta_max))
    return LB_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(z[i]) || !std::isfinite(f[i]) || z[i] < 0.0 || z[i] > H) return LB_EINVAL;
  // coarse logarithmic scan, then golden section on log(zeta) around the best grid point
  const int NG = 241;
  const double l0 = std::log(zeta_min), l1 = std::log(zeta_max), dl = (l1 - l0) / (NG - 1);
  int best = -1;
  double best_sse = INFINITY, fb = 0, fw = 0;
  for (int k = 0; k < NG; ++k) {
    const double e = solve_at(z, f, n, H, std::exp(l0 + k * dl), &fb, &fw);
    if (e < best_sse) {
      best_sse = e;
      best = k;
    }
  }
  if (best < 0) return LB_EINVAL;
  double a = l0 + std::max(best - 1, 0) * dl, b = l0 + std::min(best + 1, NG - 1) * dl;
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double c = b - gr * (b - a), d = a + gr * (b - a);
  double fc = solve_at(z, f, n, H, std::exp(c), &fb, &fw), fd = solve_at(z, f, n, H, std::exp(d), &fb, &fw);
  for (int it = 0; it < 200 && b - a > 1e-15; ++it) {
    if (fc <= fd) {
      b = d;
      d = c;
      fd = fc;
      c = b - gr * (b - a);
      fc = solve_at(z, f, n, H, std::exp(c), &fb, &fw);
    } else {
      a = c;
      c = d;
      fc = fd;
      d = a + gr * (b - a);
      fd = solve_at(z, f, n, H, std::exp(d), &fb, &fw);
    }
  }
  const double zeta = std::exp(0.5 * (a + b));
  const double sse = solve_at(z, f, n, H, zeta, &fb, &fw);
  if (!std::isfinite(sse)) return LB_EINVAL;
  out[0] = zeta;
  out[1] = fb;
  out[2] = fw;
  out[3] = std::sqrt(sse / n);
  return LB_OK;
}

int lb_disjoining_pressure(const double *h, const double *gamma_f, int32_t n, double *pi) {
  if (!h || !gamma_f || !pi || n < 2) return LB_EINVAL;
  // sort the thicknesses (stable order of the input indices), distinct and finite
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(h[i]) || !std::isfinite(gamma_f[i]) || !(h[i] > 0.0)) return LB_EINVAL;
    order[i] = i;
  }
  std::sort(order.begin(), order.end(), [&](int a, int b) { return h[a] < h[b]; });
  for (int k = 1; k < n; ++k)
    if (!(h[order[k]] > h[order[k - 1]])) return LB_EINVAL;
  // eq. (doppiasigma) differentiated: d gamma_f = h d Pi; Pi = 0 at the thickest film and, with
  // gamma_f linear on each interval, the integral of gamma_f'(h) / h over it is
  // slope * ln(h_hi / h_lo)
  pi[order[n - 1]] = 0.0;
  double acc = 0.0;
  for (int k = n - 2; k >= 0; --k) {
    const int lo = order[k], hi = order[k + 1];
    const double slope = (gamma_f[hi] - gamma_f[lo]) / (h[hi] - h[lo]);
    acc -= slope * std::log(h[hi] / h[lo]);
    pi[lo] = acc;
  }
  return LB_OK;
}

}  // extern "C"
