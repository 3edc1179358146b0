// Host FP64 background scalars for one step (Sec. 2.1 Eqs. 1-4, Sec. 2.2
// Eqs. 7-9, Sec. 2.4 Eq. 10).  Conformal time in units of 1/H0.
//
// The conformal interval int da / (a^2 E(a)) is taken in the variable
// u = sqrt(a), where the integrand 2 / (u^3 E(u^2)) is smooth (and constant
// for a matter-only universe), with composite 16-point Gauss-Legendre
// quadrature.  The nodes are computed once by Newton's method on the
// Legendre polynomial P_16.
#include <cmath>
#include <mutex>

#include "internal.h"

namespace sdpm {
namespace {

constexpr int kGL = 16;
constexpr int kPanels = 16;

struct GaussLegendre {
  double x[kGL];
  double w[kGL];
  GaussLegendre() {
    for (int i = 0; i < kGL; ++i) {
      // initial guess (Tricomi), then Newton on P_n; the weight uses P_n'
      // at the converged node
      double z = std::cos(M_PI * (i + 0.75) / (kGL + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= kGL; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = kGL * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussLegendre& gl() {
  static const GaussLegendre rule;
  return rule;
}

double integrand_u(double u, double om, double ol) {
  const double a = u * u;
  return 2.0 / (u * u * u * hubble_e(a, om, ol));
}

}  // namespace

double hubble_e(double a, double om, double ol) {
  const double ok = 1.0 - om - ol;
  return std::sqrt(om / (a * a * a) + ok / (a * a) + ol);
}

double conformal_dtau(double a0, double a1, double om, double ol) {
  if (a1 == a0) return 0.0;
  const GaussLegendre& r = gl();
  const double u0 = std::sqrt(a0), u1 = std::sqrt(a1);
  const double du = (u1 - u0) / kPanels;
  double sum = 0.0;
  for (int p = 0; p < kPanels; ++p) {
    const double lo = u0 + p * du;
    const double mid = lo + 0.5 * du, half = 0.5 * du;
    double s = 0.0;
    for (int i = 0; i < kGL; ++i) s += r.w[i] * integrand_u(mid + half * r.x[i], om, ol);
    sum += s * half;
  }
  return sum;
}

double conformal_midpoint(double a0, double a1, double om, double ol) {
  const double target = 0.5 * conformal_dtau(a0, a1, om, ol);
  double a = 0.5 * (a0 + a1);
  for (int it = 0; it < 60; ++it) {
    const double f = conformal_dtau(a0, a, om, ol) - target;
    const double fp = 1.0 / (a * a * hubble_e(a, om, ol));
    double next = a - f / fp;
    if (next < a0) next = 0.5 * (a + a0);
    if (next > a1) next = 0.5 * (a + a1);
    if (std::fabs(next - a) <= 4e-16 * a) return next;
    a = next;
  }
  return a;
}

double lightcone_radius(double a, double om, double ol, double c_light) {
  if (a >= 1.0) return 0.0;
  return c_light * conformal_dtau(a, 1.0, om, ol);
}

StepScalars step_scalars(const sdpm_config& cfg, double a, double da) {
  StepScalars s{};
  const double a1 = a + da;
  s.dtau = conformal_dtau(a, a1, cfg.omega_m, cfg.omega_l);
  s.a_half = conformal_midpoint(a, a1, cfg.omega_m, cfg.omega_l);
  s.s_half = 1.5 * cfg.omega_m / s.a_half;
  const double h = cfg.box / cfg.ng;
  s.c_g = cfg.c_grav < 0.0 ? 0.019 * h * cfg.c_light : cfg.c_grav;
  if (s.c_g == 0.0) {
    s.kappa1_h2 = s.kappa2_h2 = 0.0;
  } else {
    const double denom = s.c_g * s.c_g * 0.5 * s.dtau;
    s.kappa1_h2 = 3.0 * s.a_half * hubble_e(s.a_half, cfg.omega_m, cfg.omega_l) * h * h / denom;
    s.kappa2_h2 = 3.0 * a1 * hubble_e(a1, cfg.omega_m, cfg.omega_l) * h * h / denom;
  }
  s.r_lc_end = lightcone_radius(a1, cfg.omega_m, cfg.omega_l, cfg.c_light);
  return s;
}

}  // namespace sdpm
