// FP64 host computation of everything that depends on a but not on particles:
// background Q(a), growth factors and their T derivatives, the COLA kick and drift
// factors, and the BBKS spectrum with its sigma8 normalisation.
//
// Paper passages: Appendix A.1 eq. (eom) (T = Q d/da, Q = a^3 H/H0, and the force
// whose linearisation gives T^2[D1] = (3/2) Om a D1); Appendix A.3 (D1(1) = 1,
// second-order growth T^2[D2] = (3/2) Om a (D2 - D1^2)); eq. (KDKALC) (u = a^nLPT,
// kick (u(a_f) - u(a_i)) / T[u](a_c), drift int u/Q da / u(a_c)); eq. (KDKALCstd)
// and eq. (KDKStd) for the variant flags; eq. (ALCtimestep) with midpoints
// a_{i+1/2} = (a_i + a_{i+1})/2 and steps uniform in a (Appendix A.3.2).
#include "cosmology.hpp"

#include <cmath>

namespace cola {

namespace {
constexpr double kAStart = 1e-5;
constexpr int kGrowthSteps = 20000;

struct Y4 {
  double d1, v1, d2, v2;
};

Y4 growth_rhs_lna(const Cosmo& c, double lna, const Y4& y) {
  // d/dln a = a d/da; dD/da = T[D]/Q, dT[D]/da = T^2[D]/Q.
  const double a = std::exp(lna);
  const double q = c.Q(a);
  const double src = 1.5 * c.omega_m * a;
  return {a * y.v1 / q, a * src * y.d1 / q, a * y.v2 / q, a * src * (y.d2 - y.d1 * y.d1) / q};
}

Y4 axpy(const Y4& y, double h, const Y4& k) {
  return {y.d1 + h * k.d1, y.v1 + h * k.v1, y.d2 + h * k.d2, y.v2 + h * k.v2};
}

// Classical RK4 in ln a from the growing mode at kAStart to a.
Y4 integrate_growth(const Cosmo& c, double a) {
  const double q0 = c.Q(kAStart);
  Y4 y{kAStart, q0, -3.0 / 7.0 * kAStart * kAStart, -6.0 / 7.0 * kAStart * q0};
  const double x0 = std::log(kAStart), x1 = std::log(a);
  const double h = (x1 - x0) / kGrowthSteps;
  for (int s = 0; s < kGrowthSteps; ++s) {
    const double x = x0 + s * h;
    const Y4 k1 = growth_rhs_lna(c, x, y);
    const Y4 k2 = growth_rhs_lna(c, x + 0.5 * h, axpy(y, 0.5 * h, k1));
    const Y4 k3 = growth_rhs_lna(c, x + 0.5 * h, axpy(y, 0.5 * h, k2));
    const Y4 k4 = growth_rhs_lna(c, x + h, axpy(y, h, k3));
    y.d1 += h / 6.0 * (k1.d1 + 2 * k2.d1 + 2 * k3.d1 + k4.d1);
    y.v1 += h / 6.0 * (k1.v1 + 2 * k2.v1 + 2 * k3.v1 + k4.v1);
    y.d2 += h / 6.0 * (k1.d2 + 2 * k2.d2 + 2 * k3.d2 + k4.d2);
    y.v2 += h / 6.0 * (k1.v2 + 2 * k2.v2 + 2 * k3.v2 + k4.v2);
  }
  return y;
}

// 20-panel composite 8-point Gauss-Legendre rule on [lo, hi].
template <class F>
double gauss_legendre(F&& f, double lo, double hi, int panels = 20) {
  static const double x[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
  static const double w[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
  const double h = (hi - lo) / panels;
  double tot = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = lo + (p + 0.5) * h, half = 0.5 * h;
    double s = 0.0;
    for (int j = 0; j < 4; ++j) s += w[j] * (f(mid - half * x[j]) + f(mid + half * x[j]));
    tot += s * half;
  }
  return tot;
}
}  // namespace

double Cosmo::E(double a) const {
  const double ok = 1.0 - omega_m - omega_l;
  return std::sqrt(omega_m / (a * a * a) + ok / (a * a) + omega_l);
}

double Cosmo::Q(double a) const { return a * a * a * E(a); }

Growth Cosmo::growth(double a) const {
  const Y4 one = integrate_growth(*this, 1.0);
  const Y4 y = integrate_growth(*this, a);
  const double c = one.d1;
  Growth g;
  g.d1 = y.d1 / c;
  g.td1 = y.v1 / c;
  g.d2 = y.d2 / (c * c);
  g.td2 = y.v2 / (c * c);
  g.t2d1 = 1.5 * omega_m * a * g.d1;
  g.t2d2 = 1.5 * omega_m * a * (g.d2 - g.d1 * g.d1);
  return g;
}

double Cosmo::u(double a) const { return std::pow(a, n_lpt); }
double Cosmo::tu(double a) const { return Q(a) * n_lpt * std::pow(a, n_lpt - 1.0); }

double Cosmo::int_u_over_q(double lo, double hi) const {
  return gauss_legendre([this](double a) { return u(a) / Q(a); }, lo, hi);
}
double Cosmo::int_1_over_q(double lo, double hi) const {
  return gauss_legendre([this](double a) { return 1.0 / Q(a); }, lo, hi);
}
double Cosmo::int_a_over_q(double lo, double hi) const {
  return gauss_legendre([this](double a) { return a / Q(a); }, lo, hi);
}

// --- BBKS spectrum --------------------------------------------------------------
double Cosmo::bbks(double k) const {
  const double q = k / (omega_m * h);
  const double x = 2.34 * q;
  const double lead = x > 1e-8 ? std::log1p(x) / x : 1.0 - 0.5 * x;
  const double poly = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
  return lead * std::pow(poly, -0.25);
}

static double tophat(double x) {
  if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0;
  return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

void Cosmo::normalise_sigma8() {
  // sigma^2(8) = 1/(2 pi^2) int k^3 P(k) W(8k)^2 dln k over [1e-5, 1e3] h/Mpc.
  const double lo = std::log(1e-5), hi = std::log(1e3);
  auto f = [this](double lnk) {
    const double k = std::exp(lnk);
    const double t = bbks(k), w = tophat(8.0 * k);
    return k * k * k * std::pow(k, n_s) * t * t * w * w;
  };
  const double integral = gauss_legendre(f, lo, hi, 4000);
  amplitude = sigma8 * sigma8 / (integral / (2.0 * M_PI * M_PI));
}

double Cosmo::power(double k) const {
  const double t = bbks(k);
  return amplitude * std::pow(k, n_s) * t * t;
}

// --- Step table ------------------------------------------------------------------
std::vector<StepRow> build_step_table(const Cosmo& c, double a_init, double a_final, int n, uint32_t flags) {
  std::vector<double> a(n + 1), am(n);
  const bool log_steps = flags & kFlagLogA;
  for (int i = 0; i <= n; ++i) {
    a[i] = log_steps ? a_init * std::pow(a_final / a_init, (double)i / n)
                     : a_init + (a_final - a_init) * (double)i / n;
  }
  a[n] = a_final;
  for (int i = 0; i < n; ++i) am[i] = 0.5 * (a[i] + a[i + 1]);

  std::vector<StepRow> t(n + 1);
  for (int i = 0; i <= n; ++i) {
    StepRow& r = t[i];
    r.a = a[i];
    r.g = c.growth(a[i]);
    const double lo = (i == 0) ? a[0] : am[i - 1];
    const double hi = (i == n) ? a[n] : am[i];
    if (flags & (kFlagKdkStd | kFlagNoLpt)) {
      // eq. (KDKALCstd) / (KDKStd): int (a / a_c) / Q da over the kick interval;
      // KDKStd carries the force's a_c inside its a-weighted integral, the same factor.
      r.alpha = c.int_a_over_q(lo, hi) / a[i];
    } else {
      r.alpha = (c.u(hi) - c.u(lo)) / c.tu(a[i]);
    }
    if (i < n) {
      r.a_mid = am[i];
      // eq. (KDKALC) drift int u/Q da / u(a_c); with u = 1 (the footnote's variant, kick
      // unchanged) and in the standard schemes it is int 1/Q da
      r.beta = (flags & (kFlagKdkStd | kFlagNoLpt | kFlagU1Drift)) ? c.int_1_over_q(a[i], a[i + 1])
                                                                    : c.int_u_over_q(a[i], a[i + 1]) / c.u(am[i]);
    }
    r.force = 1.5 * c.omega_m * a[i];
  }
  for (int i = 0; i < n; ++i) {
    t[i].dd1 = t[i + 1].g.d1 - t[i].g.d1;
    t[i].dd2 = t[i + 1].g.d2 - t[i].g.d2;
  }
  return t;
}

}  // namespace cola
