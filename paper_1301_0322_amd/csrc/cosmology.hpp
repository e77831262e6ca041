// FP64 host cosmology: background, growth factors, spectrum and step table.
#pragma once

#include <cstdint>
#include <vector>

namespace cola {

constexpr uint32_t kFlagKdkStd = 0x1u;
constexpr uint32_t kFlagNoLpt = 0x2u;
constexpr uint32_t kFlagLogA = 0x4u;
constexpr uint32_t kFlagU1Drift = 0x8u;

struct Growth {
  double d1 = 0, d2 = 0, td1 = 0, td2 = 0, t2d1 = 0, t2d2 = 0;
};

struct Cosmo {
  double omega_m = 0.3, omega_l = 0.7, h = 0.7, n_s = 0.96, sigma8 = 0.8, n_lpt = -2.5;
  double amplitude = 0.0;  // P(k) = amplitude k^ns T(k)^2 after normalise_sigma8()

  double E(double a) const;
  double Q(double a) const;
  Growth growth(double a) const;  // normalised to D1(1) = 1
  double u(double a) const;
  double tu(double a) const;
  double int_u_over_q(double lo, double hi) const;
  double int_1_over_q(double lo, double hi) const;
  double int_a_over_q(double lo, double hi) const;
  double bbks(double k) const;
  void normalise_sigma8();
  double power(double k) const;
};

struct StepRow {
  double a = 0, a_mid = 0;
  Growth g;
  double alpha = 0, beta = 0, dd1 = 0, dd2 = 0, force = 0;
};

std::vector<StepRow> build_step_table(const Cosmo& c, double a_init, double a_final, int n, uint32_t flags);

}  // namespace cola
