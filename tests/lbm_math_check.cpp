// Host build of the chemical potential's logarithms (paper_2403_11167_amd/
// csrc/lbm_math.h) against long-double references: prints the worst error
// in ulps of each function over sweeps that cover the whole exponent range,
// arguments near 1 (and near 0 for log1p), the reduction's switch point
// 1/sqrt2, and the densities of the paper's workloads.
#include <cmath>
#include <cstdio>
#include <random>

#include "lbm_math.h"

static double ulp_of(double x) { return std::nextafter(std::fabs(x), INFINITY) - std::fabs(x); }
static double ulp_of(float x) {
  return (double)(std::nextafter(std::fabs(x), INFINITY) - std::fabs(x));
}

int main() {
  std::mt19937_64 rng(20240317);
  std::uniform_real_distribution<double> u01(0.0, 1.0);
  double w64 = 0.0, w32 = 0.0;
  for (int i = 0; i < 2000000; ++i) {
    double x;
    switch (i % 5) {
      case 0: x = std::exp(-700.0 + 1400.0 * u01(rng)); break;
      case 1: x = 1.0 + (u01(rng) - 0.5) * std::pow(10.0, -(double)(i % 16)); break;
      case 2: x = 1e-3 + 20.0 * u01(rng); break;
      case 3: x = std::ldexp(0.70 + 0.02 * u01(rng), (i % 41) - 20); break;
      default: x = std::ldexp(1.0, (i % 2000) - 1000) * (1.0 + 1e-15 * u01(rng)); break;
    }
    const long double ref = logl((long double)x);
    if (ref == 0.0L) continue;
    const double e = (double)fabsl((long double)lbmm::ln_f64(x) - ref) / ulp_of((double)ref);
    if (e > w64) w64 = e;
  }
  for (int i = 0; i < 2000000; ++i) {
    float v;
    switch (i % 4) {
      case 0: v = (float)(-0.999 + 101.0 * u01(rng)); break;
      case 1: v = (float)((2.0 * u01(rng) - 1.0) * std::pow(10.0, -(double)(i % 31))); break;
      case 2: v = (float)std::exp(-80.0 + 160.0 * u01(rng)); break;
      default: v = (float)(std::sqrt(0.5) - 1.0 + 0.02 * (u01(rng) - 0.5)); break;
    }
    const long double ref = log1pl((long double)v);
    if (ref == 0.0L) continue;
    const double e = (double)fabsl((long double)lbmm::ln1p_f32(v) - ref) / ulp_of((float)ref);
    if (e > w32) w32 = e;
  }
  const bool nan_ok = std::isnan(lbmm::ln_f64(0.0)) && std::isnan(lbmm::ln_f64(-1.0)) &&
                      std::isnan(lbmm::ln_f64(INFINITY)) && std::isnan(lbmm::ln_f64(NAN)) &&
                      std::isnan(lbmm::ln1p_f32(-1.0f)) && std::isnan(lbmm::ln1p_f32(-3.0f)) &&
                      std::isnan(lbmm::ln1p_f32(NAN));
  std::printf("%.6f %.6f %d %.17g %.9g\n", w64, w32, nan_ok ? 1 : 0, lbmm::ln_f64(1.0),
              (double)lbmm::ln1p_f32(0.0f));
  return 0;
}
