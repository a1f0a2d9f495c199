// Calls every host-theory entry point of the library (thermo.cpp, built
// alone with g++) over both equations of state and a range of temperatures,
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Prints
// the number of calls that did not return LBM_OK where they should have.
#include <cmath>
#include <cstdio>

#include "lbm.h"

int main() {
  int fails = 0;
  for (int eos = 0; eos < 2; ++eos) {
    const double a = eos == LBM_EOS_CS ? 0.25 : 9.0 / 49.0;
    const double b = eos == LBM_EOS_CS ? 4.0 : 2.0 / 21.0;
    double Tc, rc, pc;
    fails += lbm_eos_critical(eos, a, b, 1.0, &Tc, &rc, &pc) != LBM_OK;
    for (double Tr = 0.55; Tr < 0.96; Tr += 0.1) {
      const double T = Tr * Tc;
      double rl, rv, p0, p, dp, eps, sig, kp, kli, w, gam;
      fails += lbm_maxwell(eos, a, b, 1.0, T, &rl, &rv, &p0) != LBM_OK;
      fails += lbm_eos_eval(eos, a, b, 1.0, T, 0.5 * (rl + rv), &p, &dp) != LBM_OK;
      if (eos == LBM_EOS_CS) {
        fails += lbm_sigma_li_theory(eos, a, b, 1.0, T, &eps, &sig) != LBM_OK;
        fails += lbm_match_p_to_fe(eos, a, b, 1.0, T, 0.5 * a, 5.0, &sig, &kp, &kli) != LBM_OK;
      }
      fails += lbm_fe_planar_theory(eos, a, b, 1.0, T, 0.5 * a, &w, &gam) != LBM_OK;
      (void)lbm_eos_eval(eos, a, b, 1.0, T, -1.0, &p, &dp);  // out of domain: an error code
    }
  }
  std::printf("%d\n", fails);
  return fails != 0;
}
