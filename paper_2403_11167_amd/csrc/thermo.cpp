// thermo.cpp -- host-side thermodynamics for the lattice Boltzmann library:
// equations of state, critical points, Maxwell coexistence, the
// pseudopotential consistency coefficient sigma^Li (App. B), planar
// interface widths and surface tensions (Eq. 26, App. C Eq. 44 and 46) and
// the matching of the pseudopotential parameters to a free-energy interface
// (Sec. 3-4).  FP64, libm only; no device work.
#include <math.h>
#include <stdint.h>

#include <vector>

#include "lbm.h"

namespace {

constexpr double kG = -1.0;       // interaction sign of Eq. 11
constexpr double kCs2 = 1.0 / 3.0;

struct Eos {
  int kind;
  double a, b, R, T;

  // Upper end of the density domain (b rho < 1 vdW, b rho/4 < 1 CS).
  double rho_max() const { return kind == LBM_EOS_CS ? 4.0 / b : 1.0 / b; }

  double p(double r) const {
    if (kind == LBM_EOS_CS) {
      double e = 0.25 * b * r, om = 1.0 - e;
      return r * R * T * (1.0 + e + e * e - e * e * e) / (om * om * om) - a * r * r;
    }
    return r * R * T / (1.0 - b * r) - a * r * r;
  }
  // dp/drho
  double dp(double r) const {
    if (kind == LBM_EOS_CS) {
      double e = 0.25 * b * r, om = 1.0 - e;
      // d/drho [rho Z(e)] = Z + e Z' with Z = (1+e+e^2-e^3)/(1-e)^3; the
      // combination simplifies to (1 + 4e + 4e^2 - 4e^3 + e^4)/(1-e)^4.
      double num = 1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e * e * e + e * e * e * e;
      return R * T * num / (om * om * om * om) - 2.0 * a * r;
    }
    double om = 1.0 - b * r;
    return R * T / (om * om) - 2.0 * a * r;
  }
  // bulk chemical potential (Eq. 29 for CS; vdW antiderivative of p'/rho)
  double mu(double r) const {
    double RT = R * T;
    if (kind == LBM_EOS_CS) {
      double e = 0.25 * b * r, om = 1.0 - e;
      return RT * (3.0 - e) / (om * om * om) + RT * log(r) + RT - 2.0 * a * r;
    }
    double om = 1.0 - b * r;
    return RT * log(r / om) + RT * b * r / om - 2.0 * a * r;
  }
  // psi^2 of Eq. 11 with G = -1, and d psi/d rho
  double psi2(double r) const { return 2.0 * (r * kCs2 - p(r)); }
  double psi(double r) const { return sqrt(psi2(r)); }
  double dpsi(double r) const { return (kCs2 - dp(r)) / psi(r); }
};

bool ok_eos(int eos, double a, double b, double R) {
  return (eos == LBM_EOS_VDW || eos == LBM_EOS_CS) && isfinite(a) && isfinite(b) &&
         isfinite(R) && a > 0 && b > 0 && R > 0;
}

template <class F>
double bisect(F f, double lo, double hi, int iters = 200) {
  double flo = f(lo);
  for (int k = 0; k < iters; ++k) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double fm = f(mid);
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

// The two spinodal densities (dp/drho = 0), found by a geometric scan.
bool spinodals(const Eos& E, double* s1, double* s2) {
  double hi = E.rho_max();
  const int n = 20000;
  double prev_r = hi * 1e-7, prev = E.dp(prev_r);
  int found = 0;
  double roots[2] = {0, 0};
  for (int k = 1; k <= n && found < 2; ++k) {
    double r = hi * 1e-7 * pow(0.999999 / 1e-7, (double)k / n);
    double v = E.dp(r);
    if ((v < 0) != (prev < 0)) {
      roots[found++] = bisect([&](double x) { return E.dp(x); }, prev_r, r);
    }
    prev_r = r;
    prev = v;
  }
  if (found < 2) return false;
  *s1 = roots[0];
  *s2 = roots[1];
  return true;
}

bool maxwell(const Eos& E, double* rl, double* rv, double* p0) {
  double s1, s2;
  if (!spinodals(E, &s1, &s2)) return false;
  double pv_max = E.p(s1), pl_min = E.p(s2);
  double lo = fmax(pl_min, 0.0), hi = pv_max;
  double rtop = E.rho_max() * (1.0 - 1e-15);
  auto roots = [&](double P, double* l, double* v) {
    double rlo = 1e-300;
    *v = bisect([&](double x) { return E.p(x) - P; }, rlo, s1);
    *l = bisect([&](double x) { return E.p(x) - P; }, s2, rtop);
  };
  // mu(rho_l) - mu(rho_v) changes sign across the admissible pressures
  auto g = [&](double P) {
    double l, v;
    roots(P, &l, &v);
    return E.mu(l) - E.mu(v);
  };
  double P = bisect(g, lo + 1e-14 * (hi - lo), hi - 1e-14 * (hi - lo), 300);
  double l, v;
  roots(P, &l, &v);
  // Newton polish on p(l) = p(v), mu(l) = mu(v)
  for (int it = 0; it < 8; ++it) {
    double F1 = E.p(l) - E.p(v), F2 = E.mu(l) - E.mu(v);
    double dl = E.dp(l), dv = E.dp(v);
    double J11 = dl, J12 = -dv, J21 = dl / l, J22 = -dv / v;
    double det = J11 * J22 - J12 * J21;
    if (det == 0 || !isfinite(det)) break;
    double dL = (-F1 * J22 + F2 * J12) / det;
    double dV = (-F2 * J11 + F1 * J21) / det;
    l += dL;
    v += dV;
    if (fabs(dL) < 1e-16 * l && fabs(dV) < 1e-16 * fmax(v, 1e-300)) break;
  }
  if (!(v > 0 && l > v && isfinite(l))) return false;
  *rl = l;
  *rv = v;
  *p0 = E.p(l);
  return true;
}

// Composite Simpson rule over n (even) panels of f sampled at n + 1 points.
double simpson(const std::vector<double>& f, double h) {
  size_t n = f.size() - 1;
  double s = f[0] + f[n];
  for (size_t k = 1; k < n; ++k) s += (k & 1 ? 4.0 : 2.0) * f[k];
  return s * h / 3.0;
}

// Planar-profile tabulation on [rho_v, rho_l]: slope2[k] = (d rho/dx)^2 at
// r[k].  integrand(r) is the density integrand of the first integral and
// scale(r, I) turns the running integral into the squared slope.
template <class FI, class FS>
void planar_profile(double rv, double rl, int n, FI integrand, FS scale,
                    std::vector<double>& r, std::vector<double>& slope2) {
  r.resize(n + 1);
  slope2.assign(n + 1, 0.0);
  double h = (rl - rv) / n;
  for (int k = 0; k <= n; ++k) r[k] = rv + h * k;
  double run = 0.0, fl = integrand(r[0]);
  slope2[0] = 0.0;
  for (int k = 1; k <= n; ++k) {
    // Simpson on the single panel [r_{k-1}, r_k] with its midpoint
    double fm = integrand(r[k - 1] + 0.5 * h), fr = integrand(r[k]);
    run += h / 6.0 * (fl + 4.0 * fm + fr);
    fl = fr;
    double s2 = scale(r[k], run);
    slope2[k] = s2 > 0 ? s2 : 0.0;
  }
  slope2[n] = 0.0;
}

// Maximum of a sampled smooth function, refined by a parabola.
double sampled_max(const std::vector<double>& y) {
  size_t k = 1;
  for (size_t i = 1; i + 1 < y.size(); ++i)
    if (y[i] > y[k]) k = i;
  double y0 = y[k - 1], y1 = y[k], y2 = y[k + 1];
  double den = y0 - 2 * y1 + y2;
  if (den == 0) return y1;
  double t = 0.5 * (y0 - y2) / den;
  return y1 - 0.25 * (y0 - y2) * t;
}

constexpr int kProfileN = 40000;

bool fe_theory(const Eos& E, double kappa, double* width, double* gamma) {
  double rl, rv, p0;
  if (!maxwell(E, &rl, &rv, &p0)) return false;
  std::vector<double> r, s2;
  // Eq. 26: (d rho/dx)^2 = (2 rho/kappa) int_{rho_v}^{rho} (p - p0)/s^2 ds
  planar_profile(
      rv, rl, kProfileN, [&](double s) { return (E.p(s) - p0) / (s * s); },
      [&](double rr, double I) { return 2.0 * rr / kappa * I; }, r, s2);
  std::vector<double> slope(s2.size());
  for (size_t k = 0; k < s2.size(); ++k) slope[k] = sqrt(s2[k]);
  *width = (rl - rv) / sqrt(sampled_max(s2));
  *gamma = kappa * simpson(slope, (rl - rv) / kProfileN);  // kappa int rho' d rho
  return true;
}

bool sigma_theory(const Eos& E, double* eps_out, double* sigma) {
  double rl, rv, p0;
  if (!maxwell(E, &rl, &rv, &p0)) return false;
  const int n = 40000;  // Simpson intervals (App. B fixes the rule, not the count)
  double h = (rl - rv) / n;
  std::vector<double> base(n + 1), lnpsi(n + 1);
  for (int k = 0; k <= n; ++k) {
    double r = rv + h * k;
    double q = E.psi2(r);
    if (!(q > 0)) return false;
    double ps = sqrt(q);
    // (p - p0) psi' / psi, the eps-independent part of the Eq. 13 integrand
    base[k] = (E.p(r) - p0) * E.dpsi(r) / ps;
    lnpsi[k] = log(ps);
  }
  double eps = 2.0;  // initial guess of App. B
  std::vector<double> f(n + 1), df(n + 1);
  for (int it = 0; it < 100; ++it) {
    for (int k = 0; k <= n; ++k) {
      double wk = base[k] * exp(-eps * lnpsi[k]);  // (p - p0) psi'/psi^(1+eps)
      f[k] = wk;
      df[k] = -wk * lnpsi[k];  // d/deps of the integrand
    }
    double F = simpson(f, h), dF = simpson(df, h);
    if (!(dF != 0) || !isfinite(F)) return false;
    double step = -F / dF;
    eps += step;
    if (fabs(step) < 1e-14 * fmax(1.0, fabs(eps))) {
      *eps_out = eps;
      *sigma = -eps / (16.0 * kG);
      return true;
    }
  }
  return false;
}

// Pseudopotential planar profile of App. C Eq. 44 at kappa^P = 1:
// max-slope width and I = int psi' (d psi/dx) d rho.
bool p_theory_unit(const Eos& E, double eps, double* width1, double* I1) {
  double rl, rv, p0;
  if (!maxwell(E, &rl, &rv, &p0)) return false;
  std::vector<double> r, z2;
  // (d psi/dx)^2 = (8 psi^eps / G) int_{rho_v}^{rho} (p0 - p) psi'/psi^(1+eps)
  planar_profile(
      rv, rl, kProfileN,
      [&](double s) { return (p0 - E.p(s)) * E.dpsi(s) / pow(E.psi(s), 1.0 + eps); },
      [&](double rr, double I) { return 8.0 * pow(E.psi(rr), eps) / kG * I; }, r, z2);
  std::vector<double> slope2(z2.size()), integrand(z2.size());
  for (size_t k = 0; k < z2.size(); ++k) {
    double d = E.dpsi(r[k]);
    slope2[k] = z2[k] / (d * d);
    integrand[k] = fabs(d) * sqrt(z2[k]);
  }
  *width1 = (rl - rv) / sqrt(sampled_max(slope2));
  *I1 = simpson(integrand, (rl - rv) / kProfileN);
  return true;
}

}  // namespace

extern "C" {

lbm_status lbm_eos_eval(int32_t eos, double a, double b, double R, double T, double rho,
                        double* p, double* dp_drho) {
  if (!p || !dp_drho || !ok_eos(eos, a, b, R) || !(T > 0.0)) return LBM_ERR_INVALID_ARG;
  Eos E{eos, a, b, R, T};
  if (!(rho > 0.0) || !(rho < E.rho_max())) return LBM_ERR_EOS_DOMAIN;
  *p = E.p(rho);
  *dp_drho = E.dp(rho);
  return LBM_OK;
}

lbm_status lbm_eos_critical(int32_t eos, double a, double b, double R, double* Tc,
                            double* rho_c, double* p_c) {
  if (!Tc || !rho_c || !p_c || !ok_eos(eos, a, b, R)) return LBM_ERR_INVALID_ARG;
  if (eos == LBM_EOS_VDW) {
    *Tc = 8.0 * a / (27.0 * b * R);
    *rho_c = 1.0 / (3.0 * b);
    *p_c = a / (27.0 * b * b);
    return LBM_OK;
  }
  // CS: with e = b rho/4 and Z(e) = (1+e+e^2-e^3)/(1-e)^3, p' = 0 and
  // p'' = 0 eliminate a and T to  Z - e Z' - e^2 Z'' = 0.
  auto Z = [](double e) { return (1 + e + e * e - e * e * e) / pow(1 - e, 3); };
  auto Zp = [](double e) {
    double N = 1 + e + e * e - e * e * e, Np = 1 + 2 * e - 3 * e * e;
    return (Np * (1 - e) + 3 * N) / pow(1 - e, 4);
  };
  auto Zpp = [](double e) {
    double N = 1 + e + e * e - e * e * e, Np = 1 + 2 * e - 3 * e * e, Npp = 2 - 6 * e;
    // derivative of (Np (1-e) + 3N) / (1-e)^4
    double num = Np * (1 - e) + 3 * N;
    double dnum = Npp * (1 - e) - Np + 3 * Np;
    return (dnum * (1 - e) + 4 * num) / pow(1 - e, 5);
  };
  double ec = bisect([&](double e) { return Z(e) - e * Zp(e) - e * e * Zpp(e); }, 0.01, 0.5);
  double rc = 4.0 * ec / b;
  // p' = RT (Z + e Z') - 2 a rho = 0
  double T = 2.0 * a * rc / (R * (Z(ec) + ec * Zp(ec)));
  *Tc = T;
  *rho_c = rc;
  *p_c = rc * R * T * Z(ec) - a * rc * rc;
  return LBM_OK;
}

lbm_status lbm_maxwell(int32_t eos, double a, double b, double R, double T, double* rho_l,
                       double* rho_v, double* p0) {
  if (!rho_l || !rho_v || !p0 || !ok_eos(eos, a, b, R) || !(T > 0) || !isfinite(T))
    return LBM_ERR_INVALID_ARG;
  double Tc, rc, pc;
  lbm_eos_critical(eos, a, b, R, &Tc, &rc, &pc);
  if (!(T < Tc)) return LBM_ERR_INVALID_ARG;
  Eos E{eos, a, b, R, T};
  if (!maxwell(E, rho_l, rho_v, p0)) return LBM_ERR_NO_CONVERGENCE;
  return LBM_OK;
}

lbm_status lbm_sigma_li_theory(int32_t eos, double a, double b, double R, double T,
                               double* eps, double* sigma_li) {
  if (!eps || !sigma_li || !ok_eos(eos, a, b, R) || !(T > 0)) return LBM_ERR_INVALID_ARG;
  double rl, rv, p0;
  lbm_status st = lbm_maxwell(eos, a, b, R, T, &rl, &rv, &p0);
  if (st != LBM_OK) return st;
  Eos E{eos, a, b, R, T};
  if (!(E.psi2(rv) > 0)) return LBM_ERR_EOS_DOMAIN;
  for (int k = 0; k <= 1000; ++k)
    if (!(E.psi2(rv + (rl - rv) * k / 1000.0) > 0)) return LBM_ERR_EOS_DOMAIN;
  if (!sigma_theory(E, eps, sigma_li)) return LBM_ERR_NO_CONVERGENCE;
  return LBM_OK;
}

lbm_status lbm_fe_planar_theory(int32_t eos, double a, double b, double R, double T,
                                double kappa, double* width, double* gamma) {
  if (!width || !gamma || !ok_eos(eos, a, b, R) || !(T > 0) || !(kappa > 0))
    return LBM_ERR_INVALID_ARG;
  double rl, rv, p0;
  lbm_status st = lbm_maxwell(eos, a, b, R, T, &rl, &rv, &p0);
  if (st != LBM_OK) return st;
  Eos E{eos, a, b, R, T};
  if (!fe_theory(E, kappa, width, gamma)) return LBM_ERR_NO_CONVERGENCE;
  return LBM_OK;
}

lbm_status lbm_match_p_to_fe(int32_t eos, double a, double b, double R, double T,
                             double kappa_fe, double target_width, double* sigma_li,
                             double* kappa_p, double* kappa_li) {
  if (!sigma_li || !kappa_p || !kappa_li || !ok_eos(eos, a, b, R) || !(T > 0) ||
      !(kappa_fe > 0))
    return LBM_ERR_INVALID_ARG;
  double eps, sig;
  lbm_status st = lbm_sigma_li_theory(eos, a, b, R, T, &eps, &sig);
  if (st != LBM_OK) return st;
  Eos E{eos, a, b, R, T};
  double wfe, gfe;
  if (!fe_theory(E, kappa_fe, &wfe, &gfe)) return LBM_ERR_NO_CONVERGENCE;
  double w1, I1;
  if (!p_theory_unit(E, eps, &w1, &I1)) return LBM_ERR_NO_CONVERGENCE;
  double wt = target_width > 0 ? target_width : wfe;
  // Eq. 44: width grows as sqrt(kappa^P), I = int psi' psi_x d rho as 1/sqrt.
  double kp = (wt / w1) * (wt / w1);
  double I = I1 / sqrt(kp);
  // Eq. 46: gamma = -(G/6) (kappa^P - kappa^Li) I  ->  solve for kappa^Li.
  *sigma_li = sig;
  *kappa_p = kp;
  *kappa_li = kp - 6.0 * gfe / (-kG * I);
  return LBM_OK;
}

}  // extern "C"
