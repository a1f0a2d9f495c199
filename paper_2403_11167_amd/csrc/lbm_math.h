// lbm_math.h -- logarithms for the bulk chemical potential of the
// free-energy step (Eq. 29 for Carnahan-Starling, the antiderivative of
// (1/rho) dp/drho for van der Waals).
//
// The free-energy step evaluates one logarithm per node (two for van der
// Waals in FP32 storage), and that step is bound by its vector ALU as much
// as by HBM.  The library logarithms carry double-word arithmetic to get
// within half an ulp; here the chemical potential only needs a few ulps (it
// enters the force through differences of neighbours, next to the rounding
// of the stored populations), so both functions use the textbook reduction
//
//   v = m 2^e with m in [1/sqrt2, sqrt2),  ln v = e ln2 + ln m,
//   ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1)/(m + 1),
//
// with |s| <= 3 - 2 sqrt2 = 0.1716, so s^2 <= 0.0295 and the series is cut
// where its next term falls below the working precision (s^21/21 in FP64,
// s^11/11 in FP32).  ln2 is split into a head and a tail that are applied
// by two fused multiply-adds.  log1p adds the first-order correction c/u for
// the rounding error c of u = 1 + v, which keeps full relative precision
// for small arguments.
//
// Accuracy (the host build of these functions, checked against long-double
// references over wide sweeps by the CPU tests): ln_f64 within 2 ulp,
// ln1p_f32 within 3 ulp.  Arguments outside the domain (v <= 0 for ln,
// v <= -1 for log1p) and non-finite arguments give NaN; the step flags such
// densities itself.
//
// The device build uses the hardware reciprocal (refined by Newton steps in
// FP64) and the hardware frexp; the host build, which exists only so the
// algorithm can be tested on a CPU, uses a division and frexp().
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__
#else
#define LBM_HD
#endif

namespace lbmm {

// 1/b for normal positive b: hardware estimate plus two Newton steps
// r <- r + r (1 - b r), each squaring the relative error.
LBM_HD inline double rcp_f64(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / b;
#endif
}

LBM_HD inline float rcp_f32(float b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(b);  // 1 ulp
#else
  return 1.0f / b;
#endif
}

// m in [0.5, 1) and e with v = m 2^e (finite, non-zero v).
LBM_HD inline double mant_f64(double v, int& e) {
#if defined(__HIP_DEVICE_COMPILE__)
  e = __builtin_amdgcn_frexp_exp(v);
  return __builtin_amdgcn_frexp_mant(v);
#else
  return frexp(v, &e);
#endif
}

LBM_HD inline float mant_f32(float v, int& e) {
#if defined(__HIP_DEVICE_COMPILE__)
  e = __builtin_amdgcn_frexp_expf(v);
  return __builtin_amdgcn_frexp_mantf(v);
#else
  return frexpf(v, &e);
#endif
}

// ln 2 = LN2_HI + LN2_LO (head: ln 2 rounded to a double; tail: the rest).
constexpr double LN2_HI = 0.69314718055994528623;
constexpr double LN2_LO = 2.3190468138462996154e-17;
constexpr float LN2F_HI = 0.693147182464599609375f;
constexpr float LN2F_LO = -1.9046542999577679e-09f;
constexpr double RSQRT2 = 0.70710678118654752440;

// Natural logarithm in FP64.
LBM_HD inline double ln_f64(double v) {
  int e;
  double m = mant_f64(v, e);
  const bool lo = m < RSQRT2;  // m in [1/sqrt2, sqrt2) after this
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double a = m - 1.0;  // exact (Sterbenz)
  const double b = m + 1.0;
  const double r = rcp_f64(b);
  double s = a * r;
  s = fma(r, fma(-s, b, a), s);  // residual correction of the quotient
  const double z = s * s;
  // atanh(s)/s - 1 = z (1/3 + z/5 + ... + z^8/19)
  double q = 1.0 / 19.0;
  q = fma(q, z, 1.0 / 17.0);
  q = fma(q, z, 1.0 / 15.0);
  q = fma(q, z, 1.0 / 13.0);
  q = fma(q, z, 1.0 / 11.0);
  q = fma(q, z, 1.0 / 9.0);
  q = fma(q, z, 1.0 / 7.0);
  q = fma(q, z, 1.0 / 5.0);
  q = fma(q, z, 1.0 / 3.0);
  const double s2 = s + s;
  const double lm = fma(s2 * z, q, s2);  // ln m = 2 atanh(s)
  const double ed = (double)e;
  const double res = fma(ed, LN2_HI, fma(ed, LN2_LO, lm));
  return v > 0.0 ? res : NAN;
}

// ln(1 + v) in FP32.
LBM_HD inline float ln1p_f32(float v) {
  const float u = 1.0f + v;
  const float c = v - (u - 1.0f);  // rounding error of u (exact)
  int e;
  float m = mant_f32(u, e);
  const bool lo = m < (float)RSQRT2;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const float s = (m - 1.0f) * rcp_f32(m + 1.0f);
  const float z = s * s;
  const float q = fmaf(fmaf(fmaf(1.0f / 9.0f, z, 1.0f / 7.0f), z, 1.0f / 5.0f), z, 1.0f / 3.0f);
  const float s2 = s + s;
  const float lm = fmaf(s2 * z, q, s2);
  const float ed = (float)e;
  float res = fmaf(ed, LN2F_HI, fmaf(ed, LN2F_LO, lm));
  res = fmaf(c, rcp_f32(u), res);  // ln(u + c) = ln u + c/u + O(c^2)
  return u > 0.0f ? res : NAN;
}

}  // namespace lbmm
