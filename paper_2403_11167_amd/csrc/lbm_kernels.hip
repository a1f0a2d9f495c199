// lbm_kernels.hip -- gfx950 kernels and C ABI of the D2Q9 multiphase lattice
// Boltzmann library (pseudopotential and well-balanced free-energy models of
// Czelusniak et al., arXiv 2403.11167).  See include/lbm.h for the contract.
//
// Data layout in HBM
//   Populations: array of structures of arrays with 64-node blocks.  Row y
//   is split into blocks of 64 columns; for each block the nine velocity
//   chunks of 64 values (Eq. 2 order) are contiguous, so element (i, x, y)
//   sits at y * rowpitch + (x / 64) * 576 + 64 i + x % 64 with rowpitch =
//   576 ceil(nx / 64).  A wavefront (64 lanes = one block) reads each
//   velocity chunk as one coalesced segment (two when shifted by one
//   column), and a workgroup's row is a few contiguous regions instead of
//   nine plane streams.  What is stored is the post-collision, pre-streaming field
//   g*_i(x) = f*_i(x) - s_i, where s_i = f_i^eq(rho_ref, u = 0) of the model
//   (w_i rho_ref for the pseudopotential, rho_ref delta_i0 for the free
//   energy) and rho_ref = 0 for FP64 storage.  A step pulls
//   f_i(x) = s_i + g*_i(x - c_i) (streaming of Eq. 1), so reads are shifted
//   by at most one node and writes are aligned and coalesced.
//
// One step = one launch of a fused kernel.  A workgroup of BX threads owns a
// strip of BX columns and a segment of LY rows and sweeps it row by row:
//   1. pull row y+H (H = 1 for P, 2 for FE) into registers, form rho
//      (Eq. 6a) and the row of psi (Eq. 11) or rho into an LDS ring that
//      also holds H halo columns on each side;
//   2. FE only: form mu = mu_b - kappa lap(rho) (Sec. 2.2, Eq. 24) for row
//      y+1 into a second LDS ring;
//   3. collide row y in moment space with the model's force / source terms
//      read from the 3x3 LDS stencil, and store it.
// Halo rows at the segment ends and the H halo columns are recomputed from
// the populations.  No MFMA: the update is a bandwidth-bound stencil.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_math.h"

// Multiply-adds are fused only within one expression, never across
// statements: the fused kernels (two steps per launch) must round exactly
// as the single-step kernels do, and cross-statement fusion depends on the
// surrounding code.
#pragma clang fp contract(on)

namespace lbmk {

enum { EOS_VDW = 0, EOS_CS = 1 };
enum { MODEL_P = 0, MODEL_FE = 1 };

// Kernel-argument parameter block in the compute type C.
template <class C>
struct KParams {
  int nx, ny;
  int nstrips, nseg, LY;
  int xcd_remap;  // 1: map workgroups so that each XCD gets a contiguous
                  // band of tiles (neighbouring tiles share its L2)
  int rowpitch;   // population elements per lattice row (576 per 64 columns)
  int walls;      // 1: no-slip walls on the rows y = 0 and ny - 1 (observation
                  // kernels; the step kernels take it as a template argument)
  C a, b, RT;
  C lam_e, lam_z, lam_q, lam_nu;  // 1/tau of the e, zeta, q, p rows (Eq. 3)
  C hl_e, hl_z, hl_q, hl_nu;      // 1 - lam/2 (Eq. 1 forcing factor)
  C sig_e, sig_z;  // P: 12 kappa^P sigma^Li/(tau - 1/2), multiplies G^2|S|^2
  C qa, qb;        // P: Q tensor coefficients, see q_terms()
  C kappa;         // FE
  C fx, fy;        // constant body force
  C ax, rho_ave;   // droplet-collision drive a(x) |rho - rho_ave| (0: off now)
  int x_split;     // a = +ax for x <= x_split, -ax beyond
  C A;             // FE: viscosity-tuning A of Eq. 20 (0: off)
  C g, grho0, gy0; // FE gravity (Sec. 2.2): p_g = grho0 g (y - gy0) in Eq. 20,
                   // buoyancy -(rho - grho0) g in y, d_y p_g = grho0 g in Eq. 21
                   // (g = 0: off; walls only)
  double* uax;     // FE with A != 0: velocity field of the current step
  double* uay;
  C rho_ref;       // sum of the storage shift s_i
  C s0, sax, sdg;  // storage shift for i = 0, axis and diagonal velocities
  // Reference terms for chemical-potential differences (shifted storage):
  C inv_rho_ref;   // 1 / rho_ref
  C om_ref;        // 1 - b rho_ref (vdW) or 1 - b rho_ref / 4 (CS)
  C inv_om_ref;    // 1 / om_ref
  C inv_om_ref3;   // 1 / om_ref^3
};


template <class C>
__device__ __forceinline__ C d_sqrt(C v) {
  if constexpr (sizeof(C) == 4) return sqrtf(v); else return sqrt(v);
}
// Logarithms of the chemical potential: the reduced-range atanh series of
// lbm_math.h (a few ulps, a third of the library functions' instructions).
template <class C>
__device__ __forceinline__ C d_log(C v) {
  if constexpr (sizeof(C) == 4) return logf(v); else return lbmm::ln_f64(v);
}

// Fused multiply-add a b + c in the compute type.
template <class C>
__device__ __forceinline__ C fmad(C a, C b, C c) {
  if constexpr (sizeof(C) == 4) return __builtin_fmaf(a, b, c); else return __builtin_fma(a, b, c);
}

// Reciprocal in the compute type.  FP32 (shifted storage) takes the
// hardware reciprocal (1 ulp) instead of the correctly rounded division
// sequence: the FP32 step is bound by its vector ALU, and an ulp here is
// below the storage rounding its error bounds already carry.  FP64 refines
// the hardware estimate by two Newton steps, r <- r + r (1 - v r), each
// squaring the relative error: within an ulp or so of 1/v for the normal,
// positive arguments the step divides by (densities and 1 - b rho), in 5
// instructions instead of the division sequence's 10 (the free-energy FP64
// step is bound by its vector ALU as much as by HBM).
template <class C>
__device__ __forceinline__ C recip(C v) {
  if constexpr (sizeof(C) == 4) {
    return __builtin_amdgcn_rcpf(v);
  } else {
    double r = __builtin_amdgcn_rcp(v);
    double e = fma(-v, r, 1.0);
    r = fma(r, e, r);
    e = fma(-v, r, 1.0);
    return fma(r, e, r);
  }
}

// ---- equations of state ---------------------------------------------------
// Carnahan-Starling (Eq. 28) and van der Waals pressure.
template <int EOS, class C>
__device__ __forceinline__ C eos_p(C rho, const KParams<C>& kp) {
  if constexpr (EOS == EOS_CS) {
    C e = kp.b * rho * C(0.25);
    C om = C(1) - e;
    C num = C(1) + e * (C(1) + e * (C(1) - e));
    return rho * kp.RT * num * recip(om * om * om) - kp.a * rho * rho;
  } else {
    return rho * kp.RT * recip(C(1) - kp.b * rho) - kp.a * rho * rho;
  }
}

// Bulk chemical potential: Eq. 29 (CS); for vdW the antiderivative of
// (1/rho) dp/drho, RT ln(rho/(1 - b rho)) + RT b rho/(1 - b rho) - 2 a rho.
template <int EOS, class C>
__device__ __forceinline__ C eos_mu(C rho, const KParams<C>& kp) {
  if constexpr (EOS == EOS_CS) {
    C e = kp.b * rho * C(0.25);
    C om = C(1) - e;
    return kp.RT * (C(3) - e) * recip(om * om * om) + kp.RT * d_log(rho) + kp.RT -
           C(2) * kp.a * rho;
  } else {
    C inv = recip(C(1) - kp.b * rho);
    return kp.RT * d_log(rho * inv) + kp.RT * kp.b * rho * inv -
           C(2) * kp.a * rho;
  }
}

template <class C>
__device__ __forceinline__ C d_log1p(C v) {
  if constexpr (sizeof(C) == 4) return lbmm::ln1p_f32(v); else return log1p(v);
}

// Chemical potential up to a constant, from the density deviation
// d = rho - rho_ref.  FP64 storage (rho_ref = 0): mu_b(d) itself.  Shifted
// storage: mu_b(rho_ref + d) - mu_b(rho_ref) written so that every term is
// O(d) with full relative precision (log1p for the logarithms; factored
// differences of the rational terms), because only differences of mu enter
// the force and an O(1) float mu_b would put 2^-24 noise on them.
//   vdW: RT ln(1 + d/rho_r) - RT ln(1 - b d/(1 - b rho_r))
//        + RT b d / ((1 - b rho)(1 - b rho_r)) - 2 a d
//   CS, u = 1 - b rho/4: RT [g(u) - g(u_r)] + RT ln(1 + d/rho_r) - 2 a d with
//        g = (2 + u)/u^3 and g(u) - g(u_r) = (b d/4) [2 (u_r^2 + u u_r + u^2)/
//        (u^3 u_r^3) + (u + u_r)/(u^2 u_r^2)]
template <int EOS, class C>
__device__ __forceinline__ C mu_dev(C d, const KParams<C>& kp) {
  if constexpr (sizeof(C) == 8) {
    return eos_mu<EOS>(kp.rho_ref + d, kp);
  } else {
    C lr = kp.RT * d_log1p(d * kp.inv_rho_ref);
    if constexpr (EOS == EOS_CS) {
      // both rational terms over the common denominator u^3 u_r^3:
      // [2 (u_r^2 + u u_r + u^2) + (u + u_r) u u_r] / (u^3 u_r^3)
      C u = kp.om_ref - kp.b * d * C(0.25), ur = kp.om_ref;
      C num = C(2) * (ur * ur + u * ur + u * u) + (u + ur) * u * ur;
      C dg = kp.b * d * C(0.25) * num * recip(u * u * u) * kp.inv_om_ref3;
      return kp.RT * dg + lr - C(2) * kp.a * d;
    } else {
      C om = kp.om_ref - kp.b * d;  // 1 - b rho
      return lr - kp.RT * d_log1p(-kp.b * d * kp.inv_om_ref) +
             kp.RT * kp.b * d * recip(om) * kp.inv_om_ref - C(2) * kp.a * d;
    }
  }
}

template <int MODEL, int EOS, class C>
__device__ __forceinline__ unsigned domain_flags(C rho, const KParams<C>& kp) {
  unsigned fl = 0;
  if (!__builtin_isfinite(rho)) fl |= LBM_FLAG_NONFINITE;
  C lim = (EOS == EOS_CS) ? kp.b * rho * C(0.25) : kp.b * rho;
  if (!(lim < C(1))) fl |= LBM_FLAG_EOS_DOMAIN;
  if (MODEL == MODEL_FE && !(rho > C(0))) fl |= LBM_FLAG_EOS_DOMAIN;
  return fl;
}

// Yuan-Schaefer potential, Eq. 11 with G = -1: psi^2 = 2 (rho c_s^2 - p).
// A negative psi^2 is clamped to zero and flagged.
template <int EOS, class C>
__device__ __forceinline__ C psi_of(C rho, const KParams<C>& kp, unsigned& fl) {
  C arg = C(2) * (rho * C(1.0 / 3.0) - eos_p<EOS>(rho, kp));
  if (arg < C(0)) {
    fl |= LBM_FLAG_PSI_CLAMP;
    arg = C(0);
  }
  return d_sqrt(arg);
}

// ---- streaming ------------------------------------------------------------
// Population loads and stores.  NT bit 0: non-temporal stores, bit 1:
// non-temporal loads (each population is read and written once per step;
// the working set is far larger than L2 and the infinity cache).
template <int NT, class S>
__device__ __forceinline__ S ld(const S* p) {
  if constexpr (NT & 2) return __builtin_nontemporal_load(p); else return *p;
}
template <int NT, class S>
__device__ __forceinline__ void st(S* p, S v) {
  if constexpr (NT & 1) __builtin_nontemporal_store(v, p); else *p = v;
}

// Column offset of x inside a row of the blocked layout.
__device__ __forceinline__ int colo(int x) { return (x >> 6) * 576 + (x & 63); }

// Pulled deviations g_i(x, y) = g*_i(x - c_i) for one node: rm / r0 / rp are
// the row offsets of y-1, y, y+1 and cm / c0 / cp the column offsets of
// x-1, x, x+1 (periodic wrap already applied); velocity i adds 64 i.
template <class S, class C, int NT = 0>
__device__ __forceinline__ void pull9(const S* __restrict__ src, int rm, int r0,
                                      int rp, int cm, int c0, int cp, C g[9]) {
  g[0] = (C)ld<NT>(&src[r0 + c0]);
  g[1] = (C)ld<NT>(&src[r0 + cm + 64]);
  g[2] = (C)ld<NT>(&src[rm + c0 + 128]);
  g[3] = (C)ld<NT>(&src[r0 + cp + 192]);
  g[4] = (C)ld<NT>(&src[rp + c0 + 256]);
  g[5] = (C)ld<NT>(&src[rm + cm + 320]);
  g[6] = (C)ld<NT>(&src[rm + cp + 384]);
  g[7] = (C)ld<NT>(&src[rp + cp + 448]);
  g[8] = (C)ld<NT>(&src[rp + cm + 512]);
}

template <class C>
__device__ __forceinline__ C sum9(const C g[9]) {
  return ((g[0] + (g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8])));
}

// ---- the 3x3 stencils -----------------------------------------------------
// Neighbour values of a field around the node, indices in Eq. 2 order:
// v[1..4] = E, N, W, S; v[5..8] = NE, NW, SW, SE; v[0] = centre.
// Shan-Chen sum S = sum_i omega_i v(x + c_i) c_i (Eq. 10).  Since
// omega_i = 3 w_i = w_i / c_s^2 this is also the 9-point gradient of Eq. 24.
template <class C>
__device__ __forceinline__ void grad_sum(const C v[9], C& sx, C& sy) {
  sx = (v[1] - v[3]) * C(1.0 / 3.0) + ((v[5] - v[7]) - (v[6] - v[8])) * C(1.0 / 12.0);
  sy = (v[2] - v[4]) * C(1.0 / 3.0) + ((v[5] - v[7]) + (v[6] - v[8])) * C(1.0 / 12.0);
}

// Q tensor of Eq. 30: with C_i_ab = alpha delta_ab + beta c_ia c_ib,
// alpha = C_1 G - C_2 c_s^2 and beta = C_2 + kappa^Li G/2 (qa, qb), returns
// Qxx + Qyy, Qxx - Qyy and Qxy.
// Neighbour differences v_i - v_0 are formed first: for a smooth field they
// are exact (Sterbenz), so the stencil sums keep full relative precision
// instead of losing it to the cancellation of four O(v) terms.
template <class C>
__device__ __forceinline__ void diff_sums(const C v[9], C& ax, C& dg) {
  C p = v[0];
  ax = ((v[1] - p) + (v[2] - p)) + ((v[3] - p) + (v[4] - p));
  dg = ((v[5] - p) + (v[6] - p)) + ((v[7] - p) + (v[8] - p));
}

template <class C>
__device__ __forceinline__ void q_terms(const C v[9], C qa, C qb, C& qs, C& qd,
                                        C& qxy) {
  C p = v[0];
  C ax, dg;
  diff_sums(v, ax, dg);
  C sw = ax * C(1.0 / 3.0) + dg * C(1.0 / 12.0);  // sum omega_i (v_i - v)
  C sc = ax * C(1.0 / 3.0) + dg * C(1.0 / 6.0);   // sum omega_i |c_i|^2 (v_i - v)
  qs = p * (C(2) * qa * sw + qb * sc);
  qd = p * qb * (((v[1] - v[2]) + (v[3] - v[4])) * C(1.0 / 3.0));
  qxy = p * qb * (((v[5] - v[6]) + (v[7] - v[8])) * C(1.0 / 12.0));
}

// 9-point Laplacian of Eq. 24: (2/c_s^2) sum_i w_i (v_i - v).
template <class C>
__device__ __forceinline__ C lap9(const C v[9]) {
  C ax, dg;
  diff_sums(v, ax, dg);
  return ax * C(2.0 / 3.0) + dg * C(1.0 / 6.0);
}

// Gather the 3x3 neighbourhood of LDS column j from three LDS rows.
template <class C>
__device__ __forceinline__ void gather(const C* bot, const C* mid, const C* top,
                                       int j, C v[9]) {
  v[0] = mid[j];
  v[1] = mid[j + 1];
  v[2] = top[j];
  v[3] = mid[j - 1];
  v[4] = bot[j];
  v[5] = top[j + 1];
  v[6] = top[j - 1];
  v[7] = bot[j - 1];
  v[8] = bot[j + 1];
}

// ---- collision in moment space --------------------------------------------
// Eq. 1 written for the deviations g = f - s (s an equilibrium at rest, so
// M s only has rho, e and zeta components):
//   m* = m - Lambda (m - m^eq) + (I - Lambda/2) mF + mC,  g* = M^-1 m*,
// with M the moment matrix of Eq. 48, M^-1 of Eq. 49 applied in factored
// form, m^eq of Eq. 4 (P) or Eq. 20 (FE), mF of Eq. 32 (P) or the moments of
// Eq. 21 (FE), mC of Eq. 13 (P).  The j rows reduce exactly to j + F.
// With AV = 1 (free energy) the equilibrium also carries the A terms of
// Eq. 20: a_div = rho A div(u) and a_xx, a_xy, their p_xx and p_xy moments.
//
// FE with gravity (Sec. 2.2): pg = p_g at the node adds w_i p_g / c_s^2
// (i > 0) and -(1 - w_0) p_g / c_s^2 (i = 0) to the equilibrium, whose
// moments are e 6 p_g and zeta -9 p_g; dpg = d_y p_g replaces F_y by
// F_y - d_y p_g in the velocity-dependent part of Eq. 21, which moves the
// e / zeta forcing by -/+ 6 u_y dpg, p_xx by 2 u_y dpg and p_xy by -u_x dpg.
template <int MODEL, int AV = 0, class C>
__device__ __forceinline__ void collide(C g[9], C drho, C rho, C Fx, C Fy,
                                        C t0, C t1, C t2, C t3,
                                        const KParams<C>& kp, C& ux_out, C& uy_out,
                                        C a_div = C(0), C a_xx = C(0), C a_xy = C(0),
                                        C pg = C(0), C dpg = C(0)) {
  // P: t0 = G^2 |S|^2, t1 = Qxx + Qyy, t2 = Qxx - Qyy, t3 = Qxy.
  // FE: t0 = d_x rho, t1 = d_y rho.
  C jx = (g[1] - g[3]) + ((g[5] - g[7]) - (g[6] - g[8]));
  C jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
  C inv = recip(rho);
  C ux = (jx + C(0.5) * Fx) * inv;  // Eq. 6b
  C uy = (jy + C(0.5) * Fy) * inv;
  ux_out = ux;
  uy_out = uy;

  C axs = (g[1] + g[2]) + (g[3] + g[4]);
  C dgs = (g[5] + g[6]) + (g[7] + g[8]);
  C me = C(-4) * g[0] - axs + C(2) * dgs;
  C mz = C(4) * g[0] - C(2) * axs + dgs;
  C dx1 = g[1] - g[3], dy1 = g[2] - g[4];
  C d57 = g[5] - g[7], d68 = g[6] - g[8];
  C mqx = C(-2) * dx1 + (d57 - d68);
  C mqy = C(-2) * dy1 + (d57 + d68);
  C mpxx = (g[1] + g[3]) - (g[2] + g[4]);
  C mpxy = (g[5] + g[7]) - (g[6] + g[8]);

  C ru2 = rho * (ux * ux + uy * uy);
  C eqe, eqz;
  if constexpr (MODEL == MODEL_P) {
    eqe = C(-2) * drho + C(3) * ru2;
    eqz = drho - C(3) * ru2;
  } else {
    eqe = C(-4) * drho + C(3) * ru2;
    eqz = C(4) * drho - C(3) * ru2;
  }
  C eqqx = -rho * ux, eqqy = -rho * uy;
  C eqpxx = rho * (ux * ux - uy * uy);
  C eqpxy = rho * ux * uy;
  if constexpr (AV != 0) {
    // moments of w_i rho (c c - c_s^2 I) : c_s^2 A S / (2 c_s^4) and of the
    // rest term -w_0 rho A div(u): e 2 rho A div u, zeta -2 rho A div u,
    // p_xx (2/3) rho A (d_x u_x - d_y u_y), p_xy (1/3) rho A (d_x u_y + d_y u_x)
    eqe += C(2) * a_div;
    eqz -= C(2) * a_div;
    eqpxx += a_xx;
    eqpxy += a_xy;
  }
  if constexpr (MODEL == MODEL_FE) {
    eqe += C(6) * pg;
    eqz -= C(9) * pg;
  }

  C uF = ux * Fx + uy * Fy;
  C Fe, Fz, Fpxx, Fpxy;
  C Ce = C(0), Cz = C(0), Cpxx = C(0), Cpxy = C(0);
  if constexpr (MODEL == MODEL_P) {
    Fe = C(6) * uF + kp.sig_e * t0;
    Fz = C(-6) * uF - kp.sig_z * t0;
    Fpxx = C(2) * (ux * Fx - uy * Fy);
    Fpxy = ux * Fy + uy * Fx;
    Ce = C(1.5) * t1 * kp.lam_e;
    Cz = C(-1.5) * t1 * kp.lam_z;
    Cpxx = -t2 * kp.lam_nu;
    Cpxy = -t3 * kp.lam_nu;
  } else {
    C ug = ux * t0 + uy * t1;
    Fe = C(6) * uF + C(4) * ug - C(6) * uy * dpg;
    Fz = -Fe;
    Fpxx = C(2) * (ux * Fx - uy * Fy) + C(2.0 / 3.0) * (ux * t0 - uy * t1) + C(2) * uy * dpg;
    Fpxy = ux * Fy + uy * Fx + C(1.0 / 3.0) * (ux * t1 + uy * t0) - ux * dpg;
  }

  C se = me - kp.lam_e * (me - eqe) + kp.hl_e * Fe + Ce;
  C sz = mz - kp.lam_z * (mz - eqz) + kp.hl_z * Fz + Cz;
  C sjx = jx + Fx;
  C sjy = jy + Fy;
  C sqx = mqx - kp.lam_q * (mqx - eqqx) - kp.hl_q * Fx;
  C sqy = mqy - kp.lam_q * (mqy - eqqy) - kp.hl_q * Fy;
  C spxx = mpxx - kp.lam_nu * (mpxx - eqpxx) + kp.hl_nu * Fpxx + Cpxx;
  C spxy = mpxy - kp.lam_nu * (mpxy - eqpxy) + kp.hl_nu * Fpxy + Cpxy;

  // M^-1 (Eq. 49) in factored form.  The rest population is closed on the
  // mass, g*_0 = rho* - sum_{i>0} g*_i (row 0 of M is all ones), which is
  // the same number without the bias a rounded 1/9 would put on the mass.
  // (the multiply-adds written out: each population is two fused steps)
  C r9 = drho * C(1.0 / 9.0);
  C Aax = r9 - se * C(1.0 / 36.0) - sz * C(1.0 / 18.0);
  C Adg = r9 + se * C(1.0 / 18.0) + sz * C(1.0 / 36.0);
  C dX = sjx - sqx, dY = sjy - sqy;
  C X5 = sjx * C(1.0 / 6.0) + sqx * C(1.0 / 12.0);
  C Y5 = sjy * C(1.0 / 6.0) + sqy * C(1.0 / 12.0);
  C Ap = Adg + X5, Am = Adg - X5;
  g[1] = fmad(spxx, C(0.25), fmad(dX, C(1.0 / 6.0), Aax));
  g[2] = fmad(-spxx, C(0.25), fmad(dY, C(1.0 / 6.0), Aax));
  g[3] = fmad(spxx, C(0.25), fmad(-dX, C(1.0 / 6.0), Aax));
  g[4] = fmad(-spxx, C(0.25), fmad(-dY, C(1.0 / 6.0), Aax));
  g[5] = fmad(spxy, C(0.25), Ap + Y5);
  g[6] = fmad(-spxy, C(0.25), Am + Y5);
  g[7] = fmad(spxy, C(0.25), Am - Y5);
  g[8] = fmad(-spxy, C(0.25), Ap - Y5);
  g[0] = drho - (((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8])));
}

// ---- tile mapping -----------------------------------------------------------
__device__ __forceinline__ int tile_index(int xcd_remap) {
  int b = blockIdx.x;
  if (!xcd_remap) return b;
  // Workgroups are dispatched round-robin over the 8 XCDs; give XCD k the
  // contiguous band [k*nb/8, (k+1)*nb/8) of tiles so that a tile's
  // neighbours (and their shared halo lines) usually sit in the same L2.
  int nb = gridDim.x;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Sticky-flag commit at the end of a kernel, called by every thread of the
// workgroup: OR the flag bits across each wavefront by ballot, then across
// the workgroup in LDS, and issue one global atomic per workgroup, only if
// it adds bits not yet set (a run that has gone non-finite would otherwise
// issue one atomic per node and step).
__device__ __forceinline__ void commit_flags(unsigned fl, unsigned* __restrict__ flags,
                                             unsigned* s_flag) {
  unsigned long long b0 = __ballot(fl & 1u), b1 = __ballot(fl & 2u), b2 = __ballot(fl & 4u);
  unsigned w = (b0 ? 1u : 0u) | (b1 ? 2u : 0u) | (b2 ? 4u : 0u);
  if (w && (threadIdx.x & 63) == 0) atomicOr(s_flag, w);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned v = *s_flag;
    if (v && (v & ~__atomic_load_n(flags, __ATOMIC_RELAXED))) atomicOr(flags, v);
  }
}

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ---- no-slip walls (Sec. 5.3) -----------------------------------------------
// Rows y = 0 and ny - 1 are wall rows: fluid nodes held at u = 0 by the
// closure of Zou and He.  Past a wall the density stencils see the mirror
// image of the rows inside.
__device__ __forceinline__ int seen_row(int y, int ny) {
  return y < 0 ? -y : (y > ny - 1 ? 2 * (ny - 1) - y : y);
}

// +1 on the bottom wall row (the populations with c_y = +1 arrive from
// outside), -1 on the top one, 0 elsewhere.
__device__ __forceinline__ int wall_side(int y, int ny) {
  return y == 0 ? 1 : (y == ny - 1 ? -1 : 0);
}

// The closure in two parts.  A wall node must carry sum_i g_i c_i =
// (jx, jy) = -F/2 so that Eq. 6b gives u = 0; the normal unknown equals its
// opposite (non-equilibrium bounce-back at zero wall velocity) and the two
// diagonal unknowns take the rest.  wall_fill applies jy = -fy/2 with
// jx = 0: the diagonal pair's sum, hence the density, does not depend on jx.
// wall_fx adds the jx = -Fx/2 part once the tangential force is known.  The
// deviations g = f - s obey the same relations since the shift s is
// symmetric under c -> -c.
template <class C>
__device__ __forceinline__ void wall_fill(C g[9], int side, C fy) {
  // both walls' values from the original populations, then selected by
  // value: branches on `side` writing different slots would be merged into
  // indexed stores, which put g[] in scratch memory
  const C t = C(0.5) * (g[1] - g[3]);
  const C h = C(-0.25) * fy;  // jy / 2
  const bool b = side > 0;
  const C n2 = g[4], n5 = g[7] - t + h, n6 = g[8] + t + h;  // bottom wall
  const C s4 = g[2], s7 = g[5] + t - h, s8 = g[6] - t - h;  // top wall
  g[2] = b ? n2 : g[2];
  g[5] = b ? n5 : g[5];
  g[6] = b ? n6 : g[6];
  g[4] = b ? g[4] : s4;
  g[7] = b ? g[7] : s7;
  g[8] = b ? g[8] : s8;
}

// Closure of a free-energy wall row, whose normal force is fy plus, with
// gravity, the buoyancy -(rho - rho_0) g of its own density: the density
// with the normal part closed at zero, r0, moves by side j_y with
// j_y = -F_y(rho)/2, a linear equation for rho.  Without gravity this is
// wall_fill with fy.
template <class C>
__device__ __forceinline__ void wall_fill_fe(C g[9], int side, const KParams<C>& kp) {
  C fy = kp.fy;
  if (kp.g != C(0)) {
    // r0: the known populations plus the unknowns closed at j_y = 0 (the
    // normal one equals its opposite, the diagonal pair sums to the pair
    // opposite it): g0 + g1 + g3 + 2 (g4 + g7 + g8) on the bottom wall,
    // g0 + g1 + g3 + 2 (g2 + g5 + g6) on the top one
    const bool b = side > 0;
    const C in = b ? (g[4] + g[7]) + g[8] : (g[2] + g[5]) + g[6];
    const C r0 = kp.rho_ref + ((g[0] + (g[1] + g[3])) + C(2) * in);
    const C sd = b ? C(1) : C(-1);
    const C rho = (r0 - sd * C(0.5) * (kp.fy + kp.g * kp.grho0)) / (C(1) - sd * C(0.5) * kp.g);
    fy = kp.fy - (rho - kp.grho0) * kp.g;
  }
  wall_fill(g, side, fy);
}

template <class C>
__device__ __forceinline__ void wall_fx(C g[9], int side, C Fx) {
  const C q = C(0.25) * Fx;  // -jx / 2
  const bool b = side > 0;
  g[5] = b ? g[5] - q : g[5];
  g[6] = b ? g[6] + q : g[6];
  g[7] = b ? g[7] : g[7] + q;
  g[8] = b ? g[8] : g[8] - q;
}

// ---- per-tile step bodies -------------------------------------------------
// One workgroup of BX threads updates the tile [x0, x0 + BX) x [y0, y0 + LY)
// of one lattice (clipped to the lattice).  The single-lattice kernels and
// the batched kernels differ only in how they find the tile.
//
// With CHK = 1 the step also measures convergence: the velocity of Eq. 6b
// at every node is compared with the one stored at the previous check
// (ck.uxp / ck.uyp, overwritten), and the workgroup's max |u - u_prev| is
// folded into *ck.du (the double's bit pattern, atomically maxed: for
// non-negative doubles the unsigned order is the numeric order).
template <class C>
struct ChkOut {
  C* uxp;
  C* uyp;
  unsigned long long* du;
};

template <int CHK, class C>
__device__ __forceinline__ void chk_node(const ChkOut<C>& ck, int n, C ux, C uy, C& dmax) {
  if constexpr (CHK != 0) {
    C dx = ux - ck.uxp[n], dy = uy - ck.uyp[n];
    C d = d_sqrt(dx * dx + dy * dy);
    dmax = (d > dmax || d != d) ? d : dmax;  // keep NaN: it must not look converged
    ck.uxp[n] = ux;
    ck.uyp[n] = uy;
  }
}

template <int CHK, class C>
__device__ __forceinline__ void chk_commit(const ChkOut<C>& ck, C dmax, double* s_du) {
  if constexpr (CHK != 0) {
    double d = (double)dmax;
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_xor(d, off, 64);
      d = (o > d || o != o) ? o : d;
    }
    if ((threadIdx.x & 63) == 0) s_du[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = s_du[0];
      for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = (s_du[i] > m || s_du[i] != s_du[i]) ? s_du[i] : m;
      unsigned long long bits = (m != m) ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(m);
      atomicMax(ck.du, bits);
    }
  }
}

// Eq. 24 gradient at (x, y) of a velocity component held in global memory
// (the A term of Eq. 20).  Past a wall the mirrored row enters with its sign
// flipped, so the velocity vanishes on the wall row as the closure imposes.
template <class C>
__device__ __forceinline__ void grad_u(const double* __restrict__ u, int nx, int ny,
                                       int walls, int x, int y, C& gx, C& gy) {
  const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  int ym = wrapi(y - 1, ny), yp = wrapi(y + 1, ny);
  C sm = C(1), sp = C(1);
  if (walls) {
    if (y == 0) { ym = 1; sm = C(-1); }
    if (y == ny - 1) { yp = ny - 2; sp = C(-1); }
  }
  const double* r0 = u + (size_t)y * nx;
  const double* rm = u + (size_t)ym * nx;
  const double* rp = u + (size_t)yp * nx;
  C v[9];
  v[0] = (C)r0[x];
  v[1] = (C)r0[xp];
  v[2] = sp * (C)rp[x];
  v[3] = (C)r0[xm];
  v[4] = sm * (C)rm[x];
  v[5] = sp * (C)rp[xp];
  v[6] = sp * (C)rp[xm];
  v[7] = sm * (C)rm[xm];
  v[8] = sm * (C)rm[xp];
  grad_sum(v, gx, gy);
}

// x force of the droplet-collision drive at column x (Sec. 5.4).
template <class C>
__device__ __forceinline__ C drive_fx(const KParams<C>& kp, int x, C rho) {
  C d = rho - kp.rho_ave;
  d = d < C(0) ? -d : d;
  return (x <= kp.x_split ? kp.ax : -kp.ax) * d;
}

// Pseudopotential step on one tile.  GEN = 1: the general kernel, which
// also takes the options switched at run time -- no-slip walls in y
// (Sec. 5.3, kp.walls) and the droplet-collision drive (Sec. 5.4, kp.ax).
template <int EOS, class S, class C, int BX, int NT, int CHK, int GEN = 0>
__device__ __forceinline__ void tile_p(const S* __restrict__ src, S* __restrict__ dst,
                                       const KParams<C>& kp, unsigned* __restrict__ flags,
                                       int x0, int y0, const ChkOut<C>& ck) {
  __shared__ C psi_s[4][BX + 2];
  __shared__ unsigned s_flag;
  __shared__ double s_du[BX / 64];
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool active = t < w;
  const int x = x0 + (active ? t : 0);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);
  // halo column handled by lanes 0 (left) and 1 (right)
  const bool hl = t < 2;
  const int hx = (t == 0) ? wrapi(x0 - 1, nx) : wrapi(x0 + w, nx);
  const int hxm = (hx == 0) ? nx - 1 : hx - 1;
  const int hxp = (hx == nx - 1) ? 0 : hx + 1;
  const int hcm = colo(hxm), hc0 = colo(hx), hcp = colo(hxp);
  const int hj = (t == 0) ? 0 : w + 1;

  unsigned fl = 0;
  C dmax = C(0);
  C gc[9], gn[9];
  C drho_c = C(0), drho_n = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };
  // row whose populations give the potential seen at row y, and its wall side
  auto seen = [&](int y) {
    if constexpr (GEN != 0) return kp.walls ? seen_row(y, ny) : y;
    else return y;
  };
  auto close = [&](int ys, C g[9]) {
    if constexpr (GEN != 0) {
      const int sd = kp.walls ? wall_side(ys, ny) : 0;
      if (sd) wall_fill(g, sd, kp.fy);
    }
  };

  // Rows y0-1 (psi only) and y0 (psi and populations).
  for (int r = 0; r < 2; ++r) {
    const int y = seen(y0 - 1 + r);
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    // halo loads first, so that they are in flight with the interior ones:
    // waiting for the interior loads then covers both (one round trip, not
    // two, for the wavefront that holds the halo lanes)
    C h[9];
    if (hl) pull9<S, C, NT>(src, rm, r0, rp, hcm, hc0, hcp, h);
    if (active) {
      C g[9];
      pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
      close(y, g);
      C dr = sum9(g);
      C rho = kp.rho_ref + dr;
      fl |= domain_flags<MODEL_P, EOS>(rho, kp);
      psi_s[r][t + 1] = psi_of<EOS>(rho, kp, fl);
      if (r == 1) {
        for (int i = 0; i < 9; ++i) gc[i] = g[i];
        drho_c = dr;
      }
    }
    if (hl) {
      close(y, h);
      C rho = kp.rho_ref + sum9(h);
      psi_s[r][hj] = psi_of<EOS>(rho, kp, fl);
    }
  }

  for (int k = 0; k < ly; ++k) {
    const int y = y0 + k;
    // pull row y+1 into the ring
    {
      const int yn = seen(y + 1);
      const int r0 = rowoff(yn), rm = rowoff(yn - 1), rp = rowoff(yn + 1);
      C* row = psi_s[(k + 2) & 3];
      C h[9];
      if (hl) pull9<S, C, NT>(src, rm, r0, rp, hcm, hc0, hcp, h);  // halo first
      if (active) {
        pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, gn);
        close(yn, gn);
        drho_n = sum9(gn);
        C rho = kp.rho_ref + drho_n;
        fl |= domain_flags<MODEL_P, EOS>(rho, kp);
        row[t + 1] = psi_of<EOS>(rho, kp, fl);
      }
      if (hl) {
        close(yn, h);
        C rho = kp.rho_ref + sum9(h);
        row[hj] = psi_of<EOS>(rho, kp, fl);
      }
    }
    __syncthreads();
    if (active) {
      C v[9];
      gather(psi_s[k & 3], psi_s[(k + 1) & 3], psi_s[(k + 2) & 3], t + 1, v);
      C sx, sy;
      grad_sum(v, sx, sy);
      // Eq. 10 with G = -1: F = psi S; |F_int|^2/psi^2 = G^2 |S|^2.
      C Fx = v[0] * sx + kp.fx;
      C Fy = v[0] * sy + kp.fy;
      C K = sx * sx + sy * sy;
      C qs, qd, qxy;
      q_terms(v, kp.qa, kp.qb, qs, qd, qxy);
      C rho = kp.rho_ref + drho_c;
      if constexpr (GEN != 0) {
        if (kp.ax != C(0)) Fx += drive_fx(kp, x, rho);
        // the mirrored rows make S_y exactly zero on a wall row, so Fy = fy
        const int sd = kp.walls ? wall_side(y, ny) : 0;
        if (sd) wall_fx(gc, sd, Fx);
      }
      C ux, uy;
      collide<MODEL_P>(gc, drho_c, rho, Fx, Fy, K, qs, qd, qxy, kp, ux, uy);
      chk_node<CHK>(ck, y * nx + x, ux, uy, dmax);
      const int off = y * kp.rowpitch + c0;
#pragma unroll
      for (int i = 0; i < 9; ++i) st<NT>(&dst[off + 64 * i], (S)gc[i]);
#pragma unroll
      for (int i = 0; i < 9; ++i) gc[i] = gn[i];
      drho_c = drho_n;
    }
  }
  commit_flags(fl, flags, &s_flag);
  chk_commit<CHK>(ck, dmax, s_du);
}

// Software-pipelined variant: the populations of row y+2 (interior and
// halo columns) are loaded at the top of the iteration that collides row y
// and only consumed one iteration later, so their memory latency overlaps
// the psi row, the barrier and the collision in between.  The interior
// loads are issued unconditionally (lanes past the lattice edge read a valid
// column and discard it) and after the halo loads, and the last row is
// peeled off the loop: the wait for a row's populations can then count the
// next row's loads as issued and leaves them in flight (a load inside a
// branch that may be skipped would force a wait for every outstanding load).
template <int EOS, class S, class C, int BX, int NT>
__device__ __forceinline__ void tile_p_pipe(const S* __restrict__ src, S* __restrict__ dst,
                                            const KParams<C>& kp, unsigned* __restrict__ flags,
                                            int x0, int y0) {
  __shared__ C psi_s[4][BX + 2];
  __shared__ unsigned s_flag;
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool active = t < w;
  const int x = x0 + (active ? t : 0);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);
  const bool hl = t < 2;
  const int hx = (t == 0) ? wrapi(x0 - 1, nx) : wrapi(x0 + w, nx);
  const int hxm = (hx == 0) ? nx - 1 : hx - 1;
  const int hxp = (hx == nx - 1) ? 0 : hx + 1;
  const int hcm = colo(hxm), hc0 = colo(hx), hcp = colo(hxp);
  const int hj = (t == 0) ? 0 : w + 1;

  unsigned fl = 0;
  C gc[9], gn[9], hn[9];
  C drho_c = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };
  auto pull_row = [&](int y, C g[9], C h[9]) {
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    if (hl) pull9<S, C, NT>(src, rm, r0, rp, hcm, hc0, hcp, h);
    pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
  };
  // psi row from pulled populations; returns the interior density deviation
  auto psi_row = [&](const C g[9], const C h[9], C* row) {
    C dr = sum9(g);
    if (active) {
      C rho = kp.rho_ref + dr;
      fl |= domain_flags<MODEL_P, EOS>(rho, kp);
      row[t + 1] = psi_of<EOS>(rho, kp, fl);
    }
    if (hl) row[hj] = psi_of<EOS>(kp.rho_ref + sum9(h), kp, fl);
    return dr;
  };
  auto collide_row = [&](int k) {
    if (active) {
      const int y = y0 + k;
      C v[9];
      gather(psi_s[k & 3], psi_s[(k + 1) & 3], psi_s[(k + 2) & 3], t + 1, v);
      C sx, sy;
      grad_sum(v, sx, sy);
      C Fx = v[0] * sx + kp.fx;
      C Fy = v[0] * sy + kp.fy;
      C K = sx * sx + sy * sy;
      C qs, qd, qxy;
      q_terms(v, kp.qa, kp.qb, qs, qd, qxy);
      C rho = kp.rho_ref + drho_c;
      C ux, uy;
      collide<MODEL_P>(gc, drho_c, rho, Fx, Fy, K, qs, qd, qxy, kp, ux, uy);
      const int off = y * kp.rowpitch + c0;
#pragma unroll
      for (int i = 0; i < 9; ++i) st<NT>(&dst[off + 64 * i], (S)gc[i]);
    }
  };

  {
    C g[9], h[9];
    pull_row(y0 - 1, g, h);
    psi_row(g, h, psi_s[0]);
    pull_row(y0, gc, h);
    drho_c = psi_row(gc, h, psi_s[1]);
    pull_row(y0 + 1, gn, hn);
  }

  for (int k = 0; k < ly - 1; ++k) {
    C g2[9], h2[9];
    pull_row(y0 + k + 2, g2, h2);
    C drho_n = psi_row(gn, hn, psi_s[(k + 2) & 3]);
    __syncthreads();
    collide_row(k);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      gc[i] = gn[i];
      gn[i] = g2[i];
      hn[i] = h2[i];
    }
    drho_c = drho_n;
  }
  {
    const int k = ly - 1;
    C drho_n = psi_row(gn, hn, psi_s[(k + 2) & 3]);
    __syncthreads();
    collide_row(k);
    (void)drho_n;
  }
  commit_flags(fl, flags, &s_flag);
}

// Two pseudopotential steps on one tile of a periodic lattice in one pass
// (temporal blocking): the populations after the first step, g*1, never go
// to HBM.  The workgroup has BX + 64 threads.  Lanes 0 .. BX-1 own the
// tile's columns x0 + t for both steps; the last wavefront (the halo
// wavefront) owns the columns the first step needs around the strip:
// h = 0..3 the four columns x0-2, x0-1, x0+w, x0+w+1, whose g*1 the second
// step pulls from or needs for its psi halo, and h = 4, 5 the psi-only
// columns x0-3, x0+w+2.  Per row a of the first step (rows y0-2 ..
// y0+ly+1):
//   1. pull row a+1 (the first step's populations), psi1 into an LDS ring;
//   2. collide row a (first step) -> g*1 row a in registers; the six
//      populations that stream along x go to LDS for the neighbours;
//   3. deposit g*1 row a into the second step's pulled populations: f_4, f_7,
//      f_8 complete row a-1, f_0, f_1, f_3 go to row a, f_2, f_5, f_6 to row
//      a+1; row a-1 then gives rho2 and psi2 (LDS ring);
//   4. collide row a-2 (second step) and store it.
// Every node does the arithmetic of the single-step kernel in the same
// order, so two steps of this kernel equal two single steps bit for bit.
// PF = 1 fetches each first-step row one iteration ahead of its use (FP64:
// the wait for a row leaves the next row's loads in flight; measured
// 0.33 vs 0.50 ms per step on 4096^2); PF = 0 waits at once (FP32, where the
// nine more live registers cost a wave of occupancy: 0.159 vs 0.171 ms).
template <int EOS, class S, class C, int BX, int NT, int PF>
__device__ __forceinline__ void tile_p2(const S* __restrict__ src, S* __restrict__ dst,
                                        const KParams<C>& kp, unsigned* __restrict__ flags,
                                        int x0, int y0) {
  __shared__ C psi1[4][BX + 6];   // columns x0-3 .. x0+w+2
  __shared__ C xb[6][BX + 4];     // x-moving g*1 of one row, columns x0-2 .. x0+w+1
  __shared__ C psi2[4][BX + 2];   // columns x0-1 .. x0+w
  __shared__ unsigned s_flag;
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool mainl = t < BX;
  const int h = t - BX;
  // step-1 column of this lane (offset from x0) and its duties
  int off;
  if (mainl) off = t;
  else off = (h == 0) ? -2 : (h == 1) ? -1 : (h == 2) ? w : (h == 3) ? w + 1 : (h == 4) ? -3 : w + 2;
  const bool act1 = mainl ? (t < w) : (h < 6);   // pulls and psi1
  const bool col1 = mainl ? (t < w) : (h < 4);   // first-step collision
  const bool dep2 = mainl ? (t < w) : (h == 1 || h == 2);  // second-step psi
  const bool col2 = mainl && t < w;               // second-step collision
  const int x = wrapi(x0 + (act1 ? off : 0), nx);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);
  const int j1 = off + 3;  // psi1 index
  const int jx = off + 2;  // xb index
  const int j2 = off + 1;  // psi2 index

  unsigned fl = 0;
  C gc[9], gn[9], g2[9];
  C drho_c = C(0);
  // The second step's pulled populations at the start of iteration a: P of
  // row a-2 (complete, collided in this iteration), Q of row a-1 (all but
  // f_4, f_7, f_8, which row a brings), R2 R5 R6 of row a (from row a-1).
  C P[9], Q[9], R2 = C(0), R5 = C(0), R6 = C(0);
  C drho_p = C(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i] = Q[i] = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };
  // The pulls are unconditional (a lane without a column reads a valid one
  // and discards it) and one row ahead of their use, so that the wait for a
  // row leaves the next row's loads in flight (see tile_p_pipe).
  // (PF = 0: only lanes with a column load)
  auto pull = [&](int y, C g[9]) {
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    if (PF != 0 || act1) pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
  };
  auto psi_row = [&](const C g[9], int slot) {
    C dr = C(0);
    if (act1) {
      dr = sum9(g);
      C rho = kp.rho_ref + dr;
      fl |= domain_flags<MODEL_P, EOS>(rho, kp);
      psi1[slot & 3][j1] = psi_of<EOS>(rho, kp, fl);
    }
    return dr;
  };

  // first-step rows y0-3 (psi1 only) and y0-2 (psi1 and populations);
  // psi1 slot of row r: (r - y0 + 3) & 3; psi2 slot of row r: (r - y0 + 1) & 3
  {
    C tmp[9];
    pull(y0 - 3, tmp);
    psi_row(tmp, 0);
    pull(y0 - 2, gc);
    drho_c = psi_row(gc, 1);
    if constexpr (PF != 0) pull(y0 - 1, gn);
  }
  for (int k = 0; k < ly + 4; ++k) {
    // first-step row a = y0 - 2 + k; with PF, row a + 2 is fetched here for
    // the next iteration and row a + 1 was fetched by the previous one
    if constexpr (PF != 0) pull(y0 + k, g2);
    else pull(y0 - 1 + k, gn);
    const C drho_n = psi_row(gn, k + 2);
    __syncthreads();
    if (col1) {
      C v[9];
      gather(psi1[k & 3], psi1[(k + 1) & 3], psi1[(k + 2) & 3], j1, v);
      C sx, sy;
      grad_sum(v, sx, sy);
      C Fx = v[0] * sx + kp.fx;
      C Fy = v[0] * sy + kp.fy;
      C K = sx * sx + sy * sy;
      C qs, qd, qxy;
      q_terms(v, kp.qa, kp.qb, qs, qd, qxy);
      C rho = kp.rho_ref + drho_c;
      C ux, uy;
      collide<MODEL_P>(gc, drho_c, rho, Fx, Fy, K, qs, qd, qxy, kp, ux, uy);
      // the single-step kernel stores the first step's output and loads it
      // back: round to the storage type the same way
#pragma unroll
      for (int i = 0; i < 9; ++i) gc[i] = (C)(S)gc[i];
      xb[0][jx] = gc[1];
      xb[1][jx] = gc[5];
      xb[2][jx] = gc[8];
      xb[3][jx] = gc[3];
      xb[4][jx] = gc[6];
      xb[5][jx] = gc[7];
    }
    __syncthreads();
    // deposit row a: +x movers arrive from the column on the left, -x
    // movers from the one on the right
    C l1 = C(0), l5 = C(0), r3 = C(0), r6 = C(0), dq = C(0);
    if (dep2) {
      l1 = xb[0][jx - 1];
      l5 = xb[1][jx - 1];
      r3 = xb[3][jx + 1];
      r6 = xb[4][jx + 1];
      Q[4] = gc[4];           // f_4(x, a-1) = g*1_4(x, a)
      Q[7] = xb[5][jx + 1];   // f_7(x, a-1) = g*1_7(x+1, a)
      Q[8] = xb[2][jx - 1];   // f_8(x, a-1) = g*1_8(x-1, a)
      dq = sum9(Q);
      if (k >= 2) {  // row a-1 >= y0-1: psi2 of a complete row
        C rho = kp.rho_ref + dq;
        fl |= domain_flags<MODEL_P, EOS>(rho, kp);
        psi2[(k - 2) & 3][j2] = psi_of<EOS>(rho, kp, fl);
      }
    }
    __syncthreads();
    if (k >= 4 && col2) {
      // second-step collision of row b = a-2 (psi2 rows b-1, b, b+1)
      const int b = y0 - 4 + k;
      C v[9];
      gather(psi2[(k - 4) & 3], psi2[(k - 3) & 3], psi2[(k - 2) & 3], j2, v);
      C sx, sy;
      grad_sum(v, sx, sy);
      C Fx = v[0] * sx + kp.fx;
      C Fy = v[0] * sy + kp.fy;
      C K = sx * sx + sy * sy;
      C qs, qd, qxy;
      q_terms(v, kp.qa, kp.qb, qs, qd, qxy);
      C rho = kp.rho_ref + drho_p;
      C ux, uy;
      collide<MODEL_P>(P, drho_p, rho, Fx, Fy, K, qs, qd, qxy, kp, ux, uy);
      const int o = b * kp.rowpitch + c0;
#pragma unroll
      for (int i = 0; i < 9; ++i) st<NT>(&dst[o + 64 * i], (S)P[i]);
    }
    // shift the second step's rows: a-1 -> P, a -> Q, a+1 -> R
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = Q[i];
    drho_p = dq;
    Q[0] = gc[0];
    Q[1] = l1;
    Q[3] = r3;
    Q[2] = R2;
    Q[5] = R5;
    Q[6] = R6;
    R2 = gc[2];
    R5 = l5;
    R6 = r6;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      gc[i] = gn[i];
      if constexpr (PF != 0) gn[i] = g2[i];
    }
    drho_c = drho_n;
  }
  commit_flags(fl, flags, &s_flag);
}

// Two free-energy steps on one tile of a periodic lattice in one pass
// (temporal blocking): the populations after the first step, g*1, never go
// to HBM.  The workgroup has BX + 64 threads.  Lanes 0 .. BX-1 own the
// tile's columns x0 + t for both steps; the last wavefront (the halo
// wavefront) owns the first step's columns around the strip.  The second
// step's density is needed two columns beyond the strip (its chemical
// potential one column beyond), so the first step collides three halo
// columns each side, needs the chemical potential on four and the density
// on five: halo lane h has the column x0-1-h/2 (h even) or x0+w+h/2 (h odd),
// and h < 10 / 8 / 6 / 4 / 2 form the first step's density / chemical
// potential / collision and the second step's density / chemical
// potential.
//
// One iteration k advances six stages, each on its own row, in three
// phases separated by barriers (r = the first-step row fetched at k):
//   phase 0: A(r)   pull row r, its density into the rho1 ring;
//            D(r-3) deposit g*1 of row r-3 into the second step's pulled
//                   populations (f_4, f_7, f_8 complete row r-4, whose
//                   density goes into the rho2 ring);
//   phase 1: B(r-1) chemical potential of row r-1 into the mu1 ring;
//            E(r-5) chemical potential of the second step, row r-5;
//   phase 2: C(r-2) pull row r-2 again (its populations were not kept),
//                   collide it (first step), the x-moving populations into
//                   LDS for the neighbours' deposits;
//            F(r-6) collide row r-6 (second step) and store it.
// Each stage reads only what earlier phases wrote, and four-row rings cover
// the rows that a phase reads while another writes.  Between the deposit
// and the collision, the second step keeps three complete rows of pulled
// populations and two partial ones in registers.  Every node does the
// single-step kernel's arithmetic in the same order and the first step's
// output is rounded to the storage type, so two steps of this kernel equal
// two single steps bit for bit.
// The first step's row r-2 reaches the collision in one of two ways:
//   HOLD = 0 (FP64, whose registers are spent): pulled a second time, two
//            iterations after A pulled it; that pull is issued at the start
//            of phase 1 and A's pull of the next row at the end of phase 2,
//            after the collisions, so that each is in flight through a
//            phase of work without adding to the registers the collisions
//            need;
//   HOLD = 1 (FP32): A's rows are kept in registers for two iterations, and
//            the pull of row r+1 is issued in phase 1 for the next
//            iteration's A, so that it stays in flight through phase 2; 27
//            more registers per lane.
// Early pulls are unconditional (a lane without a column reads a valid one),
// so that a wait for one leaves the later ones in flight (see tile_p_pipe).
template <int EOS, class S, class C, int BX, int NT, int HOLD>
__device__ __forceinline__ void tile_fe2(const S* __restrict__ src, S* __restrict__ dst,
                                         const KParams<C>& kp, unsigned* __restrict__ flags,
                                         int x0, int y0) {
  __shared__ C rho1[4][BX + 10];  // columns x0-5 .. x0+w+4 (index off + 5)
  __shared__ C mu1[4][BX + 8];    // x0-4 .. x0+w+3 (off + 4)
  __shared__ C xb[6][BX + 6];     // x-moving g*1 of one row, x0-3 .. x0+w+2 (off + 3)
  __shared__ C rho2[4][BX + 4];   // x0-2 .. x0+w+1 (off + 2)
  __shared__ C mu2[4][BX + 2];    // x0-1 .. x0+w (off + 1)
  __shared__ unsigned s_flag;
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool mainl = t < BX;
  const int h = t - BX;
  const int off = mainl ? t : ((h & 1) ? w + (h >> 1) : -1 - (h >> 1));
  const bool own = mainl && t < w;
  const bool dA = own || (!mainl && h < 10);
  const bool dB = own || (!mainl && h < 8);
  const bool dC = own || (!mainl && h < 6);
  const bool dD = own || (!mainl && h < 4);
  const bool dE = own || (!mainl && h < 2);
  const int x = wrapi(x0 + (dA ? off : 0), nx);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);

  unsigned fl = 0;
  // second step: complete pulled rows R0 (collided at this iteration), R1,
  // R2 (completed at this iteration); partial rows: p1 = row r-4 before the
  // deposit (f0 f1 f3 f2 f5 f6), p2 = row r-3 (f2 f5 f6)
  C R0[9], R1[9], R2[9];
  C p1_0 = C(0), p1_1 = C(0), p1_3 = C(0), p1_2 = C(0), p1_5 = C(0), p1_6 = C(0);
  C p2_2 = C(0), p2_5 = C(0), p2_6 = C(0);
  C k0 = C(0), k2 = C(0), k4 = C(0);  // g*1 of the own column kept from C to D
#pragma unroll
  for (int i = 0; i < 9; ++i) R0[i] = R1[i] = R2[i] = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };
  auto pull = [&](int y, C g[9]) {
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
  };
  auto mu_at = [&](const C* bot, const C* mid, const C* top, int j) {
    C v[9];
    gather(bot, mid, top, j, v);
    return mu_dev<EOS>(v[0], kp) - kp.kappa * lap9(v);
  };

  const int ra = y0 - 5;  // first-step row fetched at k = 0
  const int niter = ly + 11;
  C gA[9];         // row r, fetched one iteration ahead
  C h1[9], h2[9];  // HOLD: rows r-1 and r-2 as A pulled them
  C gC[9];         // !HOLD: row r-2, pulled again at the start of phase 1
  pull(ra, gA);
  for (int k = 0; k < niter; ++k) {
    const int r = ra + k;
    // ---- phase 0: A(r), D(r-3)
    C g[9];
    if (r <= y0 + ly + 4 && dA) {
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = gA[i];
      const C dr = sum9(g);
      if (own) fl |= domain_flags<MODEL_FE, EOS>(kp.rho_ref + dr, kp);
      rho1[r & 3][off + 5] = dr;
    }
    if (r - 3 >= y0 - 3 && r - 3 <= y0 + ly + 2 && dD) {
      const int j = off + 3;
      // f_4(x, r-4) = g*1_4(x, r-3), f_7 from x+1, f_8 from x-1
      R2[0] = p1_0; R2[1] = p1_1; R2[2] = p1_2; R2[3] = p1_3;
      R2[4] = k4; R2[5] = p1_5; R2[6] = p1_6;
      R2[7] = xb[5][j + 1];
      R2[8] = xb[2][j - 1];
      if (r - 4 >= y0 - 2) {
        const C dq = sum9(R2);
        if (own) fl |= domain_flags<MODEL_FE, EOS>(kp.rho_ref + dq, kp);
        rho2[(r - 4) & 3][off + 2] = dq;
      }
      // row r-3: f_0 own, f_1 from x-1, f_3 from x+1 (f_2 f_5 f_6 already in)
      p1_0 = k0; p1_1 = xb[0][j - 1]; p1_3 = xb[3][j + 1];
      p1_2 = p2_2; p1_5 = p2_5; p1_6 = p2_6;
      // row r-2: f_2 own, f_5 from x-1, f_6 from x+1
      p2_2 = k2; p2_5 = xb[1][j - 1]; p2_6 = xb[4][j + 1];
    }
    __syncthreads();
    // ---- phase 1: B(r-1), E(r-5)
    if constexpr (HOLD) pull(r + 1, gA);
    else pull(r - 2, gC);
    if (r - 1 >= y0 - 4 && r - 1 <= y0 + ly + 3 && dB)
      mu1[(r - 1) & 3][off + 4] = mu_at(rho1[(r - 2) & 3], rho1[(r - 1) & 3], rho1[r & 3], off + 5);
    if (r - 5 >= y0 - 1 && r - 5 <= y0 + ly && dE)
      mu2[(r - 5) & 3][off + 1] = mu_at(rho2[(r - 6) & 3], rho2[(r - 5) & 3], rho2[(r - 4) & 3], off + 2);
    __syncthreads();
    // ---- phase 2: C(r-2), F(r-6)
    const int c = r - 2;
    if (c >= y0 - 3 && c <= y0 + ly + 2 && dC) {
      C g[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = HOLD ? h2[i] : gC[i];
      const C d0 = sum9(g);
      C v[9], m[9];
      gather(rho1[(c - 1) & 3], rho1[c & 3], rho1[(c + 1) & 3], off + 5, v);
      gather(mu1[(c - 1) & 3], mu1[c & 3], mu1[(c + 1) & 3], off + 4, m);
      C grx, gry, gmx, gmy;
      grad_sum(v, grx, gry);
      grad_sum(m, gmx, gmy);
      const C rho = kp.rho_ref + d0;
      const C Fx = -rho * gmx + kp.fx;
      const C Fy = -rho * gmy + kp.fy;
      C ux, uy;
      collide<MODEL_FE>(g, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy);
      // the single-step kernel stores the first step's output and loads it
      // back: round to the storage type the same way
#pragma unroll
      for (int i = 0; i < 9; ++i) g[i] = (C)(S)g[i];
      const int j = off + 3;
      xb[0][j] = g[1];
      xb[1][j] = g[5];
      xb[2][j] = g[8];
      xb[3][j] = g[3];
      xb[4][j] = g[6];
      xb[5][j] = g[7];
      k0 = g[0];
      k2 = g[2];
      k4 = g[4];
    }
    const int b = r - 6;
    if (b >= y0 && own) {
      C v[9], m[9];
      gather(rho2[(b - 1) & 3], rho2[b & 3], rho2[(b + 1) & 3], off + 2, v);
      gather(mu2[(b - 1) & 3], mu2[b & 3], mu2[(b + 1) & 3], off + 1, m);
      C grx, gry, gmx, gmy;
      grad_sum(v, grx, gry);
      grad_sum(m, gmx, gmy);
      const C d0 = sum9(R0);
      const C rho = kp.rho_ref + d0;
      const C Fx = -rho * gmx + kp.fx;
      const C Fy = -rho * gmy + kp.fy;
      C ux, uy;
      collide<MODEL_FE>(R0, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy);
      const int o = b * kp.rowpitch + c0;
#pragma unroll
      for (int i = 0; i < 9; ++i) st<NT>(&dst[o + 64 * i], (S)R0[i]);
    }
    if constexpr (!HOLD) pull(r + 1, gA);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      R0[i] = R1[i];
      R1[i] = R2[i];
      if constexpr (HOLD) {
        h2[i] = h1[i];
        h1[i] = g[i];
      }
    }
  }
  commit_flags(fl, flags, &s_flag);
}

// Free-energy step on one tile.  GEN as for tile_p; GEN = 3 adds the A term
// of Eq. 20 (kp.A, with the velocity field in kp.uax / kp.uay).  GEN = 2 is
// the velocity pass that the A term needs: the same pull, stencils, force
// and wall closure, then Eq. 6b into kp.uax / kp.uay instead of a
// collision (nothing stored to dst).
template <int EOS, class S, class C, int BX, int NT, int CHK, int GEN = 0>
__device__ __forceinline__ void tile_fe(const S* __restrict__ src, S* __restrict__ dst,
                                        const KParams<C>& kp, unsigned* __restrict__ flags,
                                        int x0, int y0, const ChkOut<C>& ck) {
  __shared__ C rho_s[8][BX + 4];
  __shared__ C mu_s[4][BX + 2];
  __shared__ unsigned s_flag;
  __shared__ double s_du[BX / 64];
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool active = t < w;
  const int x = x0 + (active ? t : 0);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);
  // rho halo columns x0-2, x0-1, x0+w, x0+w+1 on lanes 0..3
  const bool hr = t < 4;
  const int hoff = (t < 2) ? (t - 2) : (w + t - 2);
  const int hx = wrapi(x0 + hoff, nx);
  const int hxm = (hx == 0) ? nx - 1 : hx - 1;
  const int hxp = (hx == nx - 1) ? 0 : hx + 1;
  const int hcm = colo(hxm), hc0 = colo(hx), hcp = colo(hxp);
  const int hj = hoff + 2;  // LDS index of the halo column in rho_s
  // mu halo columns x0-1 (lane 0) and x0+w (lane 1)
  const bool hm = t < 2;
  const int hmj = (t == 0) ? 0 : w + 1;  // index in mu_s

  unsigned fl = 0;
  C dmax = C(0);
  C g0[9], g1[9], g2[9];
  C d0 = C(0), d1 = C(0), d2 = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };

  // density deviation of row y into ring slot r (and the populations of
  // interior lanes)
  auto load_row = [&](int yr, int slot, C g[9], C& dr) {
    int y = yr;
    int sd = 0;
    if constexpr (GEN != 0) {
      if (kp.walls) {
        y = seen_row(yr, ny);  // past a wall: the mirrored row's density
        sd = wall_side(y, ny);
      }
    }
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    C* row = rho_s[slot & 7];
    // halo loads first, in flight with the interior ones (one round trip)
    C h[9];
    if (hr) pull9<S, C, NT>(src, rm, r0, rp, hcm, hc0, hcp, h);
    if (active) {
      pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
      if (GEN != 0 && sd) wall_fill_fe(g, sd, kp);
      dr = sum9(g);
      fl |= domain_flags<MODEL_FE, EOS>(kp.rho_ref + dr, kp);
      row[t + 2] = dr;
    }
    if (hr) {
      if (GEN != 0 && sd) wall_fill_fe(h, sd, kp);
      row[hj] = sum9(h);
    }
  };
  // mu of the row in rho slot rs into mu slot ms (needs rho slots rs-1..rs+1)
  auto mu_row = [&](int rs, int ms) {
    const C* bot = rho_s[(rs - 1) & 7];
    const C* mid = rho_s[rs & 7];
    const C* top = rho_s[(rs + 1) & 7];
    C* out = mu_s[ms & 3];
    if (active) {
      C v[9];
      gather(bot, mid, top, t + 2, v);
      out[t + 1] = mu_dev<EOS>(v[0], kp) - kp.kappa * lap9(v);
    }
    if (hm) {
      C v[9];
      gather(bot, mid, top, hmj + 1, v);
      out[hmj] = mu_dev<EOS>(v[0], kp) - kp.kappa * lap9(v);
    }
  };

  // rho_s holds density deviations rho - rho_ref (rho itself for FP64).
  // rho slots: row y0-2+r -> slot r.  mu slots: row y0-1+q -> slot q.
  {
    C tmp[9];
    C dtmp;
    load_row(y0 - 2, 0, tmp, dtmp);
    load_row(y0 - 1, 1, tmp, dtmp);
    load_row(y0, 2, g0, d0);
    load_row(y0 + 1, 3, g1, d1);
  }
  __syncthreads();
  mu_row(1, 0);  // row y0-1
  mu_row(2, 1);  // row y0

  for (int k = 0; k < ly; ++k) {
    const int y = y0 + k;
    load_row(y + 2, k + 4, g2, d2);
    __syncthreads();
    mu_row(k + 3, k + 2);  // row y+1
    __syncthreads();
    if (active) {
      C v[9], m[9];
      gather(rho_s[(k + 1) & 7], rho_s[(k + 2) & 7], rho_s[(k + 3) & 7], t + 2, v);
      gather(mu_s[k & 3], mu_s[(k + 1) & 3], mu_s[(k + 2) & 3], t + 1, m);
      C grx, gry, gmx, gmy;
      grad_sum(v, grx, gry);  // Eq. 24 gradient of rho
      grad_sum(m, gmx, gmy);  // Eq. 24 gradient of mu
      C rho = kp.rho_ref + d0;
      C Fx = -rho * gmx + kp.fx;  // F = -rho grad(mu)
      C Fy = -rho * gmy + kp.fy;
      C ux, uy;
      if constexpr (GEN != 0) {
        if (kp.ax != C(0)) Fx += drive_fx(kp, x, rho);
        // on a wall row the mirrored rows give d_y rho = d_y mu = 0 (set
        // exactly: the two sides of the mirror round differently)
        const int sd = kp.walls ? wall_side(y, ny) : 0;
        if (sd) {
          Fy = kp.fy;
          gry = C(0);
        }
        // gravity: the buoyancy joins the force (on a wall row too)
        if (kp.g != C(0)) Fy -= (rho - kp.grho0) * kp.g;
        if (sd) wall_fx(g0, sd, Fx);
        const C pg = kp.grho0 * kp.g * (C(y) - kp.gy0);
        const C dpg = kp.grho0 * kp.g;
        if constexpr (GEN == 2) {
          const C jx = (g0[1] - g0[3]) + ((g0[5] - g0[7]) - (g0[6] - g0[8]));
          const C jy = (g0[2] - g0[4]) + ((g0[5] - g0[7]) + (g0[6] - g0[8]));
          const C inv = C(1) / rho;
          kp.uax[y * nx + x] = (double)((jx + C(0.5) * Fx) * inv);
          kp.uay[y * nx + x] = (double)((jy + C(0.5) * Fy) * inv);
          ux = uy = C(0);
        }
        C a_div = C(0), a_xx = C(0), a_xy = C(0);
        if constexpr (GEN == 3) {
          C dxux, dyux, dxuy, dyuy;
          grad_u(kp.uax, nx, ny, kp.walls, x, y, dxux, dyux);
          grad_u(kp.uay, nx, ny, kp.walls, x, y, dxuy, dyuy);
          const C ra = rho * kp.A;
          a_div = ra * (dxux + dyuy);
          a_xx = C(2.0 / 3.0) * ra * (dxux - dyuy);
          a_xy = C(1.0 / 3.0) * ra * (dxuy + dyux);
        }
        if constexpr (GEN == 1)
          collide<MODEL_FE>(g0, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy, C(0), C(0),
                            C(0), pg, dpg);
        if constexpr (GEN == 3)
          collide<MODEL_FE, 1>(g0, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy, a_div,
                               a_xx, a_xy, pg, dpg);
      } else {
        collide<MODEL_FE>(g0, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy);
      }
      chk_node<CHK>(ck, y * nx + x, ux, uy, dmax);
      if constexpr (GEN != 2) {
        const int off = y * kp.rowpitch + c0;
#pragma unroll
        for (int i = 0; i < 9; ++i) st<NT>(&dst[off + 64 * i], (S)g0[i]);
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) { g0[i] = g1[i]; g1[i] = g2[i]; }
      d0 = d1;
      d1 = d2;
    }
  }
  commit_flags(fl, flags, &s_flag);
  chk_commit<CHK>(ck, dmax, s_du);
}

// Software-pipelined free-energy tile: the populations of row y+3 are
// loaded at the top of the iteration that collides row y and consumed (as
// the density row y+3) one iteration later, so their latency overlaps the
// chemical-potential row, two barriers and a collision.  Four population
// rows are live (y .. y+3).  As in tile_p_pipe, interior loads are
// unconditional and follow the halo loads, and the last row is peeled.
template <int EOS, class S, class C, int BX, int NT, int CHK>
__device__ __forceinline__ void tile_fe_pipe(const S* __restrict__ src, S* __restrict__ dst,
                                             const KParams<C>& kp, unsigned* __restrict__ flags,
                                             int x0, int y0, const ChkOut<C>& ck) {
  __shared__ C rho_s[8][BX + 4];
  __shared__ C mu_s[4][BX + 2];
  __shared__ unsigned s_flag;
  __shared__ double s_du[BX / 64];
  if (threadIdx.x == 0) s_flag = 0u;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(BX, nx - x0);
  const int ly = min(kp.LY, ny - y0);
  const int t = threadIdx.x;
  const bool active = t < w;
  const int x = x0 + (active ? t : 0);
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  const int cm = colo(xm), c0 = colo(x), cp = colo(xp);
  const bool hr = t < 4;
  const int hoff = (t < 2) ? (t - 2) : (w + t - 2);
  const int hx = wrapi(x0 + hoff, nx);
  const int hxm = (hx == 0) ? nx - 1 : hx - 1;
  const int hxp = (hx == nx - 1) ? 0 : hx + 1;
  const int hcm = colo(hxm), hc0 = colo(hx), hcp = colo(hxp);
  const int hj = hoff + 2;
  const bool hm = t < 2;
  const int hmj = (t == 0) ? 0 : w + 1;

  unsigned fl = 0;
  C dmax = C(0);
  C g0[9], g1[9], g2[9], h2[9];
  C d0 = C(0), d1 = C(0);

  auto rowoff = [&](int y) { return wrapi(y, ny) * kp.rowpitch; };
  auto pull_row = [&](int y, C g[9], C h[9]) {
    const int r0 = rowoff(y), rm = rowoff(y - 1), rp = rowoff(y + 1);
    if (hr) pull9<S, C, NT>(src, rm, r0, rp, hcm, hc0, hcp, h);
    pull9<S, C, NT>(src, rm, r0, rp, cm, c0, cp, g);
  };
  // density deviation row into ring slot; returns the interior value
  auto rho_row = [&](int slot, const C g[9], const C h[9]) {
    C dr = sum9(g);
    C* row = rho_s[slot & 7];
    if (active) {
      fl |= domain_flags<MODEL_FE, EOS>(kp.rho_ref + dr, kp);
      row[t + 2] = dr;
    }
    if (hr) row[hj] = sum9(h);
    return dr;
  };
  auto mu_row = [&](int rs, int ms) {
    const C* bot = rho_s[(rs - 1) & 7];
    const C* mid = rho_s[rs & 7];
    const C* top = rho_s[(rs + 1) & 7];
    C* out = mu_s[ms & 3];
    if (active) {
      C v[9];
      gather(bot, mid, top, t + 2, v);
      out[t + 1] = mu_dev<EOS>(v[0], kp) - kp.kappa * lap9(v);
    }
    if (hm) {
      C v[9];
      gather(bot, mid, top, hmj + 1, v);
      out[hmj] = mu_dev<EOS>(v[0], kp) - kp.kappa * lap9(v);
    }
  };
  auto collide_row = [&](int k) {
    if (active) {
      const int y = y0 + k;
      C v[9], m[9];
      gather(rho_s[(k + 1) & 7], rho_s[(k + 2) & 7], rho_s[(k + 3) & 7], t + 2, v);
      gather(mu_s[k & 3], mu_s[(k + 1) & 3], mu_s[(k + 2) & 3], t + 1, m);
      C grx, gry, gmx, gmy;
      grad_sum(v, grx, gry);  // Eq. 24 gradient of rho
      grad_sum(m, gmx, gmy);  // Eq. 24 gradient of mu
      C rho = kp.rho_ref + d0;
      C Fx = -rho * gmx + kp.fx;  // F = -rho grad(mu)
      C Fy = -rho * gmy + kp.fy;
      C ux, uy;
      collide<MODEL_FE>(g0, d0, rho, Fx, Fy, grx, gry, C(0), C(0), kp, ux, uy);
      chk_node<CHK>(ck, y * nx + x, ux, uy, dmax);
      const int off = y * kp.rowpitch + c0;
#pragma unroll
      for (int i = 0; i < 9; ++i) st<NT>(&dst[off + 64 * i], (S)g0[i]);
    }
  };

  // rho slots: row y0-2+r -> slot r.  mu slots: row y0-1+q -> slot q.
  {
    C tmp[9], th[9];
    pull_row(y0 - 2, tmp, th);
    rho_row(0, tmp, th);
    pull_row(y0 - 1, tmp, th);
    rho_row(1, tmp, th);
    pull_row(y0, g0, th);
    d0 = rho_row(2, g0, th);
    pull_row(y0 + 1, g1, th);
    d1 = rho_row(3, g1, th);
    pull_row(y0 + 2, g2, h2);
  }
  __syncthreads();
  mu_row(1, 0);  // row y0-1
  mu_row(2, 1);  // row y0

  for (int k = 0; k < ly - 1; ++k) {
    C g3[9], h3[9];
    pull_row(y0 + k + 3, g3, h3);
    C d2 = rho_row(k + 4, g2, h2);  // row y+2
    __syncthreads();
    mu_row(k + 3, k + 2);  // row y+1
    __syncthreads();
    collide_row(k);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      g0[i] = g1[i];
      g1[i] = g2[i];
      g2[i] = g3[i];
      h2[i] = h3[i];
    }
    d0 = d1;
    d1 = d2;
  }
  {
    const int k = ly - 1;
    rho_row(k + 4, g2, h2);
    __syncthreads();
    mu_row(k + 3, k + 2);
    __syncthreads();
    collide_row(k);
  }
  commit_flags(fl, flags, &s_flag);
  chk_commit<CHK>(ck, dmax, s_du);
}

// ---- single-lattice step kernels --------------------------------------------
template <int EOS, class S, class C, int BX, int NT, int WPE, int GEN = 0>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_step_p(const S* __restrict__ src, S* __restrict__ dst, const KParams<C> kp,
              unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_p<EOS, S, C, BX, NT, 0, GEN>(src, dst, kp, flags, (tile % kp.nstrips) * BX,
                                   (tile / kp.nstrips) * kp.LY,
                                   ChkOut<C>{nullptr, nullptr, nullptr});
}

template <int EOS, class S, class C, int BX, int NT, int WPE>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_step_p_pipe(const S* __restrict__ src, S* __restrict__ dst, const KParams<C> kp,
                   unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_p_pipe<EOS, S, C, BX, NT>(src, dst, kp, flags, (tile % kp.nstrips) * BX,
                                 (tile / kp.nstrips) * kp.LY);
}

// Two pseudopotential steps per launch (tile_p2): BX + 64 threads.
template <int EOS, class S, class C, int BX, int NT>
__global__ __launch_bounds__(BX + 64) void k_step2_p(const S* __restrict__ src,
                                                     S* __restrict__ dst, const KParams<C> kp,
                                                     unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_p2<EOS, S, C, BX, NT, sizeof(S) == 8 ? 1 : 0>(src, dst, kp, flags,
                                                   (tile % kp.nstrips) * BX,
                                                   (tile / kp.nstrips) * kp.LY);
}

// Two free-energy steps per launch (tile_fe2): BX + 64 threads.
// Non-temporal stores; FP32 keeps the first step's rows (HOLD).
template <int EOS, class S, class C, int BX>
__global__ __launch_bounds__(BX + 64) void k_step2_fe(const S* __restrict__ src,
                                                      S* __restrict__ dst, const KParams<C> kp,
                                                      unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_fe2<EOS, S, C, BX, 1, sizeof(S) == 4 ? 1 : 0>(src, dst, kp, flags,
                                                   (tile % kp.nstrips) * BX,
                                                   (tile / kp.nstrips) * kp.LY);
}

template <int EOS, class S, class C, int BX, int NT, int WPE, int GEN = 0>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_step_fe(const S* __restrict__ src, S* __restrict__ dst, const KParams<C> kp,
               unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_fe<EOS, S, C, BX, NT, 0, GEN>(src, dst, kp, flags, (tile % kp.nstrips) * BX,
                                    (tile / kp.nstrips) * kp.LY,
                                    ChkOut<C>{nullptr, nullptr, nullptr});
}

template <int EOS, class S, class C, int BX, int NT, int WPE>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void k_step_fe_pipe(const S* __restrict__ src, S* __restrict__ dst, const KParams<C> kp,
                    unsigned* __restrict__ flags) {
  const int tile = tile_index(kp.xcd_remap);
  tile_fe_pipe<EOS, S, C, BX, NT, 0>(src, dst, kp, flags, (tile % kp.nstrips) * BX,
                                     (tile / kp.nstrips) * kp.LY,
                                     ChkOut<C>{nullptr, nullptr, nullptr});
}

// Occupancy targets (waves per SIMD) of the register-capped variants.
template <int MODEL, class S>
constexpr int wpe_target() {
  return sizeof(S) == 8 ? (MODEL == MODEL_P ? 4 : 3) : (MODEL == MODEL_P ? 8 : 5);
}

// ---- batched step kernels -----------------------------------------------------
// One launch covers every tile of every active lattice of one (model, EOS,
// strip width) group; the tile table names the lattice and the tile origin,
// the lattice's descriptor its parameters, buffers, flags and check outputs.
// The launch is persistent: at most one round of resident workgroups walks
// the group's table with a stride of the grid, and the number of active
// tiles is read from device memory, so the host shrinks the table when
// lattices retire without changing the launch (or the graph that holds it).
// Each workgroup's loop ends at that count, which no kernel changes.
struct BatchTile {
  int inst, x0, y0, pad;
};

template <class C>
struct InstDesc {
  KParams<C> kp;
  void* fA;
  void* fB;
  C* uxp;
  C* uyp;
  unsigned* flags;
  unsigned long long* du;
};

// (the checking step of the pseudopotential FP32 kernel carries the
// velocity comparison and the tile loop: one wave less, so it does not
// spill)
template <int MODEL, class S, int CHK>
constexpr int batch_wpe() {
  return wpe_target<MODEL, S>() - ((CHK && MODEL == MODEL_P && sizeof(S) == 4) ? 1 : 0);
}

template <int MODEL, int EOS, class S, class C, int BX, int NT, int CHK>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(batch_wpe<MODEL, S, CHK>())))
void k_batch_step(const BatchTile* __restrict__ tiles, const int* __restrict__ count,
                  const InstDesc<C>* __restrict__ inst, int parity) {
  const int n = *count;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const BatchTile bt = tiles[t];
    const InstDesc<C>* d = inst + bt.inst;
    const S* src = (const S*)(parity ? d->fB : d->fA);
    S* dst = (S*)(parity ? d->fA : d->fB);
    const ChkOut<C> ck{d->uxp, d->uyp, d->du};
    if constexpr (MODEL == MODEL_P)
      tile_p<EOS, S, C, BX, NT, CHK>(src, dst, d->kp, d->flags, bt.x0, bt.y0, ck);
    else
      tile_fe<EOS, S, C, BX, NT, CHK>(src, dst, d->kp, d->flags, bt.x0, bt.y0, ck);
    __syncthreads();  // the next tile reuses the LDS rings
  }
}

// Two steps of every tile in the table (tile_p2 / tile_fe2, BX + 64 threads,
// the same row schedules and register choices as k_step2_p / k_step2_fe),
// walking the table as k_batch_step does.  The table holds the single-step
// kernel's 256-column tiles, so one table serves both kernels; the
// free-energy kernel runs 128-column strips (in FP64 the 256-column one fits
// only two workgroups per CU) and takes each tile as two halves: the first
// halves of all tiles, then the second halves, so that the halves a narrow
// lattice leaves empty fall on every workgroup alike.
template <int MODEL>
constexpr int batch2_bx() { return MODEL == MODEL_P ? 256 : 128; }

template <int MODEL, int EOS, class S, class C>
__global__ __launch_bounds__(batch2_bx<MODEL>() + 64)
void k_batch_step2(const BatchTile* __restrict__ tiles, const int* __restrict__ count,
                   const InstDesc<C>* __restrict__ inst, int parity) {
  constexpr int BX = batch2_bx<MODEL>();
  constexpr int SPLIT = 256 / BX;
  const int nt = *count;
  const int n = nt * SPLIT;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const BatchTile bt = tiles[t % nt];
    const InstDesc<C>* d = inst + bt.inst;
    const int x0 = bt.x0 + (t / nt) * BX;
    if (x0 >= d->kp.nx) continue;  // the lattice ends in the first half
    const S* src = (const S*)(parity ? d->fB : d->fA);
    S* dst = (S*)(parity ? d->fA : d->fB);
    if constexpr (MODEL == MODEL_P)
      tile_p2<EOS, S, C, BX, 1, sizeof(S) == 8 ? 1 : 0>(src, dst, d->kp, d->flags, x0, bt.y0);
    else
      tile_fe2<EOS, S, C, BX, 1, sizeof(S) == 4 ? 1 : 0>(src, dst, d->kp, d->flags, x0, bt.y0);
    __syncthreads();  // the next tile reuses the LDS rings
  }
}

// ---- initial state ------------------------------------------------------------
// Stored g*_i(x) = f^eq_i(rho0(x + c_i), 0) - s_i, so that the first pull
// yields f_i(x) = f^eq_i(rho0(x), 0) (Eq. 4: w_i rho; Eq. 20: rho delta_i0).
// FE with gravity: f^eq also carries the p_g terms of Eq. 20, with
// p_g / c_s^2 = pg1 (y - gy0) on row y (pg1 = grho0 g / c_s^2).
template <int MODEL, class S>
__global__ void k_init(const double* __restrict__ rho0, S* __restrict__ dst,
                       int nx, int ny, int rowpitch, double s0, double sax, double sdg,
                       double pg1 = 0.0, double gy0 = 0.0) {
  const size_t N = (size_t)nx * ny;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double wt[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    for (int i = 0; i < 9; ++i) {
      int xs = wrapi(x + cx[i], nx), ys = wrapi(y + cy[i], ny);
      double r = rho0[(size_t)ys * nx + xs];
      double feq = (MODEL == MODEL_P) ? wt[i] * r : ((i == 0) ? r : 0.0);
      if (MODEL == MODEL_FE && pg1 != 0.0) {
        // p_g / c_s^2 of the node the population streams to
        const double q = pg1 * ((double)ys - gy0);
        feq += (i == 0) ? -(1.0 - wt[0]) * q : wt[i] * q;
      }
      double s = (i == 0) ? s0 : (i < 5 ? sax : sdg);
      dst[y * rowpitch + colo(x) + 64 * i] = (S)(feq - s);
    }
  }
}

// ---- population import / export (post-streaming f_i(x, t)) ----------------
template <class S>
__global__ void k_get_pop(const S* __restrict__ src, double* __restrict__ f,
                          int nx, int ny, int rowpitch, double s0, double sax, double sdg) {
  const size_t N = (size_t)nx * ny;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    for (int i = 0; i < 9; ++i) {
      int xs = wrapi(x - cx[i], nx), ys = wrapi(y - cy[i], ny);
      double s = (i == 0) ? s0 : (i < 5 ? sax : sdg);
      f[i * N + n] = s + (double)src[ys * rowpitch + colo(xs) + 64 * i];
    }
  }
}

template <class S>
__global__ void k_set_pop(const double* __restrict__ f, S* __restrict__ dst,
                          int nx, int ny, int rowpitch, double s0, double sax, double sdg) {
  const size_t N = (size_t)nx * ny;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    for (int i = 0; i < 9; ++i) {
      int xs = wrapi(x + cx[i], nx), ys = wrapi(y + cy[i], ny);
      double s = (i == 0) ? s0 : (i < 5 ? sax : sdg);
      dst[y * rowpitch + colo(x) + 64 * i] = (S)(f[i * N + (size_t)ys * nx + xs] - s);
    }
  }
}

// ---- observation (FP64) -------------------------------------------------------
// Pass 1: rho (Eq. 6a) and, for P, psi (Eq. 11) on every node.
template <int MODEL, int EOS, class S>
__global__ void k_obs_rho(const S* __restrict__ src, const KParams<double> kp,
                          double* __restrict__ rho_w, double* __restrict__ aux_w,
                          unsigned* __restrict__ flags) {
  __shared__ unsigned s_flag;
  if (threadIdx.x == 0) s_flag = 0u;
  __syncthreads();
  const int nx = kp.nx, ny = kp.ny;
  const size_t N = (size_t)nx * ny;
  unsigned fl = 0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int rw = kp.rowpitch;
    int r0 = y * rw, rm = wrapi(y - 1, ny) * rw, rp = wrapi(y + 1, ny) * rw;
    double g[9];
    pull9(src, rm, r0, rp, colo(xm), colo(x), colo(xp), g);
    const int sd = kp.walls ? wall_side(y, ny) : 0;
    if (sd) wall_fill_fe(g, sd, kp);  // kp.g = 0 for the pseudopotential
    double rho = kp.rho_ref + sum9(g);
    fl |= domain_flags<MODEL, EOS>(rho, kp);
    rho_w[n] = rho;
    if (MODEL == MODEL_P) aux_w[n] = psi_of<EOS>(rho, kp, fl);
  }
  commit_flags(fl, flags, &s_flag);
}

template <class C>
__device__ __forceinline__ void gather_global(const C* __restrict__ a, int nx,
                                              int ny, int walls, int x, int y, C v[9]) {
  int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
  int ym = (walls && y == 0) ? 1 : wrapi(y - 1, ny);        // mirrored past a wall
  int yp = (walls && y == ny - 1) ? ny - 2 : wrapi(y + 1, ny);
  int r0 = y * nx, rm = ym * nx, rp = yp * nx;
  v[0] = a[r0 + x];
  v[1] = a[r0 + xp];
  v[2] = a[rp + x];
  v[3] = a[r0 + xm];
  v[4] = a[rm + x];
  v[5] = a[rp + xp];
  v[6] = a[rp + xm];
  v[7] = a[rm + xm];
  v[8] = a[rm + xp];
}

// Pass 2 (FE): mu = mu_b(rho) - kappa lap(rho).
template <int EOS>
__global__ void k_obs_mu(const KParams<double> kp, const double* __restrict__ rho_w,
                         double* __restrict__ aux_w) {
  const int nx = kp.nx, ny = kp.ny;
  const size_t N = (size_t)nx * ny;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    double v[9];
    gather_global(rho_w, nx, ny, kp.walls, x, y, v);
    aux_w[n] = eos_mu<EOS>(v[0], kp) - kp.kappa * lap9(v);
  }
}

struct ObsPartial {
  double sum_hi, sum_lo, max_u, rho_min, rho_max, du_max, pad0, pad1;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Combine two partials: compensated sum (two_sum is exact and symmetric, so
// both partners of a butterfly get bit-identical results), maxima, and a
// minimum that stays NaN once a NaN density was seen.
__device__ __forceinline__ ObsPartial obs_combine(const ObsPartial& a, const ObsPartial& b) {
  ObsPartial r;
  double s, e;
  two_sum(a.sum_hi, b.sum_hi, s, e);
  r.sum_hi = s;
  r.sum_lo = (a.sum_lo + b.sum_lo) + e;
  r.max_u = fmax(a.max_u, b.max_u);
  r.rho_min = (a.rho_min != a.rho_min || b.rho_min != b.rho_min) ? NAN : fmin(a.rho_min, b.rho_min);
  r.rho_max = fmax(a.rho_max, b.rho_max);
  r.du_max = fmax(a.du_max, b.du_max);
  r.pad0 = r.pad1 = 0.0;
  return r;
}

__device__ __forceinline__ ObsPartial obs_shfl_xor(const ObsPartial& a, int off) {
  ObsPartial b;
  b.sum_hi = __shfl_xor(a.sum_hi, off, 64);
  b.sum_lo = __shfl_xor(a.sum_lo, off, 64);
  b.max_u = __shfl_xor(a.max_u, off, 64);
  b.rho_min = __shfl_xor(a.rho_min, off, 64);
  b.rho_max = __shfl_xor(a.rho_max, off, 64);
  b.du_max = __shfl_xor(a.du_max, off, 64);
  b.pad0 = b.pad1 = 0.0;
  return b;
}

// Block reduction of one partial per thread: a butterfly of wavefront
// shuffles (every lane ends with the wavefront's result), one partial per
// wavefront through LDS, then the same butterfly in the first wavefront.
// The combination order is fixed, so the result is deterministic.  Returns
// the block's partial in thread 0.
template <int NT>
__device__ __forceinline__ ObsPartial obs_block_reduce(ObsPartial a) {
  static_assert(NT % 64 == 0 && NT <= 64 * 64, "block of whole wavefronts");
  __shared__ ObsPartial sh[NT / 64];
  for (int off = 32; off > 0; off >>= 1) a = obs_combine(a, obs_shfl_xor(a, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = a;
  __syncthreads();
  if (wave == 0) {
    a = lane < NT / 64 ? sh[lane]
                       : ObsPartial{0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
    for (int off = 32; off > 0; off >>= 1) a = obs_combine(a, obs_shfl_xor(a, off));
  }
  return a;
}

// Pass 3: force, velocity (Eq. 6b), exports, per-block partial reductions.
template <int MODEL, class S, int NT>
__global__ __launch_bounds__(NT) void k_obs_u(
    const S* __restrict__ src, const KParams<double> kp,
    const double* __restrict__ rho_w, const double* __restrict__ aux_w,
    double* __restrict__ out_rho, double* __restrict__ out_ux,
    double* __restrict__ out_uy, double* __restrict__ uxp,
    double* __restrict__ uyp, int have_prev, ObsPartial* __restrict__ part) {
  const int nx = kp.nx, ny = kp.ny;
  const size_t N = (size_t)nx * ny;
  double s_hi = 0.0, s_lo = 0.0, mu = 0.0, rmin = INFINITY, rmax = -INFINITY, du = 0.0;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
       n += (size_t)gridDim.x * blockDim.x) {
    int x = (int)(n % nx), y = (int)(n / nx);
    int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int rw = kp.rowpitch;
    int r0 = y * rw, rm = wrapi(y - 1, ny) * rw, rp = wrapi(y + 1, ny) * rw;
    double g[9];
    pull9(src, rm, r0, rp, colo(xm), colo(x), colo(xp), g);
    const int sd = kp.walls ? wall_side(y, ny) : 0;
    if (sd) wall_fill_fe(g, sd, kp);
    double rho = rho_w[n];
    double Fx, Fy;
    if (MODEL == MODEL_P) {
      double v[9], sx, sy;
      gather_global(aux_w, nx, ny, kp.walls, x, y, v);
      grad_sum(v, sx, sy);
      Fx = v[0] * sx + kp.fx;
      Fy = v[0] * sy + kp.fy;
    } else {
      double v[9], sx, sy;
      gather_global(aux_w, nx, ny, kp.walls, x, y, v);
      grad_sum(v, sx, sy);
      Fx = -rho * sx + kp.fx;  // F = -rho grad(mu), Eq. 24 gradient
      Fy = -rho * sy + kp.fy;
    }
    if (kp.ax != 0.0) Fx += drive_fx(kp, x, rho);
    if (sd) Fy = kp.fy;  // zero normal interaction force on a wall row
    if (kp.g != 0.0) Fy -= (rho - kp.grho0) * kp.g;  // buoyancy (FE gravity)
    if (sd) wall_fx(g, sd, Fx);
    double jx = (g[1] - g[3]) + ((g[5] - g[7]) - (g[6] - g[8]));
    double jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
    double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    if (out_rho) out_rho[n] = rho;
    if (out_ux) out_ux[n] = ux;
    if (out_uy) out_uy[n] = uy;
    if (have_prev) {
      double dx = ux - uxp[n], dy = uy - uyp[n];
      du = fmax(du, sqrt(dx * dx + dy * dy));
    }
    uxp[n] = ux;
    uyp[n] = uy;
    // Neumaier accumulation of the mass
    double s, e;
    two_sum(s_hi, rho, s, e);
    s_hi = s;
    s_lo += e;
    mu = fmax(mu, sqrt(ux * ux + uy * uy));
    // rho_min stays NaN once a non-finite density was seen (fmin would drop it)
    rmin = (rmin != rmin || !__builtin_isfinite(rho)) ? NAN : fmin(rmin, rho);
    rmax = fmax(rmax, rho);
  }
  const ObsPartial blk =
      obs_block_reduce<NT>(ObsPartial{s_hi, s_lo, mu, rmin, rmax, du, 0.0, 0.0});
  if (threadIdx.x == 0) part[blockIdx.x] = blk;
}

// Pass 4: one workgroup combines the partials in a fixed order and forms the
// probe observables (Sec. 5.2: pressure jump, equimolar radius).
template <int EOS, int NT>
__global__ __launch_bounds__(NT) void k_obs_final(
    const ObsPartial* __restrict__ part, int nparts, const KParams<double> kp,
    const double* __restrict__ rho_w, int cx, int cy, double* __restrict__ res) {
  ObsPartial acc{0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += NT) acc = obs_combine(acc, part[i]);
  const ObsPartial a = obs_block_reduce<NT>(acc);
  if (threadIdx.x == 0) {
    const int nx = kp.nx, ny = kp.ny;
    double mass = a.sum_hi + a.sum_lo;
    int xi = wrapi(cx, nx), yi = wrapi(cy, ny);
    int xo = wrapi(cx + nx / 2, nx), yo = wrapi(cy + ny / 2, ny);
    double rin = rho_w[(size_t)yi * nx + xi];
    double rout = rho_w[(size_t)yo * nx + xo];
    double dp = eos_p<EOS>(rin, kp) - eos_p<EOS>(rout, kp);
    double excess = mass - (double)nx * (double)ny * rout;
    double denom = 3.14159265358979323846 * (rin - rout);
    double q = (denom != 0.0) ? excess / denom : NAN;
    double req = (q > 0.0) ? sqrt(q) : NAN;
    res[0] = mass;
    res[1] = a.max_u;
    res[2] = a.rho_min;
    res[3] = a.rho_max;
    res[4] = rin;
    res[5] = rout;
    res[6] = dp;
    res[7] = req;
    res[8] = a.du_max;
  }
}

}  // namespace lbmk

// =============================================================================
// Host side
// =============================================================================
using namespace lbmk;

namespace {

constexpr int kObsThreads = 256;
constexpr int kGraphSteps = 16;  // steps per graph run of lbm_step (even)
constexpr int kObsBlocksMax = 2048;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Population elements per lattice row in the blocked layout.
size_t row_pitch(int nx) { return (size_t)576 * (size_t)((nx + 63) / 64); }

struct Layout {
  size_t pop_bytes, fA, fB, rho_w, aux_w, uxp, uyp, uax, uay, part, flags, result, total;
  int obs_blocks;
};

Layout make_layout(const lbm_params* p) {
  Layout L{};
  size_t N = (size_t)p->nx * p->ny;
  size_t es = (p->precision == LBM_FP32_SHIFTED) ? 4 : 8;
  L.pop_bytes = align_up((size_t)p->ny * row_pitch(p->nx) * es);
  size_t off = 0;
  L.fA = off; off += L.pop_bytes;
  L.fB = off; off += L.pop_bytes;
  L.rho_w = off; off += align_up(N * 8);
  L.aux_w = off; off += align_up(N * 8);
  L.uxp = off; off += align_up(N * 8);
  L.uyp = off; off += align_up(N * 8);
  // FE with A != 0: the velocity field of the current step
  const size_t ua = (p->model == LBM_MODEL_FE && p->A != 0.0) ? align_up(N * 8) : 0;
  L.uax = off; off += ua;
  L.uay = off; off += ua;
  L.obs_blocks = (int)std::min<size_t>((N + kObsThreads - 1) / kObsThreads, kObsBlocksMax);
  L.part = off; off += align_up((size_t)L.obs_blocks * sizeof(ObsPartial));
  L.flags = off; off += kAlign;
  L.result = off; off += align_up(16 * sizeof(double));
  L.total = off;
  return L;
}

bool finite(double v) { return std::isfinite(v); }

lbm_status validate(const lbm_params* p) {
  if (!p) return LBM_ERR_INVALID_ARG;
  if (p->nx < 1 || p->ny < 1) return LBM_ERR_INVALID_ARG;
  if ((int64_t)p->nx * (int64_t)p->ny >= (int64_t)1 << 31) return LBM_ERR_INVALID_ARG;
  // population offsets are 32-bit: ny * rowpitch (~ 9 nx ny) < 2^31
  if ((int64_t)p->ny * (int64_t)row_pitch(p->nx) >= (int64_t)1 << 31) return LBM_ERR_INVALID_ARG;
  if (p->model != LBM_MODEL_P && p->model != LBM_MODEL_FE) return LBM_ERR_INVALID_ARG;
  if (p->eos != LBM_EOS_VDW && p->eos != LBM_EOS_CS) return LBM_ERR_INVALID_ARG;
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_SHIFTED) return LBM_ERR_INVALID_ARG;
  if (p->boundary != LBM_BOUNDARY_PERIODIC && p->boundary != LBM_BOUNDARY_WALLS)
    return LBM_ERR_INVALID_ARG;
  if (p->boundary == LBM_BOUNDARY_WALLS && p->ny < 3) return LBM_ERR_INVALID_ARG;
  if (!finite(p->a) || !finite(p->b) || !finite(p->R) || !finite(p->T)) return LBM_ERR_INVALID_ARG;
  if (p->a < 0 || p->b <= 0 || p->R <= 0 || p->T <= 0) return LBM_ERR_INVALID_ARG;
  for (int i = 0; i < 9; ++i)
    if (!finite(p->tau[i]) || !(p->tau[i] > 0.5)) return LBM_ERR_INVALID_ARG;
  if (p->tau[3] != p->tau[5] || p->tau[4] != p->tau[6] || p->tau[7] != p->tau[8])
    return LBM_ERR_INVALID_ARG;
  if (!finite(p->sigma_li) || !finite(p->kappa_li) || !finite(p->kappa_p) ||
      !finite(p->kappa) || !finite(p->A) || !finite(p->fx) || !finite(p->fy) ||
      !finite(p->rho_ref))
    return LBM_ERR_INVALID_ARG;
  if (p->model == LBM_MODEL_FE && p->kappa < 0) return LBM_ERR_INVALID_ARG;
  if (p->A != 0.0) {
    // Eq. 23: nu = c_s^2 (tau_nu - 1/2 - A) must stay positive; FE only
    if (p->model != LBM_MODEL_FE) return LBM_ERR_UNSUPPORTED;
    if (!(p->tau[7] - 0.5 - p->A > 0.0)) return LBM_ERR_INVALID_ARG;
  }
  if (!finite(p->g) || !finite(p->grav_rho0) || !finite(p->grav_y0)) return LBM_ERR_INVALID_ARG;
  if (p->g != 0.0) {
    // gravity of the free-energy model (Sec. 2.2); p_g is not periodic
    if (p->model != LBM_MODEL_FE) return LBM_ERR_UNSUPPORTED;
    if (p->boundary != LBM_BOUNDARY_WALLS || p->grav_rho0 < 0.0) return LBM_ERR_INVALID_ARG;
    // the wall-density relation divides by 1 -+ g/2
    if (!(std::fabs(p->g) < 1.0)) return LBM_ERR_INVALID_ARG;
  }
  return LBM_OK;
}

template <class C>
KParams<C> make_kparams(const lbm_params* p, double rho_ref, int nstrips,
                        int nseg, int LY, int xcd_remap) {
  KParams<C> k{};
  k.nx = p->nx;
  k.ny = p->ny;
  k.rowpitch = (int)row_pitch(p->nx);
  k.walls = p->boundary == LBM_BOUNDARY_WALLS ? 1 : 0;
  k.nstrips = nstrips;
  k.nseg = nseg;
  k.LY = LY;
  k.xcd_remap = xcd_remap;
  k.a = (C)p->a;
  k.b = (C)p->b;
  k.RT = (C)(p->R * p->T);
  double le = 1.0 / p->tau[1], lz = 1.0 / p->tau[2], lq = 1.0 / p->tau[4],
         ln = 1.0 / p->tau[7];
  k.lam_e = (C)le;
  k.lam_z = (C)lz;
  k.lam_q = (C)lq;
  k.lam_nu = (C)ln;
  k.hl_e = (C)(1.0 - 0.5 * le);
  k.hl_z = (C)(1.0 - 0.5 * lz);
  k.hl_q = (C)(1.0 - 0.5 * lq);
  k.hl_nu = (C)(1.0 - 0.5 * ln);
  const double G = -1.0;
  // Eq. 32: 12 kappa^P sigma^Li |F_int|^2 / (psi^2 (tau - 1/2)); the kernel
  // multiplies by G^2|S|^2 = |F_int|^2/psi^2.
  k.sig_e = (C)(12.0 * p->kappa_p * p->sigma_li / (p->tau[1] - 0.5));
  k.sig_z = (C)(12.0 * p->kappa_p * p->sigma_li / (p->tau[2] - 0.5));
  // Eq. 30b-31: C_i_ab = C1 G delta + C2 (c c - c_s^2 delta) + kappa^Li (G/2) c c
  //   = (C1 G - C2/3) delta + (C2 + kappa^Li G/2) c c.
  double C1 = 5.0 / 6.0 * (p->kappa_p - 1.0);
  double C2 = 0.5 * G * (1.0 - p->kappa_p);
  k.qa = (C)(C1 * G - C2 / 3.0);
  k.qb = (C)(C2 + 0.5 * G * p->kappa_li);
  k.kappa = (C)p->kappa;
  k.fx = (C)p->fx;
  k.fy = (C)p->fy;
  k.ax = (C)0;  // the drive is switched on per step (set_drive)
  k.x_split = p->x_split;
  k.A = (C)p->A;
  k.g = (C)p->g;
  k.grho0 = (C)p->grav_rho0;
  k.gy0 = (C)p->grav_y0;
  k.uax = k.uay = nullptr;
  // rho_ref is chosen by lbm_init so that every shift value below is exact
  // in float and M s is exact (rho_ref = 36 q for P with q a short float).
  double s0, sax, sdg;
  if (p->model == LBM_MODEL_P) {
    double q = rho_ref / 36.0;
    s0 = 16.0 * q;
    sax = 4.0 * q;
    sdg = q;
  } else {
    s0 = rho_ref;
    sax = 0.0;
    sdg = 0.0;
  }
  k.s0 = (C)s0;
  k.sax = (C)sax;
  k.sdg = (C)sdg;
  k.rho_ref = (C)rho_ref;
  k.inv_rho_ref = (C)(rho_ref > 0 ? 1.0 / rho_ref : 0.0);
  const double om_ref = p->eos == LBM_EOS_CS ? 1.0 - 0.25 * p->b * rho_ref : 1.0 - p->b * rho_ref;
  k.om_ref = (C)om_ref;
  k.inv_om_ref = (C)(1.0 / om_ref);
  k.inv_om_ref3 = (C)(1.0 / (om_ref * om_ref * om_ref));
  return k;
}

// Launch shape of one lattice.
struct LaunchCfg {
  int bx;    // strip width (threads per workgroup): 64 or 256
  int ly;    // segment height
  int nt;    // 1: non-temporal population stores
  int wpe;   // 1: register-capped kernel variant
  int pipe;  // 1: pipelined row loop (pseudopotential)
  int two;   // 1: two steps per launch where the model and options allow
  int bx2;   // strip width of the two-step kernel: 128, 192 or 256
  int auto_ly;  // 1: segment height set at the first launch from occupancy
};

}  // namespace

struct lbm_ctx {
  lbm_params p;
  hipStream_t stream;
  char* ws;
  Layout L;
  int cur;  // 0: state in fA, 1: state in fB
  int64_t step;
  int have_prev;
  double rho_ref;  // storage shift reference (0 for FP64)
  double rho_ave;  // mean initial density (collision drive)
  LaunchCfg lc;
  int nstrips, nseg, xcd_remap;
  int nstrips2, nseg2, xcd_remap2;  // tiling of the two-step kernel (bx2 strips)
  KParams<double> kd;
  KParams<float> kf;
  // lbm_step replays runs of kGraphSteps steps as HIP graphs, captured on a
  // library stream (the caller's may be the null stream) per starting
  // population buffer and drive state
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  ~lbm_ctx();
};

namespace {

// Launch-shape resolution: the launch fields of lbm_params where set, else
// defaults measured on MI355X (4096^2 lattices: 256-column strips,
// non-temporal stores, the pipelined pseudopotential kernel without a
// register cap, the register-capped free-energy kernel, pipelined in FP32;
// 64-column strips for lattices narrower than 256).  Without an explicit
// segment height, a single lattice gets one chosen at its first launch so
// that its tiles fill whole rounds of resident workgroups (see tune_ly);
// the fallback here (batches) aims at a few thousand tiles.
LaunchCfg resolve_launch(const lbm_params* p) {
  const bool fp64 = p->precision == LBM_FP64;
  LaunchCfg lc{};
  lc.bx = p->tile_x ? p->tile_x : (p->nx < 256 ? 64 : 256);
  if (lc.bx != 64) lc.bx = 256;
  unsigned kf = (unsigned)p->kernel_flags;
  if (kf & LBM_KF_SET) {
    lc.nt = (kf & LBM_KF_NT_STORE) ? 1 : 0;
    lc.wpe = (kf & LBM_KF_REGCAP) ? 1 : 0;
    lc.pipe = (kf & LBM_KF_PIPELINE) ? 1 : 0;
    lc.two = (kf & LBM_KF_TWO_STEP) ? 1 : 0;
    lc.bx2 = (kf & LBM_KF_STRIP128) ? 128 : (kf & LBM_KF_STRIP192) ? 192 : 256;
  } else {
    lc.nt = 1;
    lc.wpe = p->model == LBM_MODEL_P ? 0 : 1;
    // pipelined row loop: pseudopotential always; free energy in FP32 only
    // (in FP64 its four live population rows cost a wave of occupancy)
    lc.pipe = (p->model == LBM_MODEL_P || !fp64) ? 1 : 0;
    // two steps per launch, measured per step on 4096^2: pseudopotential
    // (256-column strips) 0.338 vs 0.476 ms in FP64 and 0.152 vs 0.233 ms in
    // FP32; free energy 0.406 vs 0.486 ms in FP64 and 0.178 vs 0.249 ms in
    // FP32
    lc.two = 1;
    // free energy: FP64 128-column strips (192: 0.406 ms, 256: 0.610);
    // FP32 192-column strips (0.178 ms; 128: 0.192, 256: 0.214)
    lc.bx2 = p->model == LBM_MODEL_FE ? (fp64 ? 128 : 192) : 256;
  }
  // the pseudopotential two-step kernel runs 256-column strips only
  if (p->model == LBM_MODEL_P) lc.bx2 = 256;
  if (p->boundary == LBM_BOUNDARY_WALLS || p->ax != 0.0 || p->A != 0.0) {
    // walls, the collision drive and A != 0 run in the general kernel:
    // plain row loop, non-temporal stores
    lc.nt = 1;
    lc.wpe = 0;
    lc.pipe = 0;
    lc.two = 0;
  }
  int nstrips = (p->nx + lc.bx - 1) / lc.bx;
  int LY = p->tile_y;
  lc.auto_ly = LY <= 0 ? 1 : 0;
  if (LY <= 0) {
    // enough tiles to fill 256 CUs several times over, segments of at
    // least 8 rows so the two halo rows stay a small overhead
    int target_tiles = fp64 ? 2048 : 4096;
    int want_seg = std::max(1, target_tiles / nstrips);
    LY = std::max(8, (p->ny + want_seg - 1) / want_seg);
    LY = std::min(LY, fp64 ? 32 : 16);
  }
  lc.ly = std::max(1, std::min(LY, p->ny));
  return lc;
}

lbm_status validate_launch(const lbm_params* p) {
  if (p->tile_x != 0 && p->tile_x != 64 && p->tile_x != 256) return LBM_ERR_INVALID_ARG;
  if (p->tile_y < 0 || p->tile_y > 1024) return LBM_ERR_INVALID_ARG;
  if (p->tile_rounds < 0 || p->tile_rounds > 64) return LBM_ERR_INVALID_ARG;
  if (p->kernel_flags != 0 && !((unsigned)p->kernel_flags & LBM_KF_SET)) return LBM_ERR_INVALID_ARG;
  if (!std::isfinite(p->ax) || !std::isfinite(p->rho_ave) || p->ax_from_step < 0)
    return LBM_ERR_INVALID_ARG;
  return LBM_OK;
}

void apply_launch(lbm_ctx* c) {
  c->nstrips = (c->p.nx + c->lc.bx - 1) / c->lc.bx;
  c->nseg = (c->p.ny + c->lc.ly - 1) / c->lc.ly;
  int ntiles = c->nstrips * c->nseg;
  const bool no_remap = ((unsigned)c->p.kernel_flags & LBM_KF_SET) &&
                        ((unsigned)c->p.kernel_flags & LBM_KF_NO_XCD_REMAP);
  c->xcd_remap = (ntiles >= 64 && ntiles % 8 == 0 && !no_remap) ? 1 : 0;
  for (KParams<double>* k : {&c->kd}) {
    k->nstrips = c->nstrips;
    k->nseg = c->nseg;
    k->LY = c->lc.ly;
    k->xcd_remap = c->xcd_remap;
  }
  c->nstrips2 = (c->p.nx + c->lc.bx2 - 1) / c->lc.bx2;
  c->nseg2 = c->nseg;
  const int ntiles2 = c->nstrips2 * c->nseg2;
  c->xcd_remap2 = (ntiles2 >= 64 && ntiles2 % 8 == 0 && !no_remap) ? 1 : 0;
  c->kf.nstrips = c->nstrips;
  c->kf.nseg = c->nseg;
  c->kf.LY = c->lc.ly;
  c->kf.xcd_remap = c->xcd_remap;
}

// Segment height from occupancy: with R workgroups resident on the device
// (the kernel's blocks per CU times the CU count) the lattice is cut into
// at most k R tiles of equal height, so one launch is k full rounds of
// workgroups with no partly filled tail round; segments stay at least 16
// rows so the halo rows remain a small overhead.
bool two_step_ok(const lbm_ctx* c);

template <class K>
void tune_ly(lbm_ctx* c, K kernel, int bx, int nstrips) {
  c->lc.auto_ly = 0;
  int blocks = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, bx, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      blocks < 1 || cus < 1) {
    (void)hipGetLastError();
    return;  // keep the fallback height
  }
  // measured on 4096^2: the free-energy kernel and the two-step kernels are
  // fastest with one round, the single-step pseudopotential one with three
  const int rounds = c->p.tile_rounds > 0 ? c->p.tile_rounds
                     : (c->p.model == LBM_MODEL_P && !two_step_ok(c) ? 3 : 1);
  const int resident = blocks * cus * std::max(1, rounds);
  const int segs = std::max(1, resident / nstrips);
  int LY = (c->p.ny + segs - 1) / segs;
  LY = std::max(LY, std::min(16, c->p.ny));
  c->lc.ly = std::min(LY, c->p.ny);
  apply_launch(c);
}

template <int MODEL, int EOS, class S, class C, int BX, int NT, int WPE>
void launch_step_w(lbm_ctx* c, const KParams<C>& kp) {
  // compile-time model branches: each model instantiates only its own kernels
  if (c->lc.auto_ly) {
    if constexpr (MODEL == MODEL_P) {
      if (c->lc.pipe) tune_ly(c, k_step_p_pipe<EOS, S, C, BX, NT, WPE>, BX, c->nstrips);
      else tune_ly(c, k_step_p<EOS, S, C, BX, NT, WPE>, BX, c->nstrips);
    } else {
      if (c->lc.pipe) tune_ly(c, k_step_fe_pipe<EOS, S, C, BX, NT, WPE>, BX, c->nstrips);
      else tune_ly(c, k_step_fe<EOS, S, C, BX, NT, WPE>, BX, c->nstrips);
    }
  }
  const S* src = (const S*)(c->ws + (c->cur ? c->L.fB : c->L.fA));
  S* dst = (S*)(c->ws + (c->cur ? c->L.fA : c->L.fB));
  unsigned* flags = (unsigned*)(c->ws + c->L.flags);
  dim3 grid(c->nstrips * c->nseg), block(BX);
  if constexpr (MODEL == MODEL_P) {
    if (c->lc.pipe)
      hipLaunchKernelGGL((k_step_p_pipe<EOS, S, C, BX, NT, WPE>), grid, block, 0, c->stream, src, dst, kp, flags);
    else
      hipLaunchKernelGGL((k_step_p<EOS, S, C, BX, NT, WPE>), grid, block, 0, c->stream, src, dst, kp, flags);
  } else {
    if (c->lc.pipe)
      hipLaunchKernelGGL((k_step_fe_pipe<EOS, S, C, BX, NT, WPE>), grid, block, 0, c->stream, src, dst, kp, flags);
    else
      hipLaunchKernelGGL((k_step_fe<EOS, S, C, BX, NT, WPE>), grid, block, 0, c->stream, src, dst, kp, flags);
  }
  c->cur ^= 1;
}

int grid1d(size_t N) {
  size_t b = (N + 255) / 256;
  return (int)std::min<size_t>(std::max<size_t>(b, 1), 4096);
}

// The general kernel (walls of Sec. 5.3, the droplet-collision drive of
// Sec. 5.4, the A term of Eq. 20): plain row loop, no register cap,
// non-temporal stores.  With A != 0 the velocity field of the step is
// formed first by the observation passes (Eq. 6b at every node), because
// S = grad u + grad u^T needs the neighbours' velocities.
template <int MODEL, int EOS, class S, class C, int BX>
void launch_step_gen(lbm_ctx* c, const KParams<C>& kp) {
  // the FE kernels take the periodic kernel's register target (a tighter
  // cap spills); GEN = 3 carries the A term, GEN = 1 the other options
  constexpr int WG = (MODEL == MODEL_FE) ? wpe_target<MODEL_FE, S>() : 0;
  const bool with_a = MODEL == MODEL_FE && c->p.A != 0.0;
  if (c->lc.auto_ly) {
    if constexpr (MODEL == MODEL_P) tune_ly(c, k_step_p<EOS, S, C, BX, 1, 0, 1>, BX, c->nstrips);
    else if (with_a) tune_ly(c, k_step_fe<EOS, S, C, BX, 1, WG, 3>, BX, c->nstrips);
    else tune_ly(c, k_step_fe<EOS, S, C, BX, 1, WG, 1>, BX, c->nstrips);
  }
  const S* src = (const S*)(c->ws + (c->cur ? c->L.fB : c->L.fA));
  S* dst = (S*)(c->ws + (c->cur ? c->L.fA : c->L.fB));
  unsigned* flags = (unsigned*)(c->ws + c->L.flags);
  dim3 grid(c->nstrips * c->nseg), block(BX);
  if constexpr (MODEL == MODEL_FE) {
    if (c->p.A != 0.0)  // the step's velocity field first (GEN = 2 pass)
      hipLaunchKernelGGL((k_step_fe<EOS, S, C, BX, 1, WG, 2>), grid, block, 0, c->stream, src, dst,
                         kp, flags);
  }
  if constexpr (MODEL == MODEL_P)
    hipLaunchKernelGGL((k_step_p<EOS, S, C, BX, 1, 0, 1>), grid, block, 0, c->stream, src, dst, kp, flags);
  else if (with_a)
    hipLaunchKernelGGL((k_step_fe<EOS, S, C, BX, 1, WG, 3>), grid, block, 0, c->stream, src, dst, kp, flags);
  else
    hipLaunchKernelGGL((k_step_fe<EOS, S, C, BX, 1, WG, 1>), grid, block, 0, c->stream, src, dst, kp, flags);
  c->cur ^= 1;
}

bool needs_gen(const lbm_params& p) {
  // walls (and with them gravity), the collision drive and A != 0
  return p.boundary == LBM_BOUNDARY_WALLS || p.ax != 0.0 || p.A != 0.0;
}

template <int MODEL, int EOS, class S, class C, int BX>
void launch_step_bx(lbm_ctx* c, const KParams<C>& kp) {
  if (needs_gen(c->p)) {
    launch_step_gen<MODEL, EOS, S, C, BX>(c, kp);
    return;
  }
  constexpr int W = wpe_target<MODEL, S>();
  if (c->lc.nt) {
    if (c->lc.wpe) launch_step_w<MODEL, EOS, S, C, BX, 1, W>(c, kp);
    else launch_step_w<MODEL, EOS, S, C, BX, 1, 0>(c, kp);
  } else {
    if (c->lc.wpe) launch_step_w<MODEL, EOS, S, C, BX, 0, W>(c, kp);
    else launch_step_w<MODEL, EOS, S, C, BX, 0, 0>(c, kp);
  }
}

template <int MODEL, int EOS, class S, class C>
void launch_step(lbm_ctx* c, const KParams<C>& kp) {
  if (c->lc.bx == 64) launch_step_bx<MODEL, EOS, S, C, 64>(c, kp);
  else launch_step_bx<MODEL, EOS, S, C, 256>(c, kp);
}

// Two steps in one launch (periodic lattices): strips of bx2 columns
// (256, or 128 for the free-energy kernel, whose register budget leaves two
// 256-column workgroups per CU but four 128-column ones).  The segment
// height is chosen for this kernel even when a single step is launched
// first (odd step counts), since it carries the run.
template <int EOS, class S, class C, int BX>
void tune_two_bx(lbm_ctx* c) {
  if (c->p.model == LBM_MODEL_P) {
    if constexpr (BX == 256) {
      if (c->lc.nt) tune_ly(c, k_step2_p<EOS, S, C, BX, 1>, BX + 64, c->nstrips2);
      else tune_ly(c, k_step2_p<EOS, S, C, BX, 0>, BX + 64, c->nstrips2);
    }
  } else {
    tune_ly(c, k_step2_fe<EOS, S, C, BX>, BX + 64, c->nstrips2);
  }
}

template <int EOS, class S, class C>
void tune_two(lbm_ctx* c) {
  if (c->lc.bx2 == 128) tune_two_bx<EOS, S, C, 128>(c);
  else if (c->lc.bx2 == 192) tune_two_bx<EOS, S, C, 192>(c);
  else tune_two_bx<EOS, S, C, 256>(c);
}

void tune_two_dispatch(lbm_ctx* c) {
  const bool cs = c->p.eos == LBM_EOS_CS;
  if (c->p.precision == LBM_FP64) {
    if (cs) tune_two<EOS_CS, double, double>(c);
    else tune_two<EOS_VDW, double, double>(c);
  } else {
    if (cs) tune_two<EOS_CS, float, float>(c);
    else tune_two<EOS_VDW, float, float>(c);
  }
}

template <int EOS, class S, class C, int BX>
void launch_step2_bx(lbm_ctx* c, const KParams<C>& kp_in) {
  KParams<C> kp = kp_in;  // the two-step kernel's own tiling
  kp.nstrips = c->nstrips2;
  kp.nseg = c->nseg2;
  kp.xcd_remap = c->xcd_remap2;
  const S* src = (const S*)(c->ws + (c->cur ? c->L.fB : c->L.fA));
  S* dst = (S*)(c->ws + (c->cur ? c->L.fA : c->L.fB));
  unsigned* flags = (unsigned*)(c->ws + c->L.flags);
  dim3 grid(c->nstrips2 * c->nseg2), block(BX + 64);
  if (c->p.model == LBM_MODEL_P) {
    if constexpr (BX == 256) {
      if (c->lc.nt)
        hipLaunchKernelGGL((k_step2_p<EOS, S, C, BX, 1>), grid, block, 0, c->stream, src, dst, kp, flags);
      else
        hipLaunchKernelGGL((k_step2_p<EOS, S, C, BX, 0>), grid, block, 0, c->stream, src, dst, kp, flags);
    }
  } else {
    hipLaunchKernelGGL((k_step2_fe<EOS, S, C, BX>), grid, block, 0, c->stream, src, dst, kp, flags);
  }
  c->cur ^= 1;
}

template <int EOS, class S, class C>
void launch_step2(lbm_ctx* c, const KParams<C>& kp) {
  if (c->lc.auto_ly) tune_two<EOS, S, C>(c);
  if (c->lc.bx2 == 128) launch_step2_bx<EOS, S, C, 128>(c, kp);
  else if (c->lc.bx2 == 192) launch_step2_bx<EOS, S, C, 192>(c, kp);
  else launch_step2_bx<EOS, S, C, 256>(c, kp);
}

bool two_step_ok(const lbm_ctx* c) {
  return c->lc.two && !needs_gen(c->p) && c->lc.bx == 256;
}

void step_twice(lbm_ctx* c) {
  const bool cs = c->p.eos == LBM_EOS_CS;
  if (c->p.precision == LBM_FP64) {
    if (cs) launch_step2<EOS_CS, double, double>(c, c->kd);
    else launch_step2<EOS_VDW, double, double>(c, c->kd);
  } else {
    if (cs) launch_step2<EOS_CS, float, float>(c, c->kf);
    else launch_step2<EOS_VDW, float, float>(c, c->kf);
  }
}

template <int MODEL, int EOS>
void step_dispatch_prec(lbm_ctx* c) {
  if (c->p.precision == LBM_FP64)
    launch_step<MODEL, EOS, double, double>(c, c->kd);
  else
    launch_step<MODEL, EOS, float, float>(c, c->kf);
}

void step_once(lbm_ctx* c) {
  if (c->lc.auto_ly && two_step_ok(c)) tune_two_dispatch(c);
  if (c->p.model == LBM_MODEL_P) {
    if (c->p.eos == LBM_EOS_CS) step_dispatch_prec<MODEL_P, EOS_CS>(c);
    else step_dispatch_prec<MODEL_P, EOS_VDW>(c);
  } else {
    if (c->p.eos == LBM_EOS_CS) step_dispatch_prec<MODEL_FE, EOS_CS>(c);
    else step_dispatch_prec<MODEL_FE, EOS_VDW>(c);
  }
}


template <class S>
void launch_init(lbm_ctx* c, const double* rho0) {
  S* dst = (S*)(c->ws + c->L.fA);
  size_t N = (size_t)c->p.nx * c->p.ny;
  if (c->p.model == LBM_MODEL_P)
    hipLaunchKernelGGL((k_init<MODEL_P, S>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       rho0, dst, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg);
  else
    hipLaunchKernelGGL((k_init<MODEL_FE, S>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       rho0, dst, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg,
                       3.0 * c->p.grav_rho0 * c->p.g, c->p.grav_y0);
}

template <int MODEL, int EOS, class S>
void launch_observe(lbm_ctx* c, int cx, int cy, double* d_rho, double* d_ux, double* d_uy) {
  const S* src = (const S*)(c->ws + (c->cur ? c->L.fB : c->L.fA));
  double* rho_w = (double*)(c->ws + c->L.rho_w);
  double* aux_w = (double*)(c->ws + c->L.aux_w);
  double* uxp = (double*)(c->ws + c->L.uxp);
  double* uyp = (double*)(c->ws + c->L.uyp);
  ObsPartial* part = (ObsPartial*)(c->ws + c->L.part);
  unsigned* flags = (unsigned*)(c->ws + c->L.flags);
  double* res = (double*)(c->ws + c->L.result);
  size_t N = (size_t)c->p.nx * c->p.ny;
  hipLaunchKernelGGL((k_obs_rho<MODEL, EOS, S>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                     src, c->kd, rho_w, aux_w, flags);
  if (MODEL == MODEL_FE)
    hipLaunchKernelGGL((k_obs_mu<EOS>), dim3(grid1d(N)), dim3(256), 0, c->stream, c->kd,
                       (const double*)rho_w, aux_w);
  hipLaunchKernelGGL((k_obs_u<MODEL, S, kObsThreads>), dim3(c->L.obs_blocks),
                     dim3(kObsThreads), 0, c->stream, src, c->kd, (const double*)rho_w,
                     (const double*)aux_w, d_rho, d_ux, d_uy, uxp, uyp, c->have_prev, part);
  hipLaunchKernelGGL((k_obs_final<EOS, kObsThreads>), dim3(1), dim3(kObsThreads), 0,
                     c->stream, (const ObsPartial*)part, c->L.obs_blocks, c->kd,
                     (const double*)rho_w, cx, cy, res);
}

template <int MODEL, int EOS>
void observe_dispatch_prec(lbm_ctx* c, int cx, int cy, double* r, double* ux, double* uy) {
  if (c->p.precision == LBM_FP64)
    launch_observe<MODEL, EOS, double>(c, cx, cy, r, ux, uy);
  else
    launch_observe<MODEL, EOS, float>(c, cx, cy, r, ux, uy);
}

// Context set-up shared by lbm_init and the batch: validation already done,
// rho0 checked on the host (hrho0), workspace carved.
lbm_status ctx_setup(const lbm_params* p, void* d_workspace, const double* d_rho0,
                     const std::vector<double>& hrho0, hipStream_t stream, lbm_ctx** out) {
  size_t N = (size_t)p->nx * p->ny;
  double rmin = INFINITY;
  for (size_t n = 0; n < N; ++n) {
    double r = hrho0[n];
    if (!std::isfinite(r)) return LBM_ERR_EOS_DOMAIN;
    double lim = (p->eos == LBM_EOS_CS) ? p->b * r / 4.0 : p->b * r;
    if (!(lim < 1.0) || !(r > 0.0)) return LBM_ERR_EOS_DOMAIN;
    rmin = std::min(rmin, r);
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ERR_INVALID_ARG;
  c->p = *p;
  c->stream = stream;
  c->ws = (char*)d_workspace;
  c->L = make_layout(p);
  c->cur = 0;
  c->step = 0;
  c->have_prev = 0;
  c->rho_ref = 0.0;
  {
    // mean initial density for the collision drive: compensated sum
    double s = 0.0, e = 0.0;
    for (size_t n = 0; n < N; ++n) {
      double t = s + hrho0[n];
      e += (std::fabs(s) >= std::fabs(hrho0[n])) ? (s - t) + hrho0[n] : (hrho0[n] - t) + s;
      s = t;
    }
    c->rho_ave = (p->rho_ave > 0.0) ? p->rho_ave : (s + e) / (double)N;
  }
  if (p->precision == LBM_FP32_SHIFTED) {
    // Storage shift f^eq(rho_ref, 0) (w_i rho_ref for P, rho_ref delta_i0 for
    // FE).  The default reference is the smallest initial density: the
    // stored deviations of the thinnest phase are then near zero, so float
    // rounding stays a small fraction of every local density (a mid-range
    // reference would leave the vapour with absolute noise of the order of
    // 2^-24 rho_ref per step).  Round rho_ref so that rho_ref / 36 carries
    // at most 20 significant bits: then w_i rho_ref, their sum and M s are
    // all exact in float and the deviations carry no constant bias.
    double want = (p->rho_ref > 0.0) ? p->rho_ref : rmin;
    double q = want / 36.0;
    int ex;
    double m = frexp(q, &ex);
    m = nearbyint(ldexp(m, 20));
    q = ldexp(m, ex - 20);
    c->rho_ref = 36.0 * q;
  }
  c->lc = resolve_launch(p);
  c->kd = make_kparams<double>(p, c->rho_ref, 1, 1, c->lc.ly, 0);
  c->kf = make_kparams<float>(p, c->rho_ref, 1, 1, c->lc.ly, 0);
  c->kd.rho_ave = c->rho_ave;
  c->kf.rho_ave = (float)c->rho_ave;
  c->kd.uax = c->kf.uax = (double*)(c->ws + c->L.uax);
  c->kd.uay = c->kf.uay = (double*)(c->ws + c->L.uay);
  apply_launch(c);
  if (hipMemsetAsync(c->ws + c->L.flags, 0, kAlign, stream) != hipSuccess) {
    delete c;
    return LBM_ERR_HIP;
  }
  if (p->precision == LBM_FP64) launch_init<double>(c, d_rho0);
  else launch_init<float>(c, d_rho0);
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return LBM_ERR_HIP;
  }
  *out = c;
  return LBM_OK;
}

lbm_status read_host(const double* d, size_t n, hipStream_t stream, std::vector<double>& h) {
  h.resize(n);
  if (hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return LBM_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return LBM_ERR_HIP;
  return LBM_OK;
}

// The collision drive acts in the steps that start at t >= ax_from_step;
// the velocity observed at time t (Eq. 6b) uses the force of step t.
void set_drive(lbm_ctx* c, int64_t t) {
  const bool on = c->p.ax != 0.0 && t >= c->p.ax_from_step;
  c->kd.ax = on ? c->p.ax : 0.0;
  c->kf.ax = on ? (float)c->p.ax : 0.0f;
}

lbm_status observe_impl(lbm_ctx* c, int32_t cx, int32_t cy, lbm_obs* out,
                        double* d_rho, double* d_ux, double* d_uy) {
  set_drive(c, c->step);
  if (c->p.model == LBM_MODEL_P) {
    if (c->p.eos == LBM_EOS_CS) observe_dispatch_prec<MODEL_P, EOS_CS>(c, cx, cy, d_rho, d_ux, d_uy);
    else observe_dispatch_prec<MODEL_P, EOS_VDW>(c, cx, cy, d_rho, d_ux, d_uy);
  } else {
    if (c->p.eos == LBM_EOS_CS) observe_dispatch_prec<MODEL_FE, EOS_CS>(c, cx, cy, d_rho, d_ux, d_uy);
    else observe_dispatch_prec<MODEL_FE, EOS_VDW>(c, cx, cy, d_rho, d_ux, d_uy);
  }
  if (hipGetLastError() != hipSuccess) return LBM_ERR_HIP;
  double res[9];
  unsigned flags = 0;
  if (hipMemcpyAsync(res, c->ws + c->L.result, sizeof(res), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return LBM_ERR_HIP;
  if (hipMemcpyAsync(&flags, c->ws + c->L.flags, sizeof(flags), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return LBM_ERR_HIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_ERR_HIP;
  out->step = c->step;
  out->mass = res[0];
  out->max_u = res[1];
  out->rho_min = res[2];
  out->rho_max = res[3];
  out->rho_in = res[4];
  out->rho_out = res[5];
  out->dp = res[6];
  out->r_equimolar = res[7];
  out->du_max = c->have_prev ? res[8] : INFINITY;
  out->flags = flags;
  out->reserved = 0;
  c->have_prev = 1;
  return LBM_OK;
}

// Issue m steps: two per launch where the two-step kernel applies, else one.
void advance(lbm_ctx* c, int m) {
  int k = 0;
  if (two_step_ok(c))
    for (; k + 2 <= m; k += 2) step_twice(c);
  for (; k < m; ++k) step_once(c);
}

// Run kGraphSteps steps (an even number, so the state ends in the buffer it
// started from) as one HIP graph: captured once per starting buffer and
// drive state on the library's capture stream, then launched on the
// context's stream.  The kernels' arguments (buffers, parameters, launch
// shape) are recorded by value; they do not change once the first step has
// fixed the launch shape.
lbm_status launch_graph_run(lbm_ctx* c) {
  const int cur0 = c->cur;
  const int drv = c->kd.ax != 0.0 ? 1 : 0;
  hipGraphExec_t& ge = c->graph[cur0][drv];
  if (!ge) {
    if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
      c->cap = nullptr;
      return LBM_ERR_HIP;
    }
    hipStream_t user = c->stream;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return LBM_ERR_HIP;
    c->stream = c->cap;
    advance(c, kGraphSteps);
    c->stream = user;
    c->cur = cur0;  // the capture only recorded the launches
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (e != hipSuccess) return LBM_ERR_HIP;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      ge = nullptr;
      return LBM_ERR_HIP;
    }
  }
  return hipGraphLaunch(ge, c->stream) == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

}  // namespace

lbm_ctx::~lbm_ctx() {
  for (auto& row : graph)
    for (hipGraphExec_t& g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (cap) (void)hipStreamDestroy(cap);
}

extern "C" {

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_EOS_DOMAIN: return "density outside the equation-of-state domain";
    case LBM_ERR_UNSUPPORTED: return "unsupported option";
    case LBM_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_NO_CONVERGENCE: return "solver did not converge";
  }
  return "unknown status";
}

lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  if (!bytes) return LBM_ERR_INVALID_ARG;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  if ((st = validate_launch(p)) != LBM_OK) return st;
  *bytes = make_layout(p).total;
  return LBM_OK;
}

lbm_status lbm_init(const lbm_params* p, void* d_workspace, size_t bytes,
                    const double* d_rho0, void* hip_stream, lbm_ctx** out) {
  if (!out || !d_rho0) return LBM_ERR_INVALID_ARG;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  if ((st = validate_launch(p)) != LBM_OK) return st;
  Layout L = make_layout(p);
  if (!d_workspace || bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0)
    return LBM_ERR_WORKSPACE;
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<double> h;
  if ((st = read_host(d_rho0, (size_t)p->nx * p->ny, stream, h)) != LBM_OK) return st;
  return ctx_setup(p, d_workspace, d_rho0, h, stream, out);
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c || n < 0) return LBM_ERR_INVALID_ARG;
  lbm_status st = LBM_OK;
  int64_t k = 0;
  while (k < n && st == LBM_OK) {
    const int64_t t = c->step + k;
    // a whole graph run needs the launch shape fixed (after the first
    // launch) and one drive state throughout
    const bool drive_const = c->p.ax == 0.0 || t >= c->p.ax_from_step ||
                             t + kGraphSteps <= c->p.ax_from_step;
    if (n - k >= kGraphSteps && !c->lc.auto_ly && drive_const) {
      set_drive(c, t);
      st = launch_graph_run(c);
      k += kGraphSteps;
    } else if (two_step_ok(c) && n - k >= 2) {
      set_drive(c, t);  // (no drive: the two-step kernel is periodic only)
      step_twice(c);
      k += 2;
    } else {
      set_drive(c, t);
      step_once(c);
      k += 1;
    }
  }
  c->step += k;
  if (st != LBM_OK) return st;
  if (hipGetLastError() != hipSuccess) return LBM_ERR_HIP;
  return LBM_OK;
}

lbm_status lbm_observe(lbm_ctx* c, int32_t cx, int32_t cy, lbm_obs* out,
                       double* d_rho, double* d_ux, double* d_uy) {
  if (!c || !out) return LBM_ERR_INVALID_ARG;
  return observe_impl(c, cx, cy, out, d_rho, d_ux, d_uy);
}

lbm_status lbm_get_populations(lbm_ctx* c, double* d_f) {
  if (!c || !d_f) return LBM_ERR_INVALID_ARG;
  size_t N = (size_t)c->p.nx * c->p.ny;
  const void* src = c->ws + (c->cur ? c->L.fB : c->L.fA);
  if (c->p.precision == LBM_FP64)
    hipLaunchKernelGGL((k_get_pop<double>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       (const double*)src, d_f, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg);
  else
    hipLaunchKernelGGL((k_get_pop<float>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       (const float*)src, d_f, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status lbm_set_populations(lbm_ctx* c, const double* d_f) {
  if (!c || !d_f) return LBM_ERR_INVALID_ARG;
  size_t N = (size_t)c->p.nx * c->p.ny;
  void* dst = c->ws + (c->cur ? c->L.fB : c->L.fA);
  if (c->p.precision == LBM_FP64)
    hipLaunchKernelGGL((k_set_pop<double>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       d_f, (double*)dst, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg);
  else
    hipLaunchKernelGGL((k_set_pop<float>), dim3(grid1d(N)), dim3(256), 0, c->stream,
                       d_f, (float*)dst, c->p.nx, c->p.ny, c->kd.rowpitch, c->kd.s0, c->kd.sax, c->kd.sdg);
  c->have_prev = 0;
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  delete c;  // ~lbm_ctx releases the graphs and the capture stream
  return LBM_OK;
}

lbm_status lbm_launch_info(const lbm_ctx* c, lbm_launch* out) {
  if (!c || !out) return LBM_ERR_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  const bool two = two_step_ok(c);
  out->steps_per_launch = two ? 2 : 1;
  out->strip = two ? c->lc.bx2 : c->lc.bx;
  out->threads = two ? c->lc.bx2 + 64 : c->lc.bx;
  if (!c->lc.auto_ly) {
    out->segment = c->lc.ly;
    out->workgroups = two ? c->nstrips2 * c->nseg2 : c->nstrips * c->nseg;
  }
  return LBM_OK;
}

lbm_status lbm_autotune(const lbm_params* p, void* d_workspace, size_t bytes,
                        const double* d_rho0, void* hip_stream, int32_t steps,
                        lbm_params* best, double* best_ms_per_step) {
  if (!best || !d_rho0 || steps < 1) return LBM_ERR_INVALID_ARG;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  Layout L = make_layout(p);
  if (!d_workspace || bytes < L.total || ((uintptr_t)d_workspace % kAlign) != 0)
    return LBM_ERR_WORKSPACE;
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<double> h;
  if ((st = read_host(d_rho0, (size_t)p->nx * p->ny, stream, h)) != LBM_OK) return st;
  const bool fp64 = p->precision == LBM_FP64;
  std::vector<int> bxs = {64, 256};
  // tile_y 0: the occupancy-derived one-round segment height
  std::vector<int> lys = {0, 8, 16, 32, 64};
  std::vector<unsigned> kfs = {LBM_KF_SET | LBM_KF_NT_STORE | LBM_KF_REGCAP,
                               LBM_KF_SET | LBM_KF_NT_STORE,
                               LBM_KF_SET | LBM_KF_REGCAP};
  if (p->model == LBM_MODEL_P) {
    kfs.push_back(LBM_KF_SET | LBM_KF_NT_STORE | LBM_KF_PIPELINE);
    kfs.push_back(LBM_KF_SET | LBM_KF_NT_STORE | LBM_KF_REGCAP | LBM_KF_PIPELINE);
  }
  // two steps per launch (applies to periodic lattices with 256-column
  // strips; elsewhere these candidates run single steps)
  kfs.push_back(LBM_KF_SET | LBM_KF_NT_STORE | LBM_KF_TWO_STEP);
  if (p->model == LBM_MODEL_FE)
    kfs.push_back(LBM_KF_SET | LBM_KF_NT_STORE | LBM_KF_TWO_STEP | LBM_KF_STRIP128);
  (void)fp64;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBM_ERR_HIP;
  double best_t = INFINITY;
  lbm_params bp = *p;
  for (int bx : bxs) {
    if (bx == 256 && p->nx < 192) continue;
    for (int ly : lys) {
      if (ly > p->ny) continue;
      for (unsigned kf : kfs) {
        lbm_params q = *p;
        q.tile_x = bx;
        q.tile_y = ly;
        q.kernel_flags = (int32_t)kf;
        lbm_ctx* c = nullptr;
        if ((st = ctx_setup(&q, d_workspace, d_rho0, h, stream, &c)) != LBM_OK) break;
        advance(c, 2);  // warm-up (and first-touch of the second buffer)
        hipEventRecord(e0, stream);
        advance(c, steps);
        hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) st = LBM_ERR_HIP;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        delete c;
        if (st != LBM_OK) break;
        double t = ms / steps;
        if (t < best_t) {
          best_t = t;
          bp = q;
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != LBM_OK) return st;
  *best = bp;
  if (best_ms_per_step) *best_ms_per_step = best_t;
  return LBM_OK;
}

}  // extern "C"

// =============================================================================
// Batches of independent lattices
// =============================================================================
namespace {

struct BatchInst {
  lbm_ctx* ctx;
  size_t chk_off;   // per-instance check velocities (2 N values of type C)
  int state;        // LBM_BATCH_*
  int64_t steps;
  double du, best_du;
  int stall;        // checks without a new best du
  int checks;
  uint32_t flags;
  int64_t limit;    // retire with LBM_BATCH_MAXSTEPS once steps >= limit
  int partner;      // the other problem of its unit, or -1
  int auto_ly;      // segment height chosen per group at each table rebuild
};

// two: the group's chunks take two steps per launch (k_batch_step2)
struct GroupKey {
  int model, eos, bx, two;
  bool operator<(const GroupKey& o) const {
    return model != o.model ? model < o.model
         : eos != o.eos     ? eos < o.eos
         : bx != o.bx       ? bx < o.bx
                            : two < o.two;
  }
};

}  // namespace

struct lbm_batch {
  int n;
  int fp64;
  hipStream_t stream;      // the caller's stream: graphs are launched on it
  hipStream_t cap_stream;  // library stream the graphs are captured on
  hipStream_t launch;      // stream the step launches are issued to
  char* ws;
  std::vector<BatchInst> inst;
  size_t desc_off, tiles_off, du_off, tiles_cap;
  size_t flagptr_off, flagout_off;  // per-instance flag pointers, gathered flags
  size_t counts_off;                // active tile count of each group (device)
  int parity;  // common population parity of all instances
  // one tile table per (model, EOS, strip width) group, all in one buffer:
  // each group owns a fixed region sized for all its lattices, and its
  // launch a grid set when the graph is captured; retirement changes the
  // tables and counts, and a new graph is captured only when a group
  // empties or its grid exceeds twice its tiles
  // grid / resident: the single-step launches; grid2 / resident2: the
  // two-step launches of a two-step group
  struct Group {
    GroupKey key;
    int offset, capacity, count, grid, resident, grid2, resident2;
  };
  std::vector<Group> groups;
  bool tables_valid;
  unsigned graph_groups = 0;  // groups with tiles when the graph was captured
  hipGraphExec_t graph;
  int graph_steps;
  int graph_parity;
  // measurement: node updates issued, and GPU time between events recorded
  // around each chunk's graph launch
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int64_t node_updates = 0;
  double gpu_ms = 0.0;
  int64_t chunks = 0;
};

namespace {

struct BatchLayout {
  std::vector<size_t> inst_off, chk_off;
  size_t desc_off, tiles_off, du_off, flagptr_off, flagout_off, counts_off, total, tiles_cap;
};
constexpr int kMaxGroups = 12;  // 2 models x 2 EOS x (64, 256, 256 two-step)
// Automatic segment heights in a batch: the lowest, which sizes the tile
// tables, and the candidates above it, tallest first.
constexpr int kBatchMinLY = 4;
constexpr int kBatchLY[] = {128, 64, 32, 16, 8};

BatchLayout make_batch_layout(int n, const lbm_params* p) {
  BatchLayout B;
  size_t off = 0;
  size_t tiles = 0;
  for (int i = 0; i < n; ++i) {
    B.inst_off.push_back(off);
    off += make_layout(&p[i]).total;
    size_t N = (size_t)p[i].nx * p[i].ny;
    size_t es = p[i].precision == LBM_FP64 ? 8 : 4;
    B.chk_off.push_back(off);
    off += align_up(2 * N * es);
    LaunchCfg lc = resolve_launch(&p[i]);
    const int ly = p[i].tile_y > 0 ? lc.ly : kBatchMinLY;
    tiles += (size_t)((p[i].nx + lc.bx - 1) / lc.bx) * ((p[i].ny + ly - 1) / ly);
  }
  size_t desc = std::max(sizeof(InstDesc<double>), sizeof(InstDesc<float>));
  B.desc_off = off;
  off += align_up(n * desc);
  B.tiles_cap = tiles;
  B.tiles_off = off;
  off += align_up(tiles * sizeof(BatchTile));
  B.du_off = off;
  off += align_up(n * sizeof(unsigned long long));
  B.flagptr_off = off;
  off += align_up(n * sizeof(unsigned*));
  B.flagout_off = off;
  off += align_up(n * sizeof(unsigned));
  B.counts_off = off;
  off += align_up(kMaxGroups * sizeof(int));
  B.total = off;
  return B;
}

// Resident workgroups of a batch kernel on this device (occupancy x CUs).
template <class K>
int resident_blocks(K kernel, int bx) {
  int blocks = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, bx, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      blocks < 1 || cus < 1) {
    (void)hipGetLastError();
    return 1024;
  }
  return blocks * cus;
}

// Strips the two-step kernel of a group cuts each table tile into.
int batch2_split(const lbm_batch::Group& g) { return g.key.model == MODEL_FE ? 2 : 1; }

// Launch kinds of one group: plain step, checking step, two steps.
enum BatchLaunch { BL_RESIDENT = -2, BL_GRID = -1, BL_PLAIN = 0, BL_CHECK = 1, BL_TWO = 2 };

// BL_RESIDENT: only find the group's resident workgroups per kernel;
// BL_GRID: also fix its grids (about one round of resident workgroups, at
// most one per active tile), outside any capture
template <int MODEL, int EOS, class S, class C, int BX>
void launch_batch_group(lbm_batch* b, lbm_batch::Group& g, int kind, int parity) {
  if (kind == BL_RESIDENT || kind == BL_GRID) {
    if (g.resident == 0) g.resident = resident_blocks(k_batch_step<MODEL, EOS, S, C, BX, 1, 0>, BX);
    if constexpr (BX == 256)
      if (g.key.two && g.resident2 == 0)
        g.resident2 = resident_blocks(k_batch_step2<MODEL, EOS, S, C>, batch2_bx<MODEL>() + 64);
    if (kind == BL_GRID) {
      g.grid = std::max(1, std::min(g.count, g.resident));
      if (g.key.two) g.grid2 = std::max(1, std::min(g.count * batch2_split(g), g.resident2));
    }
    return;
  }
  const InstDesc<C>* desc = (const InstDesc<C>*)(b->ws + b->desc_off);
  const BatchTile* tiles = (const BatchTile*)(b->ws + b->tiles_off) + g.offset;
  const int* count = (const int*)(b->ws + b->counts_off) + (&g - b->groups.data());
  if (kind == BL_CHECK)
    hipLaunchKernelGGL((k_batch_step<MODEL, EOS, S, C, BX, 1, 1>), dim3(g.grid), dim3(BX), 0,
                       b->launch, tiles, count, desc, parity);
  else if (kind == BL_PLAIN)
    hipLaunchKernelGGL((k_batch_step<MODEL, EOS, S, C, BX, 1, 0>), dim3(g.grid), dim3(BX), 0,
                       b->launch, tiles, count, desc, parity);
  else if constexpr (BX == 256)
    hipLaunchKernelGGL((k_batch_step2<MODEL, EOS, S, C>), dim3(g.grid2),
                       dim3(batch2_bx<MODEL>() + 64), 0, b->launch, tiles, count, desc, parity);
}

template <class S, class C>
void batch_group_typed(lbm_batch* b, lbm_batch::Group& g, int kind, int parity) {
  const GroupKey& k = g.key;
#define LBM_GROUP(M, E, X)                                                       \
  if (k.model == M && k.eos == E && k.bx == X) launch_batch_group<M, E, S, C, X>(b, g, kind, parity)
  LBM_GROUP(MODEL_P, EOS_CS, 64);
  LBM_GROUP(MODEL_P, EOS_CS, 256);
  LBM_GROUP(MODEL_P, EOS_VDW, 64);
  LBM_GROUP(MODEL_P, EOS_VDW, 256);
  LBM_GROUP(MODEL_FE, EOS_CS, 64);
  LBM_GROUP(MODEL_FE, EOS_CS, 256);
  LBM_GROUP(MODEL_FE, EOS_VDW, 64);
  LBM_GROUP(MODEL_FE, EOS_VDW, 256);
#undef LBM_GROUP
}

void batch_group(lbm_batch* b, lbm_batch::Group& g, int kind, int parity) {
  if (b->fp64) batch_group_typed<double, double>(b, g, kind, parity);
  else batch_group_typed<float, float>(b, g, kind, parity);
}

// A problem takes two steps per launch in a batch when its launch
// configuration asks for them and its tiles are 256-column strips (the
// two-step row schedules need the halo wavefront beside the strip).
int batch_two(const lbm_ctx* c) { return c->lc.two && c->lc.bx == 256 ? 1 : 0; }

// Two-step launches of a two-step group in a chunk of `steps` (even) steps:
// the last two steps are single (the last one checking), and the launch
// count steps - m is kept even, so that every chunk ends in the buffer it
// started from.
int batch_pairs(const lbm_batch::Group& g, int steps) {
  return g.key.two ? ((steps - 2) / 2) & ~1 : 0;
}

template <class C>
InstDesc<C> make_desc(lbm_batch* b, int i) {
  InstDesc<C> d{};
  const BatchInst& I = b->inst[i];
  lbm_ctx* c = I.ctx;
  if constexpr (sizeof(C) == 8) d.kp = c->kd; else d.kp = c->kf;
  d.fA = c->ws + c->L.fA;
  d.fB = c->ws + c->L.fB;
  size_t N = (size_t)c->p.nx * c->p.ny;
  d.uxp = (C*)(b->ws + I.chk_off);
  d.uyp = d.uxp + N;
  d.flags = (unsigned*)(c->ws + c->L.flags);
  d.du = (unsigned long long*)(b->ws + b->du_off) + i;
  return d;
}

// Enqueue the copy of every instance's descriptor (launch parameters and
// buffers) to the device; `host` must stay alive until the stream has
// passed the copy.
lbm_status upload_descs(lbm_batch* b, std::vector<char>& host) {
  const size_t dsz = b->fp64 ? sizeof(InstDesc<double>) : sizeof(InstDesc<float>);
  host.assign(b->n * dsz, 0);
  for (int i = 0; i < b->n; ++i) {
    if (b->fp64) {
      InstDesc<double> d = make_desc<double>(b, i);
      memcpy(&host[i * dsz], &d, dsz);
    } else {
      InstDesc<float> d = make_desc<float>(b, i);
      memcpy(&host[i * dsz], &d, dsz);
    }
  }
  return hipMemcpyAsync(b->ws + b->desc_off, host.data(), host.size(), hipMemcpyHostToDevice,
                        b->stream) == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

// Segment height of a group's automatic-height lattices: the tallest
// candidate whose tiles (with the other lattices' own) fill at least three
// quarters of one round of the group's resident workgroups, else the lowest.
// Taller segments repeat fewer halo rows (a two-step free-energy segment
// re-runs ten), so they win while the tiles still fill the device; once few
// lattices remain, shorter ones keep more workgroups busy.
int batch_group_ly(const lbm_batch* b, const lbm_batch::Group& g, const std::vector<int>& act) {
  const int64_t G = g.key.two ? g.resident2 : g.resident;
  const int sx = g.key.two ? 256 / batch2_split(g) : g.key.bx;  // columns per launched strip
  for (int ly : kBatchLY) {
    int64_t T = 0;
    for (int i : act) {
      const lbm_ctx* c = b->inst[i].ctx;
      const int strips = (c->p.nx + sx - 1) / sx;  // strips that hold lattice columns
      T += (int64_t)strips * (b->inst[i].auto_ly ? (c->p.ny + ly - 1) / ly : c->nseg);
    }
    if (4 * T >= 3 * G) return ly;
  }
  return kBatchMinLY;
}

// Rebuild the tile tables of the active instances, largest first within
// each group, and upload them with the counts (outside any graph capture).
// The first call fixes each group's region and grid from all lattices.
lbm_status rebuild_tables(lbm_batch* b) {
  std::map<GroupKey, std::vector<BatchTile>> tabs;
  std::vector<int> order(b->n);
  for (int i = 0; i < b->n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int c) {
    const lbm_params& pa = b->inst[a].ctx->p;
    const lbm_params& pc = b->inst[c].ctx->p;
    return (int64_t)pa.nx * pa.ny > (int64_t)pc.nx * pc.ny;
  });
  if (b->groups.empty()) {
    // first call: each group's region (and launch) is sized for the tiles of
    // all its lattices, retired ones included, since a retired lattice may
    // resume (lbm_batch_set_limit)
    std::map<GroupKey, int> cap;
    for (int i = 0; i < b->n; ++i) {
      lbm_ctx* c = b->inst[i].ctx;
      cap[GroupKey{c->p.model, c->p.eos, c->lc.bx, batch_two(c)}] += c->nseg * c->nstrips;
    }
    int off = 0;
    for (auto& kv : cap) {
      b->groups.push_back({kv.first, off, kv.second, 0, 0, 0, 0, 0});
      off += kv.second;
    }
    if ((size_t)off > b->tiles_cap || b->groups.size() > (size_t)kMaxGroups)
      return LBM_ERR_WORKSPACE;
  }
  // automatic segment heights, per group, from the active lattices
  std::vector<char> descs;
  bool relaunch = false;
  for (auto& g : b->groups) {
    std::vector<int> act;
    bool any_auto = false;
    for (int i = 0; i < b->n; ++i) {
      const BatchInst& I = b->inst[i];
      const lbm_ctx* c = I.ctx;
      if (I.state != LBM_BATCH_ACTIVE || c->p.model != g.key.model || c->p.eos != g.key.eos ||
          c->lc.bx != g.key.bx || batch_two(c) != g.key.two)
        continue;
      act.push_back(i);
      any_auto |= I.auto_ly != 0;
    }
    if (!any_auto) continue;
    batch_group(b, g, BL_RESIDENT, 0);
    const int ly = batch_group_ly(b, g, act);
    for (int i : act) {
      lbm_ctx* c = b->inst[i].ctx;
      if (b->inst[i].auto_ly && c->lc.ly != ly) {
        c->lc.ly = ly;
        apply_launch(c);
        relaunch = true;
      }
    }
  }
  if (relaunch && (upload_descs(b, descs) != LBM_OK || hipStreamSynchronize(b->stream) != hipSuccess))
    return LBM_ERR_HIP;
  for (int i : order) {
    BatchInst& I = b->inst[i];
    if (I.state != LBM_BATCH_ACTIVE) continue;
    lbm_ctx* c = I.ctx;
    GroupKey key{c->p.model, c->p.eos, c->lc.bx, batch_two(c)};
    auto& v = tabs[key];
    for (int s = 0; s < c->nseg; ++s)
      for (int x = 0; x < c->nstrips; ++x) v.push_back(BatchTile{i, x * c->lc.bx, s * c->lc.ly, 0});
  }
  std::vector<BatchTile> all(b->tiles_cap);
  std::vector<int> counts(kMaxGroups, 0);
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    auto& g = b->groups[gi];
    auto it = tabs.find(g.key);
    g.count = it == tabs.end() ? 0 : (int)it->second.size();
    if (g.count > g.capacity) return LBM_ERR_WORKSPACE;  // cannot happen: sized for all
    if (g.count) std::copy(it->second.begin(), it->second.end(), all.begin() + g.offset);
    counts[gi] = g.count;
  }
  if ((!all.empty() &&
       hipMemcpyAsync(b->ws + b->tiles_off, all.data(), all.size() * sizeof(BatchTile),
                      hipMemcpyHostToDevice, b->stream) != hipSuccess) ||
      hipMemcpyAsync(b->ws + b->counts_off, counts.data(), kMaxGroups * sizeof(int),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return LBM_ERR_HIP;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_ERR_HIP;
  b->tables_valid = true;
  return LBM_OK;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Copies every lattice's sticky flags into one array, so that a check reads
// them with a single transfer.
__global__ void k_gather_flags(const unsigned* const* __restrict__ ptrs, unsigned* out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *ptrs[i];
}

// A launch with more than twice as many workgroups as tiles wastes its
// dispatch on workgroups that exit at once (the tail of a run, when a few
// slow lattices remain), and one with fewer workgroups than it could keep
// resident walks 1.5 times as many tiles (after shorter automatic segments)
// in more rounds than needed: then the graph is captured again with new
// grids, which happens a few times per group as its lattices retire.
bool grids_mismatched(const lbm_batch* b) {
  auto off = [](int count, int grid, int resident) {
    return 2 * count < grid || (grid < resident && 2 * count > 3 * grid);
  };
  for (const auto& g : b->groups) {
    if (g.count == 0) continue;
    if (off(g.count, g.grid, g.resident)) return true;
    if (g.key.two && off(g.count * batch2_split(g), g.grid2, g.resident2)) return true;
  }
  return false;
}

unsigned group_mask(const lbm_batch* b) {
  unsigned m = 0;
  for (size_t i = 0; i < b->groups.size(); ++i)
    if (b->groups[i].count > 0) m |= 1u << i;
  return m;
}

void drop_graph(lbm_batch* b) {
  if (b->graph) hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_steps = 0;
}

// Capture `steps` (even) lockstep steps as one graph: each group with
// active tiles runs its steps in order (its lattices are independent of the
// other groups'), the last one checking.  The capture runs on the library's
// own stream (the caller's stream may be the null stream, which cannot be
// captured); the graph is launched on the caller's stream.  The du slots
// are cleared by a kernel, not a memset node, before any checking step.
lbm_status capture_chunk(lbm_batch* b, int steps) {
  drop_graph(b);
  // launch grids from occupancy, before the capture
  for (auto& g : b->groups) batch_group(b, g, BL_GRID, 0);
  const int parity0 = b->parity;
  hipGraph_t g;
  if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return LBM_ERR_HIP;
  b->launch = b->cap_stream;
  hipLaunchKernelGGL(k_zero_u64, dim3((b->n + 255) / 256), dim3(256), 0, b->cap_stream,
                     (unsigned long long*)(b->ws + b->du_off), b->n);
  for (auto& gr : b->groups) {
    if (gr.count == 0) continue;  // no launch for an empty group
    const int m = batch_pairs(gr, steps);
    int par = parity0;
    for (int s = 0; s < m; ++s, par ^= 1) batch_group(b, gr, BL_TWO, par);
    for (int s = 2 * m; s < steps - 1; ++s, par ^= 1) batch_group(b, gr, BL_PLAIN, par);
    batch_group(b, gr, BL_CHECK, par);
  }
  hipLaunchKernelGGL(k_gather_flags, dim3((b->n + 255) / 256), dim3(256), 0, b->cap_stream,
                     (const unsigned* const*)(b->ws + b->flagptr_off),
                     (unsigned*)(b->ws + b->flagout_off), b->n);
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  b->launch = b->stream;
  if (e != hipSuccess) return LBM_ERR_HIP;
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return LBM_ERR_HIP;
  }
  b->graph_steps = steps;
  b->graph_parity = parity0;
  b->graph_groups = group_mask(b);
  return LBM_OK;
}


}  // namespace

extern "C" {

lbm_status lbm_batch_workspace_bytes(int32_t n, const lbm_params* p, size_t* bytes) {
  if (n < 1 || !p || !bytes) return LBM_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    lbm_status st = validate(&p[i]);
    if (st != LBM_OK) return st;
    if ((st = validate_launch(&p[i])) != LBM_OK) return st;
    if (p[i].precision != p[0].precision) return LBM_ERR_INVALID_ARG;
    if (p[i].boundary != LBM_BOUNDARY_PERIODIC || p[i].ax != 0.0 || p[i].A != 0.0 ||
        p[i].g != 0.0)
      return LBM_ERR_UNSUPPORTED;
  }
  *bytes = make_batch_layout(n, p).total;
  return LBM_OK;
}

lbm_status lbm_batch_create(int32_t n, const lbm_params* p, const double* const* d_rho0,
                            void* d_workspace, size_t bytes, void* hip_stream,
                            lbm_batch** out) {
  if (!out || !d_rho0) return LBM_ERR_INVALID_ARG;
  size_t need;
  lbm_status st = lbm_batch_workspace_bytes(n, p, &need);
  if (st != LBM_OK) return st;
  if (!d_workspace || bytes < need || ((uintptr_t)d_workspace % kAlign) != 0)
    return LBM_ERR_WORKSPACE;
  for (int i = 0; i < n; ++i)
    if (!d_rho0[i]) return LBM_ERR_INVALID_ARG;
  hipStream_t stream = (hipStream_t)hip_stream;
  BatchLayout B = make_batch_layout(n, p);
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ERR_INVALID_ARG;
  b->n = n;
  b->fp64 = p[0].precision == LBM_FP64;
  b->stream = stream;
  b->launch = stream;
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return LBM_ERR_HIP;
  }
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return LBM_ERR_HIP;
  }
  b->ws = (char*)d_workspace;
  b->desc_off = B.desc_off;
  b->tiles_off = B.tiles_off;
  b->du_off = B.du_off;
  b->flagptr_off = B.flagptr_off;
  b->flagout_off = B.flagout_off;
  b->counts_off = B.counts_off;
  b->tiles_cap = B.tiles_cap;
  b->parity = 0;
  b->tables_valid = false;
  b->graph = nullptr;
  b->graph_steps = 0;
  b->inst.resize(n);
  std::vector<double> h;
  for (int i = 0; i < n && st == LBM_OK; ++i) {
    BatchInst& I = b->inst[i];
    I = BatchInst{nullptr, B.chk_off[i], LBM_BATCH_ACTIVE, 0, INFINITY, INFINITY, 0, 0, 0u,
                  INT64_MAX, -1, p[i].tile_y <= 0 ? 1 : 0};
    st = read_host(d_rho0[i], (size_t)p[i].nx * p[i].ny, stream, h);
    if (st == LBM_OK) st = ctx_setup(&p[i], b->ws + B.inst_off[i], d_rho0[i], h, stream, &I.ctx);
    if (st == LBM_OK && I.auto_ly) {
      I.ctx->lc.ly = kBatchMinLY;  // the height the tile tables are sized for
      apply_launch(I.ctx);
    }
  }
  if (st != LBM_OK) {
    for (auto& I : b->inst) delete I.ctx;
    (void)hipEventDestroy(b->ev0);
    (void)hipEventDestroy(b->ev1);
    hipStreamDestroy(b->cap_stream);
    delete b;
    return st;
  }
  // instance descriptors
  std::vector<char> descs;
  std::vector<unsigned*> flagptrs(n);
  for (int i = 0; i < n; ++i) {
    lbm_ctx* c = b->inst[i].ctx;
    flagptrs[i] = (unsigned*)(c->ws + c->L.flags);
  }
  if (upload_descs(b, descs) != LBM_OK ||
      hipMemcpyAsync(b->ws + b->flagptr_off, flagptrs.data(), n * sizeof(unsigned*),
                     hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    for (auto& I : b->inst) delete I.ctx;
    (void)hipEventDestroy(b->ev0);
    (void)hipEventDestroy(b->ev1);
    hipStreamDestroy(b->cap_stream);
    delete b;
    return LBM_ERR_HIP;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, int32_t check_every, double du_tol, int64_t max_steps,
                         int64_t* steps_run) {
  if (!b || check_every < 1 || max_steps < 0 || !(du_tol >= 0)) return LBM_ERR_INVALID_ARG;
  int K = check_every + (check_every & 1);
  if (K < 2) K = 2;
  int64_t done = 0;
  std::vector<unsigned long long> du_bits(b->n);
  std::vector<uint32_t> fl(b->n);
  lbm_status st = LBM_OK;
  while (done < max_steps) {
    bool any = false;
    for (auto& I : b->inst) {
      if (I.state == LBM_BATCH_ACTIVE && I.steps >= I.limit) {
        I.state = LBM_BATCH_MAXSTEPS;
        b->tables_valid = false;
      }
      // a unit whose other problem became unstable (at the last check) has
      // no use for this one: it retires before any further step
      if (I.state == LBM_BATCH_ACTIVE && I.partner >= 0 &&
          b->inst[I.partner].state == LBM_BATCH_UNSTABLE) {
        I.state = LBM_BATCH_DROPPED;
        b->tables_valid = false;
      }
      any |= (I.state == LBM_BATCH_ACTIVE);
    }
    if (!any) break;
    // the graph holds fixed grids that read the tile counts from device
    // memory: a new table needs no new graph unless a group has emptied
    // (or refilled), which changes the launches the graph holds
    if (!b->tables_valid) {
      if ((st = rebuild_tables(b)) != LBM_OK) break;
      if (group_mask(b) != b->graph_groups || grids_mismatched(b)) drop_graph(b);
    }
    int chunk = (int)std::min<int64_t>(K, max_steps - done);
    chunk = std::max(2, chunk - (chunk & 1));
    if (!b->graph || b->graph_steps != chunk || b->graph_parity != b->parity)
      if ((st = capture_chunk(b, chunk)) != LBM_OK) break;
    if (hipEventRecord(b->ev0, b->stream) != hipSuccess ||
        hipGraphLaunch(b->graph, b->stream) != hipSuccess ||
        hipEventRecord(b->ev1, b->stream) != hipSuccess) { st = LBM_ERR_HIP; break; }
    for (auto& I : b->inst)
      if (I.state == LBM_BATCH_ACTIVE)
        b->node_updates += (int64_t)I.ctx->p.nx * I.ctx->p.ny * chunk;
    b->parity ^= (chunk & 1);
    done += chunk;
    if (hipMemcpyAsync(du_bits.data(), b->ws + b->du_off, b->n * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, b->stream) != hipSuccess) { st = LBM_ERR_HIP; break; }
    if (hipMemcpyAsync(fl.data(), b->ws + b->flagout_off, b->n * sizeof(uint32_t),
                       hipMemcpyDeviceToHost, b->stream) != hipSuccess) { st = LBM_ERR_HIP; break; }
    if (hipStreamSynchronize(b->stream) != hipSuccess) { st = LBM_ERR_HIP; break; }
    {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) b->gpu_ms += ms;
      b->chunks += 1;
    }
    for (int i = 0; i < b->n; ++i) {
      BatchInst& I = b->inst[i];
      if (I.state != LBM_BATCH_ACTIVE) continue;
      I.steps += chunk;
      I.ctx->step = I.steps;
      I.ctx->cur = b->parity;
      double du;
      memcpy(&du, &du_bits[i], sizeof(du));
      I.flags = fl[i];
      I.checks += 1;
      if (I.flags & (LBM_FLAG_NONFINITE | LBM_FLAG_EOS_DOMAIN)) {
        I.state = LBM_BATCH_UNSTABLE;
        b->tables_valid = false;
        continue;
      }
      if (I.checks == 1) continue;  // the first check only stores u
      I.du = du;
      if (du < I.best_du) {
        I.best_du = du;
        I.stall = 0;
      } else {
        I.stall += 1;
      }
      bool conv = du < du_tol || (I.best_du < 1e-6 && I.stall >= 5);
      if (conv) {
        I.state = LBM_BATCH_CONVERGED;
        b->tables_valid = false;
      } else if (I.stall >= LBM_BATCH_STALL_CHECKS) {
        I.state = LBM_BATCH_STALLED;
        b->tables_valid = false;
      }
    }
  }
  if (st == LBM_OK) {
    // chunks have an even number of steps, so every instance (also one
    // retired at an earlier check) holds its state in the parity-0 buffer
    for (auto& I : b->inst) {
      I.ctx->cur = b->parity;
      I.ctx->have_prev = 0;
    }
    bool any = false;
    for (auto& I : b->inst) {
      if (I.state == LBM_BATCH_ACTIVE && I.partner >= 0 &&
          b->inst[I.partner].state == LBM_BATCH_UNSTABLE) {
        I.state = LBM_BATCH_DROPPED;  // the partner failed at the last check
        b->tables_valid = false;
      }
      any |= (I.state == LBM_BATCH_ACTIVE);
    }
    if (any && done >= max_steps)
      for (auto& I : b->inst)
        if (I.state == LBM_BATCH_ACTIVE) I.state = LBM_BATCH_MAXSTEPS;
  }
  if (steps_run) *steps_run = done;
  return st;
}

lbm_status lbm_batch_set_limit(lbm_batch* b, int32_t i, int64_t max_steps) {
  if (!b || i < 0 || i >= b->n || max_steps < 0) return LBM_ERR_INVALID_ARG;
  BatchInst& I = b->inst[i];
  I.limit = max_steps;
  if (I.state == LBM_BATCH_ACTIVE && I.steps >= max_steps) {
    I.state = LBM_BATCH_MAXSTEPS;
    b->tables_valid = false;
  } else if (I.state == LBM_BATCH_MAXSTEPS && I.steps < max_steps) {
    // resume from the current state; the next check measures du against
    // velocities stored by this one, so it only stores them again
    I.state = LBM_BATCH_ACTIVE;
    I.checks = 0;
    I.stall = 0;
    I.best_du = INFINITY;
    b->tables_valid = false;
  }
  return LBM_OK;
}

lbm_status lbm_batch_set_partner(lbm_batch* b, int32_t i, int32_t j) {
  if (!b || i < 0 || i >= b->n || j < 0 || j >= b->n || i == j) return LBM_ERR_INVALID_ARG;
  BatchInst& I = b->inst[i];
  BatchInst& J = b->inst[j];
  if ((I.partner >= 0 && I.partner != j) || (J.partner >= 0 && J.partner != i))
    return LBM_ERR_INVALID_ARG;
  I.partner = j;
  J.partner = i;
  return LBM_OK;
}

lbm_status lbm_batch_state(lbm_batch* b, int32_t* state, int64_t* steps, double* du,
                           uint32_t* flags) {
  if (!b) return LBM_ERR_INVALID_ARG;
  for (int i = 0; i < b->n; ++i) {
    const BatchInst& I = b->inst[i];
    if (state) state[i] = I.state;
    if (steps) steps[i] = I.steps;
    if (du) du[i] = I.du;
    if (flags) flags[i] = I.flags;
  }
  return LBM_OK;
}

lbm_status lbm_batch_observe(lbm_batch* b, int32_t i, int32_t cx, int32_t cy, lbm_obs* out,
                             double* d_rho, double* d_ux, double* d_uy) {
  if (!b || i < 0 || i >= b->n || !out) return LBM_ERR_INVALID_ARG;
  lbm_ctx* c = b->inst[i].ctx;
  // a retired instance stopped at its own parity; active ones share b->parity
  return observe_impl(c, cx, cy, out, d_rho, d_ux, d_uy);
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_ERR_INVALID_ARG;
  drop_graph(b);
  for (auto& I : b->inst) delete I.ctx;
  (void)hipEventDestroy(b->ev0);
  (void)hipEventDestroy(b->ev1);
  hipStreamDestroy(b->cap_stream);
  delete b;
  return LBM_OK;
}

lbm_status lbm_batch_stats(const lbm_batch* b, int64_t* node_updates, double* gpu_ms,
                           int64_t* chunks) {
  if (!b) return LBM_ERR_INVALID_ARG;
  if (node_updates) *node_updates = b->node_updates;
  if (gpu_ms) *gpu_ms = b->gpu_ms;
  if (chunks) *chunks = b->chunks;
  return LBM_OK;
}

lbm_status lbm_batch_launch_info(const lbm_batch* b, int32_t i, lbm_launch* out) {
  if (!b || i < 0 || i >= b->n || !out) return LBM_ERR_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  const lbm_ctx* c = b->inst[i].ctx;
  const int two = batch_two(c);
  // a two-step free-energy group runs each 256-column tile as two strips
  const int strip = two && c->p.model == LBM_MODEL_FE ? 128 : c->lc.bx;
  out->steps_per_launch = two ? 2 : 1;
  out->strip = strip;
  out->threads = two ? strip + 64 : strip;
  out->segment = c->lc.ly;
  out->workgroups = (c->p.nx + strip - 1) / strip * c->nseg;
  return LBM_OK;
}

}  // extern "C"
