/*
 * lbm_oracle.c -- plain FP64 CPU oracle of one D2Q9 multiphase lattice
 * Boltzmann time step, for the two models compared in Czelusniak et al.,
 * "Fundamental comparison between the pseudopotential and the free energy
 * lattice Boltzmann methods" (arXiv 2403.11167):
 *
 *   model 0  modified pseudopotential (MP-LBM): Shan-Chen force (Eq. 10)
 *            with the Yuan-Schaefer potential (Eq. 11), Li's consistency
 *            forcing scaled by kappa^P (Eq. 32), source term (Eq. 13) with
 *            the width-controlling Q tensor (Eq. 30-31);
 *   model 1  improved well-balanced free energy (IWB-FE-LBM): equilibrium
 *            (Eq. 20) and forcing (Eq. 21), chemical potential
 *            mu = mu_b - kappa lap(rho) (Sec. 2.2) and the 9-point stencils
 *            of Eq. 24; A (R9) and gravity (R10) are optional.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the GPU path can be
 * checked against something slow and obviously correct.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never links or calls it.  It shares no code, header,
 * table or constant with the GPU path.
 *
 * Style rules followed on purpose:
 *   - FP64 everywhere, compiled with -ffp-contract=off (no fused multiply-add);
 *   - equilibria and the free-energy forcing are built in velocity space,
 *     then mapped to moments with explicit 9x9 products by M (Eq. 48);
 *     post-collision populations come back through M^-1 (Eq. 49), applied
 *     as its integer multiple 36 M^-1 followed by a division by 36;
 *   - every node's quantities are computed from full-field arrays in separate
 *     sweeps (density, then potential / chemical potential, then the
 *     per-node collision), so that a reader can follow the paper by eye.
 *
 * Readings of the paper adopted here (where it is ambiguous or garbled):
 *   R1  C_2 = (G/2)(1 - kappa^P)  (Eq. 31b printed without G; App. C Eq. 41b
 *       and App. E Eq. 76 both require the factor G).
 *   R2  The gradient stencil of Eq. 24 carries the weights w_i (stated in the
 *       sentence after Eq. 24, and needed for App. D Eq. 59-60).
 *   R3  |F_int|^2 / psi^2 is evaluated as G^2 |S|^2 with S the neighbour sum
 *       of Eq. 10, which is the same number and is finite where psi = 0.
 *   R4  psi^2 < 0 (an equation of state above rho c_s^2) is clamped to zero
 *       and reported through a sticky flag.
 *   R5  Within a step, forces use the density of the populations at the start
 *       of the step; all densities are formed before any collision.
 *   R6  The forcing term of Eq. 32 uses the total force F = F_int + F_b,
 *       with F_b a constant body force (zero in all standard workloads);
 *       the consistency term uses F_int only.  For the free-energy model the
 *       total force is -rho grad(mu) + F_b.
 *   R7  Walls (Sec. 5.3, optional): no-slip walls of Zou and He on the rows
 *       y = 0 and y = ny - 1, which are fluid nodes whose velocity is held at
 *       zero; x stays periodic.  The paper does not say how the stencils see
 *       past a wall: values on the rows beyond it mirror the rows inside
 *       (rho, psi, mu at y = -k equal those at y = k), so the density has no
 *       normal gradient at the wall and the normal interaction force there
 *       vanishes.
 *   R8  The droplet-collision drive (Sec. 5.4, optional): an x force
 *       a(x) |rho - rho_ave| with a(x) = +ax for x <= x_split and -ax beyond,
 *       added to the body force; rho_ave, the mean density, is a constant
 *       because the scheme conserves mass (Eq. 7a).  It joins F_b of R6.
 *   R9  Free energy with A != 0 (Eq. 20, optional): S_ab = d_a u_b +
 *       d_b u_a with the gradient stencil of Eq. 24 applied to the velocity
 *       field of the same time step (Eq. 6b at every node first); past a
 *       wall the velocity is reflected with its sign flipped, so it vanishes
 *       on the wall row as the closure imposes.  The initial equilibrium
 *       takes S from the initial velocity the same way (zero for a fluid at
 *       rest).
 *   R10 Free energy with gravity (Sec. 2.2, optional, walls only): p_g =
 *       rho_0 g (y - y_g) enters the equilibrium of Eq. 20 at every node
 *       (y the node's row, y_g the row where p_g = 0), the buoyancy force
 *       F_g = -(rho - rho_0) g in y joins the total force F, and d_y p_g =
 *       rho_0 g enters Eq. 21.  With g > 0 gravity pulls toward -y: the
 *       momentum gains -d_y p_g + F_g = -rho g.  p_g is not periodic, hence
 *       walls.  On a wall row the normal force is f_y + F_g (R7), which
 *       depends on the wall density; the closure then fixes that density
 *       through a linear equation, solved in closed form.  The initial
 *       equilibrium carries p_g too.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>

/* Lattices below this many nodes run each sweep on one thread: starting the
 * threads costs more than the sweep (a 100 x 1 planar lattice ran ten times
 * slower on 8 threads).  Results do not depend on it. */
#define ORC_PAR_MIN 16384
#endif

#define ORC_MODEL_P 0
#define ORC_MODEL_FE 1
#define ORC_EOS_VDW 0
#define ORC_EOS_CS 1

#define ORC_FLAG_NONFINITE 1u
#define ORC_FLAG_PSI_CLAMP 2u
#define ORC_FLAG_EOS_DOMAIN 4u

typedef struct {
  int32_t nx, ny;
  int32_t model; /* ORC_MODEL_P or ORC_MODEL_FE */
  int32_t eos;   /* ORC_EOS_VDW or ORC_EOS_CS */
  double a, b, R, T;
  double tau[9]; /* one relaxation time per moment row (Eq. 3) */
  double sigma_li, kappa_li, kappa_p; /* pseudopotential only */
  double kappa;                       /* free energy only */
  double fx, fy;                      /* constant body force */
  int32_t walls; /* 0: periodic in y; 1: Zou-He walls on y = 0, ny-1 (R7) */
  int32_t x_split;      /* drive (R8): +ax for x <= x_split, -ax beyond */
  double ax, rho_ave;   /* drive (R8); ax = 0: off */
  double A;             /* free energy: viscosity-tuning A of Eq. 20 (R9) */
  double g, rho0_g, y_g; /* free energy: gravity (R10); g = 0: off */
} orc_params;

/* ---- lattice (Eq. 2 and the weights stated under Eq. 4) ------------------ */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* The same weights times 36 (16, 4, 1): the equilibria and the forcing
 * multiply by these integers and divide by 36 at the end, so that the
 * weights sum to one exactly and f^eq carries exactly the mass rho (a
 * rounded 1/9 would bias every step's density, against Eq. 7a / 22a). */
static const double WGT36[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
static const double CS2 = 1.0 / 3.0; /* c_s^2 for c = 1 */
static const double G = -1.0;        /* interaction sign chosen after Eq. 11 */

/* Shan-Chen weights omega(|c|^2) of Eq. 10: 1/3 for |c|^2 = 1, 1/12 for 2. */
static double omega_sc(int i) {
  int c2 = CX[i] * CX[i] + CY[i] * CY[i];
  if (c2 == 1) return 1.0 / 3.0;
  if (c2 == 2) return 1.0 / 12.0;
  return 0.0;
}

/* ---- moment matrices: M of Eq. 48 and M^-1 as printed in Eq. 49 ---------- */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},          {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},      {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},       {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},       {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

static const double MINV[9][9] = {
    {1. / 9, -1. / 9, 1. / 9, 0, 0, 0, 0, 0, 0},
    {1. / 9, -1. / 36, -1. / 18, 1. / 6, -1. / 6, 0, 0, 1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, 0, 0, 1. / 6, -1. / 6, -1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, -1. / 6, 1. / 6, 0, 0, 1. / 4, 0},
    {1. / 9, -1. / 36, -1. / 18, 0, 0, -1. / 6, 1. / 6, -1. / 4, 0},
    {1. / 9, 1. / 18, 1. / 36, 1. / 6, 1. / 12, 1. / 6, 1. / 12, 0, 1. / 4},
    {1. / 9, 1. / 18, 1. / 36, -1. / 6, -1. / 12, 1. / 6, 1. / 12, 0, -1. / 4},
    {1. / 9, 1. / 18, 1. / 36, -1. / 6, -1. / 12, -1. / 6, -1. / 12, 0, 1. / 4},
    {1. / 9, 1. / 18, 1. / 36, 1. / 6, 1. / 12, -1. / 6, -1. / 12, 0, -1. / 4}};

/* Eq. 49 times 36: the same rational matrix with integer entries.  The
 * collision applies it and divides by 36, so that no entry is a rounded
 * fraction (a rounded 1/9 would make sum_i f*_i = 9 fl(1/9) rho*, a
 * systematic loss of mass every step, against the exact conservation of
 * Eq. 7a / 22a). */
static const double MINV36[9][9] = {
    {4, -4, 4, 0, 0, 0, 0, 0, 0},       {4, -1, -2, 6, -6, 0, 0, 9, 0},
    {4, -1, -2, 0, 0, 6, -6, -9, 0},    {4, -1, -2, -6, 6, 0, 0, 9, 0},
    {4, -1, -2, 0, 0, -6, 6, -9, 0},    {4, 2, 1, 6, 3, 6, 3, 0, 9},
    {4, 2, 1, -6, -3, 6, 3, 0, -9},     {4, 2, 1, -6, -3, -6, -3, 0, 9},
    {4, 2, 1, 6, 3, -6, -3, 0, -9}};

static void mat_vec(const double A[9][9], const double *v, double *out) {
  for (int r = 0; r < 9; ++r) {
    double s = 0.0;
    for (int c = 0; c < 9; ++c) s += A[r][c] * v[c];
    out[r] = s;
  }
}

/* ---- equations of state -------------------------------------------------- */
/* Carnahan-Starling, Eq. 28; van der Waals p = rho R T/(1 - b rho) - a rho^2. */
static double eos_pressure(const orc_params *p, double rho) {
  if (p->eos == ORC_EOS_CS) {
    double e = p->b * rho / 4.0;
    double num = 1.0 + e + e * e - e * e * e;
    double den = (1.0 - e) * (1.0 - e) * (1.0 - e);
    return rho * p->R * p->T * num / den - p->a * rho * rho;
  }
  return rho * p->R * p->T / (1.0 - p->b * rho) - p->a * rho * rho;
}

/* Bulk chemical potential.  Carnahan-Starling: Eq. 29.  Van der Waals: the
 * antiderivative of (1/rho) dp/drho (the relation -rho d(mu_b) = -dp of
 * Sec. 2.2), RT ln(rho/(1-b rho)) + RT b rho/(1-b rho) - 2 a rho.          */
static double eos_mu_b(const orc_params *p, double rho) {
  double RT = p->R * p->T;
  if (p->eos == ORC_EOS_CS) {
    double e = p->b * rho / 4.0;
    return RT * (3.0 - e) / ((1.0 - e) * (1.0 - e) * (1.0 - e)) +
           RT * log(rho) + RT - 2.0 * p->a * rho;
  }
  return RT * log(rho / (1.0 - p->b * rho)) +
         RT * p->b * rho / (1.0 - p->b * rho) - 2.0 * p->a * rho;
}

static int eos_domain_ok(const orc_params *p, double rho) {
  double lim = (p->eos == ORC_EOS_CS) ? p->b * rho / 4.0 : p->b * rho;
  if (!(lim < 1.0)) return 0;
  if (p->model == ORC_MODEL_FE && !(rho > 0.0)) return 0;
  return 1;
}

/* Yuan-Schaefer potential, Eq. 11 with G = -1 and c = dt = 1:
 * psi = sqrt(2 (p_EOS - rho c_s^2) / G).  Negative argument -> clamp (R4). */
static double psi_of_rho(const orc_params *p, double rho, unsigned *flags) {
  double arg = 2.0 * (eos_pressure(p, rho) - rho * CS2) / G;
  if (arg < 0.0) {
    *flags |= ORC_FLAG_PSI_CLAMP;
    arg = 0.0;
  }
  return sqrt(arg);
}

/* ---- equilibria in velocity space ---------------------------------------- */
/* Eq. 4 (pseudopotential). */
static void feq_standard(double rho, double ux, double uy, double *feq) {
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    double uu = ux * ux + uy * uy;
    double quad = (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2);
    feq[i] = WGT36[i] * rho * (1.0 + cu / CS2 + quad) / 36.0;
  }
}

/* Eq. 20 (free energy); c_s^4 in the i != 0 term as printed in Eq. 20.
 * pg is p_g at the node, A the viscosity-tuning parameter and du[] the
 * velocity gradient (d_x u_x, d_y u_x, d_x u_y, d_y u_y), giving
 * S_ab = d_a u_b + d_b u_a (NULL: zero). */
static void feq_well_balanced(double rho, double ux, double uy, double pg,
                              double A, const double *du, double *feq) {
  double uu = ux * ux + uy * uy;
  double Sxx = 0.0, Syy = 0.0, Sxy = 0.0;
  if (du) {
    Sxx = 2.0 * du[0];
    Syy = 2.0 * du[3];
    Sxy = du[1] + du[2];
  }
  double divu = 0.5 * (Sxx + Syy);
  feq[0] = rho - (36.0 - WGT36[0]) * pg / CS2 / 36.0 -
           WGT36[0] * rho * uu / (2.0 * CS2) / 36.0 - WGT36[0] * rho * A * divu / 36.0;
  for (int i = 1; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    /* (c_a c_b - c_s^2 delta_ab)(u_a u_b + c_s^2 A S_ab) */
    double cSc = CX[i] * CX[i] * Sxx + 2.0 * CX[i] * CY[i] * Sxy + CY[i] * CY[i] * Syy;
    double tensor = (cu * cu - CS2 * uu) + CS2 * A * (cSc - CS2 * (Sxx + Syy));
    double quad = tensor / (2.0 * CS2 * CS2);
    feq[i] = WGT36[i] * (pg / CS2 + rho * (cu / CS2 + quad)) / 36.0;
  }
}

/* Eq. 21 with d = 2: velocity-space forcing of the free-energy model, with
 * gx, gy the stencil gradient of rho and dpgy = d_y p_g. */
static void forcing_well_balanced(double ux, double uy, double Fx, double Fy,
                                  double gx, double gy, double dpgy, double *Fi) {
  double Bx = Fx + CS2 * gx, By = Fy - dpgy + CS2 * gy;
  double ug = ux * gx + uy * gy;
  for (int i = 0; i < 9; ++i) {
    double cF = CX[i] * Fx + CY[i] * Fy;
    /* (c_a c_b - c_s^2 delta_ab) u_a B_b */
    double cu = CX[i] * ux + CY[i] * uy;
    double cB = CX[i] * Bx + CY[i] * By;
    double second = cu * cB - CS2 * (ux * Bx + uy * By);
    double c2 = (double)(CX[i] * CX[i] + CY[i] * CY[i]);
    Fi[i] = WGT36[i] * (cF / CS2 + second / (CS2 * CS2) +
                        0.5 * (c2 / CS2 - 2.0) * ug) / 36.0;
  }
}

static int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

/* Row whose values a stencil sees at row y: periodic, or with walls (R7)
 * the mirror image of the rows inside. */
static int row_seen(int y, int ny, int walls) {
  if (!walls) return wrap(y, ny);
  if (y < 0) return -y;
  if (y > ny - 1) return 2 * (ny - 1) - y;
  return y;
}

/* ---- stencils on a periodic field (exposed for unit tests) --------------- */

/* Shan-Chen neighbour sum S_a = sum_{i=1..8} omega_i phi(x+c_i) c_ia, so that
 * Eq. 10 reads F_a = -G psi(x) S_a. */
static void sc_sum(int nx, int ny, int walls, const double *phi, double *Sx,
                   double *Sy) {
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int i = 1; i < 9; ++i) {
        double v = phi[row_seen(y + CY[i], ny, walls) * nx + wrap(x + CX[i], nx)];
        sx += omega_sc(i) * v * CX[i];
        sy += omega_sc(i) * v * CY[i];
      }
      Sx[y * nx + x] = sx;
      Sy[y * nx + x] = sy;
    }
}

void orc_sc_sum(int nx, int ny, const double *phi, double *Sx, double *Sy) {
  sc_sum(nx, ny, 0, phi, Sx, Sy);
}

/* Eq. 30a-b with C_1 of Eq. 31a and C_2 read as (G/2)(1 - kappa^P) (R1). */
static void q_tensor(int nx, int ny, int walls, const double *psi,
                     double kappa_p, double kappa_li, double *Qxx, double *Qyy,
                     double *Qxy) {
  double C1 = 5.0 / 6.0 * (kappa_p - 1.0);
  double C2 = 0.5 * G * (1.0 - kappa_p);
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double p0 = psi[y * nx + x];
      double q[2][2] = {{0, 0}, {0, 0}};
      for (int i = 1; i < 9; ++i) {
        double d = psi[row_seen(y + CY[i], ny, walls) * nx + wrap(x + CX[i], nx)] - p0;
        int c[2] = {CX[i], CY[i]};
        for (int al = 0; al < 2; ++al)
          for (int be = 0; be < 2; ++be) {
            double delta = (al == be) ? 1.0 : 0.0;
            double C = C1 * G * delta + C2 * (c[al] * c[be] - CS2 * delta) +
                       kappa_li * 0.5 * G * c[al] * c[be];
            q[al][be] += omega_sc(i) * C * d;
          }
      }
      Qxx[y * nx + x] = p0 * q[0][0];
      Qyy[y * nx + x] = p0 * q[1][1];
      Qxy[y * nx + x] = p0 * q[0][1];
    }
}

void orc_q_tensor(int nx, int ny, const double *psi, double kappa_p,
                  double kappa_li, double *Qxx, double *Qyy, double *Qxy) {
  q_tensor(nx, ny, 0, psi, kappa_p, kappa_li, Qxx, Qyy, Qxy);
}

/* Eq. 24, first line, with the weights w_i (R2). */
static void gradient(int nx, int ny, int walls, const double *phi, double *gx,
                     double *gy) {
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int i = 0; i < 9; ++i) {
        double v = phi[row_seen(y + CY[i], ny, walls) * nx + wrap(x + CX[i], nx)];
        sx += WGT[i] * v * CX[i];
        sy += WGT[i] * v * CY[i];
      }
      gx[y * nx + x] = sx / CS2;
      gy[y * nx + x] = sy / CS2;
    }
}

void orc_gradient(int nx, int ny, const double *phi, double *gx, double *gy) {
  gradient(nx, ny, 0, phi, gx, gy);
}

/* Eq. 24, second line. */
static void laplacian(int nx, int ny, int walls, const double *phi, double *lap) {
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double c = phi[y * nx + x], s = 0.0;
      for (int i = 0; i < 9; ++i)
        s += WGT[i] * (phi[row_seen(y + CY[i], ny, walls) * nx + wrap(x + CX[i], nx)] - c);
      lap[y * nx + x] = 2.0 * s / CS2;
    }
}

void orc_laplacian(int nx, int ny, const double *phi, double *lap) {
  laplacian(nx, ny, 0, phi, lap);
}

/* Eq. 24 gradient of a velocity component (R9): past a wall the value of
 * the mirrored row enters with its sign flipped. */
static void gradient_u(int nx, int ny, int walls, const double *u, double *gx,
                       double *gy) {
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int i = 0; i < 9; ++i) {
        int yy = y + CY[i];
        double sgn = (walls && (yy < 0 || yy > ny - 1)) ? -1.0 : 1.0;
        double v = sgn * u[row_seen(yy, ny, walls) * nx + wrap(x + CX[i], nx)];
        sx += WGT[i] * v * CX[i];
        sy += WGT[i] * v * CY[i];
      }
      gx[y * nx + x] = sx / CS2;
      gy[y * nx + x] = sy / CS2;
    }
}

/* ---- exported small helpers ---------------------------------------------- */
double orc_pressure(const orc_params *p, double rho) { return eos_pressure(p, rho); }
double orc_mu_b(const orc_params *p, double rho) { return eos_mu_b(p, rho); }
double orc_psi(const orc_params *p, double rho) {
  unsigned fl = 0;
  return psi_of_rho(p, rho, &fl);
}
void orc_matrices(double *m, double *minv, double *minv36) {
  memcpy(m, MM, sizeof(MM));
  memcpy(minv, MINV, sizeof(MINV));
  memcpy(minv36, MINV36, sizeof(MINV36));
}
void orc_feq(int32_t model, double rho, double ux, double uy, double *feq) {
  if (model == ORC_MODEL_FE)
    feq_well_balanced(rho, ux, uy, 0.0, 0.0, NULL, feq);
  else
    feq_standard(rho, ux, uy, feq);
}
/* Eq. 20 in full: p_g, A and du = (d_x u_x, d_y u_x, d_x u_y, d_y u_y). */
void orc_feq_fe_full(double rho, double ux, double uy, double pg, double A,
                     const double *du, double *feq) {
  feq_well_balanced(rho, ux, uy, pg, A, du, feq);
}
void orc_forcing_fe(double ux, double uy, double Fx, double Fy, double gx,
                    double gy, double *Fi) {
  forcing_well_balanced(ux, uy, Fx, Fy, gx, gy, 0.0, Fi);
}
void orc_forcing_fe_full(double ux, double uy, double Fx, double Fy, double gx,
                         double gy, double dpgy, double *Fi) {
  forcing_well_balanced(ux, uy, Fx, Fy, gx, gy, dpgy, Fi);
}

/* p_g of Eq. 20 on row y (R10); 0 without gravity. */
static double pg_row(const orc_params *p, int y) {
  return p->rho0_g * p->g * ((double)y - p->y_g);
}

/* Population layout: f[i * N + y * nx + x], N = nx * ny, holding f_i(x, t)
 * after streaming (the left-hand side of Eq. 1 at the previous step). */

/* Initial state: f = f^eq(rho0, u0) (Sec. 5.3 and 5.4 initialise with the
 * equilibrium; u0 may be NULL for a fluid at rest). */
void orc_init(const orc_params *p, const double *rho0, const double *ux0,
              const double *uy0, double *f) {
  int nx = p->nx, ny = p->ny;
  size_t N = (size_t)nx * ny;
  double *du[4] = {NULL, NULL, NULL, NULL};
  int with_a = p->model == ORC_MODEL_FE && p->A != 0.0 && ux0 && uy0;
  if (with_a) {
    for (int k = 0; k < 4; ++k) du[k] = (double *)calloc(N, sizeof(double));
    gradient_u(nx, ny, p->walls, ux0, du[0], du[1]);
    gradient_u(nx, ny, p->walls, uy0, du[2], du[3]);
  }
  for (size_t n = 0; n < N; ++n) {
    double feq[9];
    double ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
    if (p->model == ORC_MODEL_FE) {
      double dn[4] = {0.0, 0.0, 0.0, 0.0};
      if (with_a)
        for (int k = 0; k < 4; ++k) dn[k] = du[k][n];
      feq_well_balanced(rho0[n], ux, uy, pg_row(p, (int)(n / (size_t)nx)), p->A, dn, feq);
    } else {
      feq_standard(rho0[n], ux, uy, feq);
    }
    for (int i = 0; i < 9; ++i) f[i * N + n] = feq[i];
  }
  for (int k = 0; k < 4; ++k) free(du[k]);
}

/* ---- Zou-He no-slip walls (R7) --------------------------------------------
 * Row y is a wall row if walls are on and y is 0 or ny - 1; side +1 is the
 * bottom wall (the populations with c_y = +1 are unknown after streaming,
 * they would come from below it), side -1 the top wall. */
static int wall_side(const orc_params *p, int y) {
  if (!p->walls) return 0;
  if (y == 0) return 1;
  if (y == p->ny - 1) return -1;
  return 0;
}

/* Replace the unknown populations fn[i] (c_y = side) of a wall node so that
 * the node carries the momentum sum_i f_i c_i = (jx, jy).  Zou and He's
 * closure: the normal unknown takes the value of its opposite (the
 * non-equilibrium parts bounce back; at the wall velocity u_w = 0 the two
 * equilibria are equal), then the two diagonal unknowns solve the x and y
 * momentum balances.  For u = u_w = 0 under Eq. 6b, (jx, jy) = -F/2. */
static void wall_close(double *fn, int side, double jx, double jy) {
  int nrm = -1, opp = -1, d[2], nd = 0;
  for (int i = 1; i < 9; ++i) {
    if (CY[i] == side && CX[i] == 0) nrm = i;
    if (CY[i] == -side && CX[i] == 0) opp = i;
    if (CY[i] == side && CX[i] != 0) d[nd++] = i;
  }
  fn[nrm] = fn[opp];
  double bx = jx, by = jy;
  for (int i = 0; i < 9; ++i)
    if (i != d[0] && i != d[1]) {
      bx -= fn[i] * CX[i];
      by -= fn[i] * CY[i];
    }
  /* [CX[d0] CX[d1]; CY[d0] CY[d1]] (f_d0, f_d1) = (bx, by), Cramer's rule */
  double det = (double)(CX[d[0]] * CY[d[1]] - CX[d[1]] * CY[d[0]]);
  fn[d[0]] = (bx * CY[d[1]] - CX[d[1]] * by) / det;
  fn[d[1]] = (CX[d[0]] * by - CY[d[0]] * bx) / det;
}

/* Normal force of a wall node of density rho: the body force fy plus the
 * buoyancy of R10; the interaction force vanishes there (R7).  The node
 * carries sum f c_y = -F_y/2. */
static double wall_fy(const orc_params *p, double rho) {
  return p->fy - (rho - p->rho0_g) * p->g;
}

/* Density of a wall node on `side` whose populations closed with zero
 * normal momentum sum to s: closing with j_y = -F_y/2 moves the two
 * diagonal unknowns, whose c_y is `side`, by j_y in sum f c_y, so the
 * density is rho = s + side j_y(rho), linear in rho with F_y of wall_fy. */
static double wall_rho(const orc_params *p, int side, double s) {
  return (s - side * 0.5 * (p->fy + p->g * p->rho0_g)) / (1.0 - side * 0.5 * p->g);
}

/* Per-step field work shared by the step and by the field export: density,
 * and the model's force ingredients.  Arrays are length N. */
typedef struct {
  double *rho, *psi, *Sx, *Sy, *Qxx, *Qyy, *Qxy; /* pseudopotential */
  double *lap, *mu, *gmx, *gmy, *grx, *gry;       /* free energy */
  double *ux, *uy, *du[4];                        /* velocity, its gradient (R9) */
} orc_work;

static void work_alloc(orc_work *w, size_t N) {
  double **ptrs[] = {&w->rho, &w->psi, &w->Sx,  &w->Sy,  &w->Qxx, &w->Qyy,
                     &w->Qxy, &w->lap, &w->mu,  &w->gmx, &w->gmy, &w->grx,
                     &w->gry, &w->ux,  &w->uy,  &w->du[0], &w->du[1],
                     &w->du[2], &w->du[3]};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k)
    *ptrs[k] = (double *)calloc(N, sizeof(double));
}

static void work_free(orc_work *w) {
  free(w->rho); free(w->psi); free(w->Sx); free(w->Sy); free(w->Qxx);
  free(w->Qyy); free(w->Qxy); free(w->lap); free(w->mu); free(w->gmx);
  free(w->gmy); free(w->grx); free(w->gry); free(w->ux); free(w->uy);
  for (int k = 0; k < 4; ++k) free(w->du[k]);
}

/* Eq. 6a, then the model's field quantities (Sec. 2.1 / Sec. 2.2). */
static unsigned fields_and_forces(const orc_params *p, const double *f,
                                  orc_work *w) {
  int nx = p->nx, ny = p->ny;
  size_t N = (size_t)nx * ny;
  unsigned flags = 0;
#pragma omp parallel for schedule(static) reduction(| : flags) if(N >= ORC_PAR_MIN)
  for (size_t n = 0; n < N; ++n) {
    double fn[9], s = 0.0;
    for (int i = 0; i < 9; ++i) fn[i] = f[i * N + n];
    int side = wall_side(p, (int)(n / (size_t)nx));
    if (side) wall_close(fn, side, 0.0, 0.0);
    for (int i = 0; i < 9; ++i) s += fn[i];
    /* a wall node also carries sum f c_y = j_y, which moves its density by
     * side * j_y (+j_y on the bottom wall, -j_y on the top one); jx does not
     * change it */
    if (side) s = wall_rho(p, side, s);
    w->rho[n] = s;
    if (!isfinite(s)) flags |= ORC_FLAG_NONFINITE;
    if (!eos_domain_ok(p, s)) flags |= ORC_FLAG_EOS_DOMAIN;
  }
  if (p->model == ORC_MODEL_P) {
#pragma omp parallel for schedule(static) reduction(| : flags) if(N >= ORC_PAR_MIN)
    for (size_t n = 0; n < N; ++n) w->psi[n] = psi_of_rho(p, w->rho[n], &flags);
    sc_sum(nx, ny, p->walls, w->psi, w->Sx, w->Sy);
    q_tensor(nx, ny, p->walls, w->psi, p->kappa_p, p->kappa_li, w->Qxx, w->Qyy, w->Qxy);
  } else {
    /* mu = mu_b(rho) - kappa lap(rho) (Sec. 2.2), then grad(mu), grad(rho). */
    laplacian(nx, ny, p->walls, w->rho, w->lap);
#pragma omp parallel for schedule(static) if(N >= ORC_PAR_MIN)
    for (size_t n = 0; n < N; ++n)
      w->mu[n] = eos_mu_b(p, w->rho[n]) - p->kappa * w->lap[n];
    gradient(nx, ny, p->walls, w->mu, w->gmx, w->gmy);
    gradient(nx, ny, p->walls, w->rho, w->grx, w->gry);
  }
  return flags;
}

/* Total force at node n (R6) and, for the pseudopotential, K = |F_int|^2/psi^2
 * evaluated as G^2 |S|^2 (R3). */
/* x component of the body force at node n: the constant fx plus the drive
 * of R8. */
static double body_fx(const orc_params *p, const orc_work *w, size_t n) {
  if (p->ax == 0.0) return p->fx;
  int x = (int)(n % (size_t)p->nx);
  double a = (x <= p->x_split) ? p->ax : -p->ax;
  return p->fx + a * fabs(w->rho[n] - p->rho_ave);
}

static void node_force(const orc_params *p, const orc_work *w, size_t n,
                       double *Fx, double *Fy, double *K) {
  if (p->model == ORC_MODEL_P) {
    double fxi = -G * w->psi[n] * w->Sx[n]; /* Eq. 10 */
    double fyi = -G * w->psi[n] * w->Sy[n];
    *K = G * G * (w->Sx[n] * w->Sx[n] + w->Sy[n] * w->Sy[n]);
    *Fx = fxi + body_fx(p, w, n);
    *Fy = fyi + p->fy;
  } else {
    *Fx = -w->rho[n] * w->gmx[n] + body_fx(p, w, n); /* F = -rho grad(mu) */
    /* plus the buoyancy F_g = -(rho - rho_0) g (R10) */
    *Fy = -w->rho[n] * w->gmy[n] + p->fy - (w->rho[n] - p->rho0_g) * p->g;
    *K = 0.0;
  }
}

/* Eq. 6b at every node (after fields_and_forces), wall closure included. */
static void velocity_field(const orc_params *p, const double *f, orc_work *w) {
  size_t N = (size_t)p->nx * p->ny;
#pragma omp parallel for schedule(static) if(N >= ORC_PAR_MIN)
  for (size_t n = 0; n < N; ++n) {
    double Fx, Fy, K, jx = 0.0, jy = 0.0, fn[9];
    node_force(p, w, n, &Fx, &Fy, &K);
    for (int i = 0; i < 9; ++i) fn[i] = f[i * N + n];
    int side = wall_side(p, (int)(n / (size_t)p->nx));
    if (side) wall_close(fn, side, -0.5 * Fx, -0.5 * wall_fy(p, w->rho[n]));
    for (int i = 0; i < 9; ++i) {
      jx += fn[i] * CX[i];
      jy += fn[i] * CY[i];
    }
    w->ux[n] = (jx + 0.5 * Fx) / w->rho[n];
    w->uy[n] = (jy + 0.5 * Fy) / w->rho[n];
  }
}

/* Export rho and u (Eq. 6a-b) for the current populations. */
uint32_t orc_fields(const orc_params *p, const double *f, double *rho,
                    double *ux, double *uy) {
  size_t N = (size_t)p->nx * p->ny;
  orc_work w;
  work_alloc(&w, N);
  unsigned flags = fields_and_forces(p, f, &w);
  velocity_field(p, f, &w);
  for (size_t n = 0; n < N; ++n) {
    if (rho) rho[n] = w.rho[n];
    if (ux) ux[n] = w.ux[n];
    if (uy) uy[n] = w.uy[n];
  }
  work_free(&w);
  return flags;
}

/* One collision at node n: Eq. 1 written in moment space,
 *   m* = m - Lambda (m - m^eq) + (I - Lambda/2) mF + mC,   f* = M^-1 m*. */
static void collide_node(const orc_params *p, const double *f, size_t N,
                         const orc_work *w, size_t n, double *fstar) {
  double fn[9], feq[9], m[9], meq[9], mF[9], mC[9], ms[9];
  double Fx, Fy, K;
  double rho = w->rho[n];
  for (int i = 0; i < 9; ++i) fn[i] = f[i * N + n];
  node_force(p, w, n, &Fx, &Fy, &K);
  int side = wall_side(p, (int)(n / (size_t)p->nx));
  if (side) wall_close(fn, side, -0.5 * Fx, -0.5 * wall_fy(p, rho));

  /* Eq. 6b. */
  double jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) {
    jx += fn[i] * CX[i];
    jy += fn[i] * CY[i];
  }
  double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;

  const double *tau = p->tau;
  for (int i = 0; i < 9; ++i) mC[i] = 0.0;

  if (p->model == ORC_MODEL_P) {
    feq_standard(rho, ux, uy, feq); /* Eq. 4 */
    /* Eq. 32 (forcing moments, consistency term scaled by kappa^P). */
    double uF = ux * Fx + uy * Fy;
    double ks = p->kappa_p * p->sigma_li * K;
    mF[0] = 0.0;
    mF[1] = 6.0 * uF + 12.0 * ks / (tau[1] - 0.5);
    mF[2] = -6.0 * uF - 12.0 * ks / (tau[2] - 0.5);
    mF[3] = Fx;
    mF[4] = -Fx;
    mF[5] = Fy;
    mF[6] = -Fy;
    mF[7] = 2.0 * (ux * Fx - uy * Fy);
    mF[8] = ux * Fy + uy * Fx;
    /* Eq. 13 (source moments) with the Q of Eq. 30. */
    double qs = w->Qxx[n] + w->Qyy[n];
    mC[1] = 1.5 * qs / tau[1];
    mC[2] = -1.5 * qs / tau[2];
    mC[7] = -(w->Qxx[n] - w->Qyy[n]) / tau[7];
    mC[8] = -w->Qxy[n] / tau[8];
  } else {
    double Fi[9], dn[4] = {0.0, 0.0, 0.0, 0.0};
    if (p->A != 0.0)
      for (int k = 0; k < 4; ++k) dn[k] = w->du[k][n];
    /* Eq. 20 and Eq. 21, with p_g and d_y p_g of R10 (zero without gravity) */
    double pg = pg_row(p, (int)(n / (size_t)p->nx));
    feq_well_balanced(rho, ux, uy, pg, p->A, dn, feq);
    forcing_well_balanced(ux, uy, Fx, Fy, w->grx[n], w->gry[n], p->rho0_g * p->g, Fi);
    mat_vec(MM, Fi, mF);
  }

  mat_vec(MM, fn, m);
  mat_vec(MM, feq, meq);
  for (int k = 0; k < 9; ++k) {
    double lam = 1.0 / tau[k];
    ms[k] = m[k] - lam * (m[k] - meq[k]) + (1.0 - 0.5 * lam) * mF[k] + mC[k];
  }
  mat_vec(MINV36, ms, fstar);
  for (int i = 0; i < 9; ++i) fstar[i] /= 36.0;
}

/* Advance nsteps time steps in place.  Returns the OR of the sticky flags
 * raised on the way.  Streaming: f_i(x + c_i, t + 1) = f*_i(x, t), periodic.
 * With walls, what streams across a wall lands in the unknown slots of the
 * opposite wall row, which the closure overwrites before any use. */
uint32_t orc_step(const orc_params *p, double *f, int64_t nsteps) {
  int nx = p->nx, ny = p->ny;
  size_t N = (size_t)nx * ny;
  double *fnew = (double *)malloc(9 * N * sizeof(double));
  orc_work w;
  work_alloc(&w, N);
  unsigned flags = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    flags |= fields_and_forces(p, f, &w);
    if (p->model == ORC_MODEL_FE && p->A != 0.0) {
      /* S of Eq. 20 needs the velocity of this step at every node (R9) */
      velocity_field(p, f, &w);
      gradient_u(nx, ny, p->walls, w.ux, w.du[0], w.du[1]);
      gradient_u(nx, ny, p->walls, w.uy, w.du[2], w.du[3]);
    }
#pragma omp parallel for schedule(static) if((size_t)nx * ny >= ORC_PAR_MIN)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t n = (size_t)y * nx + x;
        double fstar[9];
        collide_node(p, f, N, &w, n, fstar);
        for (int i = 0; i < 9; ++i) {
          size_t dst = (size_t)wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx);
          fnew[i * N + dst] = fstar[i];
        }
      }
    memcpy(f, fnew, 9 * N * sizeof(double));
  }
  for (size_t k = 0; k < 9 * N; ++k)
    if (!isfinite(f[k])) {
      flags |= ORC_FLAG_NONFINITE;
      break;
    }
  work_free(&w);
  free(fnew);
  return flags;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
