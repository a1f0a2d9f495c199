/* Drives the FP64 oracle (oracle/lbm_oracle.c, included as one translation
 * unit) through every option of its step on small lattices, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: periodic P and FE
 * (both EOS), Zou-He walls with normal and tangential forces, the
 * collision drive, A != 0 and free-energy gravity.  Exits 0 when every run
 * stays finite. */
#include "../oracle/lbm_oracle.c"

#include <stdio.h>

static int run(orc_params p, int steps) {
  const size_t N = (size_t)p.nx * p.ny;
  double *rho0 = (double *)malloc(N * sizeof(double));
  double *f = (double *)malloc(9 * N * sizeof(double));
  double *rho = (double *)malloc(N * sizeof(double));
  double *ux = (double *)malloc(N * sizeof(double));
  double *uy = (double *)malloc(N * sizeof(double));
  const double rm = p.eos == ORC_EOS_VDW ? 3.5 : 0.1;  /* near the critical density */
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x)
      rho0[(size_t)y * p.nx + x] = rm * (1.0 + 0.02 * sin(0.7 * x) * cos(0.9 * y));
  orc_init(&p, rho0, NULL, NULL, f);
  uint32_t fl = orc_step(&p, f, steps);
  fl |= orc_fields(&p, f, rho, ux, uy);
  int bad = 0;
  for (size_t n = 0; n < N; ++n) bad |= !(rho[n] == rho[n]);
  free(rho0); free(f); free(rho); free(ux); free(uy);
  return bad || (fl & 1u);
}

int main(void) {
  orc_params base;
  memset(&base, 0, sizeof(base));
  base.nx = 23; base.ny = 17;
  base.a = 0.25; base.b = 4.0; base.R = 1.0; base.T = 0.02;  /* C-S: Tr about 0.85 */
  for (int i = 0; i < 9; ++i) base.tau[i] = 1.0;
  int fails = 0;
  for (int model = 0; model < 2; ++model)
    for (int eos = 0; eos < 2; ++eos) {
      orc_params p = base;
      p.model = model; p.eos = eos;
      if (eos == ORC_EOS_VDW) { p.a = 9.0 / 49.0; p.b = 2.0 / 21.0; p.T = 0.95 * 4.0 / 7.0; }
      p.sigma_li = 0.1; p.kappa_p = 0.8; p.kappa_li = 0.2;
      p.kappa = eos == ORC_EOS_VDW ? 0.02 : 0.5;  /* kappa rho_l well below 1/3 */
      p.tau[1] = 0.8; p.tau[4] = p.tau[6] = 1.0 / 1.99;
      fails += run(p, 20);
      orc_params w = p;  /* walls with forces */
      w.walls = 1; w.fx = 1e-6; w.fy = -1e-6;
      fails += run(w, 20);
      orc_params d = p;  /* collision drive */
      d.ax = 1e-6; d.x_split = 11; d.rho_ave = eos == ORC_EOS_VDW ? 3.5 : 0.1;
      fails += run(d, 20);
      if (model == ORC_MODEL_FE) {
        orc_params a = p;
        a.A = 0.1;
        fails += run(a, 20);
        orc_params g = p;  /* gravity between walls */
        g.walls = 1; g.g = 1e-6; g.rho0_g = eos == ORC_EOS_VDW ? 3.5 : 0.1; g.y_g = 8.0;
        fails += run(g, 20);
      }
    }
  printf("%d\n", fails);
  return fails != 0;
}
