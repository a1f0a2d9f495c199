/*
 * lbm_cdemo.c -- a plain C client of the C ABI in include/lbm.h (no Python,
 * no torch): allocates device memory with the HIP runtime, sets up a static
 * droplet (Sec. 5.2 geometry) for the chosen model, advances it and prints
 * the observables as one JSON line.
 *
 *   lbm_cdemo MODEL NX NY STEPS     MODEL: 0 pseudopotential, 1 free energy
 *
 * Carnahan-Starling EOS with a = 0.25, b = 4, R = 1 at Tr = 0.8; droplet of
 * radius min(NX, NY)/4 between the Maxwell densities (tanh profile of width
 * 5); free energy: kappa = 0.5, tau_e = 0.75; pseudopotential: the App. B
 * sigma^Li with kappa^P and kappa^Li matched to the free-energy model,
 * tau_q = 1/1.99.  Exit status 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

#define CHECK(call)                                                        \
  do {                                                                     \
    lbm_status st_ = (call);                                               \
    if (st_ != LBM_OK) {                                                   \
      fprintf(stderr, "%s: %s\n", #call, lbm_status_string(st_));          \
      return 1;                                                            \
    }                                                                      \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s MODEL NX NY STEPS\n", argv[0]);
    return 2;
  }
  const int model = atoi(argv[1]), nx = atoi(argv[2]), ny = atoi(argv[3]);
  const long steps = atol(argv[4]);
  const double a = 0.25, b = 4.0, R = 1.0;
  double Tc, rc, pc, rl, rv, p0;
  CHECK(lbm_eos_critical(LBM_EOS_CS, a, b, R, &Tc, &rc, &pc));
  const double T = 0.8 * Tc;
  CHECK(lbm_maxwell(LBM_EOS_CS, a, b, R, T, &rl, &rv, &p0));

  lbm_params p = {0};
  p.nx = nx;
  p.ny = ny;
  p.model = model;
  p.eos = LBM_EOS_CS;
  p.precision = LBM_FP64;
  p.a = a;
  p.b = b;
  p.R = R;
  p.T = T;
  for (int i = 0; i < 9; ++i) p.tau[i] = 1.0;
  if (model == LBM_MODEL_FE) {
    p.tau[1] = 0.75;
    p.kappa = 0.5;
  } else {
    p.tau[4] = p.tau[6] = 1.0 / 1.99;
    CHECK(lbm_match_p_to_fe(LBM_EOS_CS, a, b, R, T, 0.5, 0.0, &p.sigma_li, &p.kappa_p,
                            &p.kappa_li));
  }

  /* initial density on the host, then on the device */
  const size_t N = (size_t)nx * ny;
  double* h_rho = (double*)malloc(N * sizeof(double));
  if (!h_rho) return 1;
  const double r0 = 0.25 * (nx < ny ? nx : ny);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double r = hypot(x - 0.5 * nx, y - 0.5 * ny);
      h_rho[(size_t)y * nx + x] = 0.5 * (rl + rv) - 0.5 * (rl - rv) * tanh(2.0 * (r - r0) / 5.0);
    }
  size_t bytes = 0;
  CHECK(lbm_workspace_bytes(&p, &bytes));
  void* d_ws = NULL;
  double* d_rho0 = NULL;
  if (hipMalloc(&d_ws, bytes) != hipSuccess || hipMalloc((void**)&d_rho0, N * sizeof(double)) != hipSuccess ||
      hipMemcpy(d_rho0, h_rho, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "HIP allocation or copy failed\n");
    return 1;
  }
  lbm_ctx* ctx = NULL;
  CHECK(lbm_init(&p, d_ws, bytes, d_rho0, NULL, &ctx));
  lbm_obs o0, o1;
  CHECK(lbm_observe(ctx, nx / 2, ny / 2, &o0, NULL, NULL, NULL));
  CHECK(lbm_step(ctx, steps));
  CHECK(lbm_observe(ctx, nx / 2, ny / 2, &o1, NULL, NULL, NULL));
  printf("{\"model\": %d, \"nx\": %d, \"ny\": %d, \"steps\": %lld, \"mass0\": %.17g, "
         "\"mass\": %.17g, \"rho_in\": %.17g, \"rho_out\": %.17g, \"dp\": %.17g, "
         "\"r_equimolar\": %.17g, \"max_u\": %.17g, \"flags\": %u}\n",
         model, nx, ny, (long long)o1.step, o0.mass, o1.mass, o1.rho_in, o1.rho_out, o1.dp,
         o1.r_equimolar, o1.max_u, o1.flags);
  CHECK(lbm_destroy(ctx));
  hipFree(d_ws);
  hipFree(d_rho0);
  free(h_rho);
  return 0;
}
