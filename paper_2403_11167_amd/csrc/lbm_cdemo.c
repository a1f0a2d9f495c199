/*
 * lbm_cdemo.c -- a plain C client of the C ABI in include/lbm.h (no Python,
 * no torch): allocates device memory with the HIP runtime, sets up a static
 * droplet (Sec. 5.2 geometry), advances it and prints the observables as
 * JSON.
 *
 *   lbm_cdemo MODEL NX NY STEPS     one lattice; MODEL: 0 pseudopotential,
 *                                   1 free energy; one JSON line
 *   lbm_cdemo batch NX NY STEPS     a batch of two lattices, the same droplet
 *                                   under each model, paired as one unit and
 *                                   run in lockstep (checks every 50 steps,
 *                                   no convergence test); one JSON line per
 *                                   problem
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
#include <string.h>

#include "lbm.h"

#define CHECK(call)                                                        \
  do {                                                                     \
    lbm_status st_ = (call);                                               \
    if (st_ != LBM_OK) {                                                   \
      fprintf(stderr, "%s: %s\n", #call, lbm_status_string(st_));          \
      return 1;                                                            \
    }                                                                      \
  } while (0)

static const double A_EOS = 0.25, B_EOS = 4.0, R_EOS = 1.0;

/* Parameters of one droplet lattice under the given model at T. */
static int droplet_params(int model, int nx, int ny, double T, lbm_params* p) {
  memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->model = model;
  p->eos = LBM_EOS_CS;
  p->precision = LBM_FP64;
  p->a = A_EOS;
  p->b = B_EOS;
  p->R = R_EOS;
  p->T = T;
  for (int i = 0; i < 9; ++i) p->tau[i] = 1.0;
  if (model == LBM_MODEL_FE) {
    p->tau[1] = 0.75;
    p->kappa = 0.5;
  } else {
    p->tau[4] = p->tau[6] = 1.0 / 1.99;
    CHECK(lbm_match_p_to_fe(LBM_EOS_CS, A_EOS, B_EOS, R_EOS, T, 0.5, 0.0, &p->sigma_li,
                            &p->kappa_p, &p->kappa_li));
  }
  return 0;
}

static void print_obs(int model, int nx, int ny, double mass0, const lbm_obs* o) {
  printf("{\"model\": %d, \"nx\": %d, \"ny\": %d, \"steps\": %lld, \"mass0\": %.17g, "
         "\"mass\": %.17g, \"rho_in\": %.17g, \"rho_out\": %.17g, \"dp\": %.17g, "
         "\"r_equimolar\": %.17g, \"max_u\": %.17g, \"flags\": %u}\n",
         model, nx, ny, (long long)o->step, mass0, o->mass, o->rho_in, o->rho_out, o->dp,
         o->r_equimolar, o->max_u, o->flags);
}

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s MODEL|batch NX NY STEPS\n", argv[0]);
    return 2;
  }
  const int batch = strcmp(argv[1], "batch") == 0;
  const int model = batch ? 0 : atoi(argv[1]);
  const int nx = atoi(argv[2]), ny = atoi(argv[3]);
  const long steps = atol(argv[4]);
  double Tc, rc, pc, rl, rv, p0;
  CHECK(lbm_eos_critical(LBM_EOS_CS, A_EOS, B_EOS, R_EOS, &Tc, &rc, &pc));
  const double T = 0.8 * Tc;
  CHECK(lbm_maxwell(LBM_EOS_CS, A_EOS, B_EOS, R_EOS, T, &rl, &rv, &p0));

  /* initial density on the host, then on the device */
  if (nx < 1 || ny < 1) return 2;
  const size_t N = (size_t)nx * ny;
  double* h_rho = (double*)malloc(N * sizeof(double));
  if (!h_rho) return 1;
  const double r0 = 0.25 * (nx < ny ? nx : ny);
  double mass0 = 0.0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      double r = hypot(x - 0.5 * nx, y - 0.5 * ny);
      double v = 0.5 * (rl + rv) - 0.5 * (rl - rv) * tanh(2.0 * (r - r0) / 5.0);
      h_rho[(size_t)y * nx + x] = v;
      mass0 += v;
    }
  double* d_rho0 = NULL;
  if (hipMalloc((void**)&d_rho0, N * sizeof(double)) != hipSuccess ||
      hipMemcpy(d_rho0, h_rho, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    fprintf(stderr, "HIP allocation or copy failed\n");
    return 1;
  }

  if (!batch) {
    lbm_params p;
    if (droplet_params(model, nx, ny, T, &p)) return 1;
    size_t bytes = 0;
    CHECK(lbm_workspace_bytes(&p, &bytes));
    void* d_ws = NULL;
    if (hipMalloc(&d_ws, bytes) != hipSuccess) {
      fprintf(stderr, "HIP allocation failed\n");
      return 1;
    }
    lbm_ctx* ctx = NULL;
    CHECK(lbm_init(&p, d_ws, bytes, d_rho0, NULL, &ctx));
    lbm_obs o0, o1;
    CHECK(lbm_observe(ctx, nx / 2, ny / 2, &o0, NULL, NULL, NULL));
    CHECK(lbm_step(ctx, steps));
    CHECK(lbm_observe(ctx, nx / 2, ny / 2, &o1, NULL, NULL, NULL));
    print_obs(model, nx, ny, o0.mass, &o1);
    CHECK(lbm_destroy(ctx));
    hipFree(d_ws);
  } else {
    /* problem 0: pseudopotential, problem 1: free energy, same droplet */
    lbm_params p[2];
    if (droplet_params(LBM_MODEL_P, nx, ny, T, &p[0]) ||
        droplet_params(LBM_MODEL_FE, nx, ny, T, &p[1]))
      return 1;
    const double* d0[2] = {d_rho0, d_rho0};
    size_t bytes = 0;
    CHECK(lbm_batch_workspace_bytes(2, p, &bytes));
    void* d_ws = NULL;
    if (hipMalloc(&d_ws, bytes) != hipSuccess) {
      fprintf(stderr, "HIP allocation failed\n");
      return 1;
    }
    lbm_batch* b = NULL;
    CHECK(lbm_batch_create(2, p, d0, d_ws, bytes, NULL, &b));
    CHECK(lbm_batch_set_partner(b, 0, 1));
    int64_t ran = 0;
    CHECK(lbm_batch_run(b, 50, 0.0, steps, &ran));
    int32_t st[2];
    int64_t ns[2];
    CHECK(lbm_batch_state(b, st, ns, NULL, NULL));
    for (int i = 0; i < 2; ++i) {
      lbm_obs o;
      CHECK(lbm_batch_observe(b, i, nx / 2, ny / 2, &o, NULL, NULL, NULL));
      if (st[i] != LBM_BATCH_MAXSTEPS || ns[i] != ran) {
        fprintf(stderr, "problem %d: state %d after %lld of %lld steps\n", i, st[i],
                (long long)ns[i], (long long)ran);
        return 1;
      }
      print_obs(p[i].model, nx, ny, mass0, &o);
    }
    CHECK(lbm_batch_destroy(b));
    hipFree(d_ws);
  }
  hipFree(d_rho0);
  free(h_rho);
  return 0;
}
