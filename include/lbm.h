/*
 * lbm.h -- C ABI of the MI355X D2Q9 multiphase lattice Boltzmann library.
 *
 * The library advances a periodic D2Q9 lattice with one of the two models
 * compared by Czelusniak et al., "Fundamental comparison between the
 * pseudopotential and the free energy lattice Boltzmann methods"
 * (arXiv 2403.11167):
 *
 *   LBM_MODEL_P   modified pseudopotential model (Sec. 2.1 and Sec. 4):
 *                 MRT lattice Boltzmann equation (Eq. 1) with the standard
 *                 equilibrium (Eq. 4), Shan-Chen force (Eq. 10) on the
 *                 Yuan-Schaefer potential psi(rho) (Eq. 11, G = -1), the
 *                 kappa^P-scaled consistency forcing (Eq. 32) and the source
 *                 term (Eq. 13) built on the width-controlling Q tensor
 *                 (Eq. 30-31, with C_2 = (G/2)(1 - kappa^P), the reading that
 *                 App. C Eq. 41b and App. E Eq. 76 require);
 *   LBM_MODEL_FE  improved well-balanced free-energy model (Sec. 2.2):
 *                 equilibrium of Eq. 20 and forcing of Eq. 21 with A = 0 and
 *                 p_g = 0, force F = -rho grad(mu), mu = mu_b(rho) -
 *                 kappa lap(rho), 9-point stencils of Eq. 24 (with weights).
 *
 * Equations of state: Carnahan-Starling (Eq. 28, mu_b from Eq. 29) and van
 * der Waals (p = rho R T/(1 - b rho) - a rho^2).  Lattice units throughout:
 * c = dx = dt = 1, c_s^2 = 1/3.
 *
 * Memory and streams.  All device memory is owned by the caller: a workspace
 * of lbm_workspace_bytes() bytes and the initial density field.  The context
 * returned by lbm_init() is a small host object holding non-owning pointers
 * into that workspace; it must not outlive it.  Every device operation is
 * enqueued on the HIP stream given to lbm_init() (NULL = the null stream).
 * Only lbm_observe() and the lbm_batch_run() / lbm_batch_observe() calls
 * synchronise that stream.  One context per stream; contexts on different
 * streams are independent.  The library holds no global state apart from
 * the fixed device array of lbm_mlp_grad_noalloc (below).
 *
 * Errors.  Every entry point returns an lbm_status.  Invalid arguments are
 * detected on the host before any device work is enqueued and leave all
 * state untouched.  Conditions that arise on the device during a run are
 * not errors: they raise sticky flags (LBM_FLAG_*) reported by
 * lbm_observe().
 *
 * Layout.  Node (x, y) has linear index n = y * nx + x (x fastest).  Field
 * arrays (densities, velocities) are nx * ny contiguous doubles in that
 * order.  Populations are stored structure-of-arrays, one plane of nx * ny
 * values per velocity, velocities in the order of Eq. 2:
 * c_0 = (0,0), c_1..c_4 = (1,0),(0,1),(-1,0),(0,-1), c_5..c_8 = (1,1),
 * (-1,1),(-1,-1),(1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = -1,  /* bad pointer, size or parameter value        */
  LBM_ERR_EOS_DOMAIN = -2,   /* equation of state undefined for an input    */
  LBM_ERR_UNSUPPORTED = -3,  /* valid request the library does not implement */
  LBM_ERR_WORKSPACE = -4,    /* workspace missing, too small or misaligned  */
  LBM_ERR_HIP = -5,          /* a HIP runtime call failed                   */
  LBM_ERR_NO_CONVERGENCE = -6 /* a host-side solver did not converge        */
} lbm_status;

typedef enum { LBM_MODEL_P = 0, LBM_MODEL_FE = 1 } lbm_model;
typedef enum { LBM_EOS_VDW = 0, LBM_EOS_CS = 1 } lbm_eos;
typedef enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1 } lbm_precision;
/* Boundary in y (x is always periodic).  LBM_BOUNDARY_WALLS puts no-slip
 * walls of Zou and He on the rows y = 0 and y = ny - 1, as in the two-phase
 * channel flow of Sec. 5.3: those rows are fluid nodes held at zero
 * velocity (under Eq. 6b); the populations entering from outside are
 * rebuilt each step, the normal one equal to its opposite and the two
 * diagonal ones from the momentum -F/2 that u = 0 requires.  The density
 * stencils (psi, mu, grad rho) see mirrored rows past a wall, so the
 * density has no normal gradient there.  A force normal to the walls (fy,
 * gravity) enters the closure through -F/2; the wall density then carries
 * the normal momentum (+j_y on the bottom wall, -j_y on the top one).  Needs
 * ny >= 3; single lattices only (a batch with walls returns
 * LBM_ERR_UNSUPPORTED). */
typedef enum { LBM_BOUNDARY_PERIODIC = 0, LBM_BOUNDARY_WALLS = 1 } lbm_boundary;

/* Sticky device flags (lbm_obs.flags). */
#define LBM_FLAG_NONFINITE 1u  /* a density became NaN or infinite          */
#define LBM_FLAG_PSI_CLAMP 2u  /* p_EOS > rho c_s^2 somewhere: psi^2 < 0 was
                                  clamped to 0 (pseudopotential only)        */
#define LBM_FLAG_EOS_DOMAIN 4u /* a density left the EOS domain (b rho >= 1
                                  vdW, b rho/4 >= 1 CS, rho <= 0 for FE)     */

/* Problem statement (Sec. 2, Sec. 5).  Plain data; copied by lbm_init(). */
typedef struct {
  int32_t nx, ny;       /* lattice, 1 <= nx, ny, and
                            ny * 576 * ceil(nx / 64) < 2^31 (population
                            offsets are 32-bit): about 2.4e8 nodes, e.g.
                            15360 x 15360; larger is LBM_ERR_INVALID_ARG  */
  int32_t model;        /* lbm_model                                        */
  int32_t eos;          /* lbm_eos                                          */
  int32_t precision;    /* lbm_precision                                    */
  int32_t boundary;     /* lbm_boundary (y direction; x is periodic)         */
  double a, b, R, T;    /* EOS constants and absolute temperature (> 0)     */
  double tau[9];        /* relaxation time of each moment row of M (Eq. 3,
                           order rho, e, zeta, j_x, q_x, j_y, q_y, p_xx,
                           p_xy); every tau > 1/2; tau[3] == tau[5],
                           tau[4] == tau[6], tau[7] == tau[8]               */
  double sigma_li;      /* P: consistency coefficient sigma^Li (Eq. 32)     */
  double kappa_li;      /* P: surface-tension coefficient kappa^Li (Eq. 30) */
  double kappa_p;       /* P: interface-width coefficient kappa^P (Eq. 30-32) */
  double kappa;         /* FE: gradient coefficient kappa (Sec. 2.2), >= 0  */
  double A;             /* FE: viscosity-tuning A of Eq. 20 (nu = c_s^2
                           (tau[7] - 1/2 - A) > 0, Eq. 23).  A != 0 forms
                           the velocity field of each step before the step
                           (S = grad u + grad u^T with the Eq. 24 stencil;
                           past a wall u is reflected with its sign flipped);
                           P: LBM_ERR_UNSUPPORTED; batches: unsupported    */
  double fx, fy;        /* constant body force added to the model force     */
  double rho_ref;       /* FP32_SHIFTED: reference density of the storage
                           shift (<= 0: the smallest initial density)       */
  /* Launch shape; 0 selects the tuned default (see lbm_autotune).  Results
     do not depend on these, only the speed does. */
  int32_t tile_x;       /* columns per workgroup strip: 0, 64 or 256         */
  int32_t tile_y;       /* rows per workgroup segment: 1 .. 1024, or 0: set at
                           the first step so that the tiles fill whole rounds
                           of resident workgroups (at least 16 rows)        */
  int32_t kernel_flags; /* 0, or LBM_KF_SET | any of the LBM_KF_* below
                           (with walls: ignored, non-temporal stores only) */
  int32_t tile_rounds;  /* with tile_y = 0: the rounds of resident
                           workgroups the tiles fill, 0 .. 64 (0: 1 for the
                           two-step and free-energy kernels, 3 for the
                           single-step pseudopotential one)                 */
  /* Droplet-collision drive (Sec. 5.4): an x force a(x) |rho - rho_ave|
     added to fx, with a = +ax for x <= x_split and -ax beyond, in the steps
     that start at t >= ax_from_step (the paper: a_x = 5e-6, x_split = 100 on
     a 200-wide box, from t = 2000).  ax = 0 turns it off.  Periodic
     lattices and single lattices only (batches: LBM_ERR_UNSUPPORTED). */
  int32_t x_split;
  double ax;
  double rho_ave;       /* <= 0: the mean of the initial density (the scheme
                           conserves mass, so the mean stays constant)      */
  int64_t ax_from_step; /* >= 0                                              */
  /* Gravity of the free-energy model (Sec. 2.2): p_g = grav_rho0 g
     (y - grav_y0) in the equilibrium of Eq. 20 (also at t = 0), the
     buoyancy F_g = -(rho - grav_rho0) g in y added to the force, and
     d_y p_g = grav_rho0 g in the forcing of Eq. 21; g > 0 pulls toward -y
     (the momentum gains -d_y p_g + F_g = -rho g).  g = 0 turns it off.
     Needs LBM_BOUNDARY_WALLS (p_g is not periodic), |g| < 1 and
     grav_rho0 >= 0, else LBM_ERR_INVALID_ARG; the pseudopotential model and
     batches return LBM_ERR_UNSUPPORTED.  On a wall row the normal force is
     fy + F_g of the wall node's density.  The row grav_y0 where p_g = 0
     only moves rounding: results do not depend on it otherwise. */
  double g;
  double grav_rho0;
  double grav_y0;
} lbm_params;

#define LBM_KF_SET 0x80000000u  /* kernel_flags given explicitly            */
#define LBM_KF_NT_STORE 1u      /* non-temporal population stores           */
#define LBM_KF_REGCAP 2u        /* register-capped kernel, higher occupancy */
#define LBM_KF_PIPELINE 4u      /* software-pipelined row loop (P only)     */
#define LBM_KF_TWO_STEP 16u     /* two time steps per launch (periodic
                                   lattices at least 256 wide, both models):
                                   the intermediate populations stay on
                                   chip; results are bit-identical to two
                                   single steps                            */
#define LBM_KF_STRIP128 32u     /* the free-energy two-step kernel on
                                   128-column strips (the default)         */
#define LBM_KF_STRIP192 64u     /* ... on 192-column strips                */
#define LBM_KF_NO_XCD_REMAP 8u  /* keep the dispatch order of the tiles
                                   (default: a contiguous band of tiles per
                                   XCD, whose L2 the neighbours share)      */

/* Observables of the current state (Eq. 6a-b and Sec. 5.2). */
typedef struct {
  int64_t step;         /* time steps taken since lbm_init                   */
  double mass;          /* sum of rho (FP64, compensated)                    */
  double max_u;         /* max |u| over the lattice                          */
  double rho_min, rho_max;
  double rho_in;        /* rho at the probe node (cx, cy)                    */
  double rho_out;       /* rho at (cx + nx/2, cy + ny/2), periodic           */
  double dp;            /* p_EOS(rho_in) - p_EOS(rho_out)                    */
  double r_equimolar;   /* sqrt((mass - N rho_out)/(pi (rho_in - rho_out)))  */
  double du_max;        /* max |u - u_prev| since the previous observe
                           (+inf on the first observe)                       */
  uint32_t flags;       /* OR of LBM_FLAG_* raised since lbm_init            */
  uint32_t reserved;
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;

/* Human-readable text for a status code (static storage). */
const char* lbm_status_string(lbm_status s);

/* Size in bytes of the device workspace a problem needs.  Host only. */
lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Validate p, carve d_workspace (>= lbm_workspace_bytes, 256-byte aligned,
 * device memory) and enqueue f_i = f_i^eq(rho0, u = 0) on hip_stream, the
 * initial state of Sec. 5.3-5.4 (Eq. 4 for P, Eq. 20 for FE).  d_rho0 is a
 * device array of nx*ny doubles, read by the enqueued work.  Returns
 * LBM_ERR_EOS_DOMAIN if a density of d_rho0 is outside the EOS domain
 * (checked on the host from a copy).  On success *out receives a new
 * context. */
lbm_status lbm_init(const lbm_params* p, void* d_workspace, size_t bytes,
                    const double* d_rho0, void* hip_stream, lbm_ctx** out);

/* Enqueue n >= 0 time steps of Eq. 1 (pull streaming, fused with the
 * model's stencils and the moment-space collision).  Asynchronous. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Compute the observables of the current state and, for each non-NULL
 * pointer, export rho, u_x, u_y (device arrays of nx*ny doubles).  The
 * probe (cx, cy) is taken modulo the lattice.  Synchronises the stream. */
lbm_status lbm_observe(lbm_ctx* ctx, int32_t cx, int32_t cy, lbm_obs* out,
                       double* d_rho, double* d_ux, double* d_uy);

/* Copy the current post-streaming populations f_i(x, t) into d_f (device,
 * 9*nx*ny doubles, plane i at offset i*nx*ny) / overwrite the state from
 * d_f (checkpoint and resume).  With walls, the entries of the populations
 * that enter a wall row from outside are unspecified (the next step rebuilds
 * them), so a get / set round trip still resumes exactly.  Asynchronous. */
lbm_status lbm_get_populations(lbm_ctx* ctx, double* d_f);
lbm_status lbm_set_populations(lbm_ctx* ctx, const double* d_f);

/* Free the host context (device memory stays with the caller). */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* The launch shape that carries a run (not part of the paper's method; it
 * lets a caller relate measured kernel times to the work of one launch). */
typedef struct {
  int32_t steps_per_launch; /* 2 where two steps run per launch, else 1     */
  int32_t strip;            /* columns per workgroup strip of that kernel    */
  int32_t segment;          /* rows per segment; 0 until the first lbm_step
                               has fixed an automatic height                 */
  int32_t workgroups;       /* workgroups per launch (0 before that step)    */
  int32_t threads;          /* threads per workgroup                         */
  int32_t reserved[3];
} lbm_launch;

/* Fill *out for ctx.  Host only, no synchronisation.  LBM_ERR_INVALID_ARG
 * for NULL arguments. */
lbm_status lbm_launch_info(const lbm_ctx* ctx, lbm_launch* out);

/* Time the step kernel for p (its lattice size, model, EOS and precision)
 * over a list of launch shapes and kernel variants (strip width, segment
 * height, store kind, register cap, pipelined row loop, one or two steps
 * per launch and the two-step kernel's strip width), `steps` steps each, on
 * a scratch state started from d_rho0, and return the fastest in
 * best->tile_x / tile_y / kernel_flags (the other fields are copied from p).
 * Uses d_workspace (lbm_workspace_bytes(p)); synchronises the stream; the
 * results of a run never depend on the choice, only its speed. */
lbm_status lbm_autotune(const lbm_params* p, void* d_workspace, size_t bytes,
                        const double* d_rho0, void* hip_stream, int32_t steps,
                        lbm_params* best, double* best_ms_per_step);

/* ---- batches of independent lattices --------------------------------------
 * A batch advances n independent problems (sizes, models, EOS and
 * parameters may differ; the precision is common) in lockstep: each time
 * step is one launch per (model, EOS, strip width) group over a table of all
 * tiles of all active problems, and runs of steps are captured in a HIP
 * graph.  Problems on 256-column strips whose kernel_flags allow two steps
 * per launch (0, or LBM_KF_TWO_STEP set) form groups of their own that take
 * two steps per launch (free energy: each tile as two 128-column strips),
 * except the last two to four steps of each check interval; results are the
 * same bit for bit.  A problem with tile_y = 0 has its
 * segment height chosen again for its group whenever the active problems
 * change (4 to 128 rows: the tallest whose tiles fill about one round of
 * resident workgroups); tile_rounds is ignored in a batch.  Every
 * check_every steps a checking step measures, per problem,
 * max |u(t) - u(t - check_every)|; a problem retires as converged when that
 * is below du_tol (or stays below 1e-6 without falling for 5 checks, the
 * floor of FP32 storage), as unstable when it raises NONFINITE or
 * EOS_DOMAIN, or as stalled when that maximum has not fallen below its
 * lowest value for LBM_BATCH_STALL_CHECKS checks without either rule being
 * met (its velocity field stopped settling: it would run to any step limit
 * without converging).  Retired problems keep their state for
 * lbm_batch_observe(). */
typedef struct lbm_batch lbm_batch;

#define LBM_BATCH_ACTIVE 0
#define LBM_BATCH_CONVERGED 1
#define LBM_BATCH_UNSTABLE 2
#define LBM_BATCH_MAXSTEPS 3
#define LBM_BATCH_DROPPED 4 /* retired because its partner became unstable */
#define LBM_BATCH_STALLED 5 /* no new lowest max |du| in LBM_BATCH_STALL_CHECKS
                               checks, and not converged */
#define LBM_BATCH_STALL_CHECKS 100

lbm_status lbm_batch_workspace_bytes(int32_t n, const lbm_params* p, size_t* bytes);

/* p: host array of n problems (common precision, periodic boundaries:
 * LBM_BOUNDARY_WALLS returns LBM_ERR_UNSUPPORTED); d_rho0: host array of n
 * device pointers to each problem's initial density (nx*ny doubles). */
lbm_status lbm_batch_create(int32_t n, const lbm_params* p, const double* const* d_rho0,
                            void* d_workspace, size_t bytes, void* hip_stream,
                            lbm_batch** out);

/* Run until every problem has retired or max_steps more steps were taken.
 * check_every is rounded up to an even number >= 2.  *steps_run (may be
 * NULL) receives the number of lockstep steps executed.  Synchronises. */
lbm_status lbm_batch_run(lbm_batch* b, int32_t check_every, double du_tol,
                         int64_t max_steps, int64_t* steps_run);

/* Step limit of problem i (total steps since creation; default INT64_MAX).
 * An active problem retires with LBM_BATCH_MAXSTEPS at the first check at
 * which its step count has reached the limit, so it may overshoot by up to
 * check_every - 1 steps; one already at or past the limit retires at once.
 * A problem in state LBM_BATCH_MAXSTEPS whose step count is below the new
 * limit becomes active again and continues from its current state at the
 * next lbm_batch_run().  Host-only; no device work. */
lbm_status lbm_batch_set_limit(lbm_batch* b, int32_t i, int64_t max_steps);

/* Problems i and j form one unit, such as the flat and the droplet lattice
 * of one calibration tuple, whose results are only of use together: when
 * either becomes LBM_BATCH_UNSTABLE, the other, if still active, retires
 * with LBM_BATCH_DROPPED before the next step (it keeps its state and step
 * count, and a later lbm_batch_set_limit() does not resume it).  A pair
 * may be set again; i == j, an index out of range, or a problem that
 * already has a different partner gives LBM_ERR_INVALID_ARG.  Host-only; no
 * device work. */
lbm_status lbm_batch_set_partner(lbm_batch* b, int32_t i, int32_t j);

/* Measurement of the runs so far (not part of the paper's method): node
 * updates issued (lattice nodes of the active problems times the steps of
 * each chunk), GPU time between events recorded on the stream around each
 * chunk's graph launch, and the number of chunks.  Each pointer may be
 * NULL.  Host only. */
lbm_status lbm_batch_stats(const lbm_batch* b, int64_t* node_updates, double* gpu_ms,
                           int64_t* chunks);

/* The launch shape of problem i in the batch (not part of the paper's
 * method): steps_per_launch 2 when its group takes two steps per launch,
 * strip and threads of that kernel (a two-step free-energy group runs each
 * 256-column tile as two 128-column strips), segment its current segment
 * height (with tile_y = 0 it may change whenever the active problems
 * change), and workgroups the strip-by-segment tiles of that kernel that
 * hold its columns.  Host only. */
lbm_status lbm_batch_launch_info(const lbm_batch* b, int32_t i, lbm_launch* out);

/* Per-problem state (LBM_BATCH_*), steps taken, last measured max |du| and
 * sticky flags; each pointer may be NULL, else points to n elements. */
lbm_status lbm_batch_state(lbm_batch* b, int32_t* state, int64_t* steps, double* du,
                           uint32_t* flags);

/* lbm_observe() for problem i of the batch. */
lbm_status lbm_batch_observe(lbm_batch* b, int32_t i, int32_t cx, int32_t cy, lbm_obs* out,
                             double* d_rho, double* d_ux, double* d_uy);

lbm_status lbm_batch_destroy(lbm_batch* b);

/* ---- host thermodynamics (no device work) ------------------------------ */

/* Pressure and dp/drho of the EOS at density rho (Eq. 28 for
 * Carnahan-Starling; van der Waals p = rho R T/(1 - b rho) - a rho^2).
 * LBM_ERR_EOS_DOMAIN outside 0 < rho < rho_max. */
lbm_status lbm_eos_eval(int32_t eos, double a, double b, double R, double T, double rho,
                        double* p, double* dp_drho);

/* Critical point of the EOS: van der Waals in closed form, Carnahan-Starling
 * from p' = p'' = 0 (Sec. 3).  Outputs may not be NULL. */
lbm_status lbm_eos_critical(int32_t eos, double a, double b, double R,
                            double* Tc, double* rho_c, double* p_c);

/* Maxwell equal-area coexistence at temperature T: p(rho_v) = p(rho_l) = p0
 * and the integral of (p - p0)/rho^2 over [rho_v, rho_l] vanishes (Eq. 27).
 * LBM_ERR_INVALID_ARG above the critical temperature. */
lbm_status lbm_maxwell(int32_t eos, double a, double b, double R, double T,
                       double* rho_l, double* rho_v, double* p0);

/* epsilon and sigma^Li = -epsilon/(16 G) that make the pseudopotential
 * mechanical-stability integral (Eq. 18) vanish at the Maxwell densities:
 * Newton iteration on Simpson integrals (App. B, Eq. 13-14).
 * LBM_ERR_EOS_DOMAIN if psi is not real on [rho_v, rho_l]. */
lbm_status lbm_sigma_li_theory(int32_t eos, double a, double b, double R,
                               double T, double* eps, double* sigma_li);

/* Free-energy planar theory (Eq. 26, App. B Eq. 15): max-slope interface
 * width (rho_l - rho_v)/max|d rho/dx| and surface tension
 * kappa * integral of (d rho/dx) d rho. */
lbm_status lbm_fe_planar_theory(int32_t eos, double a, double b, double R,
                                double T, double kappa, double* width,
                                double* gamma);

/* Parameters that match the pseudopotential model to a free-energy
 * interface (Sec. 3-4, App. B-C): sigma^Li from App. B; kappa^P such that
 * the max-slope width of App. C Eq. 44 equals target_width (<= 0: the FE
 * width for kappa_fe); kappa^Li such that the surface tension of Eq. 46
 * equals the FE one for kappa_fe (Eq. 26). */
lbm_status lbm_match_p_to_fe(int32_t eos, double a, double b, double R,
                             double T, double kappa_fe, double target_width,
                             double* sigma_li, double* kappa_p,
                             double* kappa_li);

/* ---- calibration surrogate --------------------------------------------------
 * The paper fixes the pseudopotential parameters by preliminary simulations
 * at each temperature (Sec. 3 and 5.1-5.2).  The surrogate replaces that
 * search by a multilayer perceptron 4 -> 128 -> 128 -> 128 -> 4 (GELU after
 * each hidden layer) mapping a calibration tuple x = (model, Tr, width
 * parameter w, kappa) to y = (rho_l, rho_v, sigma, W) as measured by
 * equilibrium runs of this library, and seeds near-equilibrium initial
 * profiles for new runs.
 *
 * Parameters: LBM_MLP_NPARAMS floats in device memory, per layer the n_in x
 * n_out weights input-major (W[k][j] at k * n_out + j) followed by the n_out
 * biases; layers 4x128, 128x128, 128x128, 128x4.  Normalisation: network
 * input (x - x_shift) * x_scale; network output o gives y = exp(o * y_scale
 * + y_shift); the loss is the mean over samples and outputs of
 * (o - (log y - y_shift) / y_scale)^2.  Feature and target arrays are
 * row-major n x 4 floats; targets must be positive.  Flag LBM_MLP_BF16
 * rounds every product operand (layer inputs, weights) to bfloat16 and
 * accumulates in FP32; 0 computes in FP32.  All calls are asynchronous on
 * hip_stream; the caller owns every buffer. */
#define LBM_MLP_NPARAMS 34180
#define LBM_MLP_BF16 1

typedef struct {
  float x_shift[4], x_scale[4];
  float y_shift[4], y_scale[4];  /* y_scale != 0 */
} lbm_mlp_norm;

/* Predictions y (n x 4) for features x (n x 4); n == 0 is a no-op. */
lbm_status lbm_mlp_forward(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                           int32_t n, float* d_y, int32_t flags, void* hip_stream);

/* Workspace for a gradient over n samples (about n / 16 * 137 KB, at most
 * 17.5 MB), 256-byte aligned. */
lbm_status lbm_mlp_workspace_bytes(int32_t n, size_t* bytes);

/* Loss and gradient (LBM_MLP_NPARAMS floats, overwritten) over n samples of
 * a data set of n_rows rows: sample s is row d_idx[s] (d_idx may be NULL:
 * rows 0..n-1).  A row index outside [0, n_rows) makes *d_loss NaN and the
 * sample contributes nothing.  d_loss (one float) may be NULL.  The
 * gradient is summed per workgroup and then in a fixed order, so repeated
 * calls give identical results. */
lbm_status lbm_mlp_grad(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                        const float* d_y, int32_t n_rows, const int32_t* d_idx, int32_t n,
                        float* d_grad, float* d_loss, int32_t flags, void* d_workspace,
                        size_t bytes, void* hip_stream);

/* One Adam update (Kingma and Ba, 2015, with bias correction) of the
 * parameters with moment buffers d_m, d_v (LBM_MLP_NPARAMS floats each,
 * zero before step t = 1). */
lbm_status lbm_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t t,
                        float lr, float beta1, float beta2, float eps, void* hip_stream);

/* lbm_mlp_grad followed by lbm_mlp_adam with beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8. */
lbm_status lbm_mlp_train_step(float* d_params, float* d_m, float* d_v, int64_t t, float lr,
                              const lbm_mlp_norm* norm, const float* d_x, const float* d_y,
                              int32_t n_rows, const int32_t* d_idx, int32_t n, float* d_grad,
                              float* d_loss, int32_t flags, void* d_workspace, size_t bytes,
                              void* hip_stream);

/* ---- allocation-free gradient -------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training loops, harnesses that forbid hipMalloc):
 * lbm_mlp_grad without the workspace argument.  The per-workgroup gradient
 * partials live in a fixed device array inside the library (about 8.4 MiB,
 * the partials of LBM_MLP_NOALLOC_MAX_N samples), one copy per GPU, held
 * until the process ends; its address is looked up on the first call on
 * each device.  The call allocates nothing (no hipMalloc, no library
 * allocator), and its results are identical to lbm_mlp_grad's for the same
 * arguments.  n > LBM_MLP_NOALLOC_MAX_N returns LBM_ERR_WORKSPACE with no
 * device work; other arguments and errors as lbm_mlp_grad.  The array is
 * shared by every call on that GPU: two calls whose work overlaps in time on
 * one GPU (different streams or threads) race on it and give wrong
 * results; calls in one stream are ordered and safe. */
#define LBM_MLP_NOALLOC_MAX_N 1024

lbm_status lbm_mlp_grad_noalloc(const float* d_params, const lbm_mlp_norm* norm,
                                const float* d_x, const float* d_y, int32_t n_rows,
                                const int32_t* d_idx, int32_t n, float* d_grad, float* d_loss,
                                int32_t flags, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
