/*
 * grmhd.h -- C ABI of the MI355X (gfx950) GR-MHD stepper.
 *
 * The library advances ideal GR-MHD in a fixed Kerr metric with the conservative
 * finite-volume scheme of the cuHARM paper (arXiv 2205.02484): PLM/MC reconstruction,
 * Lax-Friedrichs or HLL face fluxes with the simplified dispersion relation, the centred
 * geometric source, flux-CT, the RK2 midpoint step with a CFL time step, and the
 * Newton-Raphson / Brent / entropy conserved-to-primitive inversion with floors, ceilings,
 * the Lorentz cap and neighbour-average fixups (Secs. 2.1-2.4, 4.1, 4.2).
 *
 * Conventions shared by every entry point
 *   - Primitive order (Sec. 2.1, vector P): rho, u, u~1, u~2, u~3, B1, B2, B3, with u~ the
 *     normal-observer velocity and B^i = *F^{it}, contravariant components in the code
 *     coordinates (MKS or flat Cartesian).
 *   - Conserved order (Sec. 2.1, vector U plus the entropy of Sec. 2.1):
 *     sqrt(-g) (rho u^t, T^t_t, T^t_1, T^t_2, T^t_3, B1, B2, B3, S u^t), S = p / rho^(gamma-1).
 *   - Arrays are FP64, C order [var][n1][n2][n3] with n3 (phi) fastest, interior cells only.
 *   - Pointers are host pointers unless the matching `*_on_device` flag is non-zero, in which
 *     case they are device pointers on the context's device.  The caller owns every buffer it
 *     passes; the library copies inputs and owns its device state.
 *   - A context is bound to one HIP stream and is not thread-safe; distinct contexts are
 *     independent.
 *   - Functions return a GRMHD_* code and never throw or abort; the text of the last error of
 *     the calling thread is available from grmhd_last_error().  Inputs holding NaN are rejected
 *     with GRMHD_EINVAL.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GRMHD_OK = 0,
    GRMHD_EINVAL = -1,    /* bad argument */
    GRMHD_ENOMEM = -2,    /* device allocation failed */
    GRMHD_EDEVICE = -3,   /* HIP runtime error */
    GRMHD_ENUMERIC = -4,  /* cells left unfixable by the fixup rounds (state kept valid) */
    GRMHD_EAGAIN = -5,    /* ensemble: job does not fit the memory budget right now */
    GRMHD_ENOTFOUND = -6  /* ensemble: unknown job id */
};

enum { GRMHD_MKS = 0, GRMHD_MINKOWSKI_CART = 1 };
enum { GRMHD_LLF = 0, GRMHD_HLL = 1 };
/* Reconstruction of the face states (Sec. 2.2): piecewise linear with the MC limiter, or PPM
 * (Colella & Woodward 1984, the upgrade Sec. 2.2 names), which needs >= 3 cells along every
 * direction with more than one cell. */
enum { GRMHD_PLM = 0, GRMHD_PPM = 1 };

/* Grid.  GRMHD_MKS (Sec. 4.1): r = exp(X1) on [r_in, r_out], theta = pi X2 + (1-h)/2 sin(2 pi X2)
 * on X2 in [0,1], phi = X3 on [0, 2 pi); radial inflow/outflow, polar reflection, periodic phi.
 * GRMHD_MINKOWSKI_CART: flat space on the box [xmin, xmax], periodic in every direction (used
 * for wave and conservation tests).  A direction with n = 1 is inactive (n3 = 1 is the 2D
 * axisymmetric case; it keeps only the E^3 component of flux-CT). */
typedef struct {
    int32_t n1, n2, n3;
    int32_t coords;
    double r_in, r_out, h;
    double xmin[3], xmax[3];
    /* MKS radial map (Sec. 4.1, R_0 = 0): r = exp(X1) for X1 < ln r_br and
     * r = exp(X1 + (X1 - ln r_br)^n_x) beyond; r_br <= 0 keeps exp(X1) on the whole grid
     * (EINVAL unless r_br > r_in and 2 <= n_x <= 16 when r_br > 0).  X1 spans [ln r_in, X1_out]
     * with r(X1_out) = r_out in n1 equal cells. */
    double r_br;
    int32_t n_x;
    /* MKS polar velocity interpolation (Sec. 4.1, boundary conditions): in the pole_fix cells
     * next to each pole, u~2 is replaced by the straight line in X2 from zero at the pole to its
     * value at the centre of cell pole_fix (resp. n2-1-pole_fix), in each stage's input before the
     * ghosts are filled.  0 (default) turns it off; the paper uses 2.  EINVAL unless
     * 0 <= pole_fix and 2 pole_fix < n2, and pole_fix = 0 on flat grids. */
    int32_t pole_fix;
} grmhd_grid;

/* Physics and numerics.  Defaults (grmhd_params_default) are the paper's values: cfl 0.45
 * (Sec. 2.2), floors rho >= max(1e-20, 1e-5 r^-1/2), u >= max(1e-20, 1e-5/3 r^-5/2), b^2/rho < 50,
 * b^2/u < 2500, Lorentz factor <= 50 (Sec. 2.4), entropy inversion below beta = 1e-2 and
 * Newton-Raphson tolerance 1e-10 (Sec. 2.3). */
typedef struct {
    double spin, gam, cfl;
    int32_t riemann;   /* GRMHD_LLF or GRMHD_HLL */
    int32_t recon;     /* GRMHD_PLM (default) or GRMHD_PPM */
    double rho_fl_coef, rho_fl_pow, u_fl_coef, u_fl_pow, fl_abs;
    double bsq_rho_max, bsq_u_max, gamma_max, beta_entropy;
    double c2p_tol;
    int32_t c2p_maxit, fixup_max_rounds;
} grmhd_params;

typedef struct grmhd_ctx grmhd_ctx;
typedef struct grmhd_batch grmhd_batch;

/* Fill `p` with the paper's defaults (spin 0, gamma 4/3). */
void grmhd_params_default(grmhd_params* p);

/* Create a run: copies the primitive fields `prims` ([8][n1][n2][n3], taken as given: the caller
 * supplies a floored state) and builds the metric, inverse-metric and source tables (Sec. 4.1
 * metric, Sec. 2.2 centred source) on the device.  `hip_stream` is a hipStream_t the context
 * launches on (NULL: the library creates a non-blocking stream of its own).  EINVAL on bad
 * sizes/NaN or when (n1+6)(n2+6)n3 >= 2^29 (each per-variable device array, ghosts included,
 * must stay below 4 GiB: kernels address it with 32-bit byte offsets; about 800^3 cells per run),
 * ENOMEM when the device state does not fit. */
int grmhd_init(grmhd_ctx** out, const grmhd_grid* grid, const grmhd_params* params,
               const double* prims, int32_t prims_on_device, void* hip_stream);

/* One RK2 step (Sec. 2.2).  dt > 0: fixed step; dt <= 0: CFL step from the stage-1 face wave
 * speeds, dt = cfl / sum_d max(c_w / dX^d).  When `dt_used` is non-NULL the call waits for the
 * step and returns the dt taken; ENUMERIC if cells were left unfixed in this step. */
int grmhd_step(grmhd_ctx* ctx, double dt, double* dt_used);

/* Enqueue `nsteps` RK2 steps on the context's stream without waiting (replays one captured
 * HIP graph per step).  Same dt convention as grmhd_step. */
int grmhd_steps(grmhd_ctx* ctx, int32_t nsteps, double dt);

/* Conserved-to-primitive inversion only (Sec. 2.3), no floors or fixups: `U` is [9][n1][n2][n3],
 * `P` holds the guess on entry (also used for the beta switch) and the result on exit; `code`
 * ([n1][n2][n3], may be NULL) receives 0 Newton-Raphson, 1 Brent on W, 2 entropy, -1 failure
 * (P of a failed cell keeps the guess except B).  Uses the context's grid and metric. */
int grmhd_cons2prim(grmhd_ctx* ctx, const double* U, double* P, int8_t* code, int32_t on_device);

/* Conserved vector U ([9][n1][n2][n3]) of the primitive fields P (Sec. 2.1). */
int grmhd_prim2cons(grmhd_ctx* ctx, const double* P, double* U, int32_t on_device);

/* Horizon diagnostics of the current state (Sec. 4.2): mdot = sum sqrt(-g) rho u^1 dX2 dX3 and
 * phi_b = 1/2 sum sqrt(-g) |B^1| dX2 dX3 on the first radial cell with r >= r_horizon.  MKS only. */
int grmhd_diag(grmhd_ctx* ctx, double* mdot, double* phi_b);

/* Accretion diagnostics of the current state on the horizon shell (Sec. 4.2, Eqs. diag_Mdot,
 * diag_MAD, angular_momentum_horizon, energy_flux_horizon and the MAD parameter), each a sum over
 * the (j, k) cells of the first radial index whose centre has r >= r_horizon, weighted by
 * dX2 dX3 (the MKS sums equal the paper's theta-phi integrals).  MKS only. */
typedef struct {
    double mdot;        /* sum sqrt(-g) rho u^1 (signed: negative for inflow) */
    double phi_b;       /* 1/2 sum sqrt(-g) |B^1| */
    double ldot;        /* sum sqrt(-g) T^1_3 */
    double edot;        /* -sum sqrt(-g) T^1_0 */
    double phi_b_norm;  /* phi_b / sqrt(|mdot|), 0 when mdot is 0 */
    int32_t i_h;        /* radial index of the horizon shell */
    int32_t reserved_;
} grmhd_horizon;

/* Fills *hz and, when `radial` is non-NULL, the radial profiles radial[6][n1] (host, caller-owned):
 * rows 0-3 the four shell sums above for every radial index i, row 4 the inward angular-momentum
 * flux sum sqrt(-g)(rho + u + p + b^2) u^1 u_3 / row 0 (Eq. lin), row 5 the outward one
 * sum sqrt(-g) b^1 b_3 / row 0 (Eq. lout); rows 4-5 are NaN where row 0 is 0.  Waits for the
 * context's stream.  EINVAL for a non-MKS grid or one that does not reach the horizon. */
int grmhd_diag_full(grmhd_ctx* ctx, grmhd_horizon* hz, double* radial);

/* Largest radial size n1 that grmhd_diag_full_noalloc accepts. */
#define GRMHD_NOALLOC_MAX_N1 16384

/* grmhd_diag_full for callers that cannot allocate memory (code between replays of captured HIP
 * graphs, tight serving loops, harnesses that forbid hipMalloc): the call makes no device or host
 * allocation.  Its shell sums go to one fixed device array of 6 * GRMHD_NOALLOC_MAX_N1 doubles per
 * GPU, which the library holds from the first grmhd_init on that GPU until the process ends.
 * Arguments, results and errors are those of grmhd_diag_full (bit for bit the same values), plus
 * EINVAL when the run's n1 exceeds GRMHD_NOALLOC_MAX_N1.  Every call on a GPU shares that array and
 * each call overwrites what it reads: calls that overlap on one GPU (several host threads, or
 * contexts on several streams) race, so the caller serialises them. */
int grmhd_diag_full_noalloc(grmhd_ctx* ctx, grmhd_horizon* hz, double* radial);

/* Copy the current primitive fields out ([8][n1][n2][n3]). */
int grmhd_get_prims(grmhd_ctx* ctx, double* out, int32_t out_on_device);

/* Time, step count and the number of cells left unfixed since init. */
int grmhd_get_time(grmhd_ctx* ctx, double* t, int64_t* nstep, int64_t* nfail_total);

/* Set the run's time and step count, so that a restart continues the original clock: a context
 * created by grmhd_init from primitives read back with grmhd_get_prims, given the time and step
 * count grmhd_get_time reported with them, steps exactly as the uninterrupted run (the RK2 step of
 * Sec. 2.2 carries nothing from one step to the next but the primitives: it recomputes the
 * conserved variables from them, and the CFL dt depends only on the current state).  Waits for the
 * work already enqueued on the context's stream.  EINVAL for a NULL ctx, a non-finite t or
 * nstep < 0. */
int grmhd_set_time(grmhd_ctx* ctx, double t, int64_t nstep);

/* Method codes of the last inversion stage, [n1][n2][n3]: 0 NR, 1 Brent W, 2 entropy,
 * 3 fixed by neighbour averaging, -1 left unfixed. */
int grmhd_get_codes(grmhd_ctx* ctx, int8_t* codes);

/* Raw Riemann fluxes of direction d (1..3, before flux-CT) of the current state on the faces of
 * interior cells, as [9][n1+(d==1)][n2+(d==2)][n3+(d==3)] (host), plus the largest c_w over
 * those faces.  Diagnostic entry point for flux parity. */
int grmhd_debug_fluxes(grmhd_ctx* ctx, int32_t d, double* F, double* cmax);

/* Fixup rounds of Sec. 2.3 (averaging procedure) on a given state.  `pout` ([8][n1][n2][n3], host,
 * in/out) is a stage output whose cells with code[] == -1 failed (their values are not read),
 * `pin` the stage input; code[] (host, in/out, values -1..3) marks the failed cells.  The device
 * fixup kernel runs its Jacobi rounds (at most params.fixup_max_rounds): on return pout holds the
 * fixed state (floors applied to fixed cells; cells left unfixed carry the pin values of rho, u and
 * u~ and keep the pout field, which the flux-CT update produced), code[]
 * is 3 for cells fixed by averaging and still -1 for cells left unfixed, *left (nullable) counts
 * those.  The context's state becomes the returned pout.  Diagnostic entry point for fixup
 * parity; EINVAL on NULL pointers, NaN in pin or codes outside -1..3. */
int grmhd_debug_fixup(grmhd_ctx* ctx, double* pout, const double* pin, int8_t* code, int64_t* left);

/* Measurement: with timing on, later steps run as plain launches with a HIP event pair recorded
 * on the context's stream around every kernel.  grmhd_kernel_times waits for them and returns
 * the average duration (ms) and launch count per kernel kind, in this order: 0 boundary ghosts,
 * 1-3 face fluxes X1/X2/X3, 4 CFL step, 5 update + Newton-Raphson inversion, 6 fixup,
 * 7 full inversion of the cells the fast path hands over (beta switch, Brent, entropy, ceilings),
 * 8 flux-CT edge EMFs (at most 9 kinds are filled).  Turning timing on or off clears the
 * accumulated figures. */
int grmhd_kernel_timing(grmhd_ctx* ctx, int32_t on);
int grmhd_kernel_times(grmhd_ctx* ctx, double* avg_ms, int64_t* launches, int32_t n);

/* Autotuner: runs `steps_per_candidate` ordinary RK2 steps (CFL dt, counted in the run's time)
 * under each candidate launch shape -- threads per workgroup 64/128/256 and the block-to-XCD
 * order -- and keeps, per stage-kernel kind (ghosts, X1/X2/X3 fluxes, update), the fastest.
 * Results do not depend on the shape.  `report` (may be NULL) receives a text summary. */
int grmhd_autotune(grmhd_ctx* ctx, int32_t steps_per_candidate, char* report, int32_t report_len);

void grmhd_destroy(grmhd_ctx* ctx);

/* Text of the last error of the calling thread ("" if none). */
const char* grmhd_last_error(void);

/* Device bytes one run of this grid occupies (state, fluxes, metric tables, fixup lists). */
int64_t grmhd_footprint_bytes(const grmhd_grid* grid);

/* ---------------------------------------------------------------------------------------- */
/* Ensemble: independent runs of different grids and physics advanced together.              */
/* Each admitted job keeps its state resident in device memory until released; all active    */
/* jobs advance in one kernel chain per step (one launch per stage kernel for the whole       */
/* ensemble), each with its own CFL dt, until it has taken its requested number of steps.    */
/* ---------------------------------------------------------------------------------------- */

/* `hbm_budget_bytes` bounds the summed footprint of resident jobs (<= 0: 90% of free memory). */
int grmhd_batch_create(grmhd_batch** out, int64_t hbm_budget_bytes, int32_t max_jobs, void* hip_stream);

/* Admit a job (copies `prims`); EAGAIN if its footprint does not fit the budget now. */
int grmhd_batch_admit(grmhd_batch* b, const grmhd_grid* grid, const grmhd_params* params,
                      const double* prims, int32_t prims_on_device, int64_t nsteps, int64_t* job_id);

/* Advance every unfinished job by up to `steps` RK2 steps (CFL dt per job); enqueue only. */
int grmhd_batch_advance(grmhd_batch* b, int32_t steps);

/* Autotuner of the ensemble's launch shapes (see grmhd_autotune); the steps count for the jobs. */
int grmhd_batch_autotune(grmhd_batch* b, int32_t steps_per_candidate, char* report, int32_t report_len);

/* grmhd_kernel_timing / grmhd_kernel_times for the batch's engine: with timing on, later advances
 * run every kernel as a plain launch with an event pair on the batch's stream (no graph, no
 * parallel branches), so each figure is the kernel over all active jobs alone on the device. */
int grmhd_batch_kernel_timing(grmhd_batch* b, int32_t on);
int grmhd_batch_kernel_times(grmhd_batch* b, double* avg_ms, int64_t* launches, int32_t n);

/* Waits for the enqueued work, then lists up to `cap` finished jobs not yet reported. */
int grmhd_batch_poll(grmhd_batch* b, int64_t* done_ids, int32_t cap, int32_t* n_done);

/* Copy a job's primitives (host, [8][n1][n2][n3]), time and step count out. */
int grmhd_batch_fetch(grmhd_batch* b, int64_t job_id, double* prims, double* t, int64_t* nstep);

/* Time, step count and number of cells left unfixed since admission of a job (as grmhd_get_time:
 * the cells that the fixup rounds of Sec. 2.3 could not repair, so that a served run reports its
 * numerical failures).  Nullable outputs.  Waits for the work already enqueued on the batch's
 * stream.  ENOTFOUND for an unknown or released job. */
int grmhd_batch_get_time(grmhd_batch* b, int64_t job_id, double* t, int64_t* nstep, int64_t* nfail_total);

/* Accretion diagnostics of a job's current state (Sec. 4.2, as grmhd_diag_full: the same horizon
 * values in *hz and, when `radial` is non-NULL, the same radial profiles radial[6][n1], host and
 * caller-owned), so that ensemble and served runs report them without leaving the batch.  Ordered
 * after the work already enqueued on the batch's stream, and waits for it.  ENOTFOUND for an
 * unknown or released job; EINVAL for a NULL batch or hz, or for a job whose grid is not MKS or does
 * not reach the horizon. */
int grmhd_batch_diag_full(grmhd_batch* b, int64_t job_id, grmhd_horizon* hz, double* radial);

/* Free a job's device memory and its slot. */
int grmhd_batch_release(grmhd_batch* b, int64_t job_id);

/* Resident bytes and number of resident jobs. */
int grmhd_batch_usage(grmhd_batch* b, int64_t* bytes, int32_t* jobs);

void grmhd_batch_destroy(grmhd_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* GRMHD_H */
