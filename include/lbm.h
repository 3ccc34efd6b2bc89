/*
 * lbm.h - C ABI of the MI355X (gfx950) library for the D2Q9 pseudopotential
 * multiphase lattice Boltzmann step with high-order-difference (HDM) forces,
 * after Qin, Zhao, Chen, Zhang, Wen, "A pseudopotential multiphase lattice
 * Boltzmann model based on high-order difference" (arXiv:1712.06079).
 *
 * One time step (Sec. 2 Eq. 1) computes, per lattice site:
 *   density and momentum                                  (Sec. 2 Eq. 3)
 *   the EOS potential U = g (k p_EOS(rho, T) - rho/3)     (Eq. 8, Hu's scaling of Sec. 5,
 *        and Phi = sqrt|U| with its sign branch           Eq. 21; EOS: Eqs. 24, 27-29)
 *   the gradient of Phi (Shan-Chen) or U (Zhang-Chen) by the periodic compact
 *        sixth-order difference                           (Sec. 3.2 Eq. 20)
 *   the interaction force F = -2 s Phi grad Phi           (Eq. 22)  or  -grad U (Eq. 7)
 *   BGK collision with Kupershtokh exact-difference forcing (Eqs. 1, 2, 10)
 *   periodic streaming                                    (Eq. 1)
 * The lattice is periodic in x and y with h = dt = 1 and the D2Q9 weights
 * 4/9, 1/9, 1/36.  G cancels between Eqs. 4 and 6; the parameter g is an
 * interaction-strength multiplier on U (g = 1 is the paper's model).
 *
 * Conventions
 *  - Memory: every device buffer is owned by the caller.  A domain lives in a
 *    caller-allocated device workspace of lbm_workspace_bytes(); the handle
 *    itself is host memory freed by lbm_destroy().  The library never calls
 *    hipMalloc or hipFree.
 *  - Streams: every device call is asynchronous on the stream it is given
 *    (NULL is the null stream).  Errors of an earlier asynchronous launch
 *    surface at the next call that synchronises.
 *  - Fields: host-visible field arguments are FP64, row-major [ny][nx]
 *    (x fastest), device pointers unless stated.  FP32 domains convert on
 *    entry and exit.
 *  - Errors: every call returns an lbm_status; lbm_last_error() returns a
 *    thread-local message describing the last failure.
 *  - Population order: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1)
 *    6:(-1,1) 7:(-1,-1) 8:(1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,        /* invalid argument: sizes < 5, tau <= 1/2, null pointer, bad enum, T >= Tc where coexistence is asked */
    LBM_ENOMEM = 2,        /* workspace smaller than lbm_workspace_bytes(), or host memory exhausted */
    LBM_EDEVICE = 3,       /* a HIP call failed (message in lbm_last_error) */
    LBM_ENONFINITE = 4,    /* a non-finite density was found */
    LBM_EUNSUPPORTED = 5   /* a parameter combination the library does not implement */
} lbm_status;

typedef enum { LBM_EOS_VDW = 0, LBM_EOS_PR = 1, LBM_EOS_CS = 2, LBM_EOS_RK = 3, LBM_EOS_RKS = 4 } lbm_eos;
typedef enum { LBM_FORCE_SC = 0, LBM_FORCE_ZC = 1, LBM_FORCE_HYBRID = 2 } lbm_force;
typedef enum { LBM_GRAD_HDM = 0, LBM_GRAD_CDM = 1, LBM_GRAD_CDM9 = 2 } lbm_grad;
typedef enum { LBM_F64 = 0, LBM_F32 = 1 } lbm_prec;

/* Problem statement of one periodic domain (Secs. 2, 4, 5.2).
 *  nx, ny  lattice size, each in [5, 2^21], nx * ny <= 2^31
 *  eos     equation of state: VDW (Eq. 24), PR (Eq. 28), CS (Eq. 29 read with
 *          the Carnahan-Starling denominator (1 - b rho/4)^3), RK (Eq. 27,
 *          alpha = 1/sqrt(T)), RKS (Eq. 27 with the Soave alpha(T_r))
 *  force   Shan-Chen (Eq. 22), Zhang-Chen (Eq. 7), hybrid (Eq. 9, weight A)
 *  grad    HDM (Eq. 20), central difference along each axis (Eq. 14) or the
 *          weighted D2Q9 central difference (Eq. 15, with the factor
 *          1/c_s^2 = 3 that the printed sum lacks)
 *  prec    storage precision of the populations (FP64 or FP32); all arithmetic
 *          is FP64.  The potential field is stored in FP64, except with FP32
 *          populations and the Shan-Chen or Zhang-Chen force, where it is
 *          stored in FP32
 *  tau     relaxation time (Eq. 1), > 1/2
 *  a,b,R   EOS constants; omega is the acentric factor (PR, RKS)
 *  T       absolute temperature (T_r = T / Tc; see lbm_critical)
 *  k       Hu's EOS scaling p_m = k p_EOS (Sec. 5), > 0
 *  g       interaction-strength multiplier on U (1 = the paper)
 *  A       hybrid weight (Eq. 9), used only with LBM_FORCE_HYBRID
 *  walls   0: periodic in y; 1: no-slip walls at y = -1/2 and ny - 1/2
 *          (Sec. 5.5; halfway bounce-back, the potential continued past the
 *          wall by its mirror image for the gradient: Eq. 20 or Eq. 14 with
 *          that closure).  x is always periodic.  With walls only the tile
 *          kernels run (automatic choice, lbm_set_kernel variant 2) and
 *          Eq. 15 and the reverse step are LBM_EUNSUPPORTED.
 *  reserved  must be 0                                                     */
typedef struct lbm_params {
    int32_t nx, ny;
    int32_t eos, force, grad, prec;
    double tau;
    double a, b, R, omega;
    double T;
    double k;
    double g;
    double A;
    int32_t walls;
    int32_t reserved;
} lbm_params;

typedef struct lbm_domain lbm_domain;

/* Critical point of the EOS in p (host, synchronous): solves dp/drho =
 * d2p/drho2 = 0 (Sec. 5.2; alpha(Tc) = 1 for PR and RKS).  Independent of k,
 * g and T.  Returns LBM_EINVAL for bad constants. */
lbm_status lbm_critical(const lbm_params* p, double* Tc, double* rhoc);

/* Maxwell equal-area coexistence at temperature T (host, synchronous;
 * Sec. 5.2): rho_v < rho_l with equal pressure and equal chemical potential;
 * p0 (nullable) receives the unscaled coexistence pressure.  The densities do
 * not depend on k.  LBM_EINVAL if T >= Tc or T <= 0. */
lbm_status lbm_maxwell(const lbm_params* p, double T, double* rho_v, double* rho_l, double* p0);

/* Explicit circulant row of the periodic compact difference (Sec. 3.2 Eq. 20)
 * on n >= 5 points, as the kernels use it (host, synchronous): d[0..*taps-1]
 * receive d_1..d_taps with (D u)_i = sum_j d_j (u_{i+j} - u_{i-j}); taps =
 * min(radius, (n-1)/2) with radius 39 for LBM_F64 and 28 for LBM_F32.  d must
 * hold 40 doubles. */
lbm_status lbm_hdm_row(int32_t n, int32_t prec, double* d, int32_t* taps);

/* ---- flat interfaces (host, synchronous; host arrays) ----------------------
 * The square-gradient fluid of Sec. 5.1 Eq. 25 (constant kappa, the k-scaled
 * EOS p_m = k p_EOS of p's eos, a, b, R, omega at temperature p->T; k = p->k).
 * In a flat interface Eq. 26 keeps P_yy = p_m - kappa rho rho'' +
 * (kappa/2) rho'^2 equal to the coexistence pressure, whose first integral is
 * (kappa/2) rho'^2 = W(rho) = rho * integral_{rho_b}^{rho} (p_m(s) - k p0)/s^2 ds
 * (rho_b either Maxwell density, p0 the Maxwell pressure).  LBM_EINVAL for
 * bad arguments or no coexistence at T. */

/* W(rho[i]) for n densities (each inside (0, pole)). */
lbm_status lbm_interface_excess(const lbm_params* p, int32_t n, const double* rho, double* W);

/* The "exact" equilibrium profile of Sec. 5.1: rho and rho' at
 * y_i = (i - (n - 1)/2) h, i < n, for the interface rising with y through the
 * mean of the Maxwell densities at y = 0 (kappa > 0, h > 0). */
lbm_status lbm_flat_profile(const lbm_params* p, double kappa, double h, int32_t n, double* rho, double* drho);

/* Surface tension by the integration method of Sec. 5.3 with the tensor of
 * Eq. 25, sigma = integral (P_N - P_T) dy = kappa integral rho'^2 dy, for one
 * interface of a slab: rho is a periodic density column of n >= 5 sites
 * (h = 1, two interfaces), rho' is Eq. 20 along it (drho, nullable, receives
 * it) and *sigma = (kappa/2) sum rho'^2. */
lbm_status lbm_sigma_slab(double kappa, int32_t n, const double* rho, double* drho, double* sigma);

/* Device workspace needed by one domain with these parameters (bytes): two
 * population buffers f[9] per site (Sec. 2, Eqs. 1-3; FP64 or FP32 storage),
 * two planes of the potential field (Phi of Eq. 21 signed, or U of Eq. 8),
 * reduction partials and the coefficient tables of the Eq. 20 stencil
 * (Sec. 3.2).  Host, synchronous; LBM_EINVAL for invalid parameters or a NULL
 * `bytes`. */
lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a domain in `workspace` (device, >= lbm_workspace_bytes, 256-byte
 * aligned, owned by the caller and kept alive until lbm_destroy) and set
 * f = f^eq(rho0, u0) (Eq. 2).  rho0 is a device FP64 field [ny][nx]; ux0 and
 * uy0 may be NULL (u0 = 0).  Validates the parameters (LBM_EINVAL) and the
 * initial density (rho0 must be finite, > 0 and inside the EOS pole: checked
 * on `stream`, which this call synchronises).  On success *out owns host state
 * only. */
lbm_status lbm_init(const lbm_params* p, void* workspace, size_t workspace_bytes, const double* rho0,
                    const double* ux0, const double* uy0, hipStream_t stream, lbm_domain** out);

/* Advance the domain by nsteps >= 0 time steps (asynchronous): each step is
 * Sec. 2 Eq. 1 with the density and momentum of Eq. 3, the potential of Eq. 8
 * / Eq. 21 (Hu's scaling, Sec. 5), the gradient of Eq. 20 (Sec. 3.2; or
 * Eq. 14 / Eq. 15 of Sec. 3.1), the force of Eq. 22, Eq. 7 or Eq. 9, the
 * exact-difference forcing of Eq. 10 with the equilibrium of Eq. 2, and
 * periodic streaming.  LBM_EINVAL for a NULL domain or nsteps < 0,
 * LBM_EUNSUPPORTED when the selected kernel variant cannot run this domain;
 * launch failures return LBM_EDEVICE. */
lbm_status lbm_step(lbm_domain* d, int64_t nsteps, hipStream_t stream);

/* Output moments of the current state (asynchronous): rho (Eq. 3), the
 * half-step velocity v = (j + F/2)/rho (Eq. 11) and the bulk pressure
 * p = rho/3 + U.  Any of rho, ux, uy, p may be NULL; each is a device FP64
 * field [ny][nx].  totals (nullable, device, 4 doubles) receives
 * {sum rho, sum rho v_x, sum rho v_y, max |v|}, reduced in a fixed order
 * (bitwise reproducible; a non-finite field gives non-finite totals). */
lbm_status lbm_moments(lbm_domain* d, double* rho, double* ux, double* uy, double* p, double* totals,
                       hipStream_t stream);

/* Copy the populations out of / into the domain as a device FP64 array
 * [9][ny][nx] in the documented velocity order (asynchronous).  set also
 * refreshes the potential field so the next step sees the new state. */
lbm_status lbm_get_populations(lbm_domain* d, double* f, hipStream_t stream);
lbm_status lbm_set_populations(lbm_domain* d, const double* f, hipStream_t stream);

/* Number of steps taken since lbm_init (host). */
int64_t lbm_step_count(const lbm_domain* d);

/* Select the step kernel (host; for tuning and tests).  All variants compute
 * the same step (Sec. 2-3); they differ in how the lattice is decomposed:
 *   0  fused single pass, chosen automatically (the default): the strip-
 *      marching kernel when the HDM gradient takes its geometric form along y
 *      (grad = HDM and ny > 2R + 1, R = 39 for FP64 and 28 for FP32
 *      populations) and its automatic chunks keep >= 16 rows each (11 with
 *      FP32 populations; large lattices), otherwise independent tiles of the smallest height (4, 8
 *      or 16 rows) whose tiles all fit one set of resident workgroups, or
 *      where none does, of a height that gives at least one tile per
 *      compute unit;
 *   1  two-pass reference pair (force + collision + push streaming, then the
 *      potential field), tile_y <= 8 or 16 rows;
 *   2  fused single pass over independent 64 x tile_y tiles, tile_y in
 *      {0 (default), 4, 8, 16};
 *   3  fused strip-marching kernel, tile_y = rows per block in {0 (8), 4, 8};
 *      LBM_EUNSUPPORTED from lbm_step when the domain is not eligible.
 * The variant also picks how the reverse step (lbm_adjoint_step*) takes its y
 * derivatives where the HDM gradient has its geometric form along y (ny > 79;
 * Sec. 3.2, Eq. 20): by column marches under 3, from tiles under 1 and 2, and
 * under 0 by column marches once the lattice gives every compute unit 1.5
 * 64-row column chunks (2 x nxb * floor(ny / 64) >= 3 x compute units, nxb
 * the number of 64-column strips).  The results agree to rounding.
 * LBM_EINVAL for unknown values. */
lbm_status lbm_set_kernel(lbm_domain* d, int32_t variant, int32_t tile_y);

/* Number of y chunks each 64-column strip is split into by the marching
 * kernel (host; for tuning and tests): 0 = automatic (the most chunks whose
 * workgroups are all resident at once), otherwise min(nchunk, ny).
 * LBM_EINVAL for nchunk < 0. */
lbm_status lbm_set_chunks(lbm_domain* d, int32_t nchunk);

/* How the marching kernel reads and writes the populations and writes the
 * next potential field, each touched once per step (host; results are the
 * same bitwise in every mode): 0 = automatic (plain, cached accesses when the
 * domain's state, both population and potential buffers, fits in the 256 MiB
 * last-level cache of gfx950 so that the next step reads it from there,
 * otherwise non-temporal), 1 = non-temporal, 2 = plain.  Odd N_x always uses
 * non-temporal accesses.  LBM_EINVAL for other values. */
lbm_status lbm_set_access(lbm_domain* d, int32_t access);

/* What lbm_step launches for this domain under its current settings (host;
 * for tuning and tests; the first call per tile or block height queries the
 * device's occupancy): *kernel 1 (two-pass reference), 2 (tiles) or 3 (strip
 * march); *rows the tile height or the march's rows per block; *chunks the
 * march's y chunks per 64-column strip (0 for the other kernels); *cached 1
 * when the march uses plain (cached) population accesses, else 0.
 * LBM_EUNSUPPORTED where lbm_step would fail the same way (variant 3 on a
 * domain it cannot march, variant 1 with walls); LBM_EINVAL for NULL. */
lbm_status lbm_kernel_choice(lbm_domain* d, int32_t* kernel, int32_t* rows, int32_t* chunks, int32_t* cached);

/* Check the current density (Eq. 3) for non-finite values (synchronises
 * `stream`): *ok = 1 if every rho is finite, else 0 (and the call returns
 * LBM_ENONFINITE).  A non-finite density is how a run that has left the
 * stable range of Hu's scaling (Sec. 5) shows itself.  LBM_EINVAL for NULL
 * arguments. */
lbm_status lbm_check_finite(lbm_domain* d, int32_t* ok, hipStream_t stream);

/* ---- state snapshots (checkpoint / restart) ------------------------------ */

/* Bytes of one snapshot of the domain: its populations followed by the
 * potential field of that state (Eq. 8 / Eq. 21), device, library layout. */
lbm_status lbm_state_bytes(const lbm_domain* d, size_t* bytes);

/* Copy the current state into `state` (device, lbm_state_bytes, 256-byte
 * aligned) / make `state` the current state (asynchronous).  The step counter
 * is not changed. */
lbm_status lbm_save_state(lbm_domain* d, void* state, hipStream_t stream);
lbm_status lbm_load_state(lbm_domain* d, const void* state, hipStream_t stream);

/* Record a trajectory (asynchronous): slot 0 of `states` receives the current
 * state, and slot t+1 the state after step t+1 (the step of Sec. 2, Eq. 1),
 * for t < nsteps; slot t starts at byte t * stride (stride >= lbm_state_bytes,
 * a multiple of 256; states 256-byte aligned, nsteps + 1 slots, caller-owned).
 * The steps are computed from slot to slot without copies; afterwards the
 * domain holds the last state and its step counter has advanced by nsteps.
 * This is the recomputation of a checkpointed segment of a reverse sweep. */
lbm_status lbm_record(lbm_domain* d, int64_t nsteps, void* states, size_t stride, hipStream_t stream);

/* ---- reverse mode ---------------------------------------------------------- */

/* Device scratch needed by lbm_adjoint_step and lbm_adjoint_steps for this
 * domain (bytes): four FP64 planes of the padded lattice, per-tile partials,
 * and one FP64 plane of the lattice that only lbm_adjoint_steps uses. */
lbm_status lbm_adjoint_workspace_bytes(const lbm_domain* d, size_t* bytes);

/* One reverse-mode step (asynchronous), the transpose of the Jacobian of the
 * step of Sec. 2 Eq. 1 (density Eq. 3, potential Eqs. 8 and 21 with Hu's
 * scaling, gradient Eq. 20, force Eq. 22 or Eq. 7, EDM-BGK collision Eqs. 2
 * and 10, streaming) at the state `state_t` (a snapshot from lbm_save_state):
 *   lam_t = (d f_{t+1} / d f_t)^T lam_next,
 *   grad[0] += dJ/dg,  grad[1] += dJ/dT   (J the objective whose dJ/df_{t+1} is lam_next).
 * lam_next, lam_t: device FP64 [9][ny][nx] (distinct buffers); grad: device,
 * 2 doubles; adj_ws: device scratch of lbm_adjoint_workspace_bytes, 256-byte
 * aligned.  The domain's own state is not touched.  state_t carries the
 * potential field of its populations (lbm_save_state, lbm_record).  LBM_EUNSUPPORTED for FP32
 * domains and for the hybrid force. */
lbm_status lbm_adjoint_step(lbm_domain* d, const void* state_t, const double* lam_next, double* lam_t, double* grad,
                            void* adj_ws, size_t adj_ws_bytes, hipStream_t stream);

/* nsteps reverse-mode steps over a recorded trajectory (asynchronous): with
 * states as written by lbm_record (slot t = the state before step t+1) and
 * lam = dJ/df_nsteps on entry, lam = dJ/df_0 on return, i.e. lbm_adjoint_step
 * applied at slots nsteps-1 .. 0 in turn; grad[0] += dJ/dg, grad[1] += dJ/dT
 * over all the steps (per-workgroup partials are summed step after step and
 * reduced once, in a fixed order).  lam_tmp: device FP64 [9][ny][nx] scratch,
 * distinct from lam; adj_ws as for lbm_adjoint_step.  Errors as for
 * lbm_adjoint_step. */
lbm_status lbm_adjoint_steps(lbm_domain* d, const void* states, size_t stride, int64_t nsteps, double* lam,
                             double* lam_tmp, double* grad, void* adj_ws, size_t adj_ws_bytes, hipStream_t stream);

/* lbm_adjoint_step without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight loops, hosts
 * that forbid allocation).  Same contract and result as lbm_adjoint_step; the
 * scratch of its kernels is a fixed device array inside the library, one per
 * GPU, of lbm_adjoint_noalloc_max_bytes() bytes (32 MiB: lattices up to about
 * 1000 x 1000; one step's scratch is 4 FP64 planes of the padded lattice
 * plus per-tile partials).  LBM_EINVAL
 * when the domain needs more.  Nothing is allocated and nothing needs
 * clearing (every scratch word is written before it is read in a call).  All
 * calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (different streams or threads) race and must be serialised by the caller. */
lbm_status lbm_adjoint_step_noalloc(lbm_domain* d, const void* state_t, const double* lam_next, double* lam_t,
                                    double* grad, hipStream_t stream);

/* Size of the fixed scratch array of lbm_adjoint_step_noalloc (bytes). */
size_t lbm_adjoint_noalloc_max_bytes(void);

/* dJ/drho0 from dJ/df_0 for the initial state f_0 = f^eq(rho0, u0) of Eq. 2 at
 * fixed u0 (asynchronous): drho0 = sum_i lam0_i f^eq_i(1, u0).  lam0 device
 * FP64 [9][ny][nx]; ux0, uy0 device [ny][nx] or NULL (u0 = 0); drho0 device [ny][nx]. */
lbm_status lbm_adjoint_rho0(lbm_domain* d, const double* lam0, const double* ux0, const double* uy0, double* drho0,
                            hipStream_t stream);

/* ---- batched sweep ------------------------------------------------------- */

/* Many independent periodic domains that differ in size, EOS, temperature
 * and constants (the coexistence-curve sweep of Sec. 5.2, Fig. 5) but share
 * precision and force (and either all or none use the Eq. 15 gradient; the
 * hybrid weight A and the other gradients may differ), advanced together: one
 * launch per step of a worklist
 * kernel whose tiles cover every domain, replayed from a captured hipGraph.
 * A scheduler setting (tile height, worklist order, workgroups of the
 * persistent launch) is picked by lbm_batch_autotune. */
typedef struct lbm_batch lbm_batch;

/* Device workspace for a batch of n >= 1 domains (bytes). */
lbm_status lbm_batch_workspace_bytes(const lbm_params* params, int32_t n, size_t* bytes);

/* Create a batch in `workspace` (device, 256-byte aligned, caller-owned, kept
 * until lbm_batch_destroy) with domain i = params[i] initialised to
 * f^eq(rho0s[i], 0) (Eq. 2).  rho0s is a host array of n device pointers to
 * FP64 fields [ny_i][nx_i].  Validates like lbm_init (LBM_EINVAL also when
 * the domains differ in precision, force or use of Eq. 15); synchronises
 * `stream`. */
lbm_status lbm_batch_create(const lbm_params* params, int32_t n, void* workspace, size_t workspace_bytes,
                            const double* const* rho0s, hipStream_t stream, lbm_batch** out);

/* Advance every domain by nsteps (the step of lbm_step: Sec. 2 Eq. 1 with
 * Eqs. 2, 3, 8, 10, 20-22): one batched launch per step, in captured graphs of
 * 16 launches (asynchronous).  LBM_EINVAL for a NULL batch or nsteps < 0;
 * LBM_EDEVICE if a graph cannot be captured or launched. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps, hipStream_t stream);

/* The same evolution with one single-domain fused launch per domain per step
 * (the plain path the batched launch is measured against; asynchronous). */
lbm_status lbm_batch_step_separate(lbm_batch* b, int64_t nsteps, hipStream_t stream);

/* Handle of domain i for lbm_moments, lbm_get_populations, lbm_check_finite
 * (owned by the batch; NULL if i is out of range). */
lbm_domain* lbm_batch_domain(lbm_batch* b, int32_t i);

/* Scheduler setting: tile_y rows per tile (4 or 8), order (0 = domain order,
 * 1 = largest domains first, 2 = round robin over domains, 3 = each domain's
 * tiles on the workgroups of one XCD: worklist position p goes to workgroup
 * p mod grid, which the hardware places on XCD (p mod grid) mod 8), grid =
 * workgroups of the persistent launch (0 = one per tile).  set copies the new worklist on
 * `stream` and synchronises it: batched steps queued on `stream` before the
 * call finish with the old schedule.  Steps queued on other streams must be
 * complete (the caller synchronises them).  LBM_EINVAL for other values. */
lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t tile_y, int32_t order, int32_t grid, hipStream_t stream);
lbm_status lbm_batch_get_schedule(const lbm_batch* b, int32_t* tile_y, int32_t* order, int32_t* grid);

/* Time every scheduler candidate (tile_y 4 and 8, the four orders, grid 0,
 * 256, 512, 1024, 2048) over probe_steps batched steps with HIP events, keep
 * the fastest, and restore every domain's state as it was on entry
 * (synchronises `stream`).  report (nullable) receives a JSON object of the
 * per-step times in ms, "cached": false and the choice.  The choice is kept
 * for the rest of the process under a key of the device architecture, the
 * batch's precision, force and domains in order (shape, gradient, walls); a later call
 * for a batch with the same key applies it without timing (report
 * {"cached": true, "best": ...}). */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t probe_steps, hipStream_t stream, char* report, size_t report_len);

/* Forget every autotuner choice kept by this process (thread-safe). */
void lbm_batch_tune_cache_clear(void);

/* Per-domain non-finite check (synchronises): flags[i] = 1 if domain i holds a
 * non-finite density (host array of n int32); returns LBM_ENONFINITE if any. */
lbm_status lbm_batch_check_finite(lbm_batch* b, int32_t* flags, hipStream_t stream);

/* Free the host state of a batch and its domains (the workspace stays with the caller). */
void lbm_batch_destroy(lbm_batch* b);

/* Free the host state of a domain (the workspace stays with the caller). */
void lbm_destroy(lbm_domain* d);

/* ---- diagnostics ---------------------------------------------------------- */

/* Streaming probe (asynchronous): one launch of a plain hand-written kernel
 * that measures the HBM rate attainable on the device, the practical ceiling
 * beside the 8 TB/s peak for the bandwidth-bound step.  16-byte elements with
 * non-temporal loads and stores, a grid-stride loop over `grid` workgroups of
 * 256 threads.  kind 0 copy (dst = src, reads and writes `bytes`), 1 read
 * (reads `bytes` of src, writes one double per workgroup to dst, which must
 * hold `grid` doubles), 2 write (dst = 1.0, writes `bytes`; src unused).
 * Device buffers 16-byte aligned, bytes a positive multiple of 16, grid in
 * [1, 2^24]; LBM_EINVAL otherwise. */
lbm_status lbm_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes, int32_t grid, hipStream_t stream);

/* Thread-local description of the last failure in this thread. */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
