/*
 * lbm.h -- C ABI of liblbm, an MI355X (gfx950) implementation of one coupled time step of the
 * central-moment pseudopotential lattice Boltzmann method for forced-convection boiling on a
 * heated cylinder (Saito et al., "Lattice Boltzmann modeling and simulation of forced-convection
 * boiling on a cylinder", arXiv:1912.02018).
 *
 * One step of a run (Sec. II of the paper) is
 *   streaming of the post-collision populations (eq. streaming) with the velocity inlet, the
 *   convective outlet and the interpolated bounce-back cylinder (Sec. IV A);
 *   density and momentum (Sec. II A); pseudopotential psi(rho, T) from the Peng-Robinson EOS
 *   (eq. potential, eq. eos); the 24-neighbour interaction force (eq. interForce) plus gravity;
 *   the central-moment collision with consistent forcing and the thermodynamic-consistency
 *   terms (eq. postColl2), reconstructed as f* = M^-1 N(-u) k* (Appendix A);
 *   the finite-difference temperature equation (eq. energy) with Runge-Kutta stages, third-order
 *   upwind convection and the isotropic gradient/Laplacian of the interaction stencil;
 *   FP64 reductions of the total mass and of the wall heat flux / Nusselt number (Sec. IV B).
 *
 * Conventions
 *   * Fields are row-major [ny][nx] (x fastest); node (x, y) has index y*nx + x.  Populations
 *     follow the paper's velocity order c_x = {0,1,-1,0,0,1,-1,1,-1}, c_y = {0,0,0,1,-1,1,-1,-1,1}.
 *   * The state of a run after n steps is: the post-collision populations f* of step n-1, the
 *     post-streaming populations 2, 6, 8 of the last column from step n-1 (outlet history) and
 *     the temperature T^n.  Density and velocity are derived by streaming (lbm_fields).
 *   * The caller owns the device workspace (size from lbm_workspace_bytes, 256-byte aligned)
 *     and the HIP stream; both must outlive the handle.  The library allocates no device memory.
 *     Every device action is enqueued on that stream; only calls that return host data wait for
 *     it.  Host pointers belong to the caller and are not retained.
 *   * Errors are negative return codes; lbm_last_error() gives a message.  A handle is not
 *     thread-safe; calls on one handle must not overlap.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_handle lbm_handle;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument or configuration */
    LBM_ENOMEM = -2,    /* workspace too small */
    LBM_EDEVICE = -3,   /* a HIP call failed */
    LBM_EUNSTABLE = -4, /* non-finite state detected (e.g. negative psi radicand, blow-up) */
    LBM_ESTATE = -5     /* call not valid in the handle's state */
};

/* arithmetic of the step: FP64; FP32; FP32 compute with populations stored as FP16 or BF16
 * holding f_i - w_i * rho_ref_shift (temperature and macroscopic fields stay FP32);
 * LBM_F64_TANGENT: the FP64 step in forward-mode dual numbers, every value carrying its
 * derivatives along LBM_TANGENTS parameter directions (see lbm_nu_tangent) */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2, LBM_BF16S = 3, LBM_F64_TANGENT = 4 };
enum { LBM_TANGENTS = 4 };

/* x boundaries; y is always periodic.  LBM_BC_INLET_OUTLET: Zou-He velocity inlet (u_in, 0) at
 * x = 0 and convective outlet (speed per outlet_kind, default u_in) at x = nx-1 (Sec. IV A).  LBM_BC_WALL_OUTLET: heated
 * no-slip wall at x = -1/2 (halfway bounce-back; T = T_w, and behind it rho_wall, u = 0 like the
 * cylinder's solid nodes) with the same convective outlet: the Stefan problem (Sec. III E).  The
 * default state of a wall run is at rest.  FP64 and FP32 only. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_INLET_OUTLET = 1, LBM_BC_WALL_OUTLET = 2 };
enum { LBM_OUTLET_U_IN = 0, LBM_OUTLET_LOCAL = 1 };

typedef struct {
    int32_t nx, ny;         /* grid (>= 4 each) */
    int32_t bc_x;           /* LBM_BC_PERIODIC, LBM_BC_INLET_OUTLET or LBM_BC_WALL_OUTLET */
    int32_t rk_stages;      /* temperature update: 0 none, 2 Heun, 4 classical RK4 */
    int32_t warmup_steps;   /* first steps with neither forcing nor temperature update (Sec. IV A) */
    int32_t cyl_x, cyl_y, cyl_r; /* cylinder centre / radius in lattice units; cyl_r <= 0: none.
                                    Solid nodes: (x-cyl_x)^2 + (y-cyl_y)^2 <= cyl_r^2.  The
                                    cylinder must keep 3 nodes from the x ends and 2 from y. */
    int32_t upwind_kind;    /* 0: third-order upwind (dissipation 1/12), 1: Kawamura-Kuwahara (1/4) */
    int32_t diag_every;     /* > 0: accumulate Nu of the state every diag_every steps */
    double nu;              /* kinematic viscosity; omega = (nu/cs^2 + 1/2)^-1 (Sec. II A) */
    double eos_a, eos_b, eos_R, acentric; /* Peng-Robinson constants (eq. eos) */
    double Tr_sat;          /* saturation temperature / T_c, T_c = 0.0778 a / (0.4572 b R) */
    double dTr_wall;        /* wall superheat / T_c */
    double G, sigma;        /* interaction sign/strength (eq. potential), consistency constant */
    double gx, gy;          /* gravity: body force (rho - rho_gref) g */
    double rho_gref;        /* < 0 selects rho_l */
    double rho_l, rho_v;    /* coexistence densities; both <= 0: Maxwell construction at T_sat */
    double rho_wall;        /* density of solid nodes for psi; <= 0 selects rho_l */
    double u_in;            /* inlet velocity (also the outlet convection speed) */
    double alpha_T;         /* thermal diffusivity */
    double cv;              /* specific heat at constant volume */
    int32_t precision;      /* LBM_FP64 ... LBM_F64_TANGENT; all runs of a handle share it */
    int32_t check_every;    /* > 0: lbm_step checks the state for non-finite values */
    double rho_ref_shift;   /* reduced-precision storage offset rho_ref (f_i - w_i rho_ref); <= 0 selects
                               rho_l, which keeps the liquid's populations near zero (rho_ref = 1 is the
                               literal f_i - w_i) */
    double nu_vapor;        /* > 0: phase-dependent viscosity: nu is the liquid value, nu_vapor the
                               vapour's, linear in rho between rho_v and rho_l (constant outside);
                               <= 0: nu everywhere.  FP64 and FP32 only. */
    double alpha_vapor;     /* > 0: phase-dependent thermal diffusivity, likewise with alpha_T the
                               liquid value; lambda = rho c_v alpha(rho) in the energy equation and
                               lambda_v = rho_v c_v alpha_vapor in Nu.  <= 0: alpha_T everywhere. */
    int32_t outlet_kind;    /* convection speed U of the convective outlet (Sec. IV A):
                               LBM_OUTLET_U_IN: U = u_in;
                               LBM_OUTLET_LOCAL: U = max(0, x velocity of the outlet node's
                               post-collision populations of the previous step), the local outflow
                               speed (lets liquid displaced by growing vapour leave a closed-inlet
                               domain such as the heated wall's).  FP64 and FP32 only. */
    int32_t pad_;           /* reserved, 0 */
} lbm_config;

/* Bytes of device workspace needed for n_runs runs (cfgs[0..n_runs-1]); 0 on invalid input. */
size_t lbm_workspace_bytes(const lbm_config *cfgs, int n_runs);

/* Create a handle for n_runs runs stepped together.  Copies the configs, derives the constants,
 * carves dev_workspace and initialises every run to its default state: saturated liquid
 * (rho_l) moving with (u_in, 0) at T_sat, solid nodes at T_w (Sec. IV A).  hip_stream is a
 * hipStream_t (NULL: default stream).  On error *out is NULL. */
int lbm_create(const lbm_config *cfgs, int n_runs, void *dev_workspace, size_t ws_bytes,
               void *hip_stream, lbm_handle **out);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): lbm_create without a caller workspace.  The handle's workspace
 * is a static device array of LBM_STATIC_WORKSPACE_BYTES that the library holds on every device it
 * runs on until the process ends; this call allocates no device memory.  Every static handle of a
 * device shares that device's array: creating one waits for the device (hipDeviceSynchronize) and
 * takes the array over, after which every earlier static handle of the device refuses further
 * calls with LBM_ESTATE (lbm_destroy still releases it); static handles of one device must not be
 * used concurrently.  Runs whose workspace (lbm_workspace_bytes) exceeds the array are refused with
 * LBM_ENOMEM.  Otherwise as lbm_create (same arguments, states and results). */
#define LBM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int lbm_create_static(const lbm_config *cfgs, int n_runs, void *hip_stream, lbm_handle **out);

/* Advance every run by n_steps coupled steps (asynchronous unless check_every > 0, in which
 * case the call waits at its end and returns LBM_EUNSTABLE if a check failed). */
int lbm_step(lbm_handle *h, int n_steps);

/* Host copies of the macroscopic fields of the current state of one run: rho, u = (j + F/2)/rho,
 * T; solid nodes report rho = 0, u = 0, T = T_w and mask = 1.  Each pointer may be NULL.
 * Waits for the stream. */
int lbm_fields(lbm_handle *h, int run, double *rho, double *ux, double *uy, double *T,
               uint8_t *solid_mask);

/* Set a run's state from host fields: f* := f^eq(rho, u) (full Hermite, eq. equi) at every node,
 * outlet history := f^eq of the last column, T := T (NULL: T_sat), solid T := T_w.  Resets the
 * step counter of the handle and the Nu accumulators of the run.  Waits for the stream. */
int lbm_set_fields(lbm_handle *h, int run, const double *rho, const double *ux, const double *uy,
                   const double *T);

/* Raw state of one run as FP64 host copies: fstar [9][ny][nx] (values at solid nodes are
 * unspecified), hist [3][ny] (populations 2, 6, 8), T [ny][nx].  Each pointer may be NULL. */
int lbm_get_state(lbm_handle *h, int run, double *fstar, double *hist, double *T);

/* Checkpoints of the whole handle.  lbm_save copies, byte for byte, every run's current populations
 * (storage format), outlet history, temperature (compute format, derivatives included in the tangent
 * precision) and FP64 heat-flux / Nu accumulators, with the step counter and a header, into host_buf
 * (at least lbm_checkpoint_bytes(h) bytes); it waits for the stream.  lbm_load restores such a
 * checkpoint into a handle of the same runs (same count, precision and grids; LBM_EINVAL otherwise):
 * stepping on from it reproduces the uninterrupted run bit for bit, including the time-averaged Nu.
 * The checkpoint format is that of this library build (not a portable file format). */
size_t lbm_checkpoint_bytes(const lbm_handle *h);
int lbm_save(lbm_handle *h, void *host_buf, size_t bytes);
int lbm_load(lbm_handle *h, const void *host_buf, size_t bytes);

/* Replace the raw state of one run (converted to the storage precision) and set the step
 * counter of the handle to `step`. */
int lbm_set_state(lbm_handle *h, int run, const double *fstar, const double *hist,
                  const double *T, int64_t step);

/* Wall heat flux of the current state (Sec. IV B): N_p = 8 ceil(pi R / 4) probes at radius
 * R + 1.5, q_p = rho_p c_v alpha (T_w - T_p) / 1.5 with bilinear rho_p, T_p; q_mean is their
 * mean, nu = q_mean 2R / (rho_v c_v alpha dT); nu_time_avg is the mean of the Nu values
 * accumulated during lbm_step (0 if none).  FP64.  Waits for the stream. */
int lbm_wall_heat_flux(lbm_handle *h, int run, double *q_mean, double *nu, double *nu_time_avg);

/* Sensitivities of the wall Nusselt number (tangent precision only; LBM_EINVAL otherwise).
 * The tangent directions are the parameters, in this order:
 *   0  dTr_wall  (wall superheat / T_c; T_w = T_sat + dTr_wall T_c)
 *   1  u_in      (inlet velocity, also the outlet convection speed)
 *   2  acentric  (Peng-Robinson acentric factor, through kappa, eq. eos)
 *   3  tau       (relaxation time 3 nu + 1/2, with alpha_T scaled alongside so that nu/alpha_T
 *                 is held)
 * with the coexistence densities rho_l, rho_v (and every density derived from them), T_sat, c_v
 * and the geometry held fixed.  dnu[k] = d Nu / d theta_k of the current state; dnu_time_avg[k]
 * = d/d theta_k of the time average reported by lbm_wall_heat_flux.  The default state of
 * lbm_create carries d u / d u_in = 1; states set by lbm_set_fields / lbm_set_state carry zero
 * derivatives.  Derivatives are exact for the discrete step (forward mode) up to FP64 rounding.
 * Either pointer may be NULL (4 doubles each).  Waits for the stream. */
int lbm_nu_tangent(lbm_handle *h, int run, double *dnu, double *dnu_time_avg);

/* Reverse-mode adjoint (discrete adjoint of the step, hand-written), for objectives built from the
 * wall Nusselt number of Sec. IV B, with respect to the same four parameters as lbm_nu_tangent
 * (dTr_wall, u_in, acentric, tau; rho_l, rho_v, T_sat, c_v and the geometry held).  Covers FP64 runs
 * (precision LBM_FP64) with bc_x LBM_BC_PERIODIC or LBM_BC_INLET_OUTLET, constant transport
 * properties (nu_vapor, alpha_vapor <= 0), outlet_kind LBM_OUTLET_U_IN and nx, ny >= 5; other runs
 * are refused with LBM_EINVAL.
 *
 * lbm_adjoint_step: the adjoint of one step of run `run` from its current state n (the handle is
 * not advanced).  adj_in holds the adjoint of state n+1, adj_out receives that of state n; both are
 * device buffers of lbm_adjoint_state_bytes bytes in FP64, laid out with P = ny * pitch and
 * pitch = nx rounded up to a multiple of 64: lambda_f*[i] at element i*P + y*pitch + x (i = 0..8),
 * lambda_T at 9P + y*pitch + x, lambda_hist[m] (populations 2, 6, 8 of the last column) at
 * 10P + m*ny + y, and the gradient accumulated so far, dJ/dtheta[4], at 10P + 3ny; adj_out's
 * gradient is adj_in's plus this step's contribution.  nu_weight is dJ/dNu_n, the weight of this
 * step's Nu sample (the Nu of state n that lbm_step accumulates) in the objective (0: none).
 * scratch: device memory of lbm_adjoint_scratch_bytes bytes (intermediates of the recomputed
 * step).  dJ_dparams (host, 4 doubles, may be NULL) receives adj_out's gradient (the call then
 * waits for the stream).  The adjoint is exact for the discrete FP64 step up to rounding: it agrees
 * with the tangent precision's derivatives.  The *_bytes calls return 0 for unsupported runs. */
size_t lbm_adjoint_state_bytes(lbm_handle *h, int run);
size_t lbm_adjoint_scratch_bytes(lbm_handle *h, int run);
int lbm_adjoint_step(lbm_handle *h, int run, double nu_weight, const void *adj_in, void *adj_out, void *scratch,
                     size_t scratch_bytes, double *dJ_dparams);

/* J = mean Nu of the states average_from .. steps-1 of the next `steps` steps of a one-run handle,
 * and dJ/dtheta[4] by the reverse sweep: the forward run stores a checkpoint of the state every
 * checkpoint_every steps in dev_ws; then, segment by segment from the last, the segment is
 * recomputed from its checkpoint keeping every state, and lbm_adjoint_step runs over it backwards.
 * The gradient is that of J through the steps taken here, from the current state taken as given;
 * a run still in lbm_create's default state also gets that state's dependence on u_in, and solid
 * nodes' T_w always counts.  The handle ends in the state after `steps` steps with the Nu time
 * average of the window (as lbm_step would leave it with diag_every = 1 and the average restarted
 * at average_from).  dev_ws: caller-owned device memory, 256-byte aligned, of
 * lbm_nu_gradient_bytes(h, steps, checkpoint_every) bytes (about (steps / checkpoint_every +
 * checkpoint_every) FP64 states).  J and dJ_dparams (host) may be NULL.  Waits for the stream. */
size_t lbm_nu_gradient_bytes(lbm_handle *h, int steps, int checkpoint_every);
int lbm_nu_gradient(lbm_handle *h, int steps, int average_from, int checkpoint_every, void *dev_ws, size_t ws_bytes,
                    double *J, double *dJ_dparams);

/* Restart the time average of Nu (and of its tangents) of one run: the next lbm_step
 * accumulations start a new window.  Waits for the stream. */
int lbm_reset_time_average(lbm_handle *h, int run);

/* FP64 sum of rho over the fluid nodes of the current state.  Waits for the stream. */
int lbm_total_mass(lbm_handle *h, int run, double *mass);

/* Saturation state of a configuration's Peng-Robinson fluid (eq. eos; host only, no device
 * needed): out6 = [T_c, T_sat, p_sat, rho_l, rho_v, h_fg].  T_c = 0.0778 a / (0.4572 b R); the
 * coexistence densities follow the Maxwell equal-area construction in specific volume (Sec. III D);
 * the latent heat h_fg = T_sat (s_v - s_l), with the entropy difference integrated from the
 * Maxwell relation (ds/dv)_T = (dp/dT)_v of the EOS (equivalent to Clausius-Clapeyron on the
 * saturation curve).  Uses eos_a, eos_b, eos_R, acentric and Tr_sat of *cfg.  LBM_EINVAL if there
 * is no coexistence (see lbm_last_error(NULL)). */
int lbm_saturation(const lbm_config *cfg, double *out6);

/* Derived constants of a run: [Tc, T_sat, T_w, rho_l, rho_v, rho_w, rho_gref, omega]. */
int lbm_derived(lbm_handle *h, int run, double *out8);

/* Timing hook: enqueue n_launches back-to-back launches of one kernel of the step on the current
 * state of every run, without advancing it (the kernels write only the spare buffers and the
 * macroscopic fields of the current state).  kernel: 0 = streaming + collision (k_lbm),
 * 1 = temperature update (k_thermal; every run must have rk_stages > 0).  Asynchronous. */
enum { LBM_KERNEL_STREAM_COLLIDE = 0, LBM_KERNEL_THERMAL = 1 };
int lbm_time_kernel(lbm_handle *h, int kernel, int n_launches);

/* Launch variants of the stencil kernels (kernel 0: k_lbm, 1: k_thermal): each is a tile of
 * tx x ty nodes per workgroup of `threads` threads, compiled with a register budget for min_waves
 * waves per SIMD if min_waves > 0 (any output pointer may be NULL).  A temperature variant with
 * ty = 0 is a strip of tx columns marching down a chunk of rows whose length is chosen when the tile
 * tables are built, so that one launch spreads over the workgroups the GPU holds at once.  lbm_set_variant rebuilds the tile tables
 * (waits for the stream); lbm_autotune times every variant of both kernels on the handle's
 * current state with HIP events (`launches` pseudo-steps each, without advancing the state, or whole
 * steps with LBM_OPT_TUNE_STEPS; 20 if 0) and keeps the fastest, writing
 * the chosen indices to best[2] if not NULL.  Every tuning is remembered for the rest of the process
 * per device and workload shape (precision, RK stages, heated-wall / phase-property launch, and each
 * run's nx, ny, cylinder radius and x boundary); launches < 0 takes the remembered choice for the
 * handle's shape without timing anything, and tunes with 20 launches when there is none. */
int lbm_variant_count(int precision, int kernel);
int lbm_variant_shape(int precision, int kernel, int variant, int *tx, int *ty, int *threads, int *min_waves);
int lbm_set_variant(lbm_handle *h, int kernel, int variant);
int lbm_get_variant(const lbm_handle *h, int kernel);
int lbm_autotune(lbm_handle *h, int launches, int *best);

/* Advances every run by n_steps steps (1 <= n_steps <= LBM_MAX_PROFILE_STEPS), launching each
 * step directly (no graph replay) with the stream-and-collide and temperature kernels timed by
 * start / stop events of their own dispatches, so the durations are those inside the running
 * step sequence (caches as a step leaves them), not of repeated isolated launches.  Writes the
 * mean milliseconds per dispatch to kernel_ms[0] (k_lbm) and kernel_ms[1] (k_thermal; 0 if no
 * step advanced the temperature), and to kernel_ms[2] the time of the diagnostic reductions
 * (heat flux, Nu, mass; events around them) per step, averaged over all n_steps steps.
 * Synchronises the stream.  The state advances exactly as with lbm_step.  Errors: LBM_EINVAL
 * (NULL handle or kernel_ms, count out of range), LBM_EDEVICE. */
#define LBM_MAX_PROFILE_STEPS 4096
int lbm_profile_steps(lbm_handle *h, int n_steps, double *kernel_ms);

/* Options.  LBM_OPT_GRAPHS (default 1): lbm_step captures one period of its launch pattern
 * (2 steps, or the least common multiple with diag_every / check_every) into a HIP graph once
 * every run is past its warm-up, and replays it; 0 launches every kernel directly. */
enum { LBM_OPT_GRAPHS = 0, LBM_OPT_STREAM_GROUPS = 1, LBM_OPT_TUNE_STEPS = 2 };
int lbm_set_option(lbm_handle *h, int option, int value);

/* LBM_OPT_STREAM_GROUPS (default 1): with G > 1 (1 <= G <= min(LBM_MAX_STREAM_GROUPS, n_runs)),
 * lbm_step splits the runs into G contiguous ranges of about equal node counts and steps each range
 * on a private stream of its own (default priority), forked from and joined back to the handle's
 * stream by events, so that one range's temperature update runs beside another range's streaming.
 * With LBM_OPT_GRAPHS the window of steps, fork and join included, is captured into one HIP graph
 * whose groups are parallel branches, and replayed on the handle's stream.  Each run sees the same
 * launches in the same order as with one stream, so results are bitwise the same.  Setting the option waits for the handle's
 * stream.  lbm_get_option returns the current value (-1 for an unknown option or a NULL handle);
 * lbm_stream_group_runs gives the runs [run0, run1) of group `group` (LBM_EINVAL if out of range). */
#define LBM_MAX_STREAM_GROUPS 8
/* LBM_OPT_TUNE_STEPS (default 0): 1 makes lbm_autotune time whole steps of the handle instead of
 * pseudo-steps on the unchanged state, so the state advances by the steps it times (per variant of
 * each kernel, two rounds of launches + 3 steps, directly launched on the handle's stream).  Whole
 * steps alternate the double buffers as stepping does, and the caches with them: on the 1024x512
 * channel pseudo-steps rank a stream-and-collide tile first that whole steps find 4 % slower. */
int lbm_get_option(const lbm_handle *h, int option);
int lbm_stream_group_runs(const lbm_handle *h, int group, int *run0, int *run1);

/* Steps taken since creation / the last set_fields / set_state. */
int64_t lbm_step_count(const lbm_handle *h);

/* Message of the last error on this handle (or of the last failed lbm_create if h is NULL). */
const char *lbm_last_error(const lbm_handle *h);

/* Release the handle (does not free the caller's workspace; waits for the stream). */
void lbm_destroy(lbm_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
