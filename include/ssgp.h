/*
 * ssgp.h -- C ABI of the MI355X split-step Crank-Nicolson (SS-CN) stepper for
 * the spin-1 spin-orbit- and Rabi-coupled Gross-Pitaevskii equations of
 * arXiv:2009.13507 (Eqs. (1)-(2), App. A).
 *
 * One step n -> n+1 applies, in this order, with k = i (real time) or k = 1
 * (imaginary time, Delta -> -i Delta):
 *   CALCNU  psi_j <- exp(-k dt phi_j) psi_j, phi_j the square brackets of
 *           Eqs. (1)-(2) with V = (x^2 + kappa^2 y^2)/2, densities of the input;
 *   HERM    psi <- exp(-k dt A) psi with the 3x3 Hermitian A of App. A,
 *           Eq. (eq:nu), a = c2 psi_{-1}^* psi_0 + Omega/sqrt2,
 *           b = c2 psi_0^* psi_{+1} + Omega/sqrt2 (frozen at the input);
 *   SO      psi <- psi - k dt H_SO psi, explicit, central differences
 *           (App. A, Eqs. (p1)-(p2); the H_SO forms of Sec. 2);
 *   LUX/LUY Crank-Nicolson kinetic steps along x then y:
 *           (I + k dt/2 T) psi' = (I - k dt/2 T) psi, T = -1/2 d^2 on the
 *           three-point stencil with zero values outside the box (Table 1);
 *   RENORM  imaginary time only: psi_j <- d_j psi_j, d_j of App. A
 *           Eq. (DJ) (fixed magnetisation m) or Eq. (DJ2) (norm only).
 *
 * Data layout.  A state is 3 planes (components +1, 0, -1) of ny rows of nx
 * points, x fastest: element (j, iy, ix) at index (j*ny + iy)*nx + ix, as
 * interleaved (re, im) pairs: complex128 (SSGP_C128) or complex64
 * (SSGP_C64).  1D grids use ny = 1.  Grid points are x_i = -nx dx/2 + i dx
 * and y_i = -ny dy/2 + i dy.
 *
 * Ownership.  State buffers are device memory owned by the caller (e.g. a
 * torch tensor); the library keeps borrowed pointers and never frees them.
 * The library owns its workspace (coefficient tables, reduction partials)
 * and frees it in ssgp_destroy / ssgp_destroy_batch.
 *
 * Streams.  Every call is enqueued on the HIP stream given at creation and
 * returns without waiting, except ssgp_observables, ssgp_obs_log_reserve,
 * ssgp_obs_log_read, ssgp_batch_observables and ssgp_omega_grad, which
 * synchronise that stream.
 *
 * Errors.  Every entry point returns SSGP_OK (0) or a negative code and never
 * throws; ssgp_last_error() returns the message of the calling thread's last
 * error.  Invalid arguments leave the object unchanged.
 */
#ifndef SSGP_H
#define SSGP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssgp_grid_s *ssgp_grid;
typedef struct ssgp_batch_s *ssgp_batch;

enum ssgp_status {
    SSGP_OK = 0,
    SSGP_EINVAL = -1,      /* invalid argument or unsupported combination   */
    SSGP_ENOMEM = -2,      /* device or host allocation failed              */
    SSGP_EDEVICE = -3,     /* a HIP call failed                             */
    SSGP_ESTATE = -4,      /* call out of order (e.g. no parameters set)    */
    SSGP_ENONFINITE = -5   /* a reduction met NaN or Inf in the state       */
};

enum ssgp_dtype { SSGP_C128 = 0, SSGP_C64 = 1 };

/* Spin-orbit forms (OPT_SO of Table 2).  1D: gamma p_x Sigma_{x,y,z}.
 * 2D: gamma (eta p_y Sigma_x - p_x Sigma_y) with eta = 1 (Rashba),
 * -1 (Dresselhaus), 0 (equal mixture); SSGP_SO_PX_SX is also accepted in 2D
 * (x derivative only).  gamma p_x Sigma_y uses the Hermitian form derived
 * from Sigma_y of Eq. (3): f_{+-1} = -+ gamma~ d_x psi_0,
 * g = gamma~ d_x (psi_{+1} - psi_{-1}). */
enum ssgp_so {
    SSGP_SO_NONE = 0, SSGP_SO_PX_SX = 1, SSGP_SO_PX_SY = 2, SSGP_SO_PX_SZ = 3,
    SSGP_SO_RASHBA = 4, SSGP_SO_DRESSELHAUS = 5, SSGP_SO_ERD = 6
};

/* RENORM rule.  AUTO: Eq. (DJ) with m = mag0 when Omega = 0 and the
 * spin-orbit term commutes with Sigma_z (none, p_x Sigma_z, or gamma = 0),
 * else Eq. (DJ2).  Eq. (DJ) falls back to Eq. (DJ2) when |m| >= 1, N_{+1} or
 * N_{-1} is zero, or a radicand is negative. */
enum ssgp_renorm { SSGP_RENORM_AUTO = 0, SSGP_RENORM_NORM = 1, SSGP_RENORM_FIXED_M = 2 };

/* Time-stepping scheme (ssgp_set_scheme).  PAPER: the splitting of Sec. 2 and
 * App. A, with the explicit SO sub-step of Eqs. (p1)-(p2).  UNITARY_SO (opt-in,
 * beyond the paper): the SO term is taken by Crank-Nicolson together with the
 * x kinetic term.  STRANG (opt-in, beyond the paper): a second-order splitting
 * around the same joined solve. */
enum ssgp_scheme { SSGP_SCHEME_PAPER = 0, SSGP_SCHEME_UNITARY_SO = 1, SSGP_SCHEME_STRANG = 2 };

typedef struct {
    double c0, c2;     /* density couplings of Eqs. (1)-(2)                 */
    double gamma;      /* spin-orbit strength                              */
    double omega;      /* Rabi strength Omega                              */
    double kappa;      /* trap aspect ratio in V = (x^2 + kappa^2 y^2)/2     */
    double dt;         /* time step Delta > 0                              */
    double mag0;       /* magnetisation m for Eq. (DJ)                     */
    int so;            /* enum ssgp_so                                     */
    int renorm;        /* enum ssgp_renorm                                 */
} ssgp_params;

/* Observables of the current state (Eqs. (4)-(5), rectangle rule):
 * N[j] = dA sum |psi_j|^2 (j = +1, 0, -1), Ntot, M = N[0] - N[2], energy E
 * of Eq. (5) with parts {kinetic, trap, c0, c2, Rabi, spin-orbit}; the
 * kinetic part is the forward difference over every link including the two
 * links to the zero ghosts of each line; rms[j] = sqrt(sum r^2 rho_j /
 * sum rho_j) (0 for an empty component), rms_tot for the total density. */
typedef struct {
    double N[3], Ntot, M, E, E_parts[6], rms[3], rms_tot;
} ssgp_obs;

/* Creates a grid bound to the caller's state buffer psi_dev (3*ny*nx complex
 * elements of dtype, device memory, must outlive the grid) and stream
 * hip_stream (a hipStream_t, or NULL for the default stream).
 * dim = 1 (ny must be 1) or 2.  1 <= nx, ny <= 2048 (one row of all three
 * components is staged in LDS, and a line is solved by one wavefront of 64
 * lanes with chunks of at most 32 points).
 * dx > 0, dy > 0 (dy ignored in 1D).  On success *out owns the workspace. */
int ssgp_create_grid(int dim, int nx, int ny, double dx, double dy, int dtype,
                     void *psi_dev, void *hip_stream, ssgp_grid *out);

/* Rebinds the state buffer (same shape and dtype). */
int ssgp_set_state(ssgp_grid g, void *psi_dev);

/* Validates and stores the model parameters (Table 2: C_0, C_2, OPT_SO,
 * GAM0, OMEGA0, MAG_0, DT).  EINVAL for dt <= 0, non-finite values, an
 * unknown so/renorm value, a y-dependent SO form on a 1D grid, a 1D-only SO
 * form (p_x Sigma_y, p_x Sigma_z) on a 2D grid, or |mag0| > 1. */
int ssgp_set_params(ssgp_grid g, const ssgp_params *p);

/* Selects the time-stepping scheme (default SSGP_SCHEME_PAPER).
 * SSGP_SCHEME_UNITARY_SO, for the x-derivative SO forms (1D: gamma p_x
 * Sigma_{x,y,z}; 2D: gamma p_x Sigma_x and the equal mixture, which is
 * -gamma p_x Sigma_y) or no SO: each step is CALCNU, HERM,
 * then one Crank-Nicolson solve of every x line with
 * H_x = T (x) I + gamma (-i d_x) (x) S_a (the SO sub-step of Eqs. (p1)-(p2)
 * and LUX of Table 1 joined, S_a the spin-1 matrix of Eq. (3), central
 * differences, zero ghosts), then LUY (2D) and, in imaginary time, RENORM.
 * In real time the step then conserves the norm exactly for gamma != 0.  The
 * library solves each line in the eigenbasis of S_a.
 * SSGP_SCHEME_STRANG, for the same SO forms: each step is P2(dt/2), the
 * joined x solve and LUY of UNITARY_SO, P2(dt/2), then RENORM in imaginary
 * time (and in real time with ssgp_set_renorm_real).  P2(tau) takes the
 * pointwise part of Eqs. (1)-(2) (CALCNU's diagonal terms and HERM's matrix of
 * App. A) over tau by the exponential midpoint rule: a predictor
 * psi_m = HERM(tau/2) CALCNU(tau/2) psi, then exp(-k tau/2 Phi(psi_m))
 * exp(-k tau A(psi_m)) exp(-k tau/2 Phi(psi_m)) psi.  The step is second order
 * in dt (the paper's splitting is first order).  On 2D grids in real time the
 * last P2 of a step is merged into the next step's x-pass and the last one of
 * a call (or of an Omega segment) runs as its own pass; with RENORM it runs as
 * its own pass every step.
 * Both: EINVAL for an unknown scheme or parameters with a y-derivative SO
 * form (ssgp_set_params then refuses those too); a step call returns EINVAL
 * when the symmetrised line matrix is not diagonally dominant (real time:
 * dt gamma >= 2 dx).  The adjoint entry points (ssgp_step_real_seq,
 * ssgp_step_real_adjoint) return ESTATE under these schemes.  Drops the
 * captured step graphs. */
int ssgp_set_scheme(ssgp_grid g, int scheme);

/* on = 1: apply the RENORM rule (Eqs. (DJ)/(DJ2), as chosen by the renorm
 * parameter) after every real-time step as well, as App. A does after each
 * time step of the propagation; the sample real-time output of Sec. 3 keeps
 * its energy constant that way.  on = 0 (default): real-time steps are not
 * rescaled, so the norm and magnetisation can be tracked.  Either scheme.
 * EINVAL for another value.  While on, the adjoint entry points
 * (ssgp_step_real_seq, ssgp_step_real_adjoint) return ESTATE.  Drops the
 * captured step graphs. */
int ssgp_set_renorm_real(ssgp_grid g, int on);

/* Piecewise-constant Rabi control for real-time steps: the step with index
 * n (see ssgp_set_step_index) uses omega[n / steps_per_seg] (clamped to the
 * last segment).  nseg = 0 removes the schedule (then params.omega is used).
 * The array is copied. */
int ssgp_set_omega_schedule(ssgp_grid g, const double *omega, int nseg, int steps_per_seg);

/* Index of the next real-time step (for the Omega schedule); real-time
 * steps advance it, adjoint steps move it back. */
int ssgp_set_step_index(ssgp_grid g, long long n);
long long ssgp_get_step_index(ssgp_grid g);

/* nsteps >= 0 full imaginary-time steps on the bound state, in place;
 * RENORM after every step; the state is normalised on return.  On 2D grids
 * runs of steps are enqueued as HIP graph replays (captured once per run
 * length on a library-owned stream, launched on the grid's stream; kernel-
 * timed steps are launched one by one); the stream ordering is the same
 * either way.  The y-derivative SO forms (Rashba, Dresselhaus) take a
 * 3*nx*ny state-sized device scratch buffer, allocated at the first such
 * call and held until ssgp_destroy. */
int ssgp_step_imag(ssgp_grid g, int nsteps);

/* nsteps >= 0 full real-time steps on the bound state, in place (graph
 * replays as for ssgp_step_imag, split where the Omega schedule changes). */
int ssgp_step_real(ssgp_grid g, int nsteps);

/* nsteps real-time steps starting from src_dev, writing the state after step
 * k (k = 1..nsteps) to dst_dev + (k-1) * (3*ny*nx) elements.  src_dev is not
 * modified; the bound state is not used.  Advances the step index. */
int ssgp_step_real_seq(ssgp_grid g, const void *src_dev, void *dst_dev, int nsteps);

/* Observables of the bound state; synchronises the stream.  Returns
 * SSGP_ENONFINITE (with *out filled) when the norm is NaN or Inf.  The Rabi
 * part of E (Eq. (5)) uses params.omega after ssgp_set_params, and after a
 * step call the Omega of the last step taken (imaginary time: params.omega;
 * real time: the schedule's value for that step's index). */
int ssgp_observables(ssgp_grid g, ssgp_obs *out);

/* Observables sampled inside a stepping loop without a host synchronisation
 * (the same sums as ssgp_observables, Eqs. (4)-(5), Omega rule as there).
 * ssgp_obs_log_reserve synchronises the stream, allocates a device log of
 * capacity samples (12 doubles each; capacity = 0 keeps the buffer) and
 * empties it.  ssgp_obs_record enqueues the observables of the bound state
 * into the next free sample on the grid's stream and returns at once; ESTATE
 * when the log is full or no parameters are set.  ssgp_obs_log_read
 * synchronises the stream, writes the first min(max, recorded) samples in
 * record order to out and the number recorded to *count (the log is kept;
 * reserve again to empty it); ENONFINITE when a written sample holds NaN or
 * Inf. */
int ssgp_obs_log_reserve(ssgp_grid g, int capacity);
int ssgp_obs_record(ssgp_grid g);
int ssgp_obs_log_read(ssgp_grid g, ssgp_obs *out, int max, int *count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of ssgp_observables for a state that no grid holds, with no
 * device or host allocation by the library.  psi_dev: 3*ny*nx elements of
 * dtype in the layout above (device memory, read only); dim, nx, ny, dx, dy
 * as for ssgp_create_grid (1 <= nx, ny <= 2048, ny ignored in 1D); p as for
 * ssgp_set_params (checked the same way), its omega used for the Rabi part;
 * hip_stream as for ssgp_create_grid.  The partial sums live in a fixed
 * device array of the library (about 96 KiB, one per GPU, kept until the
 * process ends): calls that overlap on one GPU (other streams or threads)
 * race on it and must be serialised by the caller.  Synchronises the stream;
 * SSGP_ENONFINITE as for ssgp_observables. */
int ssgp_observables_noalloc(int dim, int nx, int ny, double dx, double dy, int dtype,
                             const void *psi_dev, const ssgp_params *p, void *hip_stream,
                             ssgp_obs *out);

/* Adjoint of real-time steps (reverse-mode derivative in the convention
 * grad = dL/dRe(psi) + i dL/dIm(psi)).  states_dev holds the nsteps step
 * inputs psi^{n0}, ..., psi^{n0+nsteps-1} contiguously, where n0 + nsteps is
 * the current step index; lambda_dev holds dL/dpsi^{n0+nsteps} on entry and
 * dL/dpsi^{n0} on exit (in place).  Per step, in reverse order: CN_y^H,
 * CN_x^H, SO^H = I + i dt H_SO, then the transposed Jacobian of the
 * pointwise HERM o CALCNU map recomputed from the step input.  The
 * derivative of L with respect to each step's Omega is accumulated on the
 * device per schedule segment (read with ssgp_omega_grad).  Moves the step
 * index back by nsteps.  EINVAL for the SO forms with y derivatives (Rashba,
 * Dresselhaus); ESTATE under the unitary-SO scheme or real-time RENORM. */
int ssgp_step_real_adjoint(ssgp_grid g, const void *states_dev, void *lambda_dev, int nsteps);

/* Copies the accumulated dL/dOmega per segment (nseg values, one value when
 * no schedule is set) to out and, if reset != 0, clears the accumulators.
 * Synchronises the stream. */
int ssgp_omega_grad(ssgp_grid g, double *out, int nseg, int reset);

int ssgp_destroy(ssgp_grid g);

/* Batched imaginary-time stepping of n independent 2D grids held in one
 * device pool (the same step as ssgp_step_imag, App. A, per grid).  Grid i
 * is nx[i] x ny[i] points (1 <= nx, ny <= 512) with spacing dx[i] in both
 * directions, its state at pool_dev + offsets[i] elements (3*ny*nx
 * elements, the layout above; the states must not overlap), parameters p[i]
 * (every SO form without a y derivative: none, gamma p_x Sigma_x or the
 * equal mixture of Rashba and Dresselhaus couplings).  n is
 * at most 65536.  The arrays are copied; the pool stays owned by the caller
 * and must outlive the batch.  Creation synchronises the stream. */
int ssgp_create_batch(int n, const int *nx, const int *ny, const double *dx,
                      const ssgp_params *p, int dtype, void *pool_dev,
                      const long long *offsets, void *hip_stream, ssgp_batch *out);

/* nsteps imaginary-time steps of every grid of the batch; each grid is
 * normalised on return.  The steps run as graphs of 2^i steps (HIP graphs,
 * captured on first use) of the batch's launch shape: one persistent kernel
 * with device-wide barriers between the x and y sweeps, or one kernel
 * launch per sweep over all grids.  The first call times every shape on a scratch
 * copy of the pool (allocated for the duration of the tuning) unless
 * ssgp_batch_set_shape fixed one; results do not depend on the shape.  A
 * barrier wait that times out ends the kernel (every workgroup leaves) and
 * is reported by the next ssgp_batch_sync or ssgp_batch_observables. */
int ssgp_batch_step_imag(ssgp_batch b, int nsteps);

/* The same steps one grid at a time through the single-grid path (a launch
 * per sweep and grid), for comparison.  Same result up to rounding order:
 * the y lines are split into chunks differently. */
int ssgp_batch_step_imag_serial(ssgp_batch b, int nsteps);

/* Launch shape of ssgp_batch_step_imag: k > 0 is the persistent kernel with
 * k workgroups per compute unit (at most out[2] of ssgp_batch_info), -1 one
 * kernel launch per sweep, 0 re-runs the autotuner at the next step call.
 * -2 and -4 (the grids in 2 or 4 groups of about equal points, one launch
 * per sweep and group, each group on its own stream) are switched off:
 * SSGP_EINVAL, and the autotuner does not time them.
 * Synchronises the stream when the shape changes. */
int ssgp_batch_set_shape(ssgp_batch b, int shape);

/* out[0..5] = {shape in use (0 before the first step call), persistent
 * workgroups launched (0 for shapes < 0), maximum resident workgroups per compute
 * unit, tuned microseconds per step of the shape in use (0 if it was set,
 * not timed), x work items (rows), y work items (column tiles)}. */
int ssgp_batch_info(ssgp_batch b, double *out);

/* Synchronises the stream; SSGP_EDEVICE if a barrier of an earlier batched
 * launch timed out (the batch state is then invalid; the flag is cleared). */
int ssgp_batch_sync(ssgp_batch b);

/* Observables of every grid (out has n entries); synchronises the stream
 * and reports a barrier timeout as ssgp_batch_sync does. */
int ssgp_batch_observables(ssgp_batch b, ssgp_obs *out);

int ssgp_destroy_batch(ssgp_batch b);

/* Kernel timing for measurement: with every > 0, the x-pass and y-pass
 * kernels of every every-th 2D step are launched with HIP start/stop events
 * attached (hipExtLaunchKernel), which take the kernel's own start and end
 * times, for at most capacity steps (every = 0 turns it off and frees the
 * events).  ssgp_profile_read synchronises the stream and writes
 * out[0..4] = {profiled steps, mean x-pass ms, mean y-pass ms, min x-pass ms,
 * min y-pass ms}, then restarts the count. */
int ssgp_profile(ssgp_grid g, int every, int capacity);
int ssgp_profile_read(ssgp_grid g, double *out);

/* Message of the calling thread's last error ("" if none). */
const char *ssgp_last_error(void);

/* Library version string. */
const char *ssgp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SSGP_H */
