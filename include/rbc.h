/*
 * rbc.h - C ABI of the MI355X library for Parareal applied to 2D
 * Rayleigh-Benard convection (Clarke, Davies, Ruprecht, Tobias & Oishi,
 * "Performance of parallel-in-time integration for Rayleigh Benard
 * Convection").
 *
 * The library advances the Oberbeck-Boussinesq equations (section 2.1,
 * Eqs. 3-7) on a Fourier(x) x Chebyshev(z) grid (section 3.2) with
 * implicit-explicit Runge-Kutta steps (sections 3.2 and 3.6), on every
 * Parareal time slice at once, and runs the Parareal iteration (section
 * 3.1, Eq. 19) around it on the device.
 *
 * Conventions shared by every call:
 *  - Every function returns rbc_status; nothing throws across the ABI.
 *    Negative values are errors (outputs undefined), positive values are
 *    warnings with valid outputs.  rbc_last_error() describes the last one.
 *  - Units are free-fall units on z in [0, Lz]: viscosity sqrt(Pr/Ra),
 *    thermal diffusivity 1/sqrt(Ra Pr), buoyancy coefficient 1.  The
 *    paper writes Eqs. 3-5 in thermal-diffusion units on z in [-1/2, 1/2];
 *    the two differ only by the time and velocity scales.
 *  - A state is one time level of one run, FP64, laid out as
 *        [field][m][re, im][n]
 *    field 0 = streamfunction psi_m for Fourier modes m >= 1, and for
 *    m = 0 the mean horizontal velocity u_bar(z) (imaginary part zero);
 *    field 1 = temperature T_m.  m = 0..Nx/2-1 (the Nyquist mode is
 *    dropped), n = 0..Nz-1 are Chebyshev-T coefficients in
 *    zeta = 2 z / Lz - 1 (z = 0, the hot wall, is zeta = -1).  A field
 *    value is f(x, z) = f_0(z) + 2 Re sum_{m>=1} f_m(z) exp(2 pi i m x / Lx).
 *    rbc_state_size() gives the number of doubles, 4 * (Nx/2) * Nz.
 *    Arrays of states are contiguous: [slice][state].
 *  - Device pointers are caller-owned memory on the handle's device (for
 *    example torch tensors: pass data_ptr()).  The handle owns every
 *    workspace, sized once at rbc_create.
 *  - Calls are enqueued on the handle's HIP stream and return without
 *    waiting, except those that return host values (rbc_nusselt,
 *    parareal_iterate, rbc_coarse_sweep with a host defect pointer),
 *    which synchronise the stream.  A handle is not thread-safe.
 */
#ifndef RBC_H
#define RBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbc_ctx* rbc_handle;

typedef enum {
  RBC_OK = 0,
  RBC_NOT_CONVERGED = 1,    /* k_max reached with the defect above tol      */
  RBC_ERR_ARG = -1,         /* bad size, null pointer, unsupported grid      */
  RBC_ERR_OOM = -2,         /* device allocation failed at create            */
  RBC_ERR_HIP = -3,         /* a HIP runtime call failed                     */
  RBC_ERR_NONFINITE = -4,   /* NaN/Inf in an iterate (buffers kept as-is)    */
  RBC_ERR_STATE = -5        /* factorisation check failed / bad handle state */
} rbc_status;

typedef enum { RBC_FP64 = 0, RBC_MIXED = 1 } rbc_precision;

/* Diagnostic record of one state (section 2.2), RBC_DIAG doubles:
 *   Nu_V (Eq. 9), Nu_b (Eq. 10), Nu_t (Eq. 11), each divided by the
 *   conductive flux dT/Lz of the current mean temperature drop dT = <T>(z=0)
 *   - <T>(z=Lz) (dT = 1 for fixed temperatures; Nu = 1/dT for fixed flux),
 *   KE = <u^2 + w^2>/2,
 *   epsilon_U = nu <|grad u|^2> (viscous dissipation), P = <w T> (buoyancy
 *   production), all volume means in free-fall units, exact for the
 *   discrete fields.  Time averages, RBC_DIAG_AVG doubles:
 *   Nu_V, Nu_b, Nu_t, Nu_int (Eq. 13, on the averaged Nusselt numbers), KE,
 *   Re (mean of <u^2 + w^2>^(1/2) over the viscosity), epsilon_U, P,
 *   |P - epsilon_U| / P (the balance check of Eq. 15). */
#define RBC_DIAG 6
#define RBC_DIAG_AVG 9

/* Why the last parareal_iterate stopped. */
typedef enum {
  RBC_STOP_DEFECT = 0,      /* defect <= tol                                   */
  RBC_STOP_STATISTICS = 1,  /* time-averaged Nusselt numbers settled (stat_tol) */
  RBC_STOP_KMAX = 2,        /* k_max iterations                                */
  RBC_STOP_EXACT = 3        /* k = n_slices: the serial fine solution           */
} rbc_stop;
typedef enum { RBC_ARS222 = 2, RBC_ARS443 = 4 } rbc_scheme;
/* Temperature walls: fixed temperatures T_bot, T_top (Eq. 6) or fixed flux
 * dT/dz = -1 at both walls (Eq. 7; Ra is then the flux Rayleigh number Ra_f,
 * T_top is unused and the initial profile is T_bot - z).  The velocity is
 * no-slip in both. */
typedef enum { RBC_BC_TEMPERATURE = 0, RBC_BC_FLUX = 1 } rbc_bc;

/* Problem and discretisation.  Section 2.1 gives the equations and the
 * box (aspect ratio 2), section 3.2 the grid, sections 3.6-3.7 the coarse
 * propagator and the iteration. */
typedef struct {
  double Ra, Pr;           /* Rayleigh and Prandtl numbers                  */
  double Lx, Lz;           /* box size                                      */
  int32_t Nx, Nz;          /* fine grid: Nx % 4 == 0, Nz % 2 == 0, Nz >= 8 */
  int32_t Nx_c, Nz_c;      /* coarse grid (<= fine, same rules)             */
  double t0, t_end;        /* time window split into n_slices slices        */
  int32_t n_slices;        /* Parareal slices (>= 1)                        */
  double dt_f, dt_c;       /* requested steps; each slice uses
                              dT / ceil(dT / dt) so slices hold whole steps */
  int32_t scheme_f, scheme_c;   /* rbc_scheme                              */
  int32_t precision;       /* rbc_precision: RBC_FP64, or RBC_MIXED = FP32
                              transforms, products and stage history of
                              the explicit terms; FP64 state, implicit
                              solves, correction, defect and Nusselt       */
  int32_t nu_stride;       /* sample Nu every nu_stride fine steps; 0 = off */
  double nu_t_start;       /* start of the Nu time-average window           */
  double T_bot, T_top;     /* wall temperatures at z = 0 and z = Lz (Eq. 6) */
  int32_t promote_fp64;    /* RBC_MIXED only: 1 = before parareal_iterate's
                              defect meets the FP32 rounding floor (near
                              1e-7), switch to all-FP64 propagators: after
                              iteration k >= 2, still above tol, if tol <
                              1e-6 and the defect is <= 1e-3, or if the
                              defect stalls (<= 1e-4 and more than half the
                              previous one), the coarse sweeps from
                              iteration k+1 and the fine runs from k+2 (the
                              pipelined iteration starts those before the
                              defect of k is known) run in FP64.  Default 1. */
  int32_t pipelined;       /* parareal_iterate: 1 = overlap the serial coarse
                              sweep with the fine runs (each slice's fine run
                              starts as soon as its initial state is
                              corrected; results identical to 0, the
                              sweep-then-batch order).  Default 1.          */
  double stat_tol;         /* statistics-based stop (section 5; needs
                              nu_stride > 0 and a history pointer): after
                              iteration k >= 1, stop when each time-averaged
                              Nu_V, Nu_b, Nu_t changed by <= stat_tol
                              (relative) from iteration k-1.  0 = off.      */
  int32_t bc_T;            /* rbc_bc (default RBC_BC_TEMPERATURE)           */
} rbc_params;

/* Fill p with defaults (T_bot = 1, T_top = 0, ARS443, FP64, no sampling). */
rbc_status rbc_default_params(rbc_params* p);

/* Measured launch shapes (autotuning).  rbc_tuning_load reads a text
 * table, one entry per line ('#' starts a comment):
 *     role precision Nx Nz slices MT split xrows
 * role "fine" or "coarse", precision "mixed" or "fp64", the grid, the batch
 * (slices per launch: n_slices for fine plans, 1 for coarse), and the
 * choice: modes per block of the per-mode kernel (2, 4, 6, 8), 1 = the
 * split path (mixed fine grids with Nz >= 64 and Nx >= 128 only), x-pass
 * rows per block (1, 2, 4; 0 = by rule).  An entry "0 0 0" records a batch
 * whose measurement kept the built-in rules.  Later rbc_create calls use the
 * entry of the same role, precision and grid whose batch is nearest, in
 * place of the built-in rules (the environment variables RBC_MODE_TILE,
 * RBC_SPLIT, RBC_XPASS_ROWS still override).  The choice changes launch
 * shapes only, never a result beyond rounding order.  NULL clears the
 * table; the table is process-wide.  The Python binding loads the table
 * measured for gfx950 at import. */
rbc_status rbc_tuning_load(const char* path);
rbc_status rbc_tuning_entries(int32_t* n_entries);

/* Device bytes rbc_create would allocate for p (admission control). */
rbc_status rbc_query_footprint(const rbc_params* p, size_t* device_bytes);

/* Validate p, build the operator tables and band factorisations on the
 * host, allocate workspaces on the current device; hip_stream may be NULL
 * (the null stream).  On error *out is NULL.
 * The handle creates two streams of its own for the pipelined iteration
 * (three with the FP64 switch: precision RBC_MIXED and promote_fp64).
 * A process has few hardware queues (four by default), so live handles
 * beyond the one iterating can leave its streams on a shared queue,
 * where they no longer overlap: destroy handles that are done.
 * Environment, read here (measurement aids): RBC_MODE_TILE = 2, 4, 6 or 8
 * sets the modes per block of the per-mode kernel; RBC_COARSE_PRIO = 0
 * keeps the coarse-grid kernels at the default wave priority;
 * RBC_COARSE_ONE_XCD = 0 spreads the launches of a mixed coarse plan over
 * all XCDs. */
rbc_status rbc_create(const rbc_params* p, void* hip_stream, rbc_handle* out);
rbc_status rbc_destroy(rbc_handle h);

/* Description of the last error on h (NULL h: the last create error). */
const char* rbc_last_error(rbc_handle h);

/* Doubles per state on the fine (coarse = 0) or coarse (coarse = 1) grid. */
rbc_status rbc_state_size(rbc_handle h, int32_t coarse, size_t* n_doubles);

/* Steps per slice and the step actually used on the fine or coarse grid. */
rbc_status rbc_steps_per_slice(rbc_handle h, int32_t coarse, int32_t* n_steps, double* dt);

/* Initial state of section 2.1 (linear profile plus small perturbation,
 * no flow): T = T_bot + (T_top - T_bot) z/Lz + amp xi z (Lz - z)/Lz^2 on
 * the Nx x Nz collocation grid (x_i = i Lx/Nx, Chebyshev-Gauss z points),
 * transformed to coefficients; psi = u_bar = 0.  xi[ix][iz] are standard
 * normals: point p = ix*Nz + iz uses SplitMix64 outputs 2p and 2p+1 of
 * the stream started at seed as uniforms u1, u2 (top 53 bits), and
 * xi = sqrt(-2 ln(1 - u1)) cos(2 pi u2).  Writes one fine state. */
rbc_status rbc_init_state(rbc_handle h, uint64_t seed, double noise_amp, double* U0_dev);

/* The same initial state without a handle (for ensemble runs): the fine
 * state of parameters p into U0_dev, on hip_stream (NULL: the null
 * stream); synchronises that stream. */
rbc_status rbc_initial_state(const rbc_params* p, uint64_t seed, double noise_amp, double* U0_dev, void* hip_stream);

/* The fine propagator F on a batch of slices (the data-parallel half of
 * Eq. 19): n_steps IMEX steps of the fine grid on each of n_slices
 * independent states.  U_in and U_out are [n_slices][state] (they may be
 * the same pointer).  If nu_samples_dev is not NULL and nu_stride > 0 it
 * receives [n_slices][n_steps / nu_stride][RBC_DIAG] diagnostic records
 * after every nu_stride-th step.  n_slices <= the handle's n_slices. */
rbc_status rbc_fine_step_batch(rbc_handle h, const double* U_in_dev, double* U_out_dev,
                               int32_t n_slices, int32_t n_steps, double* nu_samples_dev);

/* The serial coarse sweep of Eq. 19 (G = prolong o coarse steps o restrict,
 * restriction = keep the first Nx_c/2 modes and Nz_c coefficients,
 * prolongation = zero-pad).  U_dev is [n_slices + 1][state];
 * G_dev is [n_slices][coarse state].
 *  mode 0 (predict):  for n = first_slice..S-1:
 *      g = G(U_n); U_{n+1} = g; G_n = coarse part of g.
 *  mode 1 (correct):  for n = first_slice..S-1:
 *      g = G(U_n); U_{n+1} = g + F_n - G_n; G_n = coarse part of g,
 *      with F_dev = [n_slices][state] the fine results of the last iteration.
 * If defect_host is not NULL it receives max_n ||U_{n+1}^new - U_{n+1}^old||
 * / ||U_{n+1}^new|| over the updated slices (the call then synchronises). */
rbc_status rbc_coarse_sweep(rbc_handle h, int32_t mode, int32_t first_slice,
                            double* U_dev, const double* F_dev, double* G_dev,
                            double* defect_host);

/* Parareal (section 3.1, Eq. 19) on the device.  U_dev is [n_slices+1][state];
 * on entry U_dev[0] is the initial state, on return U_dev[n] = U_n^K.
 * Iteration 0 is the coarse prediction.  Iteration k runs F on slices
 * k-1..S-1 (the earlier ones are already exact), then the coarse
 * correction sweep; its defect (section 3.7) is the maximum over slices of
 * the relative L2 change of the state vector.
 * With p.pipelined the fine run of slice n in iteration k+1 starts as soon
 * as the sweep of iteration k has corrected U_n, on a stream of its own,
 * batched with every other fine run in flight (runs of different slices and
 * iterations advance in one launch); the sweep of iteration k+1 takes each
 * F result as it completes.  The result is the same, bit for bit, as the
 * sweep-then-batch order; the work after a converged iteration is started
 * speculatively and discarded.  Stops when the defect is
 * <= tol, when the time-averaged Nusselt numbers settle (p.stat_tol), at
 * k = k_max, or at k = n_slices (then U equals the serial fine solution);
 * rbc_stop_reason tells which.  defect_hist_host[k-1] gets the defect of
 * iteration k (k_max entries).  nu_avg_hist_host, if not NULL and
 * nu_stride > 0, gets [k_max + 1][RBC_DIAG_AVG]: the time averages over
 * [nu_t_start, t_end] of the diagnostic records sampled along the
 * trajectories of iteration k (k = 0: the coarse trajectory).  Returns
 * RBC_NOT_CONVERGED if stopped by k_max with the defect above tol > 0,
 * RBC_ERR_NONFINITE on NaN/Inf. */
rbc_status parareal_iterate(rbc_handle h, double* U_dev, int32_t k_max, double tol,
                            int32_t* k_done_host, double* defect_hist_host,
                            double* nu_avg_hist_host);

/* Checkpoint and resume of the Parareal iteration at an iteration boundary
 * (section 3.1, Eq. 19).  Iteration k + 1 reads the iterate U^k, the coarse
 * propagation G(U_n^k) of every slice, and the decisions and averages of
 * iteration k; U^k is the caller's U_dev, the rest lives in the handle.
 * rbc_get_state copies the rest, as left by the last parareal_iterate on
 * h, into host memory buf of *bytes bytes (buf = NULL: *bytes gets the size
 * needed, which depends only on the parameters): the iteration k reached,
 * its defect and the previous one, the FP64-switch iterations, the time
 * averages of iteration k, the coarse parts of G(U_n^k) and each slice's
 * diagnostic samples from its latest fine run.  Synchronises.
 * RBC_ERR_STATE if no parareal_iterate has run on h.
 * rbc_set_state loads such a buffer into a handle created with the same
 * slices, grids and sampling (RBC_ERR_ARG otherwise); the next
 * parareal_iterate on h, called with U_dev = the saved U^k, then continues
 * at iteration k + 1 instead of starting with the coarse prediction: its
 * iterates, defects (defect_hist_host[j-1] for j > k) and averages
 * (nu_avg_hist_host[j] for j >= k) are those of the uninterrupted run, bit
 * for bit, in either schedule; k_max counts from iteration 0.  The buffer
 * format is the library's own (native byte order), not a file format for
 * other machines. */
rbc_status rbc_get_state(rbc_handle h, void* buf, size_t* bytes);
rbc_status rbc_set_state(rbc_handle h, const void* buf, size_t bytes);

/* Iterate history for studies of the convergence (section 4): later
 * parareal_iterate calls copy U_dev ([n_slices+1][state]) after the coarse
 * prediction and after each iteration k <= k_cap into
 * U_hist_dev[k][n_slices+1][state] (device memory of (k_cap+1) (n_slices+1)
 * states, caller-owned).  NULL disables.  With k = n_slices the last copy is
 * the serial fine solution at every slice boundary. */
rbc_status rbc_set_iterate_history(rbc_handle h, double* U_hist_dev, int32_t k_cap);

/* Why the last parareal_iterate stopped (rbc_stop; -1 before any). */
rbc_status rbc_stop_reason(rbc_handle h, int32_t* reason);

/* First iteration whose fine runs the last parareal_iterate ran in FP64
 * (promote_fp64; its coarse sweeps switched one iteration earlier), 0 if it
 * never promoted. */
rbc_status rbc_fine_fp64_from(rbc_handle h, int32_t* k_host);

/* Scheduler statistics of the last pipelined parareal_iterate (tracing):
 * host seconds spent admitting fine runs, enqueueing batched fine steps,
 * enqueueing coarse work, reading reports and waiting for the device; the
 * number of batched fine steps and of coarse chunks enqueued; the mean
 * number of fine runs per batched step; the wall time of the call, and the
 * wall time at which the report of iteration k was read (k = 0..63, the
 * rest unset).  All zero before the first pipelined call. */
typedef struct {
  double wall_s;
  double host_admit_s, host_fine_s, host_coarse_s, host_report_s, host_wait_s;
  int64_t fine_steps, coarse_chunks;
  double mean_runs_per_step;
  double report_at_s[64];
} rbc_pipeline_stats;
rbc_status rbc_get_pipeline_stats(rbc_handle h, rbc_pipeline_stats* out);

/* Nusselt numbers of section 2.2 for n_states fine states (Eqs. 9-11):
 * nu_host[i] = (Nu_V, Nu_b, Nu_t).  Nu_b, Nu_t: -dT/dz of the horizontal
 * mean at z = 0 and z = Lz.  Nu_V: volume mean of -dT/dz + sqrt(Ra Pr) w T,
 * integrated exactly for the discrete fields.  Synchronises. */
rbc_status rbc_nusselt(rbc_handle h, const double* U_dev, int32_t n_states, double* nu_host);

/* The diagnostic records (RBC_DIAG doubles each, section 2.2) of n_states
 * fine states into out_host[n_states][RBC_DIAG].  Synchronises. */
rbc_status rbc_diagnostics(rbc_handle h, const double* U_dev, int32_t n_states, double* out_host);

/* Ensembles of independent Parareal runs on one device (many runs of
 * different Rayleigh number, grid, step and horizon; section 3.1, Eq. 19 per
 * run).  Each run is the iteration of parareal_iterate in the
 * sweep-then-batch order (pipelined = 0, no FP64 switch: promote_fp64 is
 * ignored): its iterates, defects and stop are those of a handle created
 * with the same parameters, bit for bit.  One rbc_ensemble_step advances
 * every active run by one iteration (a new run: its coarse prediction):
 * the fine runs of all runs of one fine grid shape advance in one batch per
 * stage launch, ordered by their fine steps per slice (a cost-ordered work
 * list), and the serial coarse sweeps of all runs go in lock step, the
 * coarse steps of all runs of one coarse grid shape batched.  Runs may be
 * added between steps; they join at the next step (continuous batching).
 * Run buffers (iterates, fine results, coarse parts, tables) belong to the
 * ensemble from rbc_ensemble_add until rbc_ensemble_release.  Calls are
 * enqueued on the stream given at create; rbc_ensemble_step synchronises
 * (it reads the defects).  An ensemble is not thread-safe. */
typedef struct rbc_ensemble_s* rbc_ensemble;
rbc_status rbc_ensemble_create(void* hip_stream, rbc_ensemble* out);
rbc_status rbc_ensemble_destroy(rbc_ensemble e);
const char* rbc_ensemble_last_error(rbc_ensemble e);
/* Device bytes one run of these parameters needs in an ensemble (its
 * tables, buffers and its share of the batch work arrays): for admission
 * against the free device memory. */
rbc_status rbc_ensemble_footprint(const rbc_params* p, size_t* bytes);
/* Adds a run from the fine initial state U0_dev (copied; caller-owned),
 * stopping at defect <= tol, at k_max iterations or at k = n_slices;
 * *run_id identifies it (ids are not reused). */
rbc_status rbc_ensemble_add(rbc_ensemble e, const rbc_params* p, const double* U0_dev, int32_t k_max, double tol,
                            int32_t* run_id);
/* One iteration of every active run; *n_active = runs still active after it. */
rbc_status rbc_ensemble_step(rbc_ensemble e, int32_t* n_active);
/* Run state (0 active, 1 done, 2 failed on a non-finite value, 3 released),
 * iterations done, the rbc_stop of a finished run (-1 otherwise) and the
 * first hist_len defects (defect_hist may be NULL). */
rbc_status rbc_ensemble_run_info(rbc_ensemble e, int32_t run_id, int32_t* state, int32_t* k_done, int32_t* stop,
                                 double* defect_hist, int32_t hist_len);
/* Copies the run's iterate U^k ([n_slices+1][state]) to U_dev. */
rbc_status rbc_ensemble_result(rbc_ensemble e, int32_t run_id, double* U_dev);
/* Frees a finished run's buffers. */
rbc_status rbc_ensemble_release(rbc_ensemble e, int32_t run_id);
/* Device bytes the run holds. */
rbc_status rbc_ensemble_run_bytes(rbc_ensemble e, int32_t run_id, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * records of rbc_diagnostics written to caller-owned device memory
 * out_dev[n_states][RBC_DIAG], enqueued on the handle's stream without
 * waiting, and allocating nothing.  The partial sums go to a device scratch
 * array of the library (1 MiB per GPU, held until the process ends), so
 * n_states is limited to 1 MiB / (32 bytes x ceil(Nx/2 / max(1, 512/Nz)))
 * states (64 at 1024 x 256, 2048 at 256 x 64); more gives RBC_ERR_ARG.
 * Every call on a GPU shares that GPU's scratch: calls that overlap on one
 * GPU (other streams, other threads, other handles) race, so serialise
 * them.  The scratch needs no clearing (every partial is written before it
 * is read). */
rbc_status rbc_diagnostics_noalloc(rbc_handle h, const double* U_dev, int32_t n_states, double* out_dev);

/* Diagnostic: the explicit (advective) terms of one fine state in the
 * equations' bases: E_dev gets a state-shaped array whose field 0 holds
 * -S3S2S1S0 N_omega (m >= 1) and -S1 D1 <u w> (m = 0), field 1 holds
 * -S1S0 N_T, for the equation rows (the last 4 / 2 rows are zero). */
rbc_status rbc_explicit_terms(rbc_handle h, const double* U_dev, double* E_dev);

/* Kernel timing with HIP events (tracing) of the fine grid's kernels, on
 * the stream they run on (the handle's stream, or the fine-run stream of a
 * pipelined parareal_iterate).  kernel 0 = the per-mode stage kernel, 1 =
 * the x-pass, -1 = off.  While enabled, on every `every`-th batched fine
 * step of the working-precision fine plan each launch of that kernel is
 * bracketed by an event pair (at most 8192 pairs are kept).
 * rbc_kernel_timing synchronises, returns the mean duration in ms, the
 * number of timed launches and (if mean_batch is not NULL) the mean number
 * of states per timed launch, and clears the record. */
rbc_status rbc_kernel_timing_enable(rbc_handle h, int32_t kernel, int32_t every);
rbc_status rbc_kernel_timing(rbc_handle h, double* mean_ms, int64_t* count, double* mean_batch);

/* Wait for all work enqueued on the handle's stream. */
rbc_status rbc_synchronize(rbc_handle h);

#ifdef __cplusplus
}
#endif
#endif /* RBC_H */
