/*
 * rte.h -- C-ABI of the MI355X pseudospectral P_N radiative-transport stepper.
 *
 * Method: S. Powell, B. T. Cox, S. R. Arridge, "A pseudospectral method for
 * solution of the radiative transport equation" (arXiv:1801.06364).
 *
 *  - Radiance and source are expanded in spherical harmonics with weights
 *    sqrt((2l+1)/4pi) (Sec. II, eqs. 3-4). This library stores REAL
 *    harmonics (no Condon-Shortley phase) with those same weights, so moment
 *    a = l*l + l + m holds psi_{l,m}; psi_{0,0} is the fluence and
 *    (psi_{1,1}, psi_{1,-1}, psi_{1,0}) is the flux vector (Jx, Jy, Jz).
 *  - Streaming couples degree l to l+-1 (eq. 6); it is applied spectrally
 *    (Sec. II, eqs. 7-10) on a periodic grid with k = 2 pi f / (n dx) and the
 *    Nyquist wavenumber set to zero.
 *  - Loss and in-scatter are pointwise: Sigma_l = mu_a + mu_s (1 - g^l) in
 *    the real domain (eqs. 5-6); in the absorbing boundary layer (eq. 12)
 *    scattering and source are switched off and Sigma_l = mu_b, a half-cosine
 *    profile rising from pml_mu0 at the real-domain edge to pml_mu1 at the
 *    grid edge (Sec. II.B, Sec. III.B).
 *  - Time integration is the classic four-stage Runge-Kutta method applied
 *    to d psi/dt = c (-[s.grad psi] - Sigma_l psi + q) (the sign form that
 *    eqs. 1 and 6 give), evaluated in the equivalent nested form
 *    v <- u + dt/4 f(u); v <- u + dt/3 f(v); v <- u + dt/2 f(v);
 *    u <- u + dt f(v), exact for this autonomous affine right-hand side
 *    (a time-dependent source gives each stage its own source weight, see
 *    rte_set_source_profile); or, on request, the paper's first-order
 *    explicit step (eq. 11).
 *
 * Grid: n^3 voxels, voxel (z, y, x) at r = (x, y, z) * dx; every field is
 * stored [z][y][x] with x fastest; moment fields are [a][z][y][x]. The real
 * domain is [W, n-W)^3 with W = pml_width.
 *
 * Memory: the library never allocates device memory. The caller passes one
 * device workspace of at least rte_workspace_bytes() bytes (256-byte
 * aligned) that must outlive the handle. Host arrays passed in are read
 * during the call and not retained. All work is queued on the caller's HIP
 * stream; calls that return host data synchronise that stream.
 *
 * Errors: every int-returning call returns RTE_OK (0) or a negative code;
 * no exception crosses this boundary. A handle is not thread-safe; distinct
 * handles are independent.
 */
#ifndef RTE_H
#define RTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RTE_OK = 0,
  RTE_EINVAL = -1,     /* bad argument or unsupported configuration         */
  RTE_ENOMEM = -2,     /* workspace too small or misaligned                 */
  RTE_EUNSTABLE = -3,  /* non-finite fluence or runaway growth detected     */
  RTE_EDEVICE = -4     /* a HIP call failed                                 */
};

enum { RTE_FP32 = 0, RTE_FP64 = 1 };
enum { RTE_RK4 = 0, RTE_EULER = 1 };
enum { RTE_FLUENCE_NOW = 0, RTE_FLUENCE_INTEGRATED = 1 };

typedef struct rte_handle rte_handle;

typedef struct {
  int32_t n;               /* points per axis: 16, 32, 48, 64, 96, 128, 256   */
  int32_t order_N;         /* P_N order, 0 <= N <= 7; M = (N+1)^2 moments     */
  int32_t precision;       /* RTE_FP32 or RTE_FP64 for state, FFTs, stages;
                              tables are computed in FP64 and rounded once;
                              the integrated fluence is always FP64          */
  int32_t pml_width;       /* W, absorbing-layer voxels on every face,
                              0 <= W < n/2 (0: fully periodic, no layer)     */
  double dx_mm;            /* grid spacing (mm), > 0                          */
  double c_mm_ps;          /* speed of light in the medium (mm/ps), > 0       */
  double dt_ps;            /* time step (ps); <= 0 selects 0.2 * dx / c       */
  double pml_mu0;          /* layer attenuation at the real-domain edge       */
  double pml_mu1;          /* layer attenuation at the grid edge (mm^-1)      */
  int32_t n_det;           /* number of detector voxels (>= 0)                */
  int32_t scheme;          /* RTE_RK4 (classic four-stage, default) or
                              RTE_EULER (the first-order explicit step of
                              eq. 11: u <- u + dt f(u), one stage per step)  */
  const int64_t* det_index;/* n_det distinct linear voxel indices (z*n+y)*n+x,
                              host, copied at create                         */
  int64_t record_steps;    /* capacity of the per-step record (readings,
                              residuals); later steps run unrecorded         */
} rte_config;

typedef struct {           /* host arrays, FP64, read during rte_create only   */
  const double* mu_a;      /* n^3 absorption (mm^-1), >= 0                     */
  const double* mu_s;      /* n^3 scattering (mm^-1), >= 0                     */
  const double* g;         /* n^3 HG anisotropy, -1 < g < 1                    */
  const double* psi0;      /* psi0_moments*n^3 initial real-basis moments
                              (moments a < psi0_moments; the rest are 0), or
                              NULL for an all-zero initial state             */
  const double* q;         /* q_moments*n^3 time-constant source moments, or
                              NULL; zeroed inside the absorbing layer (eq. 12) */
  int32_t psi0_moments;    /* leading moments given in psi0; 0 means all M    */
  int32_t q_moments;       /* leading moments given in q; 0 means all M       */
} rte_medium;

/* Bytes of device workspace a configuration needs (0 if it is invalid). */
size_t rte_workspace_bytes(const rte_config* cfg);

/* Validate, build the FP64 tables (streaming coefficients of eq. 6 in the
 * real basis, twiddles, wavenumbers, per-degree losses with the absorbing
 * layer of eq. 12), carve the workspace and upload the medium and state.
 * The problem statement is that of Sec. II: medium (eqs. 1-2, 5), source
 * and initial radiance as moments (eqs. 3-4), order N of the truncation
 * (Sec. II.A), real domain inside the computational domain with an
 * absorbing layer (Sec. II.B, eq. 12). hip_stream is a hipStream_t (NULL =
 * the default stream). On success *out receives a handle owned by the
 * library until rte_destroy. RTE_EINVAL for an invalid configuration or
 * medium, a detector index outside the grid or one listed twice;
 * RTE_ENOMEM for a missing, misaligned or too small workspace; nothing is
 * written to the device before these checks pass. */
int rte_create(const rte_config* cfg, const rte_medium* med, void* dev_ws,
               size_t ws_bytes, void* hip_stream, rte_handle** out);

/* Queue nsteps >= 0 full time steps (asynchronous): the transient
 * solution of Sec. II.A (the paper's first-order step is eq. 11; the
 * operator of each stage is the three-part application of Sec. III). After
 * each step the fluence psi_{0,0} at the detectors (time-resolved readings,
 * as with the TCSPC measurements of Sec. II.A), the FP64 time-integrated
 * fluence (+= dt * psi_{0,0}) and the relative fluence change
 * ||phi_n - phi_{n-1}||_2 / ||phi_n||_2 are updated on the device. Once a
 * non-finite value is seen the remaining queued steps do nothing. */
int rte_step(rte_handle* h, int64_t nsteps);

/* Steady state by marching the transient solution (Sec. II.A, Sec. III.B):
 * march until the relative fluence change of a step drops below steady_tol
 * (> 0) or max_steps steps have run. The step that meets the tolerance is
 * the last one applied (later queued steps are skipped on the device).
 * *steps_taken receives the number of steps applied by this call.
 * Returns RTE_EUNSTABLE if a non-finite value or runaway growth appears. */
int rte_run(rte_handle* h, int64_t max_steps, double steady_tol,
            int64_t* steps_taken);

/* Copy the fluence psi_{0,0} (which = RTE_FLUENCE_NOW; the internal fluence
 * of Sec. III.A and III.B, the l = 0 moment of eq. 3) or the time-integrated
 * fluence (RTE_FLUENCE_INTEGRATED; the steady-state fluence of a pulse by
 * time integration, Sec. II.A) to a caller-owned FP64 host buffer of
 * len >= n^3 elements. Synchronises the stream. */
int rte_fluence(rte_handle* h, int which, double* out, size_t len);

/* Copy min(steps recorded, len / n_det) rows of detector readings
 * [step][det] (FP64; fluence at the detector voxels after each step, the
 * time-domain measurements of Sec. II.A) into out; *rows receives the row
 * count. */
int rte_readings(rte_handle* h, double* out, size_t len, int64_t* rows);

/* Copy the per-step relative fluence change (FP64; the convergence measure
 * of the marched steady state, Sec. II.A) into out (len entries max); *rows
 * receives the number written. */
int rte_residuals(rte_handle* h, double* out, size_t len, int64_t* rows);

/* Steps applied since creation (synchronises the stream). */
int rte_steps_done(rte_handle* h, int64_t* steps);

/* Read or overwrite the full real-basis moment state u (M*n^3, FP64 on the
 * host, converted to/from the working precision): the truncated moment
 * vector psi_{l,m}, l <= N, of Sec. II.A. rte_set_state starts a new run
 * from that state: it resets the step count, the record and the integrated
 * fluence, and derives the runaway-growth threshold from the new state. */
int rte_get_state(rte_handle* h, double* out, size_t len);
int rte_set_state(rte_handle* h, const double* in, size_t len);

/* Checkpoint / resume of a run (the transient solution of Sec. II.A).
 * rte_snapshot_bytes: host bytes of a snapshot of this handle (0 for NULL).
 * rte_snapshot: copy into the caller's host buffer (len >= that size) the
 * state u in the working precision (bitwise), the step count, the FP64
 * integrated fluence, the whole record of readings and residuals and the
 * run flags. Synchronises the stream.
 * rte_restore: load such a snapshot into a handle created with the same
 * configuration, detectors, maps and source (checked by a hash stored in
 * the snapshot; RTE_EINVAL on mismatch, short or corrupt input). Stepping
 * on afterwards gives bitwise the results of the uninterrupted run.
 * Synchronises the stream. */
size_t rte_snapshot_bytes(const rte_handle* h);
int rte_snapshot(rte_handle* h, void* out, size_t len);
int rte_restore(rte_handle* h, const void* in, size_t len);

/* Dense real-basis streaming matrices B_x, B_y, B_z (each M*M, row-major,
 * FP64) exactly as the library tabulates them from eq. (6). Host only, no
 * device needed. */
int rte_coupling_dense(int32_t order_N, double* bx, double* by, double* bz);

/* ---- Discrete adjoint (gradients of detector readings) ----------------
 * The derivative of a scalar loss J(readings) with respect to mu_a(r) and
 * mu_s(r) through the exact transpose of the nested RK4 step (reverse mode
 * of the discrete scheme), with the stage states recomputed from
 * checkpoints of u kept every `every` steps (sqrt(steps) balances memory
 * and recomputation). Inside the absorbing layer the loss does not depend
 * on mu_a, mu_s (eq. 12) and the gradient is zero there.
 *
 * rte_adjoint_workspace_bytes: device bytes of the second workspace the two
 * calls below share (ceil(steps/every) + every + 7 states plus FP64 maps).
 *
 * rte_forward_checkpointed: like rte_step(h, steps) from the current state,
 * additionally saving u every `every` steps into adj_ws (caller-owned,
 * 256-byte aligned). Readings are recorded as by rte_step.
 *
 * rte_adjoint: with dj_dr = dJ/d(reading) as a host FP64 array
 * [steps][n_det] for the readings of that forward run, writes dJ/dmu_a and
 * dJ/dmu_s (host FP64, n^3 each). Uses the checkpoints in adj_ws; leaves the
 * handle's state, step count and record unchanged. Synchronises. */
size_t rte_adjoint_workspace_bytes(const rte_config* cfg, int64_t steps, int64_t every);
int rte_forward_checkpointed(rte_handle* h, int64_t steps, int64_t every, void* adj_ws,
                             size_t adj_bytes);
int rte_adjoint(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes,
                const double* dj_dr, double* grad_mu_a, double* grad_mu_s);

/* ---- Device-resident inputs and outputs (gradient loops) --------------
 * For repeated forward / adjoint solves with changing mu_a, mu_s (fitting
 * the optical maps, eqs. 1-2 and 12, through torch.autograd) without host
 * copies of maps, readings or gradients. All pointers below are device
 * pointers (8-byte aligned, FP64, caller-owned; read or written during the
 * call only). RTE_EINVAL for null or misaligned pointers; values are not
 * checked on the host (they must be what rte_create would accept).
 *
 * rte_set_medium_device: replace mu_a and mu_s (n^3 each) and rebuild the
 * per-degree loss mu_a + mu_s (1 - g^l) inside the real domain on the
 * device (same arithmetic as at creation; g and the absorbing layer are
 * kept). The state and run bookkeeping are unchanged; exact propagation is
 * no longer available on the handle, and snapshots taken before no longer
 * restore into it. Synchronises.
 *
 * rte_set_state_device: as rte_set_state from `moments` leading FP64
 * moments [moments][n^3] (0 <= moments <= M; the rest set to 0); the
 * growth threshold is recomputed on the device from the new state.
 * Synchronises.
 *
 * rte_readings_device: as rte_readings into a device buffer.
 *
 * rte_adjoint_device: as rte_adjoint with dj_dr [steps][n_det] and the two
 * gradients (n^3 each) in device memory. */
int rte_set_medium_device(rte_handle* h, const double* mu_a, const double* mu_s);
int rte_set_state_device(rte_handle* h, const double* psi, int32_t moments);
int rte_readings_device(rte_handle* h, double* out, size_t len, int64_t* rows);
int rte_adjoint_device(rte_handle* h, int64_t steps, int64_t every, void* adj_ws, size_t adj_bytes,
                       const double* dj_dr, double* grad_mu_a, double* grad_mu_s);

/* ---- Time-dependent sources ------------------------------------------
 * Eq. (4) lets the source depend on time. rte_set_source_profile makes the
 * handle's source q(r) s(t): s is linear between samples[i] at
 * t = i * delta_ps (t from step 0, i.e. creation or the last
 * rte_set_state) and keeps its last value after the last sample.
 * The library turns s into per-step source weights for `rows` steps and
 * copies them (FP64) into dev_table, a caller-owned device buffer of at
 * least rows * 4 * 8 bytes (RK4) or rows * 8 bytes (Euler), 8-byte aligned,
 * that must stay allocated while the profile is set. Steps at or past
 * `rows` use the last row. RK4 step r gives its four nested stages
 * (coefficients 1/4, 1/3, 1/2, 1) the weights
 * (j + 1) / h^(j + 1) int_0^h (h - tau)^j s(t_r + tau) dtau, j = 3, 2, 1, 0,
 * which makes the step reproduce the source integral of the
 * variation-of-constants formula through the L^3 term (fourth order for any
 * s; exact moments for the piecewise-linear s); Euler step r uses s(t_r).
 * samples = NULL or rows = 0 returns to a constant source. A profile is
 * refused by rte_steady_gmres and rte_expo_advance (RTE_EINVAL); the adjoint
 * uses it (the checkpointed run is taken to end at the current step).
 * RTE_EINVAL for non-finite samples or delta_ps <= 0, RTE_ENOMEM for a
 * missing, small or misaligned table. Synchronises. */
int rte_set_source_profile(rte_handle* h, const double* samples, int64_t nsamples, double delta_ps,
                           int64_t rows, void* dev_table, size_t table_bytes);

/* ---- Steady state by a Krylov solve ---------------------------------
 * Instead of marching to steady state, solve for it with a Krylov method
 * (Sec. II.A: the time-integrated form gives an operator whose steady state
 * a Krylov solver can find; Sec. IV: host-side Krylov solvers were limited
 * by transfers). Restarted GMRES with every vector on the device; each
 * Arnoldi step (two Gram-Schmidt passes, normalisation, Givens update of
 * the Hessenberg column, convergence test) runs on the device without a
 * host round trip, and the host solves the cycle's triangular system once
 * per restart (two synchronisations per cycle). Inner product: sum over
 * moments of (2l+1) x_a y_a (orthonormal-basis coefficients). The current
 * state u is the initial guess and receives the solution (read it back with
 * rte_fluence / rte_get_state). Two operators:
 *   steps_per_apply = 0: A u = q with A = S + Sigma (streaming plus
 *     per-degree loss, so that c (-A u + q) = 0);
 *   steps_per_apply = K > 0: (I - P^K) u = P_q^K(0), P one source-free time
 *     step of the handle's scheme and P_q^K(0) K steps with the source from
 *     a zero state: the steady state as the fixed point of K steps. Fast
 *     decaying modes are damped by the steps, which leaves GMRES the few
 *     slow ones.
 *
 * rte_krylov_workspace_bytes: device bytes of the GMRES workspace
 * (restart + 3 state-sized vectors), 1 <= restart <= 31.
 * rte_steady_gmres: iterate until the relative residual of the solved
 * system (weighted norm) is <= tol or max_iters Arnoldi steps; *iters and
 * *rel_residual receive the Arnoldi steps taken and the final relative
 * residual ||q - A u|| / ||q|| of the steady-state equation. Resets the
 * run bookkeeping (step count, readings, integrated fluence). */
size_t rte_krylov_workspace_bytes(const rte_config* cfg, int32_t restart);
int rte_steady_gmres(rte_handle* h, int32_t restart, int64_t max_iters, double tol, int32_t steps_per_apply,
                     void* kws, size_t kbytes, int64_t* iters, double* rel_residual);

/* ---- Steady state without device allocation ---------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of rte_steady_gmres with its Krylov workspace in a static device array of
 * the library instead of a caller buffer. rte_static_scratch_bytes() gives
 * the array's size (128 MiB); every GPU the library runs on holds one until
 * the process ends (its address is looked up once per device, at the first
 * rte_create on that device). Allocates nothing (no hipMalloc / hipFree, no
 * host heap). Arguments and results as rte_steady_gmres without kws /
 * kbytes; RTE_ENOMEM when rte_krylov_workspace_bytes(cfg, restart) exceeds
 * the array, RTE_EDEVICE if its device address could not be looked up. All
 * calls on one GPU share the array, which keeps the last call's contents
 * (a solve initialises everything it reads): calls that overlap on one GPU
 * (from several threads or streams) race, and the caller must serialise
 * them. */
size_t rte_static_scratch_bytes(void);
int rte_steady_gmres_static(rte_handle* h, int32_t restart, int64_t max_iters, double tol,
                            int32_t steps_per_apply, int64_t* iters, double* rel_residual);

/* ---- Exact propagation in homogeneous media --------------------------
 * The paper integrates the time-domain form analytically to obtain an
 * implicit operator (Sec. II.A) and reports exponential integrators that
 * take arbitrary time steps in homogeneous media (Sec. IV). In a
 * homogeneous medium on the periodic grid (no boundary layer) every Fourier
 * mode of the moment vector evolves independently,
 *   da/dt = M(k) a + c q(k),   M(k) = -c (i k.B + Sigma),
 * so the state after a time T is exp(T M) a + int_0^T exp(s M) ds c q per
 * mode, with no time-step error and no stability limit on T.
 *
 * rte_expo_advance: advance the handle's state by t_ps picoseconds this way
 * (t_ps >= 0; 0 is a no-op). Per spectral point the exponential is a
 * truncated Taylor series in substeps whose remainder is bounded below the
 * working precision's unit roundoff (2^-24 FP32, 2^-53 FP64). Requires a
 * handle created with constant mu_a, mu_s, g and pml_width 0 (else
 * RTE_EINVAL); refuses a t_ps so large that a spectral point would need more
 * than 10^6 substeps (RTE_EINVAL: split it into shorter advances) and a
 * handle whose run was flagged unstable (RTE_EUNSTABLE). Leaves the step
 * count, readings and integrated fluence unchanged; clears a converged
 * run's stop flag. Uses the handle's spectrum buffers; synchronises. */
int rte_expo_advance(rte_handle* h, double t_ps);

/* Run nsteps steps with plain launches, timing every kernel with HIP
 * events on the handle's stream, and store the summed milliseconds of each
 * kernel class in ms[0..12] and the launch counts in counts[0..12]. Classes:
 * 0 forward plane pass, 1 z-derivative pass, 2 moment coupling pass,
 * 3 inverse plane pass with epilogue, 4 end-of-step bookkeeping; on grids
 * split into row and pencil passes (n = 256): 5 forward row pass,
 * 6 forward y pencil pass, 7 inverse y pencil pass, 8 inverse row pass with
 * epilogue; of the exact propagation: 9 forward z pass, 10 per-point
 * propagation (frame rotations and block products, or the per-point
 * series), 11 inverse z pass, 12 block-exponential table. Synchronises the
 * stream. */
int rte_profile_kernels(rte_handle* h, int64_t nsteps, double* ms, int64_t* counts);

/* rte_expo_advance with the same per-class event timing (ms[0..12],
 * counts[0..12] as for rte_profile_kernels). */
int rte_profile_expo(rte_handle* h, double t_ps, double* ms, int64_t* counts);

/* ---- Batched serving ---------------------------------------------------
 * Many independent solves of one configuration (grid, order, precision,
 * scheme, spacing, time step, layer, detector count, record length) advance
 * together: a batch holds `slots` solves in one caller-owned workspace of
 * slots * rte_batch_slot_bytes(cfg) bytes (256-byte aligned), slot s at
 * offset s * rte_batch_slot_bytes(cfg). Every kernel of a time step is
 * launched once for all resident slots (the slot is a grid coordinate), from
 * one captured graph per number of slot rows; slots that are free, finished
 * or failed return at once. Each slot is an ordinary solve (the same
 * kernels in the same order as rte_step on a single handle, so its results
 * are bitwise those of that solve), with its own maps, source, initial state,
 * detectors and step count. Grids up to 128 points per axis, orders N <= 7.
 *
 * rte_batch_slot_bytes: device bytes of one slot (0 for an unsupported
 *   configuration).
 * rte_batch_create: hip_stream (required) is the compute stream; the
 *   library creates two more streams of its own (staging and reads) and a
 *   small pinned host ring for control-block copies. cfg->det_index is
 *   ignored (each request brings its own).
 * rte_batch_admit: stage a request into a free slot: validate and build its
 *   tables and state as rte_create does (same errors), upload them on the
 *   staging stream; det_index: cfg->n_det distinct voxel indices (NULL if
 *   n_det = 0); steps >= 1 time steps to run. May be called from another
 *   thread than the one stepping the batch. The slot starts at the next
 *   rte_batch_step.
 * rte_batch_step: start the staged slots (in stream order), then queue
 *   nsteps time steps of every running slot (a slot stops by itself after
 *   its own step count) followed by an asynchronous copy of the slot control
 *   blocks. At most 4 such chunks are in flight (the call waits for the
 *   oldest otherwise).
 * rte_batch_poll: non-blocking; from the newest chunk that has completed,
 *   status[s] (RTE_SLOT_*) and steps_done[s] for every slot (arrays of
 *   `slots` entries), and the number of queued chunks not yet completed
 *   (any of the three may be NULL).
 * rte_batch_handle: the handle of a finished or failed slot, for the
 *   read-only calls (rte_fluence, rte_readings, rte_residuals,
 *   rte_get_state, rte_steps_done, rte_snapshot; stepping calls and
 *   rte_destroy refuse or ignore it); valid until the slot is released.
 * rte_batch_release: free a finished, failed or staged slot.
 * rte_batch_destroy: synchronise, release every slot and the batch. */
enum { RTE_SLOT_FREE = 0, RTE_SLOT_STAGING = 1, RTE_SLOT_STAGED = 2, RTE_SLOT_RUNNING = 3,
       RTE_SLOT_DONE = 4, RTE_SLOT_FAILED = 5 };
typedef struct rte_batch rte_batch;
size_t rte_batch_slot_bytes(const rte_config* cfg);
int rte_batch_create(const rte_config* cfg, int32_t slots, void* dev_ws, size_t ws_bytes, void* hip_stream,
                     rte_batch** out);
int rte_batch_admit(rte_batch* b, int32_t slot, const rte_medium* med, const int64_t* det_index, int64_t steps);
int rte_batch_step(rte_batch* b, int64_t nsteps);
int rte_batch_poll(rte_batch* b, int64_t* steps_done, int32_t* status, int32_t* in_flight);
int rte_batch_handle(rte_batch* b, int32_t slot, rte_handle** out);
int rte_batch_release(rte_batch* b, int32_t slot);
void rte_batch_destroy(rte_batch* b);

/* Release the handle (and its captured graph). The workspace stays the
 * caller's. Safe on NULL. */
void rte_destroy(rte_handle* h);

/* Static description of an error code. */
const char* rte_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RTE_H */
