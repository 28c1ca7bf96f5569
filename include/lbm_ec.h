/*
 * lbm_ec.h -- C ABI of the MI355X (gfx950) electroconvection time step.
 *
 * The library advances the segregated electroconvection model of Guan &
 * Novosselov, "Two Relaxation Time Lattice Boltzmann Method Coupled to Fast
 * Fourier Transform Poisson Solver" (arXiv:1812.05711):
 *   - two D2Q9 two-relaxation-time lattices, one for the fluid with the
 *     electric body force -rho_c grad(phi) (section IV.2, Eq. 5, 7, 8, 10,
 *     12, 13, 15-17) and one for the charge density with the drift velocity
 *     u - mu_b grad(phi) (Eq. 6, 9, 11, 14, 16-17);
 *   - coupled every step to a Poisson solve for phi (Eq. 4, 18-25): a DFT
 *     along the periodic x direction, then one tridiagonal solve in y per
 *     wavenumber with the electrode potentials as Dirichlet values;
 *   - electrode and wall conditions of Table I (periodic in x; halfway
 *     bounce-back of f at both electrodes; rho_c = rho0 at the injector by
 *     anti-bounce-back of g; zero normal gradient of g at the collector).
 * The governing groups are those of Eq. 26 (M, T, C, Fe).
 *
 * Conventions shared by every entry point
 *   - Lattice units: dx = dy = dt = 1, electrode gap H = ny, potential drop
 *     1 (phi = 1 at the injector y = 0, phi = 0 at the collector y = ny),
 *     fluid density about 1.  Nodes sit at y = j + 1/2, j = 0 .. ny-1, and
 *     x = 0 .. nx-1 (periodic).
 *   - All device memory is owned by the caller (allocate it with any
 *     allocator, e.g. PyTorch); the library never allocates or frees device
 *     memory.  A handle owns only host memory.
 *   - Work is enqueued asynchronously on the caller's HIP stream given at
 *     creation; the calls that wait for the stream say so (lbm_ec_create,
 *     lbm_ec_stats, the checkpoint calls and some batch calls).
 *   - Every int-returning call returns LBM_EC_OK (0) or an error code and
 *     leaves a message for lbm_ec_last_error() (thread-local).
 *   - Calls on one handle must not run concurrently from several threads.
 */
#ifndef LBM_EC_H
#define LBM_EC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
enum {
  LBM_EC_OK = 0,
  LBM_EC_EINVAL = 1,   /* invalid argument or parameter set */
  LBM_EC_ENOMEM = 2,   /* workspace smaller than lbm_ec_workspace_bytes() */
  LBM_EC_EHIP = 3,     /* a HIP runtime call or kernel launch failed */
  LBM_EC_EUNSTABLE = 4,/* the health check found non-finite or negative density */
  LBM_EC_EBUSY = 5     /* no free slot or budget (batch API) */
};

/* storage precision of the populations */
enum {
  LBM_EC_FP64 = 0,     /* FP64 storage and arithmetic everywhere */
  LBM_EC_FP32_DEV = 1, /* FP32 deviations from the hydrostatic reference rows;
                          FP64 for the x-mean (m = 0) Poisson mode and the
                          reductions */
  LBM_EC_FP32_DEV_F64MATH = 2 /* FP32_DEV storage and transforms, with the
                          collision arithmetic in FP64 (loads widened,
                          results rounded once to FP32 on store) */
};

/* initial state */
enum {
  LBM_EC_INIT_NOISE = 0, /* closed-form hydrostatic state (Eq. 27-28) times
                            (1 + noise_amp * xi), xi uniform on [-1, 1) from
                            SplitMix64 output k = j*nx + x, seeded with
                            seed + instance_id */
  LBM_EC_INIT_EQ29 = 1,  /* hydrostatic state plus the velocity perturbation
                            of Eq. 29 (section V.2) */
  LBM_EC_INIT_REST = 2   /* rho = 1, u = 0, no charge (flow tests) */
};

/* y solve of the x wavenumbers m >= 1 (lbm_ec_set_y_solver) */
enum {
  LBM_EC_Y_TRIDIAGONAL = 0, /* chunked tridiagonal systems (default) */
  LBM_EC_Y_SPECTRAL = 1     /* odd extension and transform in y (Eq. 21-25) */
};

/* which TRT rate of the charge lattice carries the diffusivity D_c */
enum {
  LBM_EC_RATES_ANTISYMMETRIC = 0, /* D_c = cs2 (1/w_g- - 1/2); Lambda_g sets
                                     w_g+.  Gives the charge diffusivity K/Fe. */
  LBM_EC_RATES_SYMMETRIC = 1      /* the labels printed in Eq. 16:
                                     D_c = cs2 (1/w_g+ - 1/2) */
};

/* Parameters of one simulation (Eq. 16-17, Eq. 26). */
typedef struct {
  int32_t nx, ny;       /* grid; nx >= 1, ny >= 3 */
  double T, C, M, Fe;   /* electric Rayleigh number, injection level, mobility
                           ratio, inverse charge diffusivity (Eq. 26) */
  double tau_plus;      /* fluid symmetric relaxation time (> 1/2); sets the
                           viscosity nu = (tau_plus - 1/2)/3, from which the
                           mobility K = nu T / M^2, permittivity (M K)^2,
                           injected charge C (M K)^2 / ny^2 and D_c = K / Fe */
  double Lambda;        /* fluid TRT product of Eq. 17 (> 0) */
  double Lambda_g;      /* charge TRT product of Eq. 17 (> 0) */
  int32_t precision;    /* LBM_EC_FP64, LBM_EC_FP32_DEV or LBM_EC_FP32_DEV_F64MATH */
  int32_t init_mode;    /* LBM_EC_INIT_* */
  double noise_amp;     /* relative charge noise amplitude (INIT_NOISE) */
  uint64_t seed;        /* noise generator seed */
  int32_t instance_id;  /* added to the seed */
  int32_t charge_rates; /* LBM_EC_RATES_* */
  double body_force_x;  /* uniform x body force density (flow tests; 0 otherwise) */
} lbm_ec_params;

typedef struct lbm_ec lbm_ec_t;

/* Fills *p with the defaults: 122 x 100, T = 200, C = 10, M = 10, Fe = 4000,
 * tau_plus = 0.8, Lambda = 1/4, Lambda_g = 1e-6, FP64, INIT_NOISE,
 * noise_amp = 1e-3, seed = 181205711.  Returns EINVAL if p is NULL. */
int lbm_ec_params_default(lbm_ec_params* p);

/* Checks a parameter set (see the field comments; also nx <= 8192 with the
 * x transform of a row pair fitting one workgroup's LDS at 512 threads: any
 * nx up to 8192 in FP32 storage, and in FP64 up to 8192 when nx has no prime
 * factor above 5 (in-place transforms), up to 5120 otherwise; every real
 * parameter finite; and the lattice mobility K = nu T / M^2, permittivity
 * eps = (M K)^2, injected charge rho0 = C eps / ny^2 and diffusivity
 * D_c = K / Fe finite, with K, eps and D_c positive).  Returns OK or
 * EINVAL. */
int lbm_ec_validate(const lbm_ec_params* p);

/* Device workspace bytes needed by lbm_ec_create for *p (0 if invalid). */
size_t lbm_ec_workspace_bytes(const lbm_ec_params* p);

/* Creates a simulation in the caller's device workspace d_ws (ws_bytes
 * bytes, 256-byte aligned, on the current HIP device) and enqueues the
 * initial state on hip_stream (a hipStream_t; NULL means the null stream).
 * The initial state is step 0: the pre-collision populations are set to
 * their equilibria (Eq. 10-11) for the chosen init mode -- the closed-form
 * hydrostatic charge and field of section V.1 (Eq. 27-28) with seeded
 * noise, or with the velocity perturbation of Eq. 29 (section V.2) --, the
 * Poisson problem is solved for them, and their first collision is done, as
 * the pull-streaming time loop expects.  Waits for the stream once.  The workspace must stay
 * allocated and untouched by the caller until lbm_ec_destroy.
 * Errors: EINVAL (bad parameters or NULL pointers), ENOMEM (ws_bytes too
 * small or misaligned), EHIP. */
int lbm_ec_create(const lbm_ec_params* p, void* d_ws, size_t ws_bytes,
                  void* hip_stream, lbm_ec_t** out);

/* Enqueues n >= 0 time steps (section IV: charge density, Poisson solve,
 * field, TRT collision and streaming of both lattices).  Asynchronous. */
int lbm_ec_step(lbm_ec_t* h, int64_t n);

/* Number of steps taken since creation. */
int64_t lbm_ec_steps_done(const lbm_ec_t* h);

/* Enqueues the conversion of the current state (after lbm_ec_steps_done
 * steps) into nondimensional FP64 fields, each a device array of ny*nx
 * doubles in row-major [y][x] order: the moments of the pre-collision
 * populations (rho and rho_c by Eq. 5-6, u by Eq. 7 with half the electric
 * force) and the potential of the Poisson solve (Eq. 4, 18-25), scaled by
 * the groups of Eq. 26:
 *   rho   -- fluid density (lattice units, about 1)
 *   ux,uy -- velocity in units of u0 = K / H
 *   rho_c -- charge density in units of eps / H^2 (C at the injector)
 *   phi   -- potential in units of the applied drop (1 at the injector)
 * Any pointer may be NULL to skip that field.  Asynchronous. */
int lbm_ec_fields(lbm_ec_t* h, double* rho, double* ux, double* uy,
                  double* rho_c, double* phi);

/* The density departure rho - 1 of the current state (Eq. 5: rho is the sum
 * of the fluid populations) into the device array rho_m1 of ny*nx doubles,
 * [y][x].  It is formed as (rho_ref - 1) + (rho - rho_ref) from the
 * hydrostatic reference row rho_ref(y), with no cancellation, so it keeps
 * its own relative precision; rho - 1 taken from the rho of lbm_ec_fields
 * loses about five digits (|rho - 1| is 1e-5 .. 1e-3).  EINVAL for a NULL
 * pointer.  Asynchronous. */
int lbm_ec_fields_rho_m1(lbm_ec_t* h, double* rho_m1);

/* Solves the Poisson problem of Eq. 4 and 18-25 for a given charge density:
 * d_rho_c and d_phi are device arrays of ny*nx doubles, [y][x], in the
 * nondimensional units of lbm_ec_fields.  Uses the handle's transforms and
 * scratch (it overwrites the handle's potential, so call it between steps
 * only for testing).  Asynchronous. */
int lbm_ec_poisson(lbm_ec_t* h, const double* d_rho_c, double* d_phi);

/* Size of the device scratch of lbm_ec_poisson_static (64 MiB), a static
 * array of the library that each GPU it runs on holds until the process
 * ends. */
#define LBM_EC_STATIC_SCRATCH_BYTES (64u << 20)

/* The Poisson solve of lbm_ec_poisson for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): no handle and no workspace.  It solves the problem
 * of the grid and lattice constants of *p (nx, ny, and the permittivity
 * (M K)^2 from T, M, tau_plus; reference rows as for p->init_mode) for the
 * nondimensional charge density d_rho_c and writes the potential to d_phi
 * (device arrays of ny*nx doubles, [y][x], units of lbm_ec_fields), with the
 * same kernels, tables and launch shapes as lbm_ec_poisson on an instance of
 * the same parameters, so the same result bit for bit.  Its scratch is a
 * file-scope device array of LBM_EC_STATIC_SCRATCH_BYTES, one per GPU: the
 * call allocates no device memory (the tables are copied into the scratch
 * from host memory, and the call waits for the stream once for that).  Every
 * call on a GPU shares that GPU's scratch and leaves its contents behind
 * (no part of the solve reads what an earlier call left); calls that overlap
 * on one GPU (other host threads, other streams) race and must be serialised
 * by the caller.  Asynchronous after the table copy, on hip_stream (NULL: the
 * null stream) of the current device.
 * Errors: EINVAL for NULL pointers, invalid parameters or a grid whose
 * scratch (lbm_ec_poisson_static_bytes) exceeds LBM_EC_STATIC_SCRATCH_BYTES;
 * EHIP. */
int lbm_ec_poisson_static(const lbm_ec_params* p, const double* d_rho_c, double* d_phi, void* hip_stream);

/* Scratch bytes lbm_ec_poisson_static needs for *p (0 if p is invalid). */
size_t lbm_ec_poisson_static_bytes(const lbm_ec_params* p);

/* Global diagnostics of the current state, computed in FP64 on the device
 * and copied to host memory out[10] (waits for the stream):
 *   out[0] steps done, out[1] sum of (rho - 1) over nodes, out[2] sum of
 *   rho_c (lattice units), out[3] rms of u_y (lattice units), out[4] max of
 *   |u| (lattice units), out[5] min rho_c, out[6] number of non-finite or
 *   non-positive-density nodes, out[7] max |E_x| (lattice units),
 *   out[8] charge the next streaming brings in through the injector and
 *   out[9] net charge it brings in through the collector (negative: the
 *   collector current), both summed over x in lattice units, from the
 *   post-collision populations and the electrode rules of Table I (their
 *   sum is the change of the total charge over that streaming).
 * Returns EUNSTABLE (after filling out) if out[6] > 0. */
int lbm_ec_stats(lbm_ec_t* h, double* out);

/* Checkpoint and restart (continuing a run, or branching several runs off
 * one state).  A checkpoint holds the post-collision populations and every
 * array lbm_ec_fields reads, in a device buffer of lbm_ec_checkpoint_bytes(h)
 * bytes owned by the caller (any device memory, e.g. a torch uint8 tensor).
 *   lbm_ec_save copies the instance's state into d_dst (ENOMEM if bytes is
 *   smaller than needed); it waits for the stream.
 *   lbm_ec_load replaces the instance's state with the checkpoint in d_src,
 *   including its step count; EINVAL unless the checkpoint was taken with the
 *   same grid, precision, charge-rate reading, physical parameters (T, C,
 *   M, Fe, tau_plus, Lambda, Lambda_g, body force) and reference rows (the
 *   stored populations are deviations from rows that are zero for an
 *   INIT_REST start and the closed-form hydrostatic rows otherwise).  Stepping a loaded
 *   instance gives bit for bit the results the saved one would have given.
 *   It waits for the stream to read the header, then copies asynchronously.
 * Checkpoints are not portable between library versions. */
size_t lbm_ec_checkpoint_bytes(const lbm_ec_t* h);
int lbm_ec_save(lbm_ec_t* h, void* d_dst, size_t bytes);
int lbm_ec_load(lbm_ec_t* h, const void* d_src, size_t bytes);

/* Continuation at another electric Rayleigh number T (section V.2: T is
 * lowered after the vortices have formed, and they persist down to T_f).  The
 * change takes effect between the last collision and the next streaming; what
 * carries over, where the paper does not say: the charge keeps its
 * nondimensional value (the post-collision charge populations, in full, are
 * scaled by eps_new / eps_old, eps = (M K)^2 the lattice permittivity, so
 * rho_c / rho0 and E are continuous), and the fluid populations keep their
 * departure from the hydrostatic state of the lattice (the stored deviations
 * are unchanged; the reference density row and the reference force become
 * those of the new T).  K, eps, rho0, D_c, the charge rates and the injector
 * constants are those of T from the next step on; the step count is kept.
 * The moments that lbm_ec_fields reads are re-expressed in the new units
 * (charge scaled; density deviation and velocity in lattice units kept).
 * Waits for the stream.  EINVAL for a T that lbm_ec_validate refuses (the
 * instance is then unchanged).  A checkpoint records T: lbm_ec_load refuses
 * one taken at another T. */
int lbm_ec_set_T(lbm_ec_t* h, double T);

/* Chooses how the Poisson solve of an instance treats the y direction of the
 * x wavenumbers m >= 1 (the x-mean mode is always solved in FP64 flux form):
 * LBM_EC_Y_TRIDIAGONAL (default) solves one tridiagonal system per m in
 * 32-row chunks with an interface system; LBM_EC_Y_SPECTRAL takes the
 * paper's route of Eq. 21-25: each column of the spectrum is extended oddly
 * about the half-cell electrode positions to length 2 ny, transformed in y,
 * divided by the symbol -(kappa_m^2 + 4 sin^2(pi k / (2 ny))) and
 * transformed back.  Both invert the same discrete operator, so they agree
 * to rounding.  The spectral route holds two columns of 2 ny complex values
 * in LDS: EINVAL when that exceeds 160 KiB (ny > 2560 in FP64 storage,
 * ny > 5120 in FP32).  Applies to lbm_ec_step and lbm_ec_poisson from the
 * next call on; batches always use the tridiagonal solve.  Waits for the
 * stream. */
int lbm_ec_set_y_solver(lbm_ec_t* h, int32_t solver);

/* Kernel timing for measurement.  lbm_ec_profile_begin starts recording a
 * HIP event pair around every kernel of the classes whose bit is set in
 * class_mask (bit k for class k) that the handle enqueues on its stream;
 * lbm_ec_profile_end stops, waits for the stream and returns, per kernel
 * class, the summed elapsed milliseconds and the launch count in ms[k] and
 * launches[k] for k < n.  Classes: 0 forward transform (with the tile edges
 * of the charge density and the FP64 row sums), 1 y solves of the m >= 1
 * modes (chunk solves and interface system), 2 inverse transform (with the
 * x-mean mode), 3 collide-stream.  Each event pair adds a few microseconds
 * to the step (the events carry no system-scope fence), so time only the
 * classes needed.  The events are created on first use and kept by the
 * handle (host-side driver objects, no device memory). */
int lbm_ec_profile_begin(lbm_ec_t* h, uint32_t class_mask);
int lbm_ec_profile_end(lbm_ec_t* h, double* ms, int64_t* launches, int32_t n);

/* Launch shapes, which never change results: threads per x-transform block
 * (64, 128, 256 or 512; EINVAL when a row pair's transform would then need
 * more than 160 KiB of LDS), threads per collide tile (collide_bx *
 * collide_by, a multiple of 64 up to 1024) and columns per collide tile
 * (collide_tw, 1 .. 1024, or 0 for the default: whole rows while ten rows
 * of them fit 160 KiB of LDS -- nx <= 4096 in FP32 storage, 2048 in FP64 --
 * and 1024-column tiles beyond).  A collide tile is a band of rows whose
 * height depends on ny only, and of collide_tw columns; a tile narrower than
 * the row also collides the two columns next to it (without storing them),
 * so every node's charge sum is formed from the same values in the same
 * order whatever the width.  Defaults: about nx / 8 transform threads
 * (64 .. 512) and nx rounded up to 64 collide threads (at most 1024) for a
 * single instance; 256 and 256 x 1 for a batch.  Applies to the following
 * steps; EINVAL for other values.  The autotuner in
 * paper_1812_05711_amd/autotune.py picks them by timing. */
int lbm_ec_set_tuning(lbm_ec_t* h, int32_t fft_threads, int32_t collide_bx, int32_t collide_by,
                      int32_t collide_tw);

/* Releases the handle (host memory only; the caller frees the workspace). */
void lbm_ec_destroy(lbm_ec_t* h);

/* ---------------------------------------------------------------- batches
 * Many independent simulations of possibly different sizes and parameters
 * advanced together: one launch per kernel type covers every live slot, the
 * step state (current buffer, step count, target) lives on the device, and
 * each advance is replayed from captured HIP graphs (rebuilt only when the
 * slot set changes).  Every slot computes exactly what it would compute
 * alone through lbm_ec_step (same kernels, same arithmetic order).  All
 * slots of a batch share one precision.  Slots are reusable, so a batch can
 * serve requests as they arrive (admit while others run, poll, release).
 *
 * Device memory: the caller provides one workspace; the batch keeps its
 * descriptor tables and per-slot diagnostics histories at its start and
 * places each admitted simulation in the remaining space (first fit). */
typedef struct lbm_ec_batch lbm_ec_batch_t;

/* Workspace bytes for a batch of max_slots slots with hist_rows history rows
 * per slot that can hold the n simulations ps[0..n-1] at once (n may be 0 to
 * get the size of the tables alone).  0 if an argument is invalid. */
size_t lbm_ec_batch_workspace_bytes(const lbm_ec_params* ps, int32_t n, int32_t max_slots, int32_t hist_rows);

/* Creates an empty batch in the caller's workspace (256-byte aligned).
 * precision: one of LBM_EC_FP64 / FP32_DEV / FP32_DEV_F64MATH for all slots.
 * emit_every: every emit_every steps (0 = never) and at its last step each
 * slot writes its moments and a history row {step, rms u_y, max |u|, sum of
 * rho_c, A1, unhealthy, I} (lattice units), A1 the largest over the rows of
 * |sum_x u_y(x) exp(-2 pi i x / nx)| / nx: the amplitude of the first x mode
 * of u_y, whose growth or decay in time locates the electroconvective
 * threshold (the linear stability test of section V); unhealthy the number
 * of nodes with non-finite moments or rho <= 0 (the health check of
 * lbm_ec_stats, per slot); I the collector current, the charge that the next
 * streaming takes out through the upper electrode (-out[9] of lbm_ec_stats),
 * the cathode current of the electric Nusselt number Ne_0 = I / I_0 of
 * section V.2.  hip_stream: stream for all batch work; NULL makes
 * the batch create its own (graphs cannot be captured on the null stream).
 * Errors: EINVAL, ENOMEM, EHIP. */
int lbm_ec_batch_create(int32_t max_slots, int32_t precision, int32_t emit_every, int32_t hist_rows, void* d_ws,
                        size_t ws_bytes, void* hip_stream, lbm_ec_batch_t** out);

/* Admits one simulation that will run n_steps steps: finds a free slot and a
 * free region of the workspace, builds and initialises it (as lbm_ec_create;
 * waits for the stream) and stores its slot index in *slot.  Returns EBUSY
 * when no slot or no large enough region is free (nothing changes). */
int lbm_ec_batch_admit(lbm_ec_batch_t* b, const lbm_ec_params* p, int64_t n_steps, int32_t* slot);

/* Enqueues n steps of the batch: every admitted slot advances by n steps or
 * until it reaches its n_steps, whichever comes first.  Asynchronous. */
int lbm_ec_batch_step(lbm_ec_batch_t* b, int64_t n);

/* Waits for the stream and stores in done_slots[0..cap-1] the slots that
 * have reached their step count since the last poll; *n_done = count. */
int lbm_ec_batch_poll(lbm_ec_batch_t* b, int32_t* done_slots, int32_t cap, int32_t* n_done);

/* Steps taken by a slot (waits for the stream); -1 for a free slot. */
int64_t lbm_ec_batch_steps_done(lbm_ec_batch_t* b, int32_t slot);

/* As lbm_ec_fields, for the state at the slot's last emitted step (its final
 * step once it is done).  Asynchronous. */
int lbm_ec_batch_fields(lbm_ec_batch_t* b, int32_t slot, double* rho, double* ux, double* uy, double* rho_c,
                        double* phi);

/* As lbm_ec_fields_rho_m1, for the slot's last emitted step.  Asynchronous. */
int lbm_ec_batch_fields_rho_m1(lbm_ec_batch_t* b, int32_t slot, double* rho_m1);

/* Copies the first `rows` history rows of a slot (7 doubles each, host
 * memory); waits for the stream.  Row r holds step (r+1) * emit_every, the
 * last row the final step when that is not a multiple of emit_every; unused
 * rows are zero. */
int lbm_ec_batch_history(lbm_ec_batch_t* b, int32_t slot, double* out, int32_t rows);

/* lbm_ec_set_T for one slot of a batch, at the step the slot has reached
 * (waits for the stream).  The slot keeps its step count and target; the
 * batch re-captures its graphs at the next step. */
int lbm_ec_batch_set_T(lbm_ec_batch_t* b, int32_t slot, double T);

/* Launch shapes for the batch's kernels (as lbm_ec_set_tuning); the graphs
 * are re-captured at the next step, which returns EINVAL if a slot's
 * transform does not fit LDS with these shapes. */
int lbm_ec_batch_set_tuning(lbm_ec_batch_t* b, int32_t fft_threads, int32_t collide_bx, int32_t collide_by,
                            int32_t collide_tw);

/* Frees a slot and its workspace region (waits for the stream). */
int lbm_ec_batch_release(lbm_ec_batch_t* b, int32_t slot);

/* Largest free contiguous region of the batch workspace, bytes. */
size_t lbm_ec_batch_free_bytes(lbm_ec_batch_t* b);

/* Releases the batch (waits for its stream; the caller frees the workspace). */
void lbm_ec_batch_destroy(lbm_ec_batch_t* b);

/* Test hooks of the failure detection, for callers that test it: a NaN is
 * written into one population of the current state of an instance (or of a
 * batch slot), so that its next steps fail the health check while other
 * instances and slots are unaffected.  Wait for the stream.  EINVAL for a
 * NULL handle or a free slot. */
int lbm_ec_debug_poison(lbm_ec_t* h);
int lbm_ec_batch_debug_poison(lbm_ec_batch_t* b, int32_t slot);

/* Message of the last error on this thread ("" if none). */
const char* lbm_ec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_EC_H */
