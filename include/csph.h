/*
 * csph.h -- C ABI of the MI355X CSPH-TVD library.
 *
 * The library advances the 3D Euler equations of an ideal gas in a static
 * external potential psi with the CSPH-TVD scheme of Khrapov, Khoperskov and
 * Khoperskov (arXiv:1912.04855): a Lagrangian predictor-corrector stage that
 * moves one particle per cell under the pressure and potential forces
 * (Sec. 2.2, Eqs. (5)-(7)), then an Eulerian stage that remaps the particles
 * onto the fixed grid with TVD-limited, offset-shifted reconstructions
 * (Eqs. (8) and (4)), with a global CFL time step.
 *
 * Conventions shared by every call:
 *  - All entry points return csph_status (0 = success).  No C++ exception
 *    crosses this interface.  On failure csph_last_error() describes the cause
 *    (thread-local text, valid until the next call on the same thread).
 *  - Host arrays are FP64, structure of arrays, x fastest:
 *      state  [5][nz][ny][nx]  CONSERVED (rho, rho u, rho v, rho w, E)
 *                              or PRIMITIVE (rho, u, v, w, p), E = rho(|u|^2/2 + eps),
 *                              p = (gamma - 1) rho eps  (Sec. 2.1)
 *      psi    [nz][ny][nx]     cell-centred potential (force f = -grad psi, Sec. 2.1)
 *    The caller owns host arrays; every copy is complete when the call returns.
 *  - Device state lives in one device allocation per simulation, either owned
 *    by the library (csph_create) or lent by the caller (csph_create_in).  The
 *    arithmetic type of the stored state and of the kernels is desc->dtype.
 *  - Work is issued on the HIP stream given at creation (NULL = the null
 *    stream).  Calls that return host data synchronise that stream.
 *  - A simulation is not thread-safe: one thread at a time per csph_sim.
 */
#ifndef CSPH_H
#define CSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t csph_status;
enum {
  CSPH_OK = 0,
  CSPH_ERR_ARG = 1,          /* invalid argument (message says which)              */
  CSPH_ERR_NOMEM = 2,        /* device allocation failed                            */
  CSPH_ERR_DEVICE = 3,       /* a HIP runtime call failed                           */
  CSPH_ERR_STATE = 4,        /* the simulation holds a sticky error; set_state clears it */
  CSPH_ERR_NONFINITE = 5,    /* a non-finite value appeared in the new state        */
  CSPH_ERR_NEG_DENSITY = 6,  /* rho < -0.01 rho_vac appeared in the new state       */
  CSPH_ERR_NO_SIGNAL = 7,    /* no non-vacuum cell: the CFL step needs dt_max > 0   */
  CSPH_ERR_BUDGET = 8,       /* a batch would exceed its device-memory budget       */
};

typedef enum { CSPH_F32 = 0, CSPH_F64 = 1 } csph_dtype;
typedef enum { CSPH_PERIODIC = 0, CSPH_OUTFLOW = 1, CSPH_INFLOW = 2, CSPH_REFLECT = 3 } csph_bc;
typedef enum { CSPH_CONSERVED = 0, CSPH_PRIMITIVE = 1 } csph_vars;
/* Eulerian-stage options (Sec. 2.2 leaves the TVD limiter and the Riemann-solver
 * style flux open; Sec. 4 lists them as options).  Slopes are limited from the
 * forward and backward differences a, b of U^n:
 *   MINMOD    0 if ab <= 0, else sign(a) min(|a|, |b|)              (default)
 *   MC        0 if ab <= 0, else sign(a) min(2|a|, 2|b|, (|a|+|b|)/2)
 *   VANLEER   0 if ab <= 0, else 2ab/(a+b)
 *   SUPERBEE  0 if ab <= 0, else sign(a) max(min(2|a|,|b|), min(|a|,2|b|))
 * Face flux (times dt) from the reconstructed states U^L, U^R and the particle
 * offsets xi_L, xi_R along the face normal:
 *   SWEPT     max(xi_L,0) U^L + min(xi_R,0) U^R (HLL with the advective speeds)
 *   LF        (xi_L U^L + xi_R U^R)/2 - max(|xi_L|,|xi_R|)(U^R - U^L)/2
 *   SWEPT_AV  SWEPT plus the acoustic (Rusanov) damping of the face velocity
 *             jump, which vanishes for a gas at rest and for uniform flow (default) */
typedef enum { CSPH_LIM_MINMOD = 0, CSPH_LIM_MC = 1, CSPH_LIM_VANLEER = 2, CSPH_LIM_SUPERBEE = 3 } csph_limiter;
typedef enum { CSPH_FLUX_SWEPT = 0, CSPH_FLUX_LF = 1, CSPH_FLUX_SWEPT_AV = 2 } csph_flux;

/* Grid and gas.  One spacing h on all three axes (Sec. 2.2: x_i = x_{i-1} + h,
 * likewise y and z).  nx, ny, nz >= 4; h > 0; gamma > 1; 0 < cfl <= 0.5;
 * rho_vac >= 0 (cells with rho <= rho_vac are vacuum: zero velocity, left out of
 * the CFL maximum).  The time step is dt = cfl h / max(c + |u| + |v| + |w|). */
typedef struct {
  int32_t nx, ny, nz;
  double h;
  double origin[3];
  double gamma;
  double cfl;
  double rho_vac;
  int32_t dtype;   /* csph_dtype */
} csph_grid_desc;

typedef struct csph_sim csph_sim;
typedef struct csph_batch csph_batch;

/* Device bytes one simulation needs (state, potential, stage scratch, control
 * block), for admission decisions and csph_create_in.  0 for an invalid desc. */
size_t csph_required_bytes(const csph_grid_desc* desc);

/* Create a simulation; the library allocates and owns its device memory.
 * Boundaries start PERIODIC on all faces, psi = 0, state = 0, t = 0.
 * Errors: CSPH_ERR_ARG (bad desc or NULL out), CSPH_ERR_NOMEM, CSPH_ERR_DEVICE. */
csph_status csph_create(const csph_grid_desc* desc, void* hip_stream, csph_sim** out);

/* Same, in caller-owned device memory dev_buf of `bytes` bytes (e.g. a torch
 * tensor's data pointer) that must outlive the simulation; it is not freed by
 * csph_destroy.  CSPH_ERR_ARG if bytes < csph_required_bytes(desc) or dev_buf
 * is not 256-byte aligned. */
csph_status csph_create_in(const csph_grid_desc* desc, void* hip_stream, void* dev_buf,
                           size_t bytes, csph_sim** out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc): the same as csph_create_in,
 * with the simulation in a static device array of CSPH_STATIC_BYTES that the
 * library holds on every GPU it runs on until the process ends.  The call makes
 * no device or host-heap allocation; the array is cleared (state = 0, psi = 0,
 * t = 0) as by the other create calls.  One such simulation per GPU at a time:
 * calls on two of them would race on the same memory, so a second creation
 * returns CSPH_ERR_STATE until the first is destroyed.  CSPH_ERR_ARG if
 * csph_required_bytes(desc) > CSPH_STATIC_BYTES (an FP32 cube of 112^3 cells
 * fits, an FP64 one of 81^3).  Every other call works on it as on any sim. */
#define CSPH_STATIC_BYTES ((size_t)128 << 20)
csph_status csph_create_static(const csph_grid_desc* desc, void* hip_stream, csph_sim** out);

/* Free what the library owns.  NULL is accepted.  CSPH_ERR_ARG (nothing freed)
 * while the simulation is a batch member. */
csph_status csph_destroy(csph_sim* sim);

/* Change the stream later work is issued on (NULL = null stream). */
csph_status csph_set_stream(csph_sim* sim, void* hip_stream);

/* Set the interior state from host FP64 `[5][nz][ny][nx]`.  PRIMITIVE input is
 * converted to conserved on the host in FP64 (m = rho u,
 * E = p/(gamma-1) + rho |u|^2/2), then rounded to the storage type.  Rejects
 * rho < 0 or (PRIMITIVE) p < 0 with CSPH_ERR_ARG.  Clears a sticky error. */
csph_status csph_set_state(csph_sim* sim, csph_vars vars, const double* host);

/* Large grids without a full host copy (all of the state lives in HBM; a
 * 1024^3 FP32 grid holds about 91 GB).  csph_fill_state sets every cell, ghosts
 * included, to one state (5 values in `vars`), on the device; the time is kept,
 * the sticky error bits are cleared.  csph_set_state_box and csph_get_state_box
 * write and read a box of the interior: lo = first cell (x, y, z), n = extent
 * (x, y, z), host array [5][n_z][n_y][n_x] (one 2D copy per plane and variable);
 * the rest of the state is untouched.  A write clears the sticky error bits and
 * applies from the next step (ghosts and the signal-speed maximum are formed
 * again).  CSPH_ERR_ARG for a box outside the interior, negative density or
 * pressure, non-finite values, or (for the writes) a batch member. */
csph_status csph_fill_state(csph_sim* sim, csph_vars vars, const double state[5]);
csph_status csph_set_state_box(csph_sim* sim, csph_vars vars, const int32_t lo[3], const int32_t n[3],
                               const double* host);
csph_status csph_get_state_box(const csph_sim* sim, csph_vars vars, const int32_t lo[3],
                               const int32_t n[3], double* host_out);

/* Set the cell-centred potential psi `[nz][ny][nx]`; NULL means psi = 0.  Its
 * ghost cells follow the boundary rules with inflow faces copying like outflow,
 * so set the boundaries first (or call this again after changing them). */
csph_status csph_set_potential(csph_sim* sim, const double* host_psi);

/* Boundary rule of one face: 0..5 = -x, +x, -y, +y, -z, +z.  PERIODIC must be set
 * on both faces of an axis before stepping.  inflow_prim = (rho, u, v, w, p) is
 * read only for CSPH_INFLOW (a Dirichlet state whose particles move by u dt).
 * CSPH_ERR_ARG for a bad face or kind, a batch member, or (while self-gravity is
 * on) a kind that would change the box's class: PERIODIC on an isolated box, any
 * other kind on a periodic one. */
csph_status csph_set_boundary(csph_sim* sim, int32_t face, csph_bc kind,
                              const double inflow_prim[5]);

/* One step with dt = min(CFL dt, dt_max if dt_max > 0).  dt_taken may be NULL;
 * when it is not, the call synchronises and stores the step taken.  Errors found
 * in the new state (CSPH_ERR_NONFINITE, CSPH_ERR_NEG_DENSITY, CSPH_ERR_NO_SIGNAL)
 * are reported by the next synchronising call and make the error sticky. */
csph_status csph_step(csph_sim* sim, double dt_max, double* dt_taken);

/* Step until t == t_end exactly (the last step is shortened to land on it) or
 * until max_steps steps; t_end = +inf gives a fixed step count.  The step loop
 * runs on the device; the host polls a completion flag every few steps.
 * steps_taken may be NULL.  Synchronises. */
csph_status csph_advance(csph_sim* sim, double t_end, int64_t max_steps, int64_t* steps_taken);

/* Read the interior state into caller-owned host FP64 `[5][nz][ny][nx]`. */
csph_status csph_get_state(const csph_sim* sim, csph_vars vars, double* host_out);

/* Time and step count of the current state; restore them for checkpoint/resume. */
csph_status csph_get_time(const csph_sim* sim, double* t, int64_t* nsteps);
csph_status csph_set_time(csph_sim* sim, double t, int64_t nsteps);

/* FP64 totals (mass, x/y/z momentum, energy) x h^3 of the state written by the
 * last step, summed on the device in a fixed order. */
csph_status csph_totals(const csph_sim* sim, double out[5]);

/* Intermediate fields of the last step, interior only, host FP64 `[nz][ny][nx]`:
 * which = 0..3 m*, E* (predictor, Eq. (5)); 4..6 xi* (predicted particle
 * offset); 7..10 m~, E~ (corrector, Eq. (6)); 11..13 xi^{n+1} (final particle
 * offset); 14 phi* = sqrt(2 p*) of the predicted particle, p* its pressure over
 * its predicted volume; 15 psi, the cell-centred potential of the step (with
 * self-gravity: the external potential plus the gas's own of rho^n); 16 (with
 * self-gravity only) the potential the corrector samples at r*: the external
 * one plus that of the density predicted for t^{n+1}.  The offsets are kept by
 * FP64 simulations only: the FP32 build recomputes them from rho, m^n, m* and
 * m~ where it needs them, and returns CSPH_ERR_ARG for which = 4..6 and 11..13. */
csph_status csph_get_stage(const csph_sim* sim, int32_t which, double* host_out);

const char* csph_last_error(void);

/* Kernel timing (benchmark support).  While enabled, every step records HIP
 * events around its kernels on the simulation's stream; csph_profile_read
 * synchronises and returns, per kernel group, the average duration in
 * milliseconds of one launch and the number of launches timed since enabling:
 * group 0 = stage P (predictor), 1 = stage C (corrector), 2 = stage E (Eulerian
 * update), 3 = ghost fills (three launches per step, timed together; the first
 * also starts the step), 4 = the launch that ends the step, 5 = self-gravity
 * (the Poisson solve and the ghosts of its two potentials, timed together per
 * step; no launches without self-gravity).  n is the capacity of both arrays
 * (<= 6). */
csph_status csph_profile_enable(csph_sim* sim, int32_t on);
csph_status csph_profile_read(csph_sim* sim, double* avg_ms, int64_t* launches, int32_t n);

/* Streaming reference (benchmark support, not part of the method): the average
 * time in milliseconds of one pass of a kernel that reads `reads` (1..16) and
 * writes `writes` (1..16) device arrays of `words` 4-byte words, each element
 * once, in address order, on hip_stream (NULL = the default stream), over `reps`
 * timed passes after one untimed pass.  This is the mix of HBM streams a stage
 * kernel moves, without its halos; the rate it reaches is a practical ceiling
 * for that kernel's bytes.  The arrays are allocated and freed inside the call.
 * Returns CSPH_ERR_ARG, CSPH_ERR_NOMEM or CSPH_ERR_DEVICE (no message is set). */
csph_status csph_stream_probe(int32_t reads, int32_t writes, int64_t words, int32_t reps,
                              void* hip_stream, double* ms_per_pass);

/* Choose the Eulerian-stage limiter and flux (see csph_limiter / csph_flux);
 * applies from the next step.  CSPH_ERR_ARG for unknown values or a batch
 * member.  csph_get_scheme returns the current pair (either pointer may be NULL). */
csph_status csph_set_scheme(csph_sim* sim, csph_limiter limiter, csph_flux flux);
csph_status csph_get_scheme(const csph_sim* sim, int32_t* limiter, int32_t* flux);

/* Viscosity (Sec. 4 names viscous flows as an extension of the method): a
 * uniform kinematic viscosity nu >= 0 (0, the default, is inviscid), applied in
 * the Lagrangian stage as the SPH viscous force of Morris et al. on the 27-point
 * neighbourhood, f_ij = nu (rho_i + rho_j)/2 lambda_ij (u_j - u_i) with the
 * lattice weight lambda_ij = -2 (r_ij . grad W_ij) / |r_ij|^2, and its work
 * f_ij . (u_i + u_j)/2 in the energy; momentum and energy stay conserved.  The
 * step is further limited to nu dt <= h^2/4.  Applies from the next step.
 * CSPH_ERR_ARG for a negative or non-finite nu or a batch member. */
csph_status csph_set_viscosity(csph_sim* sim, double nu);

/* Self-gravity (Sec. 4 names the gas's self-gravity as an extension of the
 * method), with gravitational constant G > 0 (0 switches it off; it is off by
 * default).  The box must be periodic (all six faces PERIODIC) or isolated (no
 * face PERIODIC).  Each step the gas's potential is computed on the device:
 *   periodic box: the solution of the 7-point discrete Poisson equation
 *     L7[psi] = 4 pi G (rho - mean rho), by a spectral solve;
 *   isolated box (gas in vacuum): the free-space potential of the cells,
 *     psi_i = -G h^3 sum_j rho_j phi(r_i - r_j), phi(d) = 1/|d| and phi(0) =
 *     C/h with C = 3 ln(2 + sqrt 3) - pi/2 (the integral of 1/|x| over a unit
 *     cube), as a convolution over the box zero-padded to power-of-two lengths
 *     >= 2 n_d per axis.
 * The potential the Lagrangian stage sees is the external one
 * (csph_set_potential, zero if none) plus it: the predictor, Eq. (5), takes the
 * potential of rho^n; the corrector, Eq. (6), which evaluates Q at the end of
 * the step, takes that of the density the continuity equation predicts for
 * t^{n+1}, rho^n - dt sum_d (m_d,i+1 - m_d,i-1) / (2h), so the step stays second
 * order in time; ghost cells of the potential follow the faces' rules.  Axis
 * lengths: periodic box, a power of two up to 4096 in FP32 and 2048 in FP64, or
 * any length up to 1024 (a direct transform, for small grids); isolated box, up
 * to 2048 in FP32 and 1024 in FP64.  Switching it on allocates the solve's
 * device memory (periodic: about 2 complex values per cell plus two fields;
 * isolated: mx my nz complex values plus two fields and the Green's function's
 * transform on (mx/2+1)(my/2+1)(mz/2+1) values, computed once in FP64 through
 * two such FP64 arrays of scratch; released when it is switched off or the sim
 * is destroyed) and, on a periodic box, takes the mean density of the current
 * state; applies from the next step.  CSPH_ERR_ARG for a negative or non-finite
 * G, a box with some but not all faces PERIODIC, an unsupported axis length, a
 * batch member or a static simulation (csph_create_static); CSPH_ERR_NOMEM if an
 * allocation fails.  While it is on, csph_set_boundary refuses a kind that
 * would change the box's class (PERIODIC on an isolated box, any other kind on a
 * periodic one) and csph_batch_add refuses the sim. */
csph_status csph_set_self_gravity(csph_sim* sim, double G);

/* Sources and sinks (Sec. 4 names non-stationary sources and sinks as an
 * extension of the method): a mass rate per cell, host FP64 `[nz][ny][nx]`
 * (mass per volume per time), copied to the device; NULL removes them.  A cell
 * with q > 0 gains gas at rest with specific internal energy eps >= 0 (rho +=
 * q dt, momentum unchanged, E += q dt eps); a cell with q < 0 loses gas at its
 * own specific values (rho += q dt, limited at zero, with m and E scaled by the
 * same factor).  The step applies half before and half after the hydrodynamic
 * step (Strang splitting), so the step stays second order; a sim with sources
 * runs the generic stage-E kernel, which applies the second half.  The caller
 * may change the rates between any two steps (the sources are non-stationary
 * that way); a call applies from the next step.  The first call allocates one
 * device field (released by NULL or by destroying the sim).  CSPH_ERR_ARG for
 * a non-finite rate, a negative or non-finite eps, a batch member or a static
 * simulation; CSPH_ERR_NOMEM if the allocation fails.  csph_batch_add refuses
 * a sim with sources. */
csph_status csph_set_source(csph_sim* sim, const double* host_q, double eps);

/* Tile depth: the stencil sweeps give each workgroup a tile of an x-y plane
 * (stages P and C of a single FP32 grid 64 x 4, otherwise 32 x 8) and march it
 * through tz planes along z.  Deeper tiles reuse more of the
 * halo they stage; shallower ones give more workgroups.  Each of the three
 * sweeps (stage P, stage C, stage E, in that order in tz[3]) has its own depth;
 * valid depths are 2..64.  A new simulation starts from a built-in rule, or from
 * the depths csph_autotune chose earlier in this process for the same device,
 * dtype and grid shape.  csph_set_tile_depth sets all three.  Not allowed on a
 * batch member (a batch sweeps every stage of a member at its stage-C depth). */
csph_status csph_set_tile_depth(csph_sim* sim, int32_t tz);
csph_status csph_set_tile_depths(csph_sim* sim, const int32_t tz[3]);
csph_status csph_get_tile_depths(const csph_sim* sim, int32_t tz[3]);

/* Autotuner: run trial_steps steps (1..1000) at each candidate depth (2, 4,
 * 8, ... up to the grid's nz) on a library-owned copy of the simulation (its
 * state, potential, boundaries and time; csph_required_bytes of extra device
 * memory while it runs), timing each stage's kernels with HIP events; keep each
 * stage's fastest depth on `sim` and remember them for the shape.  The
 * simulation itself is not advanced.  tz_out (three depths) and ms_per_step
 * (the step time at the chosen depths) may be NULL.  Synchronises. */
csph_status csph_autotune(csph_sim* sim, int32_t trial_steps, int32_t tz_out[3], double* ms_per_step);

/* ---------------- batches: many simulations advanced together ---------------
 * A batch references simulations of one dtype; it does not own them, and each
 * must outlive its membership.  Every member keeps its own dt, t and step
 * target; members of different sizes are flattened into one tile list, and one
 * launch per stage advances all of them.  hbm_budget bounds the summed
 * csph_required_bytes of the members (0 = unbounded).  Reads of a member
 * (state, time, totals, stage fields) first wait for the batch's stream.
 * While a simulation is a member, every call that would change it or free it
 * (csph_destroy, csph_set_stream, csph_set_state, csph_set_potential,
 * csph_set_boundary, csph_set_time, csph_set_scheme, csph_set_tile_depth(s),
 * csph_step, csph_advance, csph_autotune) returns CSPH_ERR_ARG and runs no
 * kernel: remove it from the batch (or destroy the batch) first. */
csph_status csph_batch_create(csph_dtype dtype, void* hip_stream, size_t hbm_budget,
                              csph_batch** out);
/* Add a member that stops after `steps` more steps or at t_end (first reached).
 * slot receives its index.  CSPH_ERR_BUDGET if the budget would be exceeded. */
csph_status csph_batch_add(csph_batch* b, csph_sim* sim, int64_t steps, double t_end,
                           int32_t* slot);
/* Advance every unfinished member by up to k steps; n_done (may be NULL)
 * receives the number of members finished so far.  Does not synchronise unless
 * n_done is non-NULL. */
csph_status csph_batch_advance(csph_batch* b, int32_t k_steps, int32_t* n_done);
/* List finished members (up to cap slots) without removing them.  Synchronises. */
csph_status csph_batch_poll(csph_batch* b, int32_t* done_slots, int32_t cap, int32_t* n);
/* Remove a member (finished or not); its slot is reused by later adds. */
csph_status csph_batch_remove(csph_batch* b, int32_t slot);
/* Autotuner for the batched launch: time trial_steps steps of the whole batch
 * with every member at each candidate tile depth, keep the fastest depth on all
 * members, and restore every member's state and time afterwards (a snapshot of
 * each member is held in extra device memory while it runs).  Synchronises. */
csph_status csph_batch_autotune(csph_batch* b, int32_t trial_steps, int32_t* tz_out,
                                double* ms_per_step);
csph_status csph_batch_destroy(csph_batch* b);

#ifdef __cplusplus
}
#endif
#endif
