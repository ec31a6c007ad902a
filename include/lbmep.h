/*
 * lbmep.h -- C ABI of the MI355X (gfx950) D3Q19 TRT lattice Boltzmann sweep
 * with an electrostatic body force and moving rigid spheres.
 *
 * Method: Bartuschat & Ruede, "A Scalable Multiphysics Algorithm for
 * Massively Parallel Direct Numerical Simulations of Electrophoresis",
 * arXiv:1708.08741.  Sec. 3.1 defines the lattice Boltzmann step (D3Q19,
 * incompressible equilibrium Eq. fequ_Incompr_SRT, TRT operator Eq. TRTOp
 * with lambda_e = -1/tau and the odd rate that fixes walls half-way, collide
 * Eq. LBMcollideStep and stream Eq. LBMstreamStep with the Luo force term
 * Eq. LBE_forcetermLuo and the velocity of Eq. modified_velocity).  Sec. 3.2
 * defines the particle coupling (obstacle cells = cells whose centre lies in
 * a particle, velocity bounce-back Eq. LBMMovWall, momentum-exchange force
 * Eq. LBMhydrodynForce and torque, equilibrium refill of uncovered cells).
 * Alg. 1's LBM block ("set velocity BCs of particles -> fused stream-collide
 * -> hydrodynamic force") is one call of lbmep_step.
 *
 * Units: lattice units, dx = dt = rho0 = 1, c_s^2 = 1/3.
 * Grid: nx*ny*nz cells, cell (x,y,z) has linear index x + nx*(y + ny*z)
 * (x fastest) and centre (x+1/2, y+1/2, z+1/2).  Per-cell vector fields are
 * SoA: component a of cell c at [a*N + c], N = nx*ny*nz.
 *
 * Conventions for every function:
 *   - returns LBMEP_OK (0) or a negative LBMEP_E* code; lbmep_last_error()
 *     gives a thread-local message for the last failure on this thread;
 *   - on an argument error (LBMEP_EINVAL) the lattice is left unchanged;
 *   - host arrays passed in are copied before the call returns; the library
 *     never keeps or frees caller memory;
 *   - on_device = 1 means the pointer is device memory on the lattice's
 *     device (e.g. a torch tensor's data_ptr); it must stay valid until the
 *     work enqueued on the lattice's stream has completed;
 *   - all device work is enqueued on the lattice's stream; lbmep_step is
 *     asynchronous, the lbmep_get_* functions synchronise the stream.
 */
#ifndef LBMEP_H
#define LBMEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBMEP_OK = 0,
    LBMEP_EINVAL = -1,    /* bad argument (sizes, NaN, null pointer, ...) */
    LBMEP_ENOMEM = -2,    /* device or host allocation failed */
    LBMEP_EDEVICE = -3,   /* a HIP call failed */
    LBMEP_ESTATE = -4,    /* call not allowed in the current state */
    LBMEP_ENONFINITE = -5,/* a global reduction found NaN/Inf populations */
    LBMEP_EBUSY = -6      /* serving: no capacity for the request now */
};

/* storage precision of the populations (compute precision in brackets) */
enum {
    LBMEP_FP64 = 0,    /* f_q stored as FP64 (FP64 collide)                  */
    LBMEP_FP32DEV = 1, /* f_q - w_q stored as FP32 (FP32 collide)            */
    LBMEP_FP16DEV = 2  /* (f_q - w_q) * 2^22 stored as FP16 (FP32 collide);
                          deviations up to 1.56e-2, i.e. |u| <~ 0.04 */
};

/* cell flags: FLUID/WALL are user input; OBST/NEAR are produced by mapping */
enum { LBMEP_FLUID = 0, LBMEP_WALL = 1, LBMEP_OBST = 2, LBMEP_NEAR = 3 };

/* element types of force / charge arrays */
enum { LBMEP_DTYPE_F64 = 0, LBMEP_DTYPE_F32 = 1 };

typedef struct lbmep_lattice lbmep_lattice; /* opaque; owns its device memory */

typedef struct {
    int32_t nx, ny, nz;      /* grid size, each >= 1 */
    int32_t periodic[3];     /* 1 = periodic axis; 0 = implicit resting
                                no-slip wall half a cell beyond the last cell */
    double nu;               /* kinematic viscosity, > 0 (Eq. kinVisc:
                                tau = 3 nu + 1/2, lambda_e = -1/tau) */
    double magic;            /* TRT parameter Lambda > 0; the paper's lambda_o
                                (walls half-way for every tau) is 3/16 */
    int32_t precision;       /* LBMEP_FP64 / LBMEP_FP32DEV / LBMEP_FP16DEV */
    int32_t move_particles;  /* 1: X_p(n) = X_p(0) + n U_p, re-mapped every
                                step; 0: fixed map, (U, W) only set the
                                surface velocity */
    int32_t device;          /* HIP device ordinal */
    int32_t reserved;        /* must be 0 */
    void *stream;            /* hipStream_t; NULL = the default stream */
} lbmep_config;

/* Message of the last failure on the calling thread ("" if none). */
const char *lbmep_last_error(void);

/* Create a lattice.  Allocates two population grids of the storage
 * precision, the flag field and the mapping fields on cfg->device.  The
 * initial state is the rest equilibrium f_q = w_q, all cells FLUID, no
 * particles, zero force.  Errors: EINVAL (non-positive sizes, nu <= 0 or not
 * finite, magic <= 0, unknown precision, reserved != 0), ENOMEM, EDEVICE. */
int lbmep_create(const lbmep_config *cfg, lbmep_lattice **out);

/* Release all device memory of L (synchronises its stream).  NULL is OK. */
int lbmep_destroy(lbmep_lattice *L);

/* Set the user flags (N bytes, LBMEP_FLUID or LBMEP_WALL per cell) and
 * re-map the particles on the new walls (walls are never obstacle cells).
 * Populations are not touched.  Errors: EINVAL (null, value not 0/1). */
int lbmep_set_flags(lbmep_lattice *L, const uint8_t *flags, int on_device);

/* Set the particle table (host arrays, n >= 0): centres X[3n], radii R[n]
 * (> 0), velocities U[3n], angular velocities W[3n] (NULL = 0).  Sets the
 * kinematic time level to 0, maps the spheres (Sec. 3.2: a cell is an
 * obstacle cell iff its centre is inside the closed ball, minimum image on
 * periodic axes, lowest index owns shared cells) and classifies NEAR cells.
 * Populations are not touched.  Errors: EINVAL (negative n, non-finite
 * values, R <= 0). */
int lbmep_set_particles(lbmep_lattice *L, int32_t n, const double *X, const double *R,
                        const double *U, const double *W);

/* Set a dense body force f_b (3*N SoA, dtype LBMEP_DTYPE_F64/F32) used at
 * fluid cells (Eq. LBE_forcetermLuo, Eq. modified_velocity).  It is kept in
 * the compute precision (FP64 for LBMEP_FP64, FP32 otherwise).  Replaces any
 * charge force.  Errors: EINVAL (null, bad dtype, non-finite values). */
int lbmep_set_force(lbmep_lattice *L, const void *fb, int dtype, int on_device);

/* Set the electric body force f_b = rho_e * E (Sec. 2: force on the ions of
 * the double layer) from a per-cell charge density rho_e (N values of dtype)
 * and a uniform field E[3].  Stored compactly (one scalar per cell) and
 * multiplied in the sweep.  Replaces any dense force.  Errors as above. */
int lbmep_set_charge_force(lbmep_lattice *L, const void *rho_e, int dtype, const double E[3],
                           int on_device);

/* Set the electric body force of the double layer computed from the EDL
 * potential psi (N values of dtype in cell order, x fastest; the library
 * keeps them in the compute precision and in its own storage order) in the
 * sweep itself (Sec. "Computing Electrostatic Forces on Fluid and
 * Particles"): at every fluid cell f_b = rho_e (E - grad psi) with the
 * Debye-Hueckel charge density rho_e = -kappa2_eps * psi (Eq. ChrgDensDHA;
 * kappa2_eps = kappa^2 eps_e in lattice units).  grad psi is the
 * w_q-weighted D3Q19 difference divided by the rest weight
 * (Eq. ElPotGradComp, dx = 1) at cells whose 18 neighbours are all fluid
 * cells inside the grid, and the central D3Q7 difference elsewhere, where
 * a neighbour that is an obstacle cell of particle p contributes zeta[p]
 * (the particle's surface potential; zeta == NULL: psi's own value there),
 * a wall cell psi's value, and a neighbour beyond a non-periodic edge the
 * cell's own value.  zeta has L's current particle count of values (host)
 * and is dropped by the next lbmep_set_particles.  Replaces any other
 * force.  Errors: EINVAL (null psi or E, bad dtype, non-finite
 * values), ENOMEM. */
int lbmep_set_potential_force(lbmep_lattice *L, const void *psi, int dtype, double kappa2_eps,
                              const double E[3], const double *zeta, int on_device);

/* Configure the solver of the Debye-Hueckel equation for the potential psi
 * held by lbmep_set_potential_force (Sec. "Finite Volume Discretization for
 * Electric Potential Equations": the seven-point finite-volume form
 * (6 + kappa2) psi_i - sum_q psi(x_i + e_q) = 0 with dx = 1 at every cell
 * that is neither a wall nor an obstacle cell).  Obstacle cells of particle
 * p are Dirichlet boundaries with the value b_p (zeta_p, or psi's value
 * there without zeta) on the shared face, walls and non-periodic edges
 * homogeneous Neumann boundaries (Sec. "Boundary Condition Handling for
 * Solver Module").  SOR in red-black order ((x+y+z) even first) with
 * relaxation omega (Sec. "Solver for Linear Elliptic PDEs with Moving
 * Boundaries"): at most max_iter iterations; with rf > 0 the L2 norm of the
 * residual (root mean square over the unknowns) is taken before the first
 * and after every check_every-th and the last iteration, and the solve stops
 * once it is below rf times the first.  With max_iter > 0, lbmep_step solves
 * on the current map before every collision (Alg. "Electrophoresis
 * Algorithm"), starting from the previous solution.  psi is updated in place
 * (compute precision); obstacle and wall cells keep their values.  Errors:
 * EINVAL (no potential set, kappa2 <= 0, omega outside (0, 2), max_iter < 0,
 * check_every < 1, an odd extent along a periodic axis). */
int lbmep_set_potential_solver(lbmep_lattice *L, double kappa2, double omega, int32_t max_iter,
                               double rf, int32_t check_every);

/* One solve now, on the current map, as configured.  iters (may be NULL):
 * iterations done; res (may be NULL): L2 norm of the initial and of the last
 * computed residual (-1 where not computed, i.e. rf <= 0).  Synchronises
 * when iters or res is given, and every 64 iterations when rf > 0.
 * Errors: EINVAL (no solver configured), EDEVICE. */
int lbmep_solve_potential(lbmep_lattice *L, int32_t *iters, double res[2]);

/* Iterations and residual norms of the last solve (as above); synchronises.
 * Errors: EINVAL (null, no solver configured). */
int lbmep_get_solver_stats(lbmep_lattice *L, int32_t *iters, double res[2]);

/* How a solve of L iterates (for labels of measurements): shape[0] = 1 for
 * the one-pass iteration (even nx, rows of at most 2048 cells), 0 for one
 * in-place launch per colour; shape[1] = rows per thread and shape[2] =
 * planes per workgroup of the one-pass iteration (of the in-place
 * half-sweep otherwise); shape[3] = wavefronts per row (one-pass) or per
 * tile along x (in-place).  Errors: EINVAL (null, no solver configured). */
int lbmep_get_solver_shape(const lbmep_lattice *L, int32_t shape[4]);

/* Copy psi (N values, FP64, cell order with x fastest) to host or device
 * memory.  Errors: EINVAL (null, no potential set), ENOMEM, EDEVICE. */
int lbmep_get_potential(lbmep_lattice *L, double *psi, int on_device);

/* Free-slip faces (Sec. "Lattice Boltzmann Method with Forcing": no-slip
 * and free-slip walls).  faces[6] for x-, x+, y-, y+, z-, z+: 1 makes the
 * implicit wall beyond that face of a non-periodic axis a specular
 * reflector at the half-way plane (a population whose source lies beyond it
 * comes from the tangential neighbour with the crossed components of its
 * direction mirrored; if that cell is a wall or obstacle cell the link
 * bounces back), 0 keeps the no-slip wall.  The potential's boundary
 * condition at faces stays homogeneous Neumann.  Errors: EINVAL (null, a
 * value not 0 / 1, a free-slip face on a periodic axis). */
int lbmep_set_free_slip(lbmep_lattice *L, const int32_t faces[6]);

/* Let the particles move under their forces instead of the prescribed
 * kinematics (Alg. "Electrophoresis Algorithm", last block; the force on a
 * particle's charge q E of Sec. "Computing Electrostatic Forces on Fluid and
 * Particles").  After the momentum exchange of every step, each sphere
 * (density rho_p, fluid density 1) is advanced by one explicit Newton-Euler
 * step without collisions: U += (F_h + q E)/m, Omega += M_h/I, X += U (the
 * new U), m = rho_p 4/3 pi R^3, I = 2/5 m R^2; F_h, M_h are the step's
 * hydrodynamic force and torque.  The new velocities act at the next step
 * (bounce-back, exchange, refill).  q: L's particle count of charges (host;
 * NULL: uncharged); E: the applied field for q E.  Needs move_particles = 1;
 * dropped by the next lbmep_set_particles.  A particle must stay below one
 * cell per step (lbmep_get_particles reports it).  Errors: EINVAL (null E,
 * not moving, rho_p <= 0, non-finite values), ENOMEM. */
int lbmep_set_dynamics(lbmep_lattice *L, double rho_p, const double *q, const double E[3]);

/* Current positions, velocities and angular velocities of the particles
 * (host arrays of 3 n doubles each; synchronises).  Errors: EINVAL (null
 * with n > 0; a velocity component reached one cell per step under
 * dynamics, i.e. the mapping no longer follows the body), EDEVICE. */
int lbmep_get_particles(lbmep_lattice *L, double *X, double *U, double *W);

/* Set every population to the incompressible equilibrium f^eq(rho, u)
 * (Eq. fequ_Incompr_SRT).  Errors: EINVAL (non-finite). */
int lbmep_init_equilibrium(lbmep_lattice *L, double rho, const double u[3]);

/* Overwrite / read the populations as absolute FP64 values f[q*N + c] in
 * the D3Q19 order q=0 rest, 1..6 = +x,-x,+y,-y,+z,-z, 7..18 = (+x+y),
 * (-x-y), (+x-y), (-x+y), (+x+z), (-x-z), (+x-z), (-x+z), (+y+z), (-y-z),
 * (+y-z), (-y+z).  Reduced-precision lattices convert to / from their
 * storage (rounding).  The state is post-stream, pre-collide.  After a step,
 * solid cells read as the rest state (walls) or f^eq(rho0, u_s) of their
 * particle (obstacle cells); their values never enter the fluid update. */
int lbmep_set_pdfs(lbmep_lattice *L, const double *f, int on_device);
int lbmep_get_pdfs(lbmep_lattice *L, double *f, int on_device);

/* Advance nsteps time steps (nsteps >= 0), asynchronously on the stream.
 * One step: fused collide (Eq. LBMcollideStep + force) and stream
 * (Eq. LBMstreamStep) of all fluid cells, bounce-back at walls and velocity
 * bounce-back at obstacle cells (Eq. LBMMovWall) with the momentum exchange
 * summed per particle in FP64 (Eq. LBMhydrodynForce); then, with moving
 * particles, the kinematics and re-mapping for the next time level; cells
 * uncovered there are refilled with f^eq(rho0, u_s) (Sec. 3.2).  Errors:
 * EINVAL (nsteps < 0), EDEVICE. */
int lbmep_step(lbmep_lattice *L, int32_t nsteps);

/* Wait for all work enqueued on the lattice's stream. */
int lbmep_sync(lbmep_lattice *L);

/* Macroscopic fields of the current state (Eq. MacroscopVel with the
 * velocity of Eq. modified_velocity): rho[N] and u[3N] in FP64.  Obstacle
 * cells report rho0 and their surface velocity, wall cells rho0 and 0. */
int lbmep_get_macro(lbmep_lattice *L, double *rho, double *u, int on_device);

/* Hydrodynamic force F[3n] and torque M[3n] (about the centre, M = sum
 * r x g, r = x_s - x_C) of the last step, FP64, host arrays. */
int lbmep_get_particle_ft(lbmep_lattice *L, double *F, double *M);

/* Current map: flags[N] (LBMEP_FLUID/WALL/OBST/NEAR; NEAR = fluid cell with
 * a wall, obstacle or out-of-domain neighbour) and owner[N] (particle index
 * or -1), host arrays; either may be NULL. */
int lbmep_get_map(lbmep_lattice *L, uint8_t *flags, int32_t *owner);

/* FP64 sums over fluid cells of the current state: out[0] = sum rho,
 * out[1..3] = sum_q c_q f_q.  Deterministic order.  Returns LBMEP_ENONFINITE
 * (with out filled) if a sum is not finite. */
int lbmep_get_invariants(lbmep_lattice *L, double out[4]);

/* Number of completed steps (the kinematic time level). */
int lbmep_get_time(lbmep_lattice *L, int64_t *step);

/* Per-kernel timing of the fused stream-collide launches: enable = 1 starts
 * recording a HIP event pair around every launch (on the lattice's stream),
 * 0 stops.  lbmep_get_timing synchronises, returns the summed duration in ms
 * and the launch count since the last call, and resets them. */
int lbmep_set_timing(lbmep_lattice *L, int enable);
int lbmep_get_timing(lbmep_lattice *L, double *total_ms, int64_t *launches);

/* Checkpoint: populations (storage format), flags, particle table, time
 * level and force to a file; load restores them into a lattice created with
 * the same configuration.  Continuing from a load is bitwise identical to
 * an uninterrupted run.  Errors: EINVAL (null path, mismatching file),
 * EDEVICE, ENOMEM. */
int lbmep_save_state(lbmep_lattice *L, const char *path);
int lbmep_load_state(lbmep_lattice *L, const char *path);

/* The number of particles of L's current particle table (set by
 * lbmep_set_particles or a load).  Errors: EINVAL (null). */
int lbmep_get_particle_count(const lbmep_lattice *L, int32_t *n);

/* Device bytes held by a lattice of this configuration with n particles of
 * radius at most r_max and a charge force or none (used for admission by
 * footprint).  With moving particles this includes the next level's link
 * lists of the overlapped step, n (8 (2 ceil(r_max) + 3)^3 + 4).  Not
 * counted: a potential solver (lbmep_set_potential_solver adds about 23 N
 * bytes with FP32 psi, 39 N with FP64 psi: boundary lists and their rows,
 * interior bitmaps, and for the one-pass iteration (even nx) a second psi
 * buffer, a saved copy of psi and per-entry row codes) and the per-particle
 * charges of the dynamics (8 n).  Errors: EINVAL. */
int lbmep_footprint(const lbmep_config *cfg, int32_t n_particles, double r_max, int with_charge,
                    size_t *bytes);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops): the sums of lbmep_get_invariants, out[0] = sum rho,
 * out[1..3] = sum c f over the fluid cells, written to `out`, 4 doubles in
 * DEVICE memory owned by the caller, enqueued on the lattice's stream and
 * asynchronous (no host synchronisation, no check for NaN/Inf: the caller
 * reads the values).  Same kernels and order as lbmep_get_invariants, so the
 * same bits.  Allocates nothing: its per-workgroup partial sums live in a
 * static device array of 5 * 4096 + 4 doubles (164 KiB) per GPU, held until
 * the process ends and shared by every call on that GPU, so calls that
 * overlap in time on one GPU (other streams or threads) race.  Grids needing
 * more than 4096 partial blocks are rejected (none do: the reduction uses at
 * most 4096).  Errors: EINVAL (null, device index >= 64), EDEVICE. */
int lbmep_get_invariants_noalloc(lbmep_lattice *L, double *out);

/* Measurement aid (not part of the method): copy `bytes` from src to dst,
 * both device memory, with 16-byte lanes and streaming stores, enqueued on
 * `stream` (a hipStream_t, NULL = the default stream) and asynchronous.  Its
 * rate is the achievable HBM bandwidth the sweep's roofline fraction is read
 * against, beside the 8 TB/s peak.  The caller owns both buffers.  Errors:
 * EINVAL (null pointer, pointers or size not multiples of 16 bytes),
 * EDEVICE. */
int lbmep_copy_reference(void *dst, const void *src, size_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of independent simulations on one GPU.
 *
 * Each request is a complete simulation (grid, walls, particles, charge force,
 * number of steps) starting from the rest equilibrium.  Requests are queued on
 * submit and admitted first-in first-out while a slot is free and the sum of
 * the resident requests' device footprints stays within the budget; all of
 * their device memory comes from one arena of `hbm_budget` bytes allocated at
 * creation.  Resident simulations advance together: every kernel of a time
 * step is one packed launch over all of them, enqueued in chunks of
 * `chunk_steps` steps; requests that arrive meanwhile join at the next chunk.
 * Each request computes exactly what a lattice created with the same
 * configuration and stepped `steps` times computes (Sec. 3.1-3.2, as for
 * lbmep_step): its fields, forces and torques are bitwise identical alone or
 * in any mix (the per-particle sums are taken in a fixed order: wavefront
 * sums by DPP row butterflies, then the wavefronts of a workgroup in order,
 * with no atomics).
 *
 * All lbmep_server_* calls on one server must come from one thread at a time.
 * Progress (completion, admission, enqueueing) happens inside
 * lbmep_server_poll, which never waits for the GPU except for the set-up of a
 * newly admitted request (which overlaps the resident requests' steps).
 * ------------------------------------------------------------------------ */

typedef struct lbmep_server lbmep_server; /* opaque; owns its arena and streams */

typedef struct {
    int32_t device;       /* HIP device ordinal */
    int32_t max_slots;    /* resident simulations at once, 1..64 */
    int32_t chunk_steps;  /* steps enqueued per chunk, >= 1 */
    int32_t max_queue;    /* queued requests before submit returns LBMEP_EBUSY */
    size_t hbm_budget;    /* bytes of the device arena, >= 1 MiB */
} lbmep_server_config;

typedef struct {
    lbmep_config cfg;        /* grid, periodic, nu, magic, precision, move_particles;
                                device / stream are the server's; reserved = 0 */
    const uint8_t *flags;    /* N user flags (LBMEP_FLUID / LBMEP_WALL) or NULL */
    int32_t n;               /* particles, >= 0 */
    int32_t steps;           /* time steps, >= 1 */
    const double *X, *R, *U; /* 3n, n, 3n (as lbmep_set_particles) */
    const double *W;         /* 3n angular velocities or NULL */
    const void *rho_e;       /* N charge densities (force rho_e E) or NULL */
    int32_t rho_e_dtype;     /* LBMEP_DTYPE_F64 / LBMEP_DTYPE_F32 */
    int32_t keep_fields;     /* 1: keep rho, u of the final state */
    double E[3];             /* uniform field (used with rho_e) */
} lbmep_request;

typedef struct {
    uint64_t submitted, admitted, completed, failed;
    int32_t queued, resident;
    uint64_t chunks, steps, packed_launches;
    double cell_updates;     /* lattice cells advanced (all cells of every step), enqueued */
    double cell_updates_done;/* of those, in chunks the GPU has completed */
    size_t bytes_reserved;   /* footprints of the resident requests */
    size_t bytes_in_use;     /* arena bytes allocated */
    size_t budget;           /* arena size */
} lbmep_server_stats;

/* Create a server: allocates the arena and two streams (default priority)
 * on cfg->device.  Errors: EINVAL (ranges), ENOMEM (arena), EDEVICE. */
int lbmep_server_create(const lbmep_server_config *cfg, lbmep_server **out);

/* Wait for the server's device work, free everything (also requests that are
 * queued or resident).  NULL is OK. */
int lbmep_server_destroy(lbmep_server *srv);

/* Device bytes a request holds while resident (its admission footprint). */
int lbmep_server_request_footprint(const lbmep_request *req, size_t *bytes);

/* Queue a request; every input array is copied before the call returns.
 * *id identifies it from then on.  Errors: EINVAL (bad configuration or
 * arrays, steps < 1, footprint above the budget, a grid whose two population
 * arrays reach 4 GiB), EBUSY (queue full). */
int lbmep_server_submit(lbmep_server *srv, const lbmep_request *req, uint64_t *id);

/* Make progress (retire finished requests, admit queued ones, enqueue the
 * next chunk) and return up to cap ids of requests finished since the last
 * poll (including requests whose set-up failed).  Errors: EINVAL, EDEVICE. */
int lbmep_server_poll(lbmep_server *srv, uint64_t *done_ids, int32_t cap, int32_t *ndone);

/* Results of a finished request: F[3n], M[3n] of its last step (either may be
 * NULL), inv[4] = FP64 mass and momentum sums of its final state (as
 * lbmep_get_invariants), times[3] = submit, admission and completion times in
 * seconds of the server's clock (may be NULL).  Errors: ESTATE (not finished
 * or unknown id); the request's own error code if its set-up failed. */
int lbmep_server_result(lbmep_server *srv, uint64_t id, double *F, double *M, double inv[4],
                        double times[3]);

/* Final fields rho[N], u[3N] (as lbmep_get_macro) of a request submitted with
 * keep_fields = 1.  Errors: ESTATE. */
int lbmep_server_fields(lbmep_server *srv, uint64_t id, double *rho, double *u);

/* Forget a finished request's results. */
int lbmep_server_release(lbmep_server *srv, uint64_t id);

/* Counters of the server. */
int lbmep_server_get_stats(lbmep_server *srv, lbmep_server_stats *out);

/* The server's clock (seconds since creation). */
int lbmep_server_now(lbmep_server *srv, double *t);

#ifdef __cplusplus
}
#endif
#endif
