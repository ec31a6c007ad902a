/*
 * lbm_oracle.h -- plain FP64 CPU reference of the D3Q19 TRT moving-particle
 * lattice Boltzmann step (Bartuschat & Ruede, "A Scalable Multiphysics
 * Algorithm for Massively Parallel Direct Numerical Simulations of
 * Electrophoresis", arXiv:1708.08741, Sec. 3.1 "Lattice Boltzmann Method"
 * and Sec. 3.2 "Momentum Exchange Approach").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker of the GPU library:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source with the GPU path.
 *
 * State layout: populations f[q * N + c] with c = x + nx * (y + ny * z).
 * The stored state is post-stream / pre-collide ("ready"): after every step
 * the particle map of the new time level is already applied (newly
 * uncovered cells refilled), so macroscopic read-outs are consistent.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_lattice orc_lattice;

/* flag values returned by orc_get_map */
enum { ORC_FLUID = 0, ORC_WALL = 1, ORC_OBST = 2, ORC_NEAR = 3 };

orc_lattice *orc_create(int nx, int ny, int nz, const int periodic[3],
                        double nu, double magic);
void orc_destroy(orc_lattice *L);
/* relaxation rates derived from nu and the TRT magic parameter */
void orc_get_rates(const orc_lattice *L, double out[3]); /* tau, lambda_e, lambda_o */
int orc_set_flags(orc_lattice *L, const uint8_t *flags);  /* 0 fluid, 1 wall */
int orc_set_particles(orc_lattice *L, int n, const double *X, const double *R,
                      const double *U, const double *W, int moving);
int orc_set_force(orc_lattice *L, const double *fb);      /* 3*N SoA */
/* body force rho_e(psi) (E - grad psi) from the EDL potential psi[N],
 * rho_e = -kappa2_eps psi; zeta[np] = potential at each particle's obstacle
 * cells (NULL: the field's value); recomputed when the map changes */
int orc_set_potential_force(orc_lattice *L, const double *psi, double kappa2_eps,
                            const double E[3], const double *zeta);
/* the body force field currently applied (3*N SoA) */
void orc_get_force(const orc_lattice *L, double *fb);
/* red-black SOR for the Debye-Hueckel equation of psi (after
 * orc_set_potential_force); max_iter > 0 also solves at every step.
 * Returns -1 for odd periodic extents or bad parameters. */
int orc_set_potential_solver(orc_lattice *L, double kappa2, double omega, int max_iter,
                             double rf, int check_every);
int orc_solve_potential(orc_lattice *L, int *iters, double *res0, double *res);
void orc_get_solver_stats(const orc_lattice *L, int *iters, double *res0, double *res);
double orc_dha_residual(const orc_lattice *L);
void orc_get_potential(const orc_lattice *L, double *psi);
/* Newton-Euler dynamics of the (moving) particles: density rho_p, charges
 * q[np] (NULL: 0), applied field E for q E.  Returns -1 unless the particle
 * table was set with moving = 1 and rho_p > 0.  Dropped by set_particles. */
int orc_set_dynamics(orc_lattice *L, double rho_p, const double *q, const double E[3]);
void orc_get_particles(const orc_lattice *L, double *X, double *U, double *W);
/* free-slip faces x-, x+, y-, y+, z-, z+ (1 = specular reflection; only on
 * non-periodic axes, else -1) */
int orc_set_free_slip(orc_lattice *L, const int faces[6]);
void orc_init_equilibrium(orc_lattice *L, double rho, const double u[3]);
void orc_set_pdfs(orc_lattice *L, const double *f);       /* 19*N */
void orc_get_pdfs(const orc_lattice *L, double *f);
void orc_step(orc_lattice *L, int nsteps);
long orc_get_step(const orc_lattice *L);
void orc_get_macro(const orc_lattice *L, double *rho, double *u);
void orc_get_ft(const orc_lattice *L, double *F, double *M);
void orc_get_map(const orc_lattice *L, uint8_t *flags, int32_t *owner);
void orc_get_invariants(const orc_lattice *L, double out[4]);
/* bookkeeping of the last step's re-mapping:
 * out[0] = number of uncovered cells, out[1..3] = sum rho0*u_s over them,
 * out[4] = sum rho over newly covered cells, out[5..7] = sum j over them,
 * out[8..10] = sum of f_b over the fluid cells of the streamed step */
void orc_get_bookkeeping(const orc_lattice *L, double out[11]);
/* particle centres of the current time level (wrapped) */
void orc_get_positions(const orc_lattice *L, double *X);
int orc_num_threads(void);
/* set the OpenMP thread count of later calls (timing on 1 core or all) */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
