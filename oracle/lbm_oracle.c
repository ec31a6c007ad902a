/*
 * lbm_oracle.c -- plain FP64 CPU reference of one time step of the D3Q19
 * two-relaxation-time (TRT) lattice Boltzmann method with a per-cell body
 * force and moving rigid spheres (velocity bounce-back, momentum exchange).
 *
 * TEST INFRASTRUCTURE ONLY: this is the checker of the GPU library.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product path never does.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * Paper: Bartuschat & Ruede, arXiv:1708.08741.
 *   Sec. 3.1 (TRT LBM): discrete LBE with forcing (Eq. discrLBE_extForce),
 *     incompressible equilibrium (Eq. fequ_Incompr_SRT), moments
 *     (Eq. MacroscopVel), viscosity (Eq. kinVisc), TRT operator (Eq. TRTOp)
 *     with lambda_e = -1/tau and the lambda_o that fixes walls half-way,
 *     even/odd split and equilibrium halves (Eq. EqPDF_TRT), collide and
 *     stream steps (Eq. LBMcollideStep, Eq. LBMstreamStep), Luo forcing
 *     term (Eq. LBE_forcetermLuo), modified momentum density
 *     (Eq. modified_velocity).
 *   Sec. "Computing Electrostatic Forces on Fluid and Particles": the body
 *     force rho_e(psi) (E_ext - grad psi) from an EDL potential
 *     (Eq. ChrgDensDHA, Eq. ElPotGradComp), optional.
 *   Sec. "Finite Volume Discretization for Electric Potential Equations",
 *     Sec. "Solver for Linear Elliptic PDEs with Moving Boundaries",
 *     Sec. "Boundary Condition Handling for Solver Module": the seven-point
 *     finite-volume Debye-Hueckel equation solved by red-black SOR with the
 *     particles' surface potentials as Dirichlet values, optional, once per
 *     time step before the collision (Alg. "Electrophoresis Algorithm").
 *   Alg. "Electrophoresis Algorithm" (last block) with Sec. "Computing
 *     Electrostatic Forces on Fluid and Particles": optional Newton-Euler
 *     dynamics of the spheres under the hydrodynamic force and torque of the
 *     step plus the force q E of the applied field on their charge.
 *   Sec. 3.2 (momentum exchange): cells whose centre lies in a particle are
 *     obstacle cells; velocity bounce-back (Eq. LBMMovWall); hydrodynamic
 *     force (Eq. LBMhydrodynForce) and torque; equilibrium refill of
 *     uncovered cells.
 *
 * Readings where the paper is silent or ambiguous (each is listed in the
 * design notes of the repository):
 *   - D3Q19 ordering: q=0 rest, 1..6 axis directions, 7..18 diagonals, with
 *     opposite pairs (2k-1, 2k).
 *   - Lattice units dx = dt = rho0 = 1, c_s^2 = 1/3 exactly, so 1/c_s^2 = 3
 *     and 1/c_s^4 = 9.
 *   - Forcing: the Luo term split into its even part F^e and odd part F^o,
 *     scaled by (1 + lambda_e/2) and (1 + lambda_o/2), with the velocity of
 *     Eq. modified_velocity used in the equilibrium and in the term (the
 *     second-order TRT form of the Luo/Guo force; the unscaled literal form
 *     would add f_b (1 - lambda_o/2) of momentum per step).
 *   - The population that is bounced back and enters the momentum exchange
 *     is the post-collision value plus the forcing term, f* = f~ + F.
 *   - omega_q in Eq. LBMMovWall / Eq. LBMhydrodynForce are the lattice
 *     weights w_q.
 *   - Torque: M = sum r x g with r = x_s - x_C (the printed substitution
 *     c_q x r is the same product with the opposite sign).
 *   - Cell centres at i + 1/2 (0-based); the inside test is the closed
 *     ball on the minimum-image distance; the lowest particle index owns a
 *     cell claimed by several; WALL cells are never particle cells.
 *   - Outside a non-periodic axis there is an implicit no-slip wall, or a
 *     free-slip (specular) face where set.
 *   - Newly covered cells lose their populations; newly uncovered cells get
 *     f^eq(rho0, u_s) with u_s of the previous owner at its previous place.
 *   - Prescribed kinematics X_p(n) = X_p(0) + n U_p (evaluated in that form),
 *     wrapped into [0, L) on periodic axes; with moving = 0, X_p(n) = X_p(0)
 *     and (U_p, W_p) only set the surface velocity.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19 velocity set (Sec. 3.1: Qian et al.'s model) */
static const int C[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* weights: 1/3 rest, 1/18 axis, 1/36 diagonal (Sec. 3.1) */
static double weight(int q) {
    if (q == 0) return 1.0 / 3.0;
    if (q <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* the opposite direction qbar with c_qbar = -c_q */
static int opposite(int q) {
    int k;
    for (k = 0; k < Q; ++k)
        if (C[k][0] == -C[q][0] && C[k][1] == -C[q][1] && C[k][2] == -C[q][2])
            return k;
    return -1;
}

static const double INV_CS2 = 3.0; /* 1/c_s^2, c_s^2 = 1/3 */
static const double INV_CS4 = 9.0; /* 1/c_s^4 */
static const double RHO0 = 1.0;    /* reference density (lattice units) */

struct orc_lattice {
    int nx, ny, nz, per[3];
    long N;
    double nu, magic, tau, le, lo;
    double w[Q];
    int opp[Q];
    double *f, *fstar, *fnew;
    uint8_t *wall;
    int32_t *owner, *owner_old;
    double *fb;
    /* electrostatic body force from the EDL potential (optional) */
    int potential;
    double *psi, *zeta, k_eps, Eext[3];
    /* red-black SOR for the Debye-Hueckel equation (optional) */
    /* free-slip faces x-, x+, y-, y+, z-, z+ (non-periodic axes only) */
    int slip[6];
    /* Newton-Euler dynamics of the particles (optional) */
    int dynamic;
    double rho_p, Edyn[3], *q;
    int sor_iters, sor_check;
    double kappa2, sor_omega, sor_rf;
    int last_iters;
    double last_res0, last_res;
    int np, moving;
    double *X0, *R, *U, *W;
    double *Xn;   /* positions of the current time level */
    double *Xold; /* positions of the previous time level */
    double *F, *M;
    long step;
    double book[11];
};

static inline long cell_index(const orc_lattice *L, int x, int y, int z) {
    return (long)x + (long)L->nx * ((long)y + (long)L->ny * (long)z);
}

/* minimum-image difference on a periodic axis of length len */
static double min_image(double d, int len, int periodic) {
    if (periodic) {
        double h = 0.5 * (double)len;
        if (d > h) d -= (double)len;
        else if (d < -h) d += (double)len;
    }
    return d;
}

/* centre of particle p at time level n (prescribed kinematics) */
static void particle_position(const orc_lattice *L, int p, long n, double out[3]) {
    int a;
    const int len[3] = {L->nx, L->ny, L->nz};
    for (a = 0; a < 3; ++a) {
        double x = L->X0[3 * p + a];
        if (L->moving) x = L->X0[3 * p + a] + (double)n * L->U[3 * p + a];
        if (L->per[a]) {
            x = x - (double)len[a] * floor(x / (double)len[a]);
            if (x >= (double)len[a]) x -= (double)len[a];
        }
        out[a] = x;
    }
}

/* r = centre of cell (x,y,z) minus X (minimum image) */
static void lever_arm(const orc_lattice *L, int x, int y, int z, const double X[3], double r[3]) {
    r[0] = min_image(((double)x + 0.5) - X[0], L->nx, L->per[0]);
    r[1] = min_image(((double)y + 0.5) - X[1], L->ny, L->per[1]);
    r[2] = min_image(((double)z + 0.5) - X[2], L->nz, L->per[2]);
}

/* centre of cell (x,y,z) moved by whole periods so that it is the image
 * nearest to X: image_centre - X equals the lever arm of lever_arm(), and the
 * values are exact half-integers */
static double image_coord(int i, double Xa, int len, int periodic) {
    double c = (double)i + 0.5;
    if (periodic) {
        double d = c - Xa, h = 0.5 * (double)len;
        if (d > h) c -= (double)len;
        else if (d < -h) c += (double)len;
    }
    return c;
}

static void image_centre(const orc_lattice *L, int x, int y, int z, const double X[3], double xs[3]) {
    xs[0] = image_coord(x, X[0], L->nx, L->per[0]);
    xs[1] = image_coord(y, X[1], L->ny, L->per[1]);
    xs[2] = image_coord(z, X[2], L->nz, L->per[2]);
}

/* surface velocity u_s = U + W x r of a rigid body */
static void surface_velocity(const orc_lattice *L, int p, const double r[3], double us[3]) {
    const double *U = L->U + 3 * p, *W = L->W + 3 * p;
    us[0] = U[0] + (W[1] * r[2] - W[2] * r[1]);
    us[1] = U[1] + (W[2] * r[0] - W[0] * r[2]);
    us[2] = U[2] + (W[0] * r[1] - W[1] * r[0]);
}

/* incompressible equilibrium (Eq. fequ_Incompr_SRT) */
static double f_equilibrium(const orc_lattice *L, int q, double rho_f, const double u[3]) {
    double cu = (double)C[q][0] * u[0] + (double)C[q][1] * u[1] + (double)C[q][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[q] * (rho_f + RHO0 * (cu * INV_CS2 + cu * cu * (0.5 * INV_CS4) - uu * (0.5 * INV_CS2)));
}

static inline int is_fluid(const orc_lattice *L, long c) {
    return !L->wall[c] && L->owner[c] < 0;
}

/* -------------------------------------------------------------------------
 * Obstacle mapping (Sec. 3.2): a cell is an obstacle cell of particle p if
 * its centre lies in the closed ball of p; lowest p wins; walls never map.
 * ---------------------------------------------------------------------- */
static void map_particles(orc_lattice *L, const double *Xpos, int32_t *owner) {
    long c;
    int p, a;
    const int len[3] = {L->nx, L->ny, L->nz};
    for (c = 0; c < L->N; ++c) owner[c] = -1;
    for (p = 0; p < L->np; ++p) {
        const double *X = Xpos + 3 * p;
        double R = L->R[p];
        int lo[3], cnt[3];
        for (a = 0; a < 3; ++a) {
            /* a generous box of cells around the ball, in FP64 so that huge
             * radii cannot overflow int */
            double l = floor(X[a] - R) - 1.0;
            double h = floor(X[a] + R) + 1.0;
            if (L->per[a]) {
                if (h - l + 1.0 >= (double)len[a]) { l = 0.0; h = (double)len[a] - 1.0; }
            } else {
                if (l < 0.0) l = 0.0;
                if (h > (double)len[a] - 1.0) h = (double)len[a] - 1.0;
            }
            lo[a] = (int)l;
            cnt[a] = h >= l ? (int)(h - l + 1.0) : 0;
        }
        if (cnt[0] <= 0 || cnt[1] <= 0 || cnt[2] <= 0) continue;
        {
            int i, j, k;
            for (k = 0; k < cnt[2]; ++k)
                for (j = 0; j < cnt[1]; ++j)
                    for (i = 0; i < cnt[0]; ++i) {
                        int x = lo[0] + i, y = lo[1] + j, z = lo[2] + k;
                        double r[3], d2;
                        if (L->per[0]) x = ((x % L->nx) + L->nx) % L->nx;
                        if (L->per[1]) y = ((y % L->ny) + L->ny) % L->ny;
                        if (L->per[2]) z = ((z % L->nz) + L->nz) % L->nz;
                        c = cell_index(L, x, y, z);
                        if (L->wall[c] || owner[c] >= 0) continue;
                        lever_arm(L, x, y, z, X, r);
                        d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
                        if (d2 <= R * R) owner[c] = p;
                    }
        }
    }
}

/* coordinate v on an axis of length len, wrapped if periodic; -1 if it
 * leaves a non-periodic axis */
static inline int wrap_coord(int v, int len, int periodic) {
    if (v < 0) return periodic ? v + len : -1;
    if (v >= len) return periodic ? v - len : -1;
    return v;
}

/* neighbour of (x,y,z) along +d (d a lattice direction); -1 if outside a
 * non-periodic axis */
static inline long neighbour(const orc_lattice *L, int x, int y, int z, const int d[3]) {
    int vx = wrap_coord(x + d[0], L->nx, L->per[0]);
    int vy = wrap_coord(y + d[1], L->ny, L->per[1]);
    int vz = wrap_coord(z + d[2], L->nz, L->per[2]);
    if (vx < 0 || vy < 0 || vz < 0) return -1;
    return cell_index(L, vx, vy, vz);
}

orc_lattice *orc_create(int nx, int ny, int nz, const int periodic[3], double nu, double magic) {
    orc_lattice *L;
    int q;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(nu > 0.0) || !(magic > 0.0)) return NULL;
    L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->per[0] = periodic[0] != 0; L->per[1] = periodic[1] != 0; L->per[2] = periodic[2] != 0;
    L->N = (long)nx * ny * nz;
    L->nu = nu;
    L->magic = magic;
    /* Eq. kinVisc: nu = (tau - 1/2) c_s^2 */
    L->tau = nu * INV_CS2 + 0.5;
    /* TRT rates (Sec. 3.1): lambda_e = -1/tau; lambda_o from the magic
     * parameter Lambda = (1/s_e - 1/2)(1/s_o - 1/2), s = -lambda.  The
     * paper's lambda_o = -8(2 - 1/tau)/(8 - 1/tau) is Lambda = 3/16. */
    L->le = -1.0 / L->tau;
    L->lo = -1.0 / (0.5 + magic / (L->tau - 0.5));
    for (q = 0; q < Q; ++q) { L->w[q] = weight(q); L->opp[q] = opposite(q); }
    L->f = (double *)calloc((size_t)Q * L->N, sizeof(double));
    L->fstar = (double *)calloc((size_t)Q * L->N, sizeof(double));
    L->fnew = (double *)calloc((size_t)Q * L->N, sizeof(double));
    L->wall = (uint8_t *)calloc((size_t)L->N, 1);
    L->owner = (int32_t *)malloc((size_t)L->N * sizeof(int32_t));
    L->owner_old = (int32_t *)malloc((size_t)L->N * sizeof(int32_t));
    L->fb = (double *)calloc((size_t)3 * L->N, sizeof(double));
    {
        long c;
        for (c = 0; c < L->N; ++c) { L->owner[c] = -1; L->owner_old[c] = -1; }
    }
    if (!L->f || !L->fstar || !L->fnew || !L->wall || !L->owner || !L->owner_old || !L->fb) {
        orc_destroy(L);
        return NULL;
    }
    orc_init_equilibrium(L, 1.0, (const double[3]){0.0, 0.0, 0.0});
    return L;
}

static void potential_force(orc_lattice *L);

static void free_particles(orc_lattice *L) {
    free(L->zeta);
    L->zeta = NULL;
    free(L->q);
    L->q = NULL;
    L->dynamic = 0;
    free(L->X0); free(L->R); free(L->U); free(L->W); free(L->Xn); free(L->Xold);
    free(L->F); free(L->M);
    L->X0 = L->R = L->U = L->W = L->Xn = L->Xold = L->F = L->M = NULL;
    L->np = 0;
}

void orc_destroy(orc_lattice *L) {
    if (!L) return;
    free(L->f); free(L->fstar); free(L->fnew); free(L->wall);
    free(L->owner); free(L->owner_old); free(L->fb);
    free(L->psi);
    free_particles(L); /* also the per-particle zeta */
    free(L);
}

void orc_get_rates(const orc_lattice *L, double out[3]) {
    out[0] = L->tau; out[1] = L->le; out[2] = L->lo;
}

int orc_set_flags(orc_lattice *L, const uint8_t *flags) {
    long c;
    for (c = 0; c < L->N; ++c) L->wall[c] = flags[c] == 1;
    /* re-map the particles on the new walls */
    if (L->np > 0) {
        map_particles(L, L->Xn, L->owner);
        memcpy(L->owner_old, L->owner, (size_t)L->N * sizeof(int32_t));
    }
    if (L->potential) potential_force(L);
    return 0;
}

int orc_set_particles(orc_lattice *L, int n, const double *X, const double *R,
                      const double *U, const double *W, int moving) {
    int p;
    free_particles(L);
    L->np = n;
    L->moving = moving != 0;
    if (n > 0) {
        L->X0 = (double *)malloc(sizeof(double) * 3 * n);
        L->R = (double *)malloc(sizeof(double) * n);
        L->U = (double *)malloc(sizeof(double) * 3 * n);
        L->W = (double *)calloc(3 * (size_t)n, sizeof(double));
        L->Xn = (double *)malloc(sizeof(double) * 3 * n);
        L->Xold = (double *)malloc(sizeof(double) * 3 * n);
        L->F = (double *)calloc(3 * (size_t)n, sizeof(double));
        L->M = (double *)calloc(3 * (size_t)n, sizeof(double));
        memcpy(L->X0, X, sizeof(double) * 3 * n);
        memcpy(L->R, R, sizeof(double) * n);
        memcpy(L->U, U, sizeof(double) * 3 * n);
        if (W) memcpy(L->W, W, sizeof(double) * 3 * n);
    }
    /* the particle table defines time level 0 of the kinematics */
    L->step = 0;
    for (p = 0; p < n; ++p) {
        particle_position(L, p, 0, L->Xn + 3 * p);
        memcpy(L->Xold + 3 * p, L->Xn + 3 * p, sizeof(double) * 3);
    }
    map_particles(L, L->Xn, L->owner);
    memcpy(L->owner_old, L->owner, (size_t)L->N * sizeof(int32_t));
    if (L->potential) potential_force(L);
    return 0;
}

int orc_set_force(orc_lattice *L, const double *fb) {
    L->potential = 0;
    memcpy(L->fb, fb, sizeof(double) * 3 * (size_t)L->N);
    return 0;
}

/* -------------------------------------------------------------------------
 * Electrostatic body force of the electric double layer (Sec. "Computing
 * Electrostatic Forces on Fluid and Particles"): at every fluid cell
 *     f_b = rho_e(psi) (E_ext - grad psi),  rho_e = -kappa^2 eps_e psi
 * (Eq. ChrgDensDHA).  grad psi is the w_q-weighted difference over the 18
 * D3Q19 neighbours divided by the rest weight (Eq. ElPotGradComp, dx = 1)
 * where every neighbour is a fluid cell, and the central D3Q7 difference
 * where a neighbour is a wall, obstacle or outside a non-periodic edge
 * (Sec. "Boundary Condition Handling for Solver Module": the value at a
 * boundary cell is extrapolated from the boundary value and the cell's
 * own value).  Particles carry a Dirichlet value b_p on the face shared
 * with the obstacle cell: zeta_p, or, without zeta, the field's value at
 * that obstacle cell; linear extrapolation gives 2 b_p - psi_c there.
 * Walls and non-periodic edges are homogeneous Neumann boundaries of the
 * potential (the value there is psi_c).  Recomputed whenever the map or
 * psi changes.
 * ---------------------------------------------------------------------- */

/* value of psi at neighbour (x,y,z) + d seen from a cell of value c0: the
 * boundary-extrapolated value at obstacle, wall and beyond-edge cells */
static double psi_at(const orc_lattice *L, int x, int y, int z, const int d[3], double c0) {
    long s = neighbour(L, x, y, z, d);
    if (s < 0 || L->wall[s]) return c0;
    if (L->owner[s] >= 0) {
        double b = L->zeta ? L->zeta[L->owner[s]] : L->psi[s];
        return 2.0 * b - c0;
    }
    return L->psi[s];
}

static void potential_force(orc_lattice *L) {
    const long N = L->N;
    long c;
#pragma omp parallel for schedule(static)
    for (c = 0; c < N; ++c) {
        int a, q;
        int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((long)L->nx * L->ny));
        double g[3] = {0.0, 0.0, 0.0}, rho_e;
        int near = 0;
        if (!is_fluid(L, c)) {
            for (a = 0; a < 3; ++a) L->fb[(long)a * N + c] = 0.0;
            continue;
        }
        for (q = 1; q < Q && !near; ++q) {
            long s = neighbour(L, x, y, z, C[q]);
            if (s < 0 || !is_fluid(L, s)) near = 1;
        }
        if (!near) {
            /* Eq. ElPotGradComp: (1/w_rest) sum_q w_q psi(x + e_q) e_q */
            double sum[3] = {0.0, 0.0, 0.0};
            for (q = 1; q < Q; ++q) {
                double t = L->w[q] * L->psi[neighbour(L, x, y, z, C[q])];
                for (a = 0; a < 3; ++a) {
                    if (C[q][a] > 0) sum[a] = sum[a] + t;
                    else if (C[q][a] < 0) sum[a] = sum[a] - t;
                }
            }
            for (a = 0; a < 3; ++a) g[a] = sum[a] * 3.0;
        } else {
            /* D3Q7 central difference with the boundary values */
            for (a = 0; a < 3; ++a) {
                int dp[3] = {0, 0, 0}, dm[3] = {0, 0, 0};
                dp[a] = 1;
                dm[a] = -1;
                g[a] = (psi_at(L, x, y, z, dp, L->psi[c]) - psi_at(L, x, y, z, dm, L->psi[c])) * 0.5;
            }
        }
        rho_e = -(L->k_eps * L->psi[c]);
        for (a = 0; a < 3; ++a) L->fb[(long)a * N + c] = rho_e * (L->Eext[a] - g[a]);
    }
}

int orc_set_potential_force(orc_lattice *L, const double *psi, double kappa2_eps,
                            const double E[3], const double *zeta) {
    int a;
    if (!L->psi) {
        L->psi = (double *)malloc(sizeof(double) * (size_t)L->N);
        if (!L->psi) return -1;
    }
    memcpy(L->psi, psi, sizeof(double) * (size_t)L->N);
    free(L->zeta);
    L->zeta = NULL;
    if (zeta && L->np > 0) {
        L->zeta = (double *)malloc(sizeof(double) * (size_t)L->np);
        memcpy(L->zeta, zeta, sizeof(double) * (size_t)L->np);
    }
    L->k_eps = kappa2_eps;
    for (a = 0; a < 3; ++a) L->Eext[a] = E[a];
    L->potential = 1;
    potential_force(L);
    return 0;
}

/* -------------------------------------------------------------------------
 * Debye-Hueckel equation for the EDL potential (Sec. "Finite Volume
 * Discretization for Electric Potential Equations"): at every cell i that
 * is neither a wall nor an obstacle cell (an unknown), the seven-point
 * finite-volume form with dx = 1,
 *     (6 + kappa^2) psi_i - sum_{q=1..6} psi(x_i + e_q) = 0,
 * where a neighbour that is no unknown takes its boundary-extrapolated
 * value (psi_at above: 2 b_p - psi_i at obstacle cells of particle p,
 * psi_i at walls and beyond non-periodic edges).  Moved into the stencil
 * and the right-hand side (Sec. "Boundary Condition Handling for Solver
 * Module"), this is
 *     diag_i psi_i - sum_{unknown q} psi(x_i + e_q) = rhs_i,
 *     diag_i = 6 + kappa^2 + n_D - n_N,  rhs_i = 2 sum_{obstacle q} b_p.
 * Solved by SOR in red-black order (Sec. "Solver for Linear Elliptic PDEs
 * with Moving Boundaries"): first all cells with x + y + z even, then all
 * with x + y + z odd, each relaxed as
 *     psi_i <- (1 - omega) psi_i + omega (rhs_i + sum_unknown) / diag_i,
 * until the L2 norm of the residual falls below rf times its initial value
 * (or a fixed count).  The L2 norm is the root mean square over the
 * unknowns (the reading under which the paper's initial residual is the
 * same at every problem size of its weak scaling).
 * ---------------------------------------------------------------------- */

/* diag_i, rhs_i and the sum over unknown neighbours at unknown cell c */
static void dha_row(const orc_lattice *L, long c, double *diag, double *rhs, double *sum) {
    int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((long)L->nx * L->ny));
    int a, sgn;
    *diag = 6.0 + L->kappa2;
    *rhs = 0.0;
    *sum = 0.0;
    for (a = 0; a < 3; ++a)
        for (sgn = -1; sgn <= 1; sgn += 2) {
            int d[3] = {0, 0, 0};
            long s;
            d[a] = sgn;
            s = neighbour(L, x, y, z, d);
            if (s < 0 || L->wall[s]) {
                *diag -= 1.0; /* homogeneous Neumann */
            } else if (L->owner[s] >= 0) {
                double b = L->zeta ? L->zeta[L->owner[s]] : L->psi[s];
                *diag += 1.0; /* Dirichlet on the shared face */
                *rhs += 2.0 * b;
            } else {
                *sum += L->psi[s];
            }
        }
}

static int dha_unknown(const orc_lattice *L, long c) { return !L->wall[c] && L->owner[c] < 0; }

double orc_dha_residual(const orc_lattice *L) {
    double ss = 0.0;
    long c, n = 0;
    for (c = 0; c < L->N; ++c) {
        double diag, rhs, sum, r;
        if (!dha_unknown(L, c)) continue;
        dha_row(L, c, &diag, &rhs, &sum);
        r = rhs + sum - diag * L->psi[c];
        ss += r * r;
        ++n;
    }
    return n > 0 ? sqrt(ss / (double)n) : 0.0;
}

/* one half-sweep over the cells of one colour; cells of a colour have no
 * neighbour of the same colour (even extents on periodic axes), so their
 * order does not matter */
static void sor_colour(orc_lattice *L, int colour) {
    long c;
    for (c = 0; c < L->N; ++c) {
        int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((long)L->nx * L->ny));
        double diag, rhs, sum;
        if (((x + y + z) & 1) != colour || !dha_unknown(L, c)) continue;
        dha_row(L, c, &diag, &rhs, &sum);
        L->psi[c] = (1.0 - L->sor_omega) * L->psi[c] + L->sor_omega * ((rhs + sum) / diag);
    }
}

int orc_set_potential_solver(orc_lattice *L, double kappa2, double omega, int max_iter,
                             double rf, int check_every) {
    int a;
    for (a = 0; a < 3; ++a)
        if (L->per[a] && ((a == 0 ? L->nx : a == 1 ? L->ny : L->nz) & 1)) return -1;
    if (!L->psi || !(kappa2 > 0.0) || !(omega > 0.0 && omega < 2.0) || max_iter < 0 ||
        check_every < 1)
        return -1;
    L->kappa2 = kappa2;
    L->sor_omega = omega;
    L->sor_iters = max_iter;
    L->sor_rf = rf;
    L->sor_check = check_every;
    return 0;
}

/* one solve on the current map: iterations until res < rf res0 (rf > 0,
 * checked every sor_check iterations) or sor_iters iterations */
int orc_solve_potential(orc_lattice *L, int *iters, double *res0, double *res) {
    int it = 0;
    double r0 = L->sor_rf > 0.0 ? orc_dha_residual(L) : -1.0, r = r0;
    if (!(L->sor_rf > 0.0 && r0 == 0.0)) {
        while (it < L->sor_iters) {
            sor_colour(L, 0);
            sor_colour(L, 1);
            ++it;
            if (L->sor_rf > 0.0 && (it % L->sor_check == 0 || it == L->sor_iters)) {
                r = orc_dha_residual(L);
                if (r < L->sor_rf * r0) break;
            }
        }
    }
    L->last_iters = it;
    L->last_res0 = r0;
    L->last_res = r;
    if (iters) *iters = it;
    if (res0) *res0 = r0;
    if (res) *res = r;
    if (L->potential) potential_force(L);
    return 0;
}

void orc_get_solver_stats(const orc_lattice *L, int *iters, double *res0, double *res) {
    *iters = L->last_iters;
    *res0 = L->last_res0;
    *res = L->last_res;
}

void orc_get_potential(const orc_lattice *L, double *psi) {
    memcpy(psi, L->psi, sizeof(double) * (size_t)L->N);
}

void orc_init_equilibrium(orc_lattice *L, double rho, const double u[3]) {
    long c;
    int q;
    for (q = 0; q < Q; ++q) {
        double v = f_equilibrium(L, q, rho, u);
        for (c = 0; c < L->N; ++c) L->f[(long)q * L->N + c] = v;
    }
}

void orc_set_pdfs(orc_lattice *L, const double *f) {
    memcpy(L->f, f, sizeof(double) * Q * (size_t)L->N);
}

void orc_get_pdfs(const orc_lattice *L, double *f) {
    memcpy(f, L->f, sizeof(double) * Q * (size_t)L->N);
}

/* -------------------------------------------------------------------------
 * Collide (Eq. LBMcollideStep) plus the forcing term: f*_q = f~_q + F_q.
 * ---------------------------------------------------------------------- */
static void collide_cell(const orc_lattice *L, long c) {
    const long N = L->N;
    double f[Q], rho = 0.0, j[3] = {0.0, 0.0, 0.0}, u[3], fb[3], uu, ufb;
    int q, a;
    for (q = 0; q < Q; ++q) f[q] = L->f[(long)q * N + c];
    for (a = 0; a < 3; ++a) fb[a] = L->fb[(long)a * N + c];
    /* Eq. MacroscopVel: rho_f = sum f, rho0 u = sum c f */
    for (q = 0; q < Q; ++q) rho += f[q];
    for (a = 0; a < 3; ++a)
        for (q = 0; q < Q; ++q) j[a] += (double)C[q][a] * f[q];
    /* Eq. modified_velocity: u = (sum c f + dt f_b / 2) / rho0 */
    for (a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * fb[a]) / RHO0;
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    ufb = u[0] * fb[0] + u[1] * fb[1] + u[2] * fb[2];
    for (q = 0; q < Q; ++q) {
        int qb = L->opp[q];
        double w = L->w[q];
        double cu = (double)C[q][0] * u[0] + (double)C[q][1] * u[1] + (double)C[q][2] * u[2];
        double cf = (double)C[q][0] * fb[0] + (double)C[q][1] * fb[1] + (double)C[q][2] * fb[2];
        /* Eq. EqPDF_TRT */
        double feq_e = w * (rho - uu * (0.5 * RHO0 * INV_CS2) + cu * cu * (0.5 * RHO0 * INV_CS4));
        double feq_o = w * (RHO0 * INV_CS2 * cu);
        /* even / odd parts of f */
        double fe = 0.5 * (f[q] + f[qb]);
        double fo = 0.5 * (f[q] - f[qb]);
        /* Eq. LBE_forcetermLuo split into even and odd parts:
         * w[(c - u)/cs^2 + (c.u) c/cs^4].fb = w[-u.fb/cs^2 + (c.u)(c.fb)/cs^4]
         *                                   + w (c.fb)/cs^2 */
        double Fe = w * (-ufb * INV_CS2 + cu * cf * INV_CS4);
        double Fo = w * (cf * INV_CS2);
        /* Eq. LBMcollideStep followed by the force of Eq. LBMstreamStep */
        double ft = f[q] + L->le * (fe - feq_e) + L->lo * (fo - feq_o);
        L->fstar[(long)q * N + c] = ft + (1.0 + 0.5 * L->le) * Fe + (1.0 + 0.5 * L->lo) * Fo;
    }
}

/* compensated (Kahan) summation: the global sums add ~10^6..10^8 terms of
 * size ~0.05 into totals of size ~N, where plain summation would lose the
 * per-step changes being checked */
static void kahan_add(double *sum, double *comp, double x) {
    double y = x - *comp;
    double t = *sum + y;
    *comp = (t - *sum) - y;
    *sum = t;
}

/* Neumaier's compensated summation (the Kahan-Babuska variant, which also
 * holds when a term exceeds the running sum) in long double */
typedef struct {
    long double s, c;
} xsum;

static void xsum_add(xsum *a, long double x) {
    long double t = a->s + x;
    if (fabsl(a->s) >= fabsl(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* -------------------------------------------------------------------------
 * One time step n -> n+1.
 * ---------------------------------------------------------------------- */
/* -------------------------------------------------------------------------
 * Particle dynamics (Alg. "Electrophoresis Algorithm": after the LBM sweep
 * the hydrodynamic force and torque of the momentum exchange, together with
 * the electrostatic force F_C = q E_ext on the particle's charge (Sec.
 * "Computing Electrostatic Forces on Fluid and Particles"), move the
 * particles).  Newton-Euler for homogeneous spheres without collisions,
 * one explicit update per lattice step (dt = 1), velocities first:
 *     U <- U + (F_h + q E) / m,   W <- W + M_h / I,   X <- X + U (new U),
 * m = rho_p (4/3) pi R^3, I = (2/5) m R^2.  The velocities of a level are
 * those of its bounce-back, exchange and refill.
 * ---------------------------------------------------------------------- */
static const double PI_D = 3.14159265358979323846;

static void particle_dynamics(orc_lattice *L) {
    int p, a;
    for (p = 0; p < L->np; ++p) {
        const double R = L->R[p];
        const double m = L->rho_p * (4.0 / 3.0) * PI_D * R * R * R;
        const double I = 0.4 * m * R * R;
        const double qp = L->q ? L->q[p] : 0.0;
        for (a = 0; a < 3; ++a) {
            L->U[3 * p + a] = L->U[3 * p + a] + (L->F[3 * p + a] + qp * L->Edyn[a]) / m;
            L->W[3 * p + a] = L->W[3 * p + a] + L->M[3 * p + a] / I;
        }
    }
}

/* the next position of particle p from its current one and its new
 * velocity, wrapped into [0, L) on periodic axes */
static void dynamic_position(const orc_lattice *L, int p, double out[3]) {
    int a;
    const int len[3] = {L->nx, L->ny, L->nz};
    for (a = 0; a < 3; ++a) {
        double x = L->Xold[3 * p + a] + L->U[3 * p + a];
        if (L->per[a]) {
            x = x - (double)len[a] * floor(x / (double)len[a]);
            if (x >= (double)len[a]) x -= (double)len[a];
        }
        out[a] = x;
    }
}

int orc_set_dynamics(orc_lattice *L, double rho_p, const double *q, const double E[3]) {
    int a;
    if (!L->moving || !(rho_p > 0.0)) return -1;
    free(L->q);
    L->q = NULL;
    if (q && L->np > 0) {
        L->q = (double *)malloc(sizeof(double) * (size_t)L->np);
        memcpy(L->q, q, sizeof(double) * (size_t)L->np);
    }
    L->rho_p = rho_p;
    for (a = 0; a < 3; ++a) L->Edyn[a] = E[a];
    L->dynamic = 1;
    return 0;
}

void orc_get_particles(const orc_lattice *L, double *X, double *U, double *W) {
    memcpy(X, L->Xn, sizeof(double) * 3 * (size_t)L->np);
    memcpy(U, L->U, sizeof(double) * 3 * (size_t)L->np);
    memcpy(W, L->W, sizeof(double) * 3 * (size_t)L->np);
}

/* -------------------------------------------------------------------------
 * Free-slip faces (no-slip and free-slip boundaries are the two wall
 * conditions of the paper's simulations, Sec. "Lattice Boltzmann Method with
 * Forcing"; the paper defers their form to earlier work).  Reading: a free-slip face of
 * a non-periodic axis is a plane half a cell beyond the last cell that
 * reflects populations specularly.  For fluid cell x and direction q whose
 * source x - e_q lies beyond the grid along the axes O, and every face so
 * crossed is free-slip: the population left the cell s' = x - e_q with its
 * O-components set back to x's, in the direction p = e_q mirrored in O, and
 * the reflection delivers it to x.  If s' is a wall or obstacle cell there
 * is no such population and the link takes the resting half-way
 * bounce-back; a face that is not free-slip always does.  Both keep the
 * streaming a one-to-one map of populations, so mass is conserved.
 * ---------------------------------------------------------------------- */
static int mirrored_direction(int q, const int flip[3]) {
    int k, want[3], a;
    for (a = 0; a < 3; ++a) want[a] = flip[a] ? -C[q][a] : C[q][a];
    for (k = 0; k < Q; ++k)
        if (C[k][0] == want[0] && C[k][1] == want[1] && C[k][2] == want[2]) return k;
    return -1;
}

static int free_slip_source(const orc_lattice *L, int x, int y, int z, int q, long *src, int *pdir) {
    const int len[3] = {L->nx, L->ny, L->nz};
    const int v[3] = {x, y, z};
    int flip[3] = {0, 0, 0}, w[3], a, any = 0;
    for (a = 0; a < 3; ++a) {
        int u = v[a] - C[q][a];
        w[a] = u;
        if (u >= 0 && u < len[a]) continue;
        if (L->per[a]) {
            w[a] = u < 0 ? u + len[a] : u - len[a];
            continue;
        }
        /* crosses the low (2a) or high (2a + 1) face of axis a */
        if (!L->slip[2 * a + (u < 0 ? 0 : 1)]) return 0;
        flip[a] = 1;
        w[a] = v[a];
        any = 1;
    }
    if (!any) return 0;
    *src = cell_index(L, w[0], w[1], w[2]);
    if (!is_fluid(L, *src)) return 0;
    *pdir = mirrored_direction(q, flip);
    return 1;
}

int orc_set_free_slip(orc_lattice *L, const int faces[6]) {
    int k;
    for (k = 0; k < 6; ++k)
        if (faces[k] && L->per[k / 2]) return -1;
    for (k = 0; k < 6; ++k) L->slip[k] = faces[k] != 0;
    return 0;
}

static void one_step(orc_lattice *L) {
    const long N = L->N;
    const int nx = L->nx, ny = L->ny, nz = L->nz, np = L->np;
    /* per z slab and particle: compensated sums of F[3] and M[3] */
    xsum *Sz = NULL;
    int z;
    if (np > 0) Sz = (xsum *)calloc((size_t)nz * np * 6, sizeof(xsum));

    /* 0. the EDL potential of this level's map and its body force */
    if (L->potential && L->sor_iters > 0) orc_solve_potential(L, NULL, NULL, NULL);

    /* 1. collide every fluid cell */
#pragma omp parallel for schedule(static)
    for (z = 0; z < nz; ++z) {
        int x, y;
        for (y = 0; y < ny; ++y)
            for (x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, z);
                if (is_fluid(L, c)) collide_cell(L, c);
            }
    }

    /* 2. stream (pull form of Eq. LBMstreamStep) with no-slip walls and the
     * velocity bounce-back of Eq. LBMMovWall; momentum exchange of
     * Eq. LBMhydrodynForce summed per z slab, then slabs in order. */
#pragma omp parallel for schedule(static)
    for (z = 0; z < nz; ++z) {
        int x, y, q;
        for (y = 0; y < ny; ++y)
            for (x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, z);
                if (!is_fluid(L, c)) {
                    for (q = 0; q < Q; ++q) L->fnew[(long)q * N + c] = L->f[(long)q * N + c];
                    continue;
                }
                for (q = 0; q < Q; ++q) {
                    const int back[3] = {-C[q][0], -C[q][1], -C[q][2]};
                    long s = neighbour(L, x, y, z, back); /* x - e_q */
                    int qb = L->opp[q];
                    long ss;
                    int ps;
                    if (s >= 0 && is_fluid(L, s)) {
                        L->fnew[(long)q * N + c] = L->fstar[(long)q * N + s];
                    } else if (s < 0 && free_slip_source(L, x, y, z, q, &ss, &ps)) {
                        /* specular reflection at a free-slip face */
                        L->fnew[(long)q * N + c] = L->fstar[(long)ps * N + ss];
                    } else if (s < 0 || L->wall[s]) {
                        /* resting no-slip wall half-way */
                        L->fnew[(long)q * N + c] = L->fstar[(long)qb * N + c];
                    } else {
                        int p = L->owner[s];
                        int sx = wrap_coord(x + back[0], nx, L->per[0]);
                        int sy = wrap_coord(y + back[1], ny, L->per[1]);
                        int sz = wrap_coord(z + back[2], nz, L->per[2]);
                        double r[3], xs[3], us[3], cus, mw, fq;
                        long double rl[3], g[3], gm;
                        xsum *S = Sz + ((size_t)z * np + p) * 6;
                        int a;
                        lever_arm(L, sx, sy, sz, L->Xn + 3 * p, r);
                        image_centre(L, sx, sy, sz, L->Xn + 3 * p, xs);
                        surface_velocity(L, p, r, us);
                        cus = (double)C[qb][0] * us[0] + (double)C[qb][1] * us[1] + (double)C[qb][2] * us[2];
                        mw = 2.0 * L->w[qb] * INV_CS2 * RHO0 * cus;
                        fq = L->fstar[(long)qb * N + c];
                        /* Eq. LBMMovWall: population q arrives back at x */
                        L->fnew[(long)q * N + c] = fq - mw;
                        /* Eq. LBMhydrodynForce: the link hands the particle
                         * g = [2 f*_qb - 2 (w_qb / c_s^2) rho0 c_qb . u_s] c_qb
                         * and the torque r x g, r = x_s - X (reading of the
                         * torque substitution).  The terms (~0.1 each) cancel
                         * to forces many orders smaller, so the lever arm, the
                         * terms and their sums are taken in long double with
                         * compensated summation: F and M are the plain link
                         * sums to within a few ulps of the result. */
                        for (a = 0; a < 3; ++a) rl[a] = (long double)xs[a] - (long double)L->Xn[3 * p + a];
                        gm = 2.0L * (long double)fq - (long double)mw;
                        for (a = 0; a < 3; ++a) g[a] = gm * (long double)C[qb][a];
                        for (a = 0; a < 3; ++a) xsum_add(&S[a], g[a]);
                        xsum_add(&S[3], rl[1] * g[2] - rl[2] * g[1]);
                        xsum_add(&S[4], rl[2] * g[0] - rl[0] * g[2]);
                        xsum_add(&S[5], rl[0] * g[1] - rl[1] * g[0]);
                    }
                }
            }
    }
    {
        /* slabs in order, each slab's sum and its correction term */
        int p, a;
        for (p = 0; p < np; ++p) {
            xsum t[6];
            memset(t, 0, sizeof(t));
            for (z = 0; z < nz; ++z)
                for (a = 0; a < 6; ++a) {
                    const xsum *S = Sz + ((size_t)z * np + p) * 6 + a;
                    xsum_add(&t[a], S->s);
                    xsum_add(&t[a], S->c);
                }
            for (a = 0; a < 3; ++a) {
                L->F[3 * p + a] = (double)(t[a].s + t[a].c);
                L->M[3 * p + a] = (double)(t[3 + a].s + t[3 + a].c);
            }
        }
    }
    free(Sz);

    /* Newton-Euler update of the particles with this step's force and
     * torque (see particle_dynamics) */
    if (L->dynamic) particle_dynamics(L);

    /* bookkeeping: total body force on the fluid cells of this step */
    {
        long c;
        int a;
        double comp[3] = {0.0, 0.0, 0.0};
        for (a = 0; a < 11; ++a) L->book[a] = 0.0;
        for (c = 0; c < N; ++c)
            if (is_fluid(L, c))
                for (a = 0; a < 3; ++a) kahan_add(&L->book[8 + a], &comp[a], L->fb[(long)a * N + c]);
    }
    {
        double *t = L->f;
        L->f = L->fnew;
        L->fnew = t;
    }
    L->step += 1;

    /* 3. kinematics and re-mapping for the new time level, refill of
     * uncovered cells with f^eq(rho0, u_s of the previous owner at its
     * previous position) (Sec. 3.2, last paragraph). */
    if (L->moving && np > 0) {
        int p;
        long c;
        int32_t *t;
        memcpy(L->Xold, L->Xn, sizeof(double) * 3 * np);
        for (p = 0; p < np; ++p) {
            if (L->dynamic) dynamic_position(L, p, L->Xn + 3 * p);
            else particle_position(L, p, L->step, L->Xn + 3 * p);
        }
        t = L->owner_old;
        L->owner_old = L->owner;
        L->owner = t;
        map_particles(L, L->Xn, L->owner);
        for (c = 0; c < N; ++c) {
            int q, a;
            int32_t po = L->owner_old[c], pn = L->owner[c];
            int x = (int)(c % nx), y = (int)((c / nx) % ny), zz = (int)(c / ((long)nx * ny));
            if (L->wall[c]) continue;
            if (po >= 0 && pn < 0) {
                double r[3], us[3];
                lever_arm(L, x, y, zz, L->Xold + 3 * po, r);
                surface_velocity(L, po, r, us);
                for (q = 0; q < Q; ++q) L->f[(long)q * N + c] = f_equilibrium(L, q, RHO0, us);
                L->book[0] += 1.0;
                for (a = 0; a < 3; ++a) L->book[1 + a] += RHO0 * us[a];
            } else if (po < 0 && pn >= 0) {
                double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
                for (q = 0; q < Q; ++q) rho += L->f[(long)q * N + c];
                for (a = 0; a < 3; ++a)
                    for (q = 0; q < Q; ++q) j[a] += (double)C[q][a] * L->f[(long)q * N + c];
                L->book[4] += rho;
                for (a = 0; a < 3; ++a) L->book[5 + a] += j[a];
            }
        }
    } else if (np > 0) {
        memcpy(L->Xold, L->Xn, sizeof(double) * 3 * np);
    }
    /* the body force of the new level's map */
    if (L->potential && L->moving && np > 0) potential_force(L);
}

void orc_step(orc_lattice *L, int nsteps) {
    int s;
    for (s = 0; s < nsteps; ++s) one_step(L);
}

long orc_get_step(const orc_lattice *L) { return L->step; }

void orc_get_macro(const orc_lattice *L, double *rho, double *u) {
    const long N = L->N;
    long c;
    for (c = 0; c < N; ++c) {
        int q, a;
        int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((long)L->nx * L->ny));
        if (L->wall[c]) {
            rho[c] = RHO0;
            for (a = 0; a < 3; ++a) u[(long)a * N + c] = 0.0;
        } else if (L->owner[c] >= 0) {
            double r[3], us[3];
            int p = L->owner[c];
            lever_arm(L, x, y, z, L->Xn + 3 * p, r);
            surface_velocity(L, p, r, us);
            rho[c] = RHO0;
            for (a = 0; a < 3; ++a) u[(long)a * N + c] = us[a];
        } else {
            double s = 0.0;
            for (q = 0; q < Q; ++q) s += L->f[(long)q * N + c];
            rho[c] = s;
            for (a = 0; a < 3; ++a) {
                double j = 0.0;
                for (q = 0; q < Q; ++q) j += (double)C[q][a] * L->f[(long)q * N + c];
                u[(long)a * N + c] = (j + 0.5 * L->fb[(long)a * N + c]) / RHO0;
            }
        }
    }
}

void orc_get_force(const orc_lattice *L, double *fb) {
    memcpy(fb, L->fb, sizeof(double) * 3 * (size_t)L->N);
}

void orc_get_ft(const orc_lattice *L, double *F, double *M) {
    if (L->np > 0) {
        memcpy(F, L->F, sizeof(double) * 3 * L->np);
        memcpy(M, L->M, sizeof(double) * 3 * L->np);
    }
}

void orc_get_map(const orc_lattice *L, uint8_t *flags, int32_t *owner) {
    long c;
    for (c = 0; c < L->N; ++c) {
        int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((long)L->nx * L->ny));
        uint8_t fl;
        if (L->wall[c]) fl = ORC_WALL;
        else if (L->owner[c] >= 0) fl = ORC_OBST;
        else {
            int q;
            fl = ORC_FLUID;
            for (q = 1; q < Q; ++q) {
                long s = neighbour(L, x, y, z, C[q]);
                if (s < 0 || !is_fluid(L, s)) { fl = ORC_NEAR; break; }
            }
        }
        if (flags) flags[c] = fl;
        if (owner) owner[c] = L->wall[c] ? -1 : L->owner[c];
    }
}

void orc_get_invariants(const orc_lattice *L, double out[4]) {
    const long N = L->N;
    long c;
    int q, a;
    double comp[4] = {0.0, 0.0, 0.0, 0.0};
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (c = 0; c < N; ++c) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (!is_fluid(L, c)) continue;
        for (q = 0; q < Q; ++q) rho += L->f[(long)q * N + c];
        for (a = 0; a < 3; ++a)
            for (q = 0; q < Q; ++q) j[a] += (double)C[q][a] * L->f[(long)q * N + c];
        kahan_add(&out[0], &comp[0], rho);
        for (a = 0; a < 3; ++a) kahan_add(&out[1 + a], &comp[1 + a], j[a]);
    }
}

void orc_get_bookkeeping(const orc_lattice *L, double out[11]) {
    memcpy(out, L->book, sizeof(double) * 11);
}

void orc_get_positions(const orc_lattice *L, double *X) {
    if (L->np > 0) memcpy(X, L->Xn, sizeof(double) * 3 * L->np);
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
