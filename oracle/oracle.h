/*
 * FP64 CPU oracle: lattice-Boltzmann fluid two-way coupled to Brownian point
 * particles (Yoshida, Kinjo & Washizu, "Numerical simulation method for Brownian
 * particles dispersed in incompressible fluids", arXiv:1909.13412).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Lattice units throughout: dx = dt = C = rho0 = 1, so c_s^2 = 1/3.
 *
 * Array layouts (all FP64, little endian, C order):
 *   populations  f[a][z][y][x]        a = 0..18 (velocity order in oracle.c)
 *   density      rho[z][y][x]
 *   velocity     u[3][z][y][x]
 *   force        F[3][z][y][x]
 *   particles    r[n][3], v[n][3]
 */
#ifndef LBMBP_ORACLE_H
#define LBMBP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_Q 19  /* the largest velocity set */

enum { ORA_FRICTION_STOKESLET = 0, ORA_FRICTION_POINTWISE = 1, ORA_FRICTION_BD = 2,
       ORA_FRICTION_STOKESLET_2DX = 3, ORA_FRICTION_STOKESLET_CUBE = 4 };

typedef struct ora_sim ora_sim;

/* Lattice tables (velocity e[a][3], weight w[a]) of the nineteen-velocity set,
 * or of the set with q = 19 or 15 velocities. */
void ora_lattice(int32_t e[ORA_Q][3], double w[ORA_Q]);
void ora_lattice_q(int32_t q, int32_t e[][3], double w[]);

/* Equilibrium of Eq. (s2-eq) for one node (nineteen or q velocities). */
void ora_equilibrium(double rho, const double u[3], double feq[ORA_Q]);
void ora_equilibrium_q(int32_t q, double rho, const double u[3], double feq[]);

/* Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller Gaussian triple. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ora_gauss3(uint64_t seed, uint32_t step, uint32_t particle, uint32_t replica,
                uint32_t stream, double z[3]);

/* Friction force on one particle from the velocities at its eight neighbour
 * nodes (section 2.1).  s = particle position already wrapped into the box,
 * corner p = bx + 2 by + 4 bz sits at floor(s) + (bx, by, bz);
 * u8[p][3] = fluid velocity there; V = particle velocity. */
void ora_friction_force(int mode, double R, double gamma, const double s[3],
                        const double V[3], const double u8[8][3], double FH[3]);

ora_sim *ora_create(int32_t nx, int32_t ny, int32_t nz, double tau);
/* Same with the velocity set chosen: q = 19 or 15. */
ora_sim *ora_create_q(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t q);
void ora_destroy(ora_sim *o);

/* rho == NULL -> 1 everywhere; u == NULL -> 0 everywhere. */
void ora_set_equilibrium(ora_sim *o, const double *rho, const double *u);
void ora_set_populations(ora_sim *o, const double *f);
void ora_get_populations(const ora_sim *o, double *f);
void ora_get_moments(const ora_sim *o, double *rho, double *u);
/* Constant external force density added to the particle reaction force on
 * every step (NULL clears it). */
void ora_set_body_force(ora_sim *o, const double *F);

/* radius <= 0 derives R from Stokes' law gamma = 6 pi eta R. */
int ora_set_particles(ora_sim *o, int32_t n, const double *r, const double *v,
                      double mass, double gamma, double kT, double radius,
                      uint64_t seed, uint32_t replica, int32_t friction);
void ora_get_particles(const ora_sim *o, double *r, double *v);
/* F_H and F_R used in the most recent step, [n][3] each. */
void ora_get_particle_forces(const ora_sim *o, double *fh, double *fr);
/* Constant force F_C of Eq. s2-langevin on each particle, [n][3] (NULL: none);
 * cleared by ora_set_particles. */
void ora_set_particle_force(ora_sim *o, const double *F);
/* Soft pair repulsion (Eq. s2-softpot read as the DPD conservative force):
 * a_f (1 - r/r_c) along the line of centres for r < r_c; a_f = 0 switches it
 * off.  Returns -1 for r_c outside (0, min(L)/2] or without particles;
 * cleared by ora_set_particles.  ora_get_pair_forces: last step's, [n][3]. */
int ora_set_pair_force(ora_sim *o, double a_f, double r_c);
void ora_get_pair_forces(const ora_sim *o, double *F);
double ora_radius(const ora_sim *o);

/* Velocity autocorrelation: origins every `stride` steps, lags 0..max_lag. */
int ora_vacf_config(ora_sim *o, int32_t max_lag, int32_t stride);
/* acc[n][max_lag+1] per-particle sums of V(t0).V(t0+l); cnt[max_lag+1] origins per lag. */
void ora_vacf_get(const ora_sim *o, double *acc, int64_t *cnt);

void ora_step(ora_sim *o, int32_t nsteps);
int64_t ora_step_count(const ora_sim *o);

/* out = {fluid mass, fluid momentum x,y,z, particle momentum x,y,z}. */
void ora_observables(const ora_sim *o, double out[7]);

/* Number of OpenMP threads the stepping loops use (1 without OpenMP). */
int32_t ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
