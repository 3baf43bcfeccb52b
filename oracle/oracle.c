/*
 * FP64 CPU oracle: lattice-Boltzmann fluid two-way coupled to Brownian point
 * particles (Yoshida, Kinjo & Washizu, arXiv:1909.13412).
 *
 * TEST INFRASTRUCTURE ONLY -- the plain, slow, obviously-correct reference the
 * GPU path is checked against.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  Nothing here is shared with the GPU library.
 *
 * Everything is FP64 with plain loops in the order the paper describes:
 *   moments (Eqs. s2-density, s2-fv) -> friction fit (Eq. s2-slet-v) and
 *   reaction force (first Eq. s2-force) -> collision with forcing (Eqs. s2-coll,
 *   s2-collision, s2-eq, second Eq. s2-force) -> streaming (Eq. s2-trans) ->
 *   Langevin update (Eqs. s2-langevin, s2-langevin2).
 * Readings where the paper is silent are listed next to the code that takes them.
 *
 * Lattice units: dx = dt = C = rho0 = 1.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Nineteen-velocity cubic set and the fifteen-velocity set the paper uses
 * (section 2.2); both weight sets give c_s^2 = 1/3 as Eqs. s2-eq and s2-ident3
 * require.  Opposite pairs are adjacent: 1<->2, 3<->4, ... */
static const int E19[19][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
};
static const double W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
};
/* rest, the six axis neighbours, the eight cube corners */
static const int E15[15][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},   {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},
    {-1, 1, 1},  {1, -1, -1},
};
static const double W15[15] = {
    2.0 / 9.0,
    1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
    1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0,
};

struct ora_sim {
    int32_t nx, ny, nz;
    int q;               /* 19 or 15 velocities */
    const int (*E)[3];   /* velocity table of this box */
    const double *W;     /* weights */
    int64_t ncell;
    double tau;
    double *f;    /* post-streaming populations f^n, [a][cell] */
    double *fnew; /* streaming target */
    double *rho;  /* moments of f^n */
    double *u;    /* [3][cell] */
    double *F;    /* force density F_p(x) of the current step, [3][cell] */
    double *body; /* optional constant external force density, [3][cell] */
    /* particles */
    int32_t np;
    double mass, gamma, kT, R;
    uint64_t seed;
    uint32_t replica;
    int32_t friction;
    double *r, *v, *fh, *fr; /* [np][3] */
    double *fc;              /* optional force F_C on each particle, [np][3] */
    double pair_a, pair_rc;  /* soft pair repulsion (a_f, cutoff); a_f = 0: off */
    double *fpair;           /* pair forces of the current step, [np][3] */
    int64_t step;
    /* velocity autocorrelation */
    int32_t vacf_on, max_lag, stride, nslot;
    int64_t vacf_t;       /* local clock, 0 at configuration */
    double *orig;         /* [nslot][np][3] origin velocities */
    int64_t *orig_t;      /* [nslot] origin times, -1 = empty */
    double *acc;          /* [np][max_lag+1] */
    int64_t *cnt;         /* [max_lag+1] */
};

static int64_t cell_index(const ora_sim *o, int64_t x, int64_t y, int64_t z)
{
    return (z * o->ny + y) * o->nx + x;
}

/* Periodic index: i mod n in [0, n). */
static int64_t wrap(int64_t i, int64_t n)
{
    if (i >= 0 && i < n) return i;
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

void ora_lattice_q(int32_t q, int32_t e[][3], double w[])
{
    const int (*E)[3] = q == 15 ? E15 : E19;
    const double *W = q == 15 ? W15 : W19;
    for (int a = 0; a < (q == 15 ? 15 : 19); ++a) {
        for (int k = 0; k < 3; ++k) e[a][k] = E[a][k];
        w[a] = W[a];
    }
}

void ora_lattice(int32_t e[ORA_Q][3], double w[ORA_Q]) { ora_lattice_q(19, e, w); }

/* Eq. (s2-eq): f^eq_a = w_a [rho~ + 3 e_a.u + (9/2)(e_a.u)^2 - (3/2) u.u], the
 * incompressible form in which rho~ appears only in the zeroth-order term. */
void ora_equilibrium_q(int32_t q, double rho, const double u[3], double feq[])
{
    const int (*E)[3] = q == 15 ? E15 : E19;
    const double *W = q == 15 ? W15 : W19;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < (q == 15 ? 15 : 19); ++a) {
        double eu = E[a][0] * u[0] + E[a][1] * u[1] + E[a][2] * u[2];
        feq[a] = W[a] * (rho + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

void ora_equilibrium(double rho, const double u[3], double feq[ORA_Q])
{
    ora_equilibrium_q(19, rho, u, feq);
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) ------------------ */
/* One round maps (c0,c1,c2,c3) with key (k0,k1) to
 *   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0)),
 * A = 0xD2511F53, B = 0xCD9E8D57; the key is bumped by the Weyl constants
 * (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals from one Philox block.  Counter = (step, particle,
 * replica, stream), key = (seed low word, seed high word).  Each 32-bit word x
 * maps to the open interval (0,1) as (x + 1/2) 2^-32; Box & Muller (1958) turns
 * (u0,u1) into two normals and (u2,u3) into a third (its sine partner unused). */
void ora_gauss3(uint64_t seed, uint32_t step, uint32_t particle, uint32_t replica,
                uint32_t stream, double z[3])
{
    uint32_t ctr[4] = {step, particle, replica, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    ora_philox4x32_10(ctr, key, x);
    const double two_pi = 6.283185307179586476925286766559;
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)x[k] + 0.5) * 2.3283064365386962890625e-10;
    double a = sqrt(-2.0 * log(u[0]));
    double b = sqrt(-2.0 * log(u[2]));
    z[0] = a * cos(two_pi * u[1]);
    z[1] = a * sin(two_pi * u[1]);
    z[2] = b * cos(two_pi * u[3]);
}

/* ---- friction force, section 2.1 ------------------------------------------ */
/* mode STOKESLET (the paper's method, Eq. s2-slet-v):
 *   w_p  = u^N_p - V at the eight nodes around the particle;
 *   e^N  = direction of the mean of w_p over the eight nodes;
 *   g_p  = (1 - 3R/(4 r_p)) e^N - 3R (d_p.e^N)/(4 r_p^3) d_p, the Stokeslet
 *          shape of Eq. s2-slet-v rotated to e^N and centred on the particle,
 *          with d_p the vector from the particle to node p and r_p = |d_p|;
 *   U^inf minimises sum_p |w_p - U^inf g_p|^2, i.e. sum w.g / sum g.g;
 *   u^inf = U^inf e^N + V and F_H = -gamma (V - u^inf) = gamma U^inf e^N.
 * Readings: the mean is the plain arithmetic mean; a node closer than 1e-12
 * to the particle is left out of both sums; a zero mean or a zero denominator
 * gives F_H = 0.
 * mode POINTWISE (Eq. s2-dis1): F_H = -gamma (V - u(r)), u(r) interpolated
 *   trilinearly from the same eight nodes.
 * mode BD (Eq. s2-dis0): F_H = -gamma V.
 * mode STOKESLET_2DX: the same fit on the eight corners of a cube of edge
 *   2 dx around the particle (the remedy section 2.2 suggests for large R):
 *   per axis the corners are c0 and c0 + 2 with c0 = floor(s + 1/2) - 1, so
 *   the particle lies in the middle half of the cube; u8 then holds the
 *   velocities at those corners (p -> c0 + 2 (p&1, p>>1&1, p>>2&1)).
 * mode STOKESLET_CUBE: the same fit as STOKESLET_2DX (the reaction force is
 *   then spread to the same cube; see couple_particles). */
void ora_friction_force(int mode, double R, double gamma, const double s[3],
                        const double V[3], const double u8[8][3], double FH[3])
{
    double c[3], d[8][3], wgt[8];
    const int wide = mode == ORA_FRICTION_STOKESLET_2DX || mode == ORA_FRICTION_STOKESLET_CUBE;
    for (int k = 0; k < 3; ++k) c[k] = wide ? floor(s[k] + 0.5) - 1.0 : floor(s[k]);
    for (int p = 0; p < 8; ++p) {
        int b[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
        wgt[p] = 1.0;
        for (int k = 0; k < 3; ++k) {
            d[p][k] = (c[k] + (wide ? 2 * b[k] : b[k])) - s[k];
            wgt[p] *= 1.0 - fabs(d[p][k]);
        }
    }
    if (mode == ORA_FRICTION_BD) {
        for (int k = 0; k < 3; ++k) FH[k] = -gamma * V[k];
        return;
    }
    if (mode == ORA_FRICTION_POINTWISE) {
        for (int k = 0; k < 3; ++k) {
            double ur = 0.0;
            for (int p = 0; p < 8; ++p) ur += wgt[p] * u8[p][k];
            FH[k] = -gamma * (V[k] - ur);
        }
        return;
    }
    double w[8][3], m[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < 8; ++p)
        for (int k = 0; k < 3; ++k) {
            w[p][k] = u8[p][k] - V[k];
            m[k] += w[p][k];
        }
    for (int k = 0; k < 3; ++k) m[k] /= 8.0;
    double mnorm = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    FH[0] = FH[1] = FH[2] = 0.0;
    if (mnorm == 0.0) return;
    double eN[3] = {m[0] / mnorm, m[1] / mnorm, m[2] / mnorm};
    double num = 0.0, den = 0.0;
    for (int p = 0; p < 8; ++p) {
        double rp = sqrt(d[p][0] * d[p][0] + d[p][1] * d[p][1] + d[p][2] * d[p][2]);
        if (!(rp > 1e-12)) continue;
        double de = d[p][0] * eN[0] + d[p][1] * eN[1] + d[p][2] * eN[2];
        double a = 1.0 - 3.0 * R / (4.0 * rp);
        double b = 3.0 * R * de / (4.0 * rp * rp * rp);
        double g[3];
        for (int k = 0; k < 3; ++k) g[k] = a * eN[k] - b * d[p][k];
        for (int k = 0; k < 3; ++k) {
            num += w[p][k] * g[k];
            den += g[k] * g[k];
        }
    }
    if (den == 0.0) return;
    double Uinf = num / den;
    for (int k = 0; k < 3; ++k) FH[k] = gamma * Uinf * eN[k];
}

/* ---- simulation state ------------------------------------------------------ */
ora_sim *ora_create_q(int32_t nx, int32_t ny, int32_t nz, double tau, int32_t q)
{
    if (nx < 2 || ny < 2 || nz < 2 || !(tau > 0.5) || (q != 15 && q != 19)) return NULL;
    ora_sim *o = (ora_sim *)calloc(1, sizeof(ora_sim));
    if (!o) return NULL;
    o->nx = nx; o->ny = ny; o->nz = nz;
    o->q = q;
    o->E = q == 15 ? E15 : E19;
    o->W = q == 15 ? W15 : W19;
    o->ncell = (int64_t)nx * ny * nz;
    o->tau = tau;
    size_t nc = (size_t)o->ncell;
    o->f = (double *)malloc(sizeof(double) * (size_t)q * nc);
    o->fnew = (double *)malloc(sizeof(double) * (size_t)q * nc);
    o->rho = (double *)malloc(sizeof(double) * nc);
    o->u = (double *)malloc(sizeof(double) * 3 * nc);
    o->F = (double *)malloc(sizeof(double) * 3 * nc);
    if (!o->f || !o->fnew || !o->rho || !o->u || !o->F) {
        ora_destroy(o);
        return NULL;
    }
    ora_set_equilibrium(o, NULL, NULL);
    return o;
}

ora_sim *ora_create(int32_t nx, int32_t ny, int32_t nz, double tau)
{
    return ora_create_q(nx, ny, nz, tau, 19);
}

void ora_destroy(ora_sim *o)
{
    if (!o) return;
    free(o->f); free(o->fnew); free(o->rho); free(o->u); free(o->F); free(o->body);
    free(o->r); free(o->v); free(o->fh); free(o->fr); free(o->fc); free(o->fpair);
    free(o->orig); free(o->orig_t); free(o->acc); free(o->cnt);
    free(o);
}

/* Moments of f^n at every node: Eq. (s2-density) rho~ = sum_a f_a and
 * Eq. (s2-fv) u = sum_a C e_a f_a (not divided by rho~). */
static void compute_moments(const ora_sim *o, const double *f, double *rho, double *u)
{
    const int64_t n = o->ncell;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < o->nz; ++z)
        for (int64_t y = 0; y < o->ny; ++y)
            for (int64_t x = 0; x < o->nx; ++x) {
                int64_t c = cell_index(o, x, y, z);
                double r = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
                for (int a = 0; a < o->q; ++a) {
                    double fa = f[a * n + c];
                    r += fa;
                    ux += o->E[a][0] * fa;
                    uy += o->E[a][1] * fa;
                    uz += o->E[a][2] * fa;
                }
                rho[c] = r;
                u[c] = ux;
                u[n + c] = uy;
                u[2 * n + c] = uz;
            }
}

void ora_set_equilibrium(ora_sim *o, const double *rho, const double *u)
{
    const int64_t n = o->ncell;
    for (int64_t c = 0; c < n; ++c) {
        double uc[3] = {u ? u[c] : 0.0, u ? u[n + c] : 0.0, u ? u[2 * n + c] : 0.0};
        double feq[ORA_Q];
        ora_equilibrium_q(o->q, rho ? rho[c] : 1.0, uc, feq);
        for (int a = 0; a < o->q; ++a) o->f[a * n + c] = feq[a];
    }
}

void ora_set_populations(ora_sim *o, const double *f)
{
    memcpy(o->f, f, sizeof(double) * (size_t)o->q * (size_t)o->ncell);
}

void ora_get_populations(const ora_sim *o, double *f)
{
    memcpy(f, o->f, sizeof(double) * (size_t)o->q * (size_t)o->ncell);
}

void ora_get_moments(const ora_sim *o, double *rho, double *u)
{
    compute_moments(o, o->f, rho, u);
}

void ora_set_body_force(ora_sim *o, const double *F)
{
    free(o->body);
    o->body = NULL;
    if (!F) return;
    o->body = (double *)malloc(sizeof(double) * 3 * (size_t)o->ncell);
    memcpy(o->body, F, sizeof(double) * 3 * (size_t)o->ncell);
}

int ora_set_particles(ora_sim *o, int32_t n, const double *r, const double *v,
                      double mass, double gamma, double kT, double radius,
                      uint64_t seed, uint32_t replica, int32_t friction)
{
    if (n < 0 || !(mass > 0.0) || !(gamma >= 0.0) || !(kT >= 0.0)) return -1;
    free(o->r); free(o->v); free(o->fh); free(o->fr); free(o->fc); free(o->fpair);
    o->r = o->v = o->fh = o->fr = o->fc = o->fpair = NULL;
    o->pair_a = 0.0;
    o->np = n;
    o->mass = mass; o->gamma = gamma; o->kT = kT;
    /* Stokes' law gamma = 6 pi eta R with eta = rho0 nu and nu = (tau - 1/2)/3
     * (Eq. s2-ident3) fixes R when only the friction constant is given. */
    double nu = (o->tau - 0.5) / 3.0;
    o->R = radius > 0.0 ? radius : gamma / (6.0 * 3.14159265358979323846 * nu);
    o->seed = seed; o->replica = replica; o->friction = friction;
    if (n > 0) {
        o->r = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        o->v = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        o->fh = (double *)calloc(3 * (size_t)n, sizeof(double));
        o->fr = (double *)calloc(3 * (size_t)n, sizeof(double));
        memcpy(o->r, r, sizeof(double) * 3 * (size_t)n);
        memcpy(o->v, v, sizeof(double) * 3 * (size_t)n);
    }
    return 0;
}

int ora_set_pair_force(ora_sim *o, double a_f, double r_c)
{
    free(o->fpair);
    o->fpair = NULL;
    o->pair_a = 0.0;
    if (a_f == 0.0) return 0;
    double half = 0.5 * (double)(o->nx < o->ny ? (o->nx < o->nz ? o->nx : o->nz)
                                               : (o->ny < o->nz ? o->ny : o->nz));
    if (!isfinite(a_f) || !(r_c > 0.0) || r_c > half || o->np == 0) return -1;
    o->pair_a = a_f;
    o->pair_rc = r_c;
    o->fpair = (double *)calloc(3 * (size_t)o->np, sizeof(double));
    return 0;
}

void ora_get_pair_forces(const ora_sim *o, double *F)
{
    if (o->fpair) memcpy(F, o->fpair, sizeof(double) * 3 * (size_t)o->np);
    else memset(F, 0, sizeof(double) * 3 * (size_t)o->np);
}

void ora_set_particle_force(ora_sim *o, const double *F)
{
    free(o->fc);
    o->fc = NULL;
    if (!F || o->np == 0) return;
    o->fc = (double *)malloc(sizeof(double) * 3 * (size_t)o->np);
    memcpy(o->fc, F, sizeof(double) * 3 * (size_t)o->np);
}

void ora_get_particles(const ora_sim *o, double *r, double *v)
{
    if (o->np == 0) return;
    if (r) memcpy(r, o->r, sizeof(double) * 3 * (size_t)o->np);
    if (v) memcpy(v, o->v, sizeof(double) * 3 * (size_t)o->np);
}

void ora_get_particle_forces(const ora_sim *o, double *fh, double *fr)
{
    if (o->np == 0) return;
    if (fh) memcpy(fh, o->fh, sizeof(double) * 3 * (size_t)o->np);
    if (fr) memcpy(fr, o->fr, sizeof(double) * 3 * (size_t)o->np);
}

double ora_radius(const ora_sim *o) { return o->R; }

int ora_vacf_config(ora_sim *o, int32_t max_lag, int32_t stride)
{
    if (max_lag < 0 || stride < 1) return -1;
    free(o->orig); free(o->orig_t); free(o->acc); free(o->cnt);
    o->max_lag = max_lag;
    o->stride = stride;
    o->nslot = max_lag / stride + 1;
    o->vacf_t = 0;
    size_t np = (size_t)(o->np > 0 ? o->np : 1);
    o->orig = (double *)calloc((size_t)o->nslot * np * 3, sizeof(double));
    o->orig_t = (int64_t *)malloc(sizeof(int64_t) * (size_t)o->nslot);
    o->acc = (double *)calloc(np * (size_t)(max_lag + 1), sizeof(double));
    o->cnt = (int64_t *)calloc((size_t)(max_lag + 1), sizeof(int64_t));
    for (int s = 0; s < o->nslot; ++s) o->orig_t[s] = -1;
    o->vacf_on = 1;
    return 0;
}

void ora_vacf_get(const ora_sim *o, double *acc, int64_t *cnt)
{
    if (!o->vacf_on) return;
    size_t L = (size_t)o->max_lag + 1;
    if (acc && o->np > 0) memcpy(acc, o->acc, sizeof(double) * (size_t)o->np * L);
    if (cnt) memcpy(cnt, o->cnt, sizeof(int64_t) * L);
}

/* C_v(t) = <V(0).V(t)> (section 2.1): each origin t0 = k * stride keeps V(t0);
 * every later sample with lag l = t - t0 <= max_lag adds V(t0).V(t) to the
 * particle's accumulator for lag l.  Sampled at V^n, before the update. */
static void vacf_sample(ora_sim *o)
{
    int64_t t = o->vacf_t;
    if (t % o->stride == 0) {
        int s = (int)((t / o->stride) % o->nslot);
        memcpy(o->orig + (size_t)s * o->np * 3, o->v, sizeof(double) * 3 * (size_t)o->np);
        o->orig_t[s] = t;
    }
    for (int s = 0; s < o->nslot; ++s) {
        int64_t t0 = o->orig_t[s];
        if (t0 < 0 || t - t0 > o->max_lag) continue;
        int64_t lag = t - t0;
        const double *vo = o->orig + (size_t)s * o->np * 3;
        for (int i = 0; i < o->np; ++i) {
            double dot = vo[3 * i] * o->v[3 * i] + vo[3 * i + 1] * o->v[3 * i + 1] +
                         vo[3 * i + 2] * o->v[3 * i + 2];
            o->acc[(size_t)i * (o->max_lag + 1) + lag] += dot;
        }
        o->cnt[lag] += 1;
    }
    o->vacf_t = t + 1;
}

/* Friction, random force and reaction-force spreading for every particle. */
static void couple_particles(ora_sim *o)
{
    const int64_t n = o->ncell;
    const int64_t L[3] = {o->nx, o->ny, o->nz};
    for (int i = 0; i < o->np; ++i) {
        const double *ri = o->r + 3 * i;
        const double *Vi = o->v + 3 * i;
        /* Positions are kept unwrapped; the eight neighbour nodes (section 2.1)
         * are the corners of the lattice cell holding the wrapped position s.
         * Lookups wrap periodically, the geometry d_p does not. */
        double s[3];
        int64_t c[3];
        for (int k = 0; k < 3; ++k) {
            s[k] = ri[k] - (double)L[k] * floor(ri[k] / (double)L[k]);
            c[k] = (int64_t)floor(s[k]);
        }
        double u8[8][3], wgt[8];
        int64_t node[8];
        for (int p = 0; p < 8; ++p) {
            int b[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
            node[p] = cell_index(o, wrap(c[0] + b[0], L[0]), wrap(c[1] + b[1], L[1]),
                                 wrap(c[2] + b[2], L[2]));
            wgt[p] = 1.0;
            for (int k = 0; k < 3; ++k) {
                double d = (double)(c[k] + b[k]) - s[k];
                wgt[p] *= 1.0 - fabs(d);
            }
            for (int k = 0; k < 3; ++k) u8[p][k] = o->u[k * n + node[p]];
        }
        const int cube = o->friction == ORA_FRICTION_STOKESLET_CUBE;
        if (o->friction == ORA_FRICTION_STOKESLET_2DX || cube) {
            /* the fit reads the corners of the (2 dx)^3 cube instead */
            for (int p = 0; p < 8; ++p) {
                int64_t q[3];
                for (int k = 0; k < 3; ++k)
                    q[k] = (int64_t)floor(s[k] + 0.5) - 1 + 2 * ((p >> k) & 1);
                int64_t nd = cell_index(o, wrap(q[0], L[0]), wrap(q[1], L[1]), wrap(q[2], L[2]));
                for (int k = 0; k < 3; ++k) u8[p][k] = o->u[k * n + nd];
            }
        }
        double FH[3];
        ora_friction_force(o->friction, o->R, o->gamma, s, Vi, u8, FH);
        /* Random force: discrete white noise of variance 2 gamma kT / dt per
         * component and step (Eqs. s2-rf1, s2-rf2 with sigma fixed by the
         * fluctuation-dissipation relation for the friction constant). */
        double FR[3] = {0.0, 0.0, 0.0};
        if (o->kT > 0.0) {
            double z[3];
            ora_gauss3(o->seed, (uint32_t)o->step, (uint32_t)i, o->replica, 0u, z);
            double sig = sqrt(2.0 * o->gamma * o->kT);
            for (int k = 0; k < 3; ++k) FR[k] = sig * z[k];
        }
        for (int k = 0; k < 3; ++k) {
            o->fh[3 * i + k] = FH[k];
            o->fr[3 * i + k] = FR[k];
        }
        /* First Eq. (s2-force): the fluid receives -F_H at the particle, spread
         * to the eight nodes with trilinear weights (sum 1, unit cell volume).
         * The Brownian-dynamics model leaves the solvent untouched.  The
         * weights "depending on the distance" are not printed; with the cube
         * fit (STOKESLET_CUBE) the force goes to the same eight corners of
         * the (2 dx)^3 cube the fit reads, with the cube's trilinear weights
         * prod_k (1 - |q_k - s_k| / 2) (sum 1, first moment s). */
        if (cube) {
            for (int p = 0; p < 8; ++p) {
                int64_t q[3];
                double w = 1.0;
                for (int k = 0; k < 3; ++k) {
                    q[k] = (int64_t)floor(s[k] + 0.5) - 1 + 2 * ((p >> k) & 1);
                    w *= 1.0 - fabs((double)q[k] - s[k]) / 2.0;
                }
                int64_t nd = cell_index(o, wrap(q[0], L[0]), wrap(q[1], L[1]), wrap(q[2], L[2]));
                for (int k = 0; k < 3; ++k) o->F[k * n + nd] += -FH[k] * w;
            }
        } else if (o->friction != ORA_FRICTION_BD) {
            for (int p = 0; p < 8; ++p)
                for (int k = 0; k < 3; ++k) o->F[k * n + node[p]] += -FH[k] * wgt[p];
        }
    }
}

/* Collision (Eqs. s2-coll, s2-collision) with the forcing term
 * dt w_a G_a, G_a = 3 F.e_a / (rho0 C) (second Eq. s2-force), followed by
 * streaming f(x + e_a) <- f^(x) (Eq. s2-trans), periodic in all directions. */
static void collide_stream(ora_sim *o)
{
    const int64_t n = o->ncell;
    const double tau = o->tau;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < o->nz; ++z)
        for (int64_t y = 0; y < o->ny; ++y)
            for (int64_t x = 0; x < o->nx; ++x) {
                int64_t c = cell_index(o, x, y, z);
                double uc[3] = {o->u[c], o->u[n + c], o->u[2 * n + c]};
                double Fc[3] = {o->F[c], o->F[n + c], o->F[2 * n + c]};
                double feq[ORA_Q];
                ora_equilibrium_q(o->q, o->rho[c], uc, feq);
                for (int a = 0; a < o->q; ++a) {
                    const int *e = o->E[a];
                    double fa = o->f[a * n + c];
                    double eF = e[0] * Fc[0] + e[1] * Fc[1] + e[2] * Fc[2];
                    double fhat = fa + (feq[a] - fa) / tau + o->W[a] * 3.0 * eF;
                    int64_t d = cell_index(o, wrap(x + e[0], o->nx), wrap(y + e[1], o->ny),
                                           wrap(z + e[2], o->nz));
                    o->fnew[a * n + d] = fhat;
                }
            }
    double *t = o->f;
    o->f = o->fnew;
    o->fnew = t;
}

/* Conservative inter-particle force of Eq. s2-softpot, read as the soft
 * repulsion of dissipative particle dynamics: every pair closer than the
 * cutoff r_c pushes apart with a_f (1 - r/r_c) along the line of centres
 * (the force of the potential (a_f r_c / 2)(1 - r/r_c)^2), nearest periodic
 * image, all pairs visited. */
static void pair_forces(ora_sim *o)
{
    const double L[3] = {(double)o->nx, (double)o->ny, (double)o->nz};
    for (int i = 0; i < o->np; ++i) {
        double F[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < o->np; ++j) {
            if (j == i) continue;
            double d[3], rr = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = o->r[3 * i + k] - o->r[3 * j + k];
                d[k] -= L[k] * round(d[k] / L[k]);
                rr += d[k] * d[k];
            }
            double r = sqrt(rr);
            if (!(r > 0.0) || !(r < o->pair_rc)) continue;
            double mag = o->pair_a * (1.0 - r / o->pair_rc) / r;
            for (int k = 0; k < 3; ++k) F[k] += mag * d[k];
        }
        for (int k = 0; k < 3; ++k) o->fpair[3 * i + k] = F[k];
    }
}

/* Langevin update (Eqs. s2-langevin, s2-langevin2) with the lattice time step:
 * V^{n+1} = V^n + (F_C + F_H + F_R)/M, r^{n+1} = r^n + V^{n+1}.  F_C is the
 * pair force of the step (if enabled) plus a given force per particle. */
static void advance_particles(ora_sim *o)
{
    for (int i = 0; i < o->np; ++i)
        for (int k = 0; k < 3; ++k) {
            double fc = o->fc ? o->fc[3 * i + k] : 0.0;
            if (o->fpair) fc += o->fpair[3 * i + k];
            o->v[3 * i + k] += (fc + o->fh[3 * i + k] + o->fr[3 * i + k]) / o->mass;
            o->r[3 * i + k] += o->v[3 * i + k];
        }
}

void ora_step(ora_sim *o, int32_t nsteps)
{
    const int64_t n = o->ncell;
    for (int32_t s = 0; s < nsteps; ++s) {
        compute_moments(o, o->f, o->rho, o->u);
        if (o->body)
            memcpy(o->F, o->body, sizeof(double) * 3 * (size_t)n);
        else
            memset(o->F, 0, sizeof(double) * 3 * (size_t)n);
        couple_particles(o);
        if (o->fpair) pair_forces(o);
        if (o->vacf_on && o->np > 0) vacf_sample(o);
        collide_stream(o);
        advance_particles(o);
        o->step += 1;
    }
}

int64_t ora_step_count(const ora_sim *o) { return o->step; }

void ora_observables(const ora_sim *o, double out[7])
{
    const int64_t n = o->ncell;
    double *rho = (double *)malloc(sizeof(double) * (size_t)n);
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    compute_moments(o, o->f, rho, u);
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t c = 0; c < n; ++c) {
        m += rho[c];
        px += u[c];
        py += u[n + c];
        pz += u[2 * n + c];
    }
    out[0] = m; out[1] = px; out[2] = py; out[3] = pz;
    double q[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < o->np; ++i)
        for (int k = 0; k < 3; ++k) q[k] += o->mass * o->v[3 * i + k];
    out[4] = q[0]; out[5] = q[1]; out[6] = q[2];
    free(rho);
    free(u);
}

int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
