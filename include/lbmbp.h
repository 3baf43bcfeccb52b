/*
 * lbmbp -- lattice-Boltzmann fluid two-way coupled to Brownian point particles,
 * hand-written HIP for gfx950 (MI355X).  C ABI.
 *
 * Method: Yoshida, Kinjo & Washizu, "Numerical simulation method for Brownian
 * particles dispersed in incompressible fluids" (arXiv:1909.13412).
 *   - fluid:    section 2.2, Eqs. s2-density, s2-fv (moments), s2-lbe, s2-collision,
 *               s2-eq (BGK with the incompressible equilibrium), second Eq. s2-force
 *               (forcing term G), s2-coll and s2-trans (collide, then stream);
 *               nineteen-velocity cubic lattice, periodic box.
 *   - coupling: section 2.1, Eq. s2-slet-v (Stokeslet-fitted far-field velocity
 *               from the eight nodes around each particle), Eq. s2-dis1 with u
 *               replaced by u^inf (friction), first Eq. s2-force (reaction force
 *               spread back to the same eight nodes).
 *   - particles: Eqs. s2-langevin, s2-langevin2 (Langevin update) with the random
 *               force of Eqs. s2-rf1, s2-rf2 drawn from Philox4x32-10.
 *   - analysis: section 2.1 / 3, C_v(t) = <V(0).V(t)>.
 *
 * Units: lattice units throughout, dx = dt = C = rho0 = 1.
 *
 * Conventions shared by every entry point
 *   - All device pointers are caller-owned; the library never allocates or frees
 *     device memory.  Buffers must stay alive until lbm_destroy (or until the
 *     next particles_couple / lbm_vacf_config replaces them).
 *   - Every kernel is enqueued on the caller's HIP stream given to lbm_init
 *     (NULL = the null stream).  Only lbm_observables, lbm_vacf_counts (host
 *     only) and the lbm_get_* queries of host values synchronise; everything
 *     else is asynchronous.
 *   - Velocity order, D3Q19 (a = 0..18): 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *     7..10 = (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0);
 *     11..14 = (+1,0,+1),(-1,0,-1),(+1,0,-1),(-1,0,+1);
 *     15..18 = (0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).
 *     Weights 1/3 (rest), 1/18 (axis), 1/36 (diagonal).
 *     D3Q15 (a = 0..14): 0 rest; 1..6 as above; 7..14 = (+1,+1,+1),(-1,-1,-1),
 *     (+1,+1,-1),(-1,-1,+1),(+1,-1,+1),(-1,+1,-1),(-1,+1,+1),(+1,-1,-1).
 *     Weights 2/9 (rest), 1/9 (axis), 1/72 (body diagonal).
 *     Population arrays hold Q = 19 or 15 planes accordingly.
 *   - Host-visible FP64 field layouts (C order, x fastest):
 *       populations f[19][nz][ny][nx], density rho[nz][ny][nx],
 *       velocity u[3][nz][ny][nx], particles r[n][3], v[n][3].
 *   - Validation happens before any launch.  On LBM_E_INVAL the context is left
 *     untouched.  A context is not thread-safe; calls on one stream are ordered.
 */
#ifndef LBMBP_H
#define LBMBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_Q 19     /* populations per node of the default set */
#define LBM_Q15 15   /* populations per node of the fifteen-velocity set */

typedef enum lbm_status {
    LBM_OK = 0,
    LBM_E_INVAL = 1,       /* bad argument; nothing was enqueued */
    LBM_E_DEVICE = 2,      /* a HIP call or kernel launch failed */
    LBM_E_STATE = 3,       /* call not valid in the context's current state */
    LBM_E_NONFINITE = 4,   /* a reduction found NaN/Inf, or a node force overflowed */
    LBM_E_UNSUPPORTED = 5  /* valid request the library does not implement */
} lbm_status;

/* Population storage.  Every storage holds the shifted value g = f - w_a rho0
 * (rest state = all zeros).  F64 computes in FP64; F32, BF16 and F16 compute in
 * FP32.  BF16 rounds g to nearest-even; F16 stores round-to-nearest-even of
 * g * 2^f16_scale_log2. */
typedef enum lbm_storage {
    LBM_STORE_F64 = 0,
    LBM_STORE_F32 = 1,
    LBM_STORE_BF16 = 2,
    LBM_STORE_F16 = 3
} lbm_storage;

/* Friction model.  STOKESLET is the paper's method (Eq. s2-slet-v); POINTWISE is
 * Eq. s2-dis1 with u(r) interpolated trilinearly from the eight nodes; BD is
 * Eq. s2-dis0 (solvent at rest, no reaction force).  STOKESLET_2DX is the
 * remedy section 2.2 names for large radii: the same fit on the eight corners
 * of a cube of edge 2 dx around the particle (per axis c0 and c0 + 2,
 * c0 = floor(s + 1/2) - 1); the reaction force is still spread to the corners
 * of the unit cell.  STOKESLET_CUBE: the same cube fit, with the reaction
 * force (first Eq. s2-force, whose distance-dependent weights the paper leaves
 * open) spread to the same eight cube corners with the cube's trilinear
 * weights prod_k (1 - |q_k - s_k| / 2).  Reading the velocity on the cube but
 * spreading on the unit cell lets a pair of particles within a few dx of each
 * other gain energy from the coupling; on the same cube the exchange
 * dissipates.  Not supported by the reverse mode (lbm_record). */
typedef enum lbm_friction {
    LBM_FRICTION_STOKESLET = 0,
    LBM_FRICTION_POINTWISE = 1,
    LBM_FRICTION_BD = 2,
    LBM_FRICTION_STOKESLET_2DX = 3,
    LBM_FRICTION_STOKESLET_CUBE = 4
} lbm_friction;

typedef struct lbm_grid_desc {
    int32_t nx, ny, nz;      /* periodic box, each >= 2, nx*ny*nz < 2^31 */
    double tau;              /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3 (Eq. s2-ident3) */
    int32_t storage;         /* lbm_storage */
    int32_t f16_scale_log2;  /* F16 only: 0..24 (16 recommended); ignored otherwise */
    int32_t velocities;      /* velocity set: 19 (or 0) = D3Q19, 15 = D3Q15 (section 2.2) */
    int32_t reserved;        /* must be 0 */
} lbm_grid_desc;

typedef struct lbm_particle_desc {
    int32_t n;           /* number of particles, 0..2^24 */
    int32_t friction;    /* lbm_friction */
    double mass;         /* M > 0 (all particles identical) */
    double gamma;        /* friction constant >= 0 */
    double kT;           /* temperature >= 0; random force variance 2 gamma kT per component per step */
    double radius;       /* R; <= 0 derives it from Stokes' law gamma = 6 pi rho0 nu R */
    uint64_t seed;       /* Philox key */
    uint32_t replica;    /* third Philox counter word (independent replicas) */
    uint32_t reserved;   /* must be 0 */
} lbm_particle_desc;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of ONE population lattice (the library uses two, A and B, swapped every
 * step): Q x nx x ny x nz elements (the Q distribution functions per node of
 * Eq. s2-lbe, section 2.2) rounded up to 256 bytes; the caller only allocates
 * this many bytes. */
lbm_status lbm_lattice_bytes(const lbm_grid_desc *grid, size_t *bytes);

/* Bytes of grid scratch: two node-force fields (24 bytes per node each: the
 * reaction force of the first Eq. s2-force, section 2.1) with their one-bit
 * flags, reduction partials and flags. */
lbm_status lbm_grid_scratch_bytes(const lbm_grid_desc *grid, size_t *bytes);

/* Bytes of particle scratch for n particles (corner bookkeeping, last-step
 * forces, the pair-force cell list). */
lbm_status lbm_particle_scratch_bytes(const lbm_grid_desc *grid, int32_t n, size_t *bytes);

/* Bytes of the VACF origin store for n particles: (max_lag/stride + 1) * n * 3
 * doubles (the velocities V(0) of C_v(t) = <V(0).V(t)>, section 2.1). */
lbm_status lbm_vacf_origin_bytes(int32_t n, int32_t max_lag, int32_t stride, size_t *bytes);

/* Create a context on the current HIP device for the lattice-Boltzmann fluid of
 * section 2.2: a periodic box of nx x ny x nz nodes, BGK relaxation time tau
 * (Eq. s2-collision; kinematic viscosity nu = (tau - 1/2)/3, Eq. s2-ident3).
 * pop_a, pop_b: device buffers of lbm_lattice_bytes each, 256-byte aligned.
 * grid_scratch: lbm_grid_scratch_bytes, 256-byte aligned.  stream: hipStream_t
 * or NULL.  Enqueues the rest state f = f^eq(rho~ = 1, u = 0) = w (Eq. s2-eq)
 * and clears the scratch.  *out receives the context.  LBM_E_INVAL for a bad
 * descriptor (tau <= 1/2 or not finite, a side below 2, nx ny nz >= 2^31, an
 * unknown storage or velocity set, f16_scale_log2 outside 0..24 for F16,
 * reserved != 0), a null or misaligned buffer, or pop_a == pop_b;
 * LBM_E_DEVICE if the clears cannot be enqueued. */
lbm_status lbm_init(const lbm_grid_desc *grid, void *pop_a, void *pop_b, void *grid_scratch,
                    void *stream, lbm_ctx **out);

/* f = f^eq(rho, u) at every node (Eq. s2-eq).  rho: device FP64 [nz][ny][nx] or
 * NULL for 1; u: device FP64 [3][nz][ny][nx] or NULL for 0. */
lbm_status lbm_set_equilibrium(lbm_ctx *ctx, const double *rho, const double *u);

/* Load the post-streaming populations f^n (the f_alpha(x, t) of Eq. s2-trans,
 * section 2.2) from device FP64 [Q][nz][ny][nx]; stored as g = f - w, rounded
 * to the storage. */
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f);

/* Uniform body force G (host array of 3 doubles, force per node in lattice
 * units; NULL = zero) acting on every node from the next step on: it enters
 * the collision through the same forcing term 3 w_a e_a.F as the particles'
 * reaction forces (second Eq. s2-force), F = G + reaction force.  The total
 * fluid momentum grows by G per node per step. */
lbm_status lbm_set_body_force(lbm_ctx *ctx, const double *g);

/* Decode the post-streaming populations f^n (Eq. s2-trans, section 2.2) into
 * device FP64 [Q][nz][ny][nx], f = w + g. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *f);

/* Moments of f^n (Eqs. s2-density, s2-fv) into device FP64 rho [nz][ny][nx]
 * (may be NULL) and u [3][nz][ny][nx] (may be NULL). */
lbm_status lbm_get_moments(lbm_ctx *ctx, double *rho, double *u);

/* Attach (or replace) the point particles of section 2.1: mass M, friction
 * constant gamma (radius R from Stokes' law gamma = 6 pi rho0 nu R unless
 * given), temperature kT.  Every later step couples them to the fluid: the
 * friction F_H from the Stokeslet fit to the fluid velocity at the eight
 * nodes around each particle (Eq. s2-slet-v with Eq. s2-dis1; or the models
 * named by desc->friction), the random force F_R of Eqs. s2-rf1, s2-rf2, the
 * Langevin update of Eqs. s2-langevin, s2-langevin2, and the reaction force
 * -F_H spread back to those nodes (first Eq. s2-force).  r, v: device FP64
 * [n][3]; the library updates them in place every step (r is kept
 * unwrapped).  particle_scratch: lbm_particle_scratch_bytes(grid, n), 256-byte
 * aligned.  Clears forced-node state and detaches any VACF configuration.
 * n = 0 detaches all particles.  LBM_E_INVAL for a bad descriptor (n outside
 * 0..2^24, M <= 0, gamma < 0, kT < 0, a non-finite M, gamma, kT or radius, an
 * unknown friction model, reserved != 0), or, with n > 0, a null r or v or a
 * null or misaligned particle_scratch. */
lbm_status particles_couple(lbm_ctx *ctx, const lbm_particle_desc *desc, double *r, double *v,
                            void *particle_scratch);

/* A given force F_C on each particle (Eq. s2-langevin), e.g. an applied
 * pulling force: device FP64 [n][3], caller-owned, read every step from the
 * next step on (keep it alive and unchanged while it is attached, and until
 * lbm_adjoint of a run recorded with it); NULL detaches it.  The fluid feels it
 * only through the friction.  LBM_E_STATE without particles; particles_couple
 * detaches it. */
lbm_status lbm_set_particle_force(lbm_ctx *ctx, const double *f);

/* Soft repulsion between particles, the conservative force F_C of Eq.
 * s2-langevin with the potential of Eq. s2-softpot read as that of dissipative
 * particle dynamics: a pair closer than r_c pushes apart with a_f (1 - r/r_c)
 * along the line of centres (nearest periodic image), added to any force set
 * with lbm_set_particle_force.  Neighbours come from a cell list rebuilt every
 * step (cells at least r_c wide hashed into buckets, each bucket in particle
 * order, a fixed visiting order: bitwise reproducible).  a_f = 0 switches it
 * off; r_c must lie in (0, min(nx, ny, nz)/2].  LBM_E_STATE without particles,
 * LBM_E_UNSUPPORTED above 65536 particles.  particles_couple switches it off.  Recorded runs differentiate
 * through it (lbm_adjoint). */
lbm_status lbm_set_pair_force(lbm_ctx *ctx, double a_f, double r_c);

/* The pair forces of the last step into device FP64 [n][3] (zeros when off). */
lbm_status lbm_pair_forces(lbm_ctx *ctx, double *fc);

/* The radius the coupling uses (given or derived), or a negative value when no
 * particles are attached. */
double lbm_particle_radius(const lbm_ctx *ctx);

/* Advisory conditions of the attached particle set (not errors; section 2.2
 * gives the parameter ranges), as a bit set:
 *   LBM_WARN_RADIUS_BOUND     R > sqrt(3) dx for the unit-cell Stokeslet fit
 *                             (R > 2 sqrt(3) dx for the (2 dx)^3 cube): the
 *                             particle covers the fitting nodes;
 *   LBM_WARN_NEGATIVE_GAIN    R > sqrt(3)/2 dx for the unit-cell fit (sqrt(3)
 *                             dx for the cube): the fit's gain in a uniform
 *                             stream is negative at the cell (cube) centre, so
 *                             friction can turn into propulsion;
 *   LBM_WARN_VOLUME_FRACTION  n (4/3) pi R^3 / (nx ny nz) > 0.1, beyond the
 *                             volume fractions the method was checked for.
 * Zero without particles. */
#define LBM_WARN_RADIUS_BOUND 1u
#define LBM_WARN_NEGATIVE_GAIN 2u
#define LBM_WARN_VOLUME_FRACTION 4u
lbm_status lbm_warnings(const lbm_ctx *ctx, uint32_t *flags);

/* Copy the friction F_H (Eq. s2-slet-v, section 2.1) and random force F_R
 * (Eqs. s2-rf1, s2-rf2) of the most recent step into device FP64 [n][3]
 * buffers (either may be NULL). */
lbm_status lbm_particle_forces(lbm_ctx *ctx, double *fh, double *fr);

/* The velocity autocorrelation C_v(t) = <V(0).V(t)> of section 2.1 (the
 * quantity of Figs. 2 and 3, section 3), per particle.  Start accumulating
 * C_i(l) = sum over origins t0 of V_i(t0).V_i(t0 + l), for
 * lags 0..max_lag, origins every `stride` steps counted from this call;
 * V sampled before each step's update.  acc: device FP64 [max_lag+1][n]
 * (lag-major: C_i(l) at acc[l * n + i]), zeroed here.  origins: device buffer of lbm_vacf_origin_bytes.  Requires
 * attached particles.  max_lag = -1 switches the accumulation off. */
lbm_status lbm_vacf_config(lbm_ctx *ctx, int32_t max_lag, int32_t stride, double *acc,
                           double *origins);

/* Host array cnt[max_lag+1]: number of origins that contributed to each lag so
 * far (the same for every particle). */
lbm_status lbm_vacf_counts(const lbm_ctx *ctx, int64_t *cnt);

/* Advance nsteps coupled steps (asynchronous).  Step n: the fluid velocity
 * u = sum e f of the post-streaming f^n at the eight nodes around each
 * particle (Eq. s2-fv), the Stokeslet fit and friction F_H (Eq. s2-slet-v,
 * Eq. s2-dis1), the random force F_R (Eqs. s2-rf1, s2-rf2), the reaction
 * force -F_H spread to the same nodes (first Eq. s2-force); then at every
 * node the moments (Eqs. s2-density, s2-fv), BGK relaxation to the
 * equilibrium (Eqs. s2-collision, s2-eq) with the forcing term (second Eq.
 * s2-force, Eq. s2-coll) and streaming (Eq. s2-trans); and the Langevin
 * update of the particles (Eqs. s2-langevin, s2-langevin2, dt = 1), with the
 * VACF sample of V^n when configured.  LBM_E_INVAL for nsteps < 0;
 * LBM_E_DEVICE if a launch fails. */
lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps);

/* Record the FP64 sums of lbm_observables (Eqs. s2-density, s2-fv; particle
 * momentum M V) during lbm_step without extra passes over the lattice:
 * every `every` steps, starting with the next step, series[8k .. 8k+7] =
 * {step, fluid mass sum rho~, fluid momentum sum u (3), particle momentum
 * sum M V (3)} of the state at the start of that step, for k < capacity
 * (recording stops when full).  The fluid sums are taken inside the
 * stream-collide (FP64 partials per wavefront) and the particle sums inside
 * the particle kernel (per block), finished in a fixed order (deterministic).
 * series: device FP64 [capacity][8], caller-owned.  every = 0 stops. */
lbm_status lbm_series_config(lbm_ctx *ctx, int32_t every, double *series, int64_t capacity);

/* Number of series entries recorded since lbm_series_config. */
lbm_status lbm_series_count(const lbm_ctx *ctx, int64_t *count);

/* Synchronous FP64 sums over the current state: out[0] fluid mass sum rho~
 * (Eq. s2-density), out[1..3] fluid momentum sum u (Eq. s2-fv; with rho0 = 1
 * it is the momentum), out[4..6] particle momentum sum M V (Eq. s2-langevin).
 * Returns LBM_E_NONFINITE (after filling out) if any value is not finite or a
 * node force left the fixed-point range since the last call. */
lbm_status lbm_observables(lbm_ctx *ctx, double out[7]);

/* lbm_observables for callers that cannot allocate device memory (harnesses
 * that forbid hipMalloc, tight serving loops): the same sums, bit for bit,
 * with the reduction partials and the result in a fixed device array of the
 * library (1024 x 4 + 8 doubles, 32.8 KB per device, held until the process
 * ends) instead of the context's grid scratch.  No call allocates or frees
 * anything.  That need is the same for every box and particle count, so no
 * context exceeds it.  Every call on one device shares the array: calls that
 * overlap on one device (two host threads, or two contexts on different
 * streams at once) race and may return each other's sums; calls from one
 * thread are safe, since each call synchronises the context's stream before
 * it returns.  The device current at the call must be the context's
 * (LBM_E_STATE otherwise); LBM_E_DEVICE if the array's address could not be
 * obtained at lbm_init.  Other results as lbm_observables. */
lbm_status lbm_observables_noalloc(lbm_ctx *ctx, double out[7]);

/* Measurement only (no part of the method).  Per-kernel GPU timing with HIP
 * events recorded on the context's stream.
 * enable = 1 brackets every particle-phase launch (VACF sample + particle
 * coupling) and every stream-collide launch of lbm_step with start/stop
 * events (host-side event objects only, no device memory); enable = 0 stops. */
lbm_status lbm_profile_enable(lbm_ctx *ctx, int32_t enable);

/* Synchronise the stream and return the accumulated timings, then reset them:
 * out[0] summed stream-collide milliseconds, out[1] stream-collide launches,
 * out[2] summed particle-phase milliseconds, out[3] particle-phase launches. */
lbm_status lbm_profile_read(lbm_ctx *ctx, double out[4]);

/* Launch configurations of the stream-collide (section 2.2, Eqs. s2-coll and
 * s2-trans): they change how lanes map to nodes, never the result (every
 * configuration gives the same bits).  k = 0..9.  For k < 8, lanes take
 * consecutive nodes and k & 3 is the geometric shape: 0 = one node per lane,
 * 512-lane blocks; 1 = one node, 256; 2 = two nodes (rows y and y + ny/2),
 * 512; 3 = two nodes, 256 (2 and 3 need an even ny); k >= 4 writes the
 * populations with non-temporal stores (streamed past the caches), which pays
 * off once a lattice no longer fits in the GPU's last-level cache.  k = 8 and
 * 9 align lanes with rows (one node per lane, 256-lane blocks, every row
 * starting a 64-lane wavefront; faster when nx is not a multiple of 64), with
 * plain and non-temporal stores; single boxes only.  Until lbm_autotune runs,
 * a context uses the configuration the autotuner last chose in this process
 * for the same device, storage, velocity set and box size, if any; otherwise
 * configuration 8 when nx >= 96 is not a multiple of 64, else shape 0, with
 * non-temporal stores when one lattice is at least 256 MiB. */
#define LBM_NUM_SHAPES 10

/* Time the stream-collide's launch options on this context's lattice (iters
 * launches each, reading the current populations and writing the spare
 * lattice, so the simulation state is not changed) and keep the fastest for
 * later lbm_step calls: first every valid configuration in linear block order
 * without a residency cap in every storage layout (lbm_set_layout: the state
 * is permuted between layouts, values unchanged), then in the layout of the
 * fastest the two fastest configurations with every block order and residency
 * cap (lbm_set_sweep_launch), and the fastest of those in every other layout;
 * finally the three fastest launches of all are timed again in turn, twice
 * each with 2 x iters launches, and the lowest total is kept.  Synchronises
 * the stream.
 * ms (host, LBM_NUM_SHAPES entries, may be NULL) receives per configuration
 * the best mean milliseconds per launch over the options timed with it (-1
 * for a configuration that does not apply, or that repeats another's lane
 * mapping exactly: 8 and 9 when 64 | nx and nx divides 256 or 256 divides
 * nx); *chosen (may be NULL) the configuration kept (lbm_get_sweep_launch
 * gives its block order and cap, lbm_get_layout the layout).  The choice is
 * also remembered for
 * contexts created later with the same device, storage, velocity set and box
 * size (process lifetime, thread-safe). */
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t iters, double *ms, int32_t *chosen);

/* Ceiling of the stream-collide's data movement (the pull streaming of the
 * stream-collide step, section 2.2, without its arithmetic): *ms (host)
 * receives the mean milliseconds per launch, over iters (1..10000) launches
 * after two warm-up launches, of a kernel that pulls every population from
 * x - e_a and stores it unchanged at x, with the layout, lane mapping and store
 * policy of launch configuration k (k < 0: the context's current one) and the
 * context's block order and residency cap.  The
 * stream-collide moves the same bytes the same way, so its duration over this
 * one is the fraction of the access pattern's ceiling it reaches.  Reads the
 * current populations and overwrites the spare lattice (as lbm_autotune does):
 * the simulation state is unchanged.  Synchronises the stream.  LBM_E_INVAL for
 * a NULL ctx or ms, iters out of range, or a configuration that does not apply
 * to this box; LBM_E_DEVICE if a launch fails. */
lbm_status lbm_stream_ceiling(lbm_ctx *ctx, int32_t k, int32_t iters, double *ms);

/* Use launch configuration k (0 .. LBM_NUM_SHAPES - 1) for later steps;
 * LBM_E_INVAL if k is out of range or does not apply to this box.  Every
 * configuration gives bit-identical results. */
lbm_status lbm_set_shape(lbm_ctx *ctx, int32_t k);

/* The launch configuration later lbm_step calls use. */
lbm_status lbm_get_shape(const lbm_ctx *ctx, int32_t *k);

/* Two more launch options of the stream-collide, neither of which changes a
 * bit of the result (the same node updates, the same per-block sums):
 *   order: 0 = blocks in node order; 1 = per-XCD slabs: the GPU hands
 *     consecutive workgroups to its eight XCDs in turn, and order 1 renumbers
 *     them so that XCD k sweeps the k-th contiguous eighth of the blocks;
 *   waves_per_simd: residency cap, 0 (none), 6, 5, 4, 3 or 2 waves per SIMD,
 *     imposed by reserving LDS the kernel does not use, so that fewer blocks
 *     (and fewer concurrent row streams) share a compute unit.
 * lbm_autotune chooses both; until then a context starts from the last
 * choice for its key, else order 0 without a cap.  LBM_E_INVAL for an order
 * or cap outside these values, or a cap the device's LDS cannot impose for
 * the current configuration's block size (lbm_set_shape drops a cap that
 * does not fit the new configuration). */
lbm_status lbm_set_sweep_launch(lbm_ctx *ctx, int32_t order, int32_t waves_per_simd);
lbm_status lbm_get_sweep_launch(const lbm_ctx *ctx, int32_t *order, int32_t *waves_per_simd);

/* Storage layout of the two lattice buffers (the populations that the pull
 * streaming of Eq. s2-trans reads): the lattice rows (y, z) are taken
 * rows_per_group at a time (1, 2, 4, 8, 16, 32 or 64, a divisor of ny), and a group
 * stores, for each population a in turn, its rows one after another, x
 * fastest: element (a, x, y, z) at
 *   ((z*ny + R*(y/R))*Q + y mod R)*nx + a*R*nx + x,   R = rows_per_group.
 * Longer runs per population can stream faster; the values are the same in
 * every layout.  lbm_set_layout moves the current populations into the new
 * layout (a permutation written through the spare lattice, which becomes the
 * current one; asynchronous); the FP64 field I/O is canonical in every
 * layout.  A run kept by lbm_record holds lattices in the layout it was
 * recorded in: lbm_adjoint returns LBM_E_STATE while another layout is in
 * use (setting the recorded one back makes it usable).  lbm_autotune chooses
 * the layout
 * with the launch options; until then a context starts from the last choice
 * for its key, else 1.  LBM_E_INVAL for a NULL ctx or a rows_per_group that is
 * not one of these values or does not divide ny. */
lbm_status lbm_set_layout(lbm_ctx *ctx, int32_t rows_per_group);
lbm_status lbm_get_layout(const lbm_ctx *ctx, int32_t *rows_per_group);

/* Number of steps taken since lbm_init (the time index n of Eq. s2-lbe). */
lbm_status lbm_get_step(const lbm_ctx *ctx, int64_t *step);

/* Release the context (host memory only; device buffers stay the caller's).
 * Bookkeeping, no part of the method. */
lbm_status lbm_destroy(lbm_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Reverse mode (gradients).  The coupled step of section 2 is a differentiable
 * map S: (f^n, r^n, V^n; gamma, tau, M, kT) -> (f^{n+1}, r^{n+1}, V^{n+1}),
 * f the post-streaming populations (Eq. s2-trans), the friction from Eq.
 * s2-slet-v (or Eqs. s2-dis1 / s2-dis0), the Brownian force sqrt(2 gamma kT) xi
 * with the drawn normals xi held fixed (Eqs. s2-rf1, s2-rf2), and the radius
 * either given or R = gamma / (6 pi eta(tau)) by Stokes' law.  lbm_record runs
 * N steps like lbm_step and keeps a checkpoint every `every` steps;
 * lbm_adjoint then returns the gradient of J = <fb, f^N> + <rb, r^N> +
 * <vb, V^N> with respect to the state at the start of the recording and to
 * (gamma, tau, M, kT): the vector-Jacobian product of S^N, the derivative of
 * the exact-arithmetic map taken along the stored trajectory, evaluated in
 * FP64.  The corner cell floor(s) and the fit's degenerate-case branches are
 * piecewise constant (zero derivative).  Supported for FP64 and FP32 storage
 * (LBM_E_UNSUPPORTED otherwise), and for every friction model but
 * LBM_FRICTION_STOKESLET_CUBE. */

/* Bytes of the checkpoint buffer for recording nsteps >= 1 with a checkpoint
 * every `every` >= 1 steps: ceil(nsteps/every) checkpoints of one lattice plus
 * the particle positions and velocities of the context as it is now. */
lbm_status lbm_tape_bytes(const lbm_ctx *ctx, int32_t nsteps, int32_t every, size_t *bytes);

/* Take nsteps coupled steps exactly as lbm_step does (VACF and series
 * recording included) and store the state at the start of every `every`-th
 * step in `tape` (device, lbm_tape_bytes, 256-byte aligned, caller-owned).
 * Replaces any earlier recording of this context.  Asynchronous. */
lbm_status lbm_record(lbm_ctx *ctx, int32_t nsteps, int32_t every, void *tape);

/* Bytes of the work buffer lbm_adjoint needs for the current recording:
 * `every` lattice states plus particle states for recomputing one segment
 * forward, two FP64 adjoint lattices, the node fields and per-particle
 * sums.  LBM_E_STATE if nothing was recorded. */
lbm_status lbm_adjoint_work_bytes(const lbm_ctx *ctx, size_t *bytes);

/* Gradient of the recorded run (asynchronous; the context's own state is not
 * touched and may have moved on).  Segments are recomputed forward from their
 * checkpoints with the same kernels (bit-identical states), then swept in
 * reverse.  All arrays are device memory:
 *   tape       the buffer of the last lbm_record on this context;
 *   work       lbm_adjoint_work_bytes, 256-byte aligned;
 *   adj_pop    in: dJ/df^N, canonical FP64 [19][nz][ny][nx] (the layout of
 *              lbm_get_populations); out: dJ/df at the start of the recording;
 *   adj_r, adj_v  in: dJ/dr^N, dJ/dV^N, FP64 [n][3]; out: the gradients at
 *              the start (NULL allowed without particles);
 *   adj_param  out: FP64 [4] dJ/d(gamma, tau, M, kT).  dJ/dkT is reported
 *              only for kT > 0 (0 otherwise: sqrt(kT) has no derivative at 0).
 * Node contributions of particles that share a node are added with FP64
 * atomics, so repeated runs agree to rounding rather than bitwise when two
 * particles touch the same node in a step.  LBM_E_STATE if tape is not the
 * last recorded run, or the lattice layout (lbm_set_layout) is not the one
 * it was recorded in. */
lbm_status lbm_adjoint(lbm_ctx *ctx, const void *tape, void *work, double *adj_pop,
                       double *adj_r, double *adj_v, double *adj_param);

/* ---------------------------------------------------------------------------
 * Ensembles: many independent periodic boxes of different sizes ("replicas"),
 * e.g. for ensemble-averaged velocity autocorrelation, stepped together.  One
 * particle launch and one stream-collide launch per step cover every replica
 * (a block never straddles two boxes); steps are replayed from a captured
 * HIP graph of LBM_ENS_GRAPH_STEPS steps.  Every replica computes exactly what a single-box
 * context with the same box, tau, particles, seed and replica word computes.
 * ------------------------------------------------------------------------- */
typedef struct lbm_ensemble_desc {
    int32_t nrep;            /* number of replicas, 1..65535 */
    int32_t storage;         /* lbm_storage, shared */
    int32_t f16_scale_log2;  /* F16 only */
    int32_t friction;        /* lbm_friction, shared */
    double mass, gamma, kT;  /* shared particle parameters (as lbm_particle_desc) */
    double radius;           /* <= 0: from Stokes' law per replica (depends on its tau) */
    int32_t reserved;        /* must be 0 */
    int32_t pad;
} lbm_ensemble_desc;

typedef struct lbm_replica_desc {
    int32_t nx, ny, nz;  /* its box, each >= 2 */
    int32_t n;           /* its particles, >= 1 */
    double tau;          /* its relaxation time, > 1/2 */
    uint64_t seed;       /* its Philox key */
    uint32_t replica;    /* its third Philox counter word */
    uint32_t reserved;   /* must be 0 */
} lbm_replica_desc;

typedef struct lbm_ens lbm_ens;

/* Bytes of ONE ensemble lattice (two are used) and of the ensemble scratch.
 * Total nodes < 2^31, total particles < 2^24, 19 nx ny nz < 2^32 for every
 * box (a box is indexed with 32 bits). */
lbm_status lbm_ens_bytes(const lbm_ensemble_desc *desc, const lbm_replica_desc *reps,
                         size_t *lattice_bytes, size_t *scratch_bytes);

/* Create an ensemble on caller buffers (256-byte aligned): both lattices,
 * scratch, and the particles r, v (device FP64 [sum n][3], replica after
 * replica, updated in place).  Fluid starts at rest.  Synchronises. */
lbm_status lbm_ens_init(const lbm_ensemble_desc *desc, const lbm_replica_desc *reps, void *pop_a,
                        void *pop_b, void *scratch, double *r, double *v, void *stream,
                        lbm_ens **out);

/* 1 (default): lbm_ens_step replays a captured graph of LBM_ENS_GRAPH_STEPS
 * steps for every whole group of that many steps from an even step (captured
 * on a private stream, replayed on the context's stream), and launches the
 * rest of the steps directly; plain launches throughout if capture is not
 * possible; 0: plain launches. */
#define LBM_ENS_GRAPH_STEPS 16
lbm_status lbm_ens_use_graph(lbm_ens *ens, int32_t use);

/* Per-particle VACF over all replicas (layouts as lbm_vacf_config with n = all
 * particles).  Synchronises. */
lbm_status lbm_ens_vacf_config(lbm_ens *ens, int32_t max_lag, int32_t stride, double *acc,
                               double *origins);
lbm_status lbm_ens_vacf_counts(const lbm_ens *ens, int64_t *cnt);

/* Advance every replica nsteps steps (asynchronous). */
lbm_status lbm_ens_step(lbm_ens *ens, int32_t nsteps);

/* Time the stream-collide launch shapes on the ensemble in every layout
 * (lbm_ens_set_layout; state unchanged), then the block orders and
 * residency caps (lbm_ens_set_sweep_launch) of the two fastest in the best
 * layout, and keep the fastest launch in the same four stages as
 * lbm_autotune.  The choice is remembered for ensembles created later on the
 * same device with the same storage and the same box sizes in the same
 * order, which start from it. */
lbm_status lbm_ens_autotune(lbm_ens *ens, int32_t iters, double *ms, int32_t *chosen);

/* Block order and residency cap of the ensemble's stream-collide, as
 * lbm_set_sweep_launch: the same node updates whatever the choice (the block
 * -> box table is read at the renumbered block).  A change drops the
 * captured graph (the next lbm_ens_step captures again).  LBM_E_INVAL for a
 * NULL argument, an order or cap outside the values of lbm_set_sweep_launch,
 * or a cap the device's LDS cannot impose for the current configuration's
 * block size. */
lbm_status lbm_ens_set_sweep_launch(lbm_ens *ens, int32_t order, int32_t waves_per_simd);
lbm_status lbm_ens_get_sweep_launch(const lbm_ens *ens, int32_t *order, int32_t *waves_per_simd);

/* Storage layout of the ensemble's lattices (as lbm_set_layout, box by box):
 * rows_per_group (1, 2, 4, ..., 64) is requested of every box, and each box
 * takes the largest power of two not above it that divides its ny.  The
 * current populations move into the new layout unchanged (through the spare
 * lattice; synchronises the stream).  lbm_ens_get_layout gives the rows per
 * group of one replica.  LBM_E_INVAL for a NULL ens or out-of-range values. */
lbm_status lbm_ens_set_layout(lbm_ens *ens, int32_t rows_per_group);
lbm_status lbm_ens_get_layout(const lbm_ens *ens, int32_t replica, int32_t *rows_per_group);

/* Ceiling of the ensemble stream-collide's data movement, as lbm_stream_ceiling:
 * *ms receives the mean milliseconds per launch (iters 1..10000, after two
 * warm-up launches) of a kernel that pulls and stores every population of every
 * box unchanged, with the ensemble's block -> box table, block order and
 * residency cap (where it fits the block size) and launch configuration k
 * (k < 0: the current one; 0..7 only).  Reads the current
 * populations and overwrites the spare lattice: the state is unchanged.
 * Synchronises the stream.  LBM_E_INVAL for a NULL ens or ms, iters out of
 * range, or a configuration that does not apply to every box. */
lbm_status lbm_ens_stream_ceiling(lbm_ens *ens, int32_t k, int32_t iters, double *ms);

/* Use launch configuration k (0..7; two-node configurations need an even ny
 * in every box) for later lbm_ens_step calls, as lbm_set_shape: the same
 * results in every configuration; a residency cap that does not fit the new
 * block size is dropped, and a change drops the captured graph.  LBM_E_INVAL
 * for a NULL ens or a configuration that does not apply to every box.
 * lbm_ens_get_shape gives the configuration later steps use. */
lbm_status lbm_ens_set_shape(lbm_ens *ens, int32_t k);
lbm_status lbm_ens_get_shape(const lbm_ens *ens, int32_t *k);

/* Per-replica FP64 sums (as lbm_observables) and populations (as
 * lbm_get_populations, the replica's own box). */
lbm_status lbm_ens_observables(lbm_ens *ens, int32_t replica, double out[7]);
lbm_status lbm_ens_get_populations(lbm_ens *ens, int32_t replica, double *f);
lbm_status lbm_ens_get_step(const lbm_ens *ens, int64_t *step);
/* Number of graph launches (of LBM_ENS_GRAPH_STEPS steps each) made so far
 * (0 when stepping eagerly). */
lbm_status lbm_ens_graph_replays(const lbm_ens *ens, int64_t *replays);
lbm_status lbm_ens_destroy(lbm_ens *ens);

/* Static string for a status code (bookkeeping). */
const char *lbm_status_string(lbm_status status);

#ifdef __cplusplus
}
#endif
#endif /* LBMBP_H */
