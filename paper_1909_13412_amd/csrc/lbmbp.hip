// lbmbp: lattice-Boltzmann fluid two-way coupled to Brownian point particles
// (Yoshida, Kinjo & Washizu, arXiv:1909.13412), hand-written HIP for gfx950.
//
// One coupled step n (section 2):
//   k_particle        per particle, eight lanes = eight neighbour nodes:
//                     VACF sample C_i(l) += V_i(t0).V_i(n) (section 2.1),
//                     gather u^n at the nodes (Eq. s2-fv), Stokeslet fit
//                     (Eq. s2-slet-v) -> F_H, Philox Brownian force
//                     (Eqs. s2-rf1, s2-rf2), spread -F_H into the node-force
//                     field (first Eq. s2-force), Langevin update (Eqs.
//                     s2-langevin, s2-langevin2)
//   k_stream_collide  every node: pull f^n_a(x) = A_a(x - e_a) (Eq. s2-trans of
//                     the previous step), moments (Eqs. s2-density, s2-fv),
//                     BGK (Eqs. s2-collision, s2-eq) plus forcing (second
//                     Eq. s2-force) where the node is flagged, write B_a(x)
//                     (Eq. s2-coll); A and B swap.
//
// Layout and the stream-collide kernel: collide.hpp.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <algorithm>
#include <vector>

#include "lbmbp.h"
#include "adjoint.hpp"
#include "codec.hpp"
#include "collide.hpp"
#include "velocities.hpp"
#include "pairs.hpp"
#include "particle.hpp"
#include "philox.hpp"

namespace lbmbp {

constexpr int kRedBlocks = 1024;

// ---------------------------------------------------------------------------
// Ensembles of independent boxes (replicas) of different sizes, stepped
// together: one stream-collide launch covers every replica's nodes (a block
// never straddles two replicas) and one particle launch covers every
// particle.  Step-dependent values come from a device clock so that a
// captured graph of several steps can be replayed.
// ---------------------------------------------------------------------------
struct Replica {
    Grid g;
    uint64_t pop_off;              // first element of this box in the lattices
    uint64_t cell_off;             // first node in the node-force fields
    uint32_t mask_off;             // first word of its forcing flags
    uint32_t first_block[4];       // first stream-collide block, per launch shape
    uint32_t part_off, npart;      // its particles in the concatenated arrays
    uint32_t replica_id;           // Philox third counter word
    uint32_t pad;
    uint64_t seed;                 // Philox key
    double omega;                  // 1 / tau
    double R;                      // particle radius
};

struct EnsClock {
    int64_t step;    // Philox first counter word and field parity
    int64_t vacf_t;  // VACF sample clock
};

template <class C, int CPT, int BS, bool NTS>
__global__ __launch_bounds__(BS) void k_ens_collide(const typename C::T *__restrict__ A,
                                                    typename C::T *__restrict__ B,
                                                    const Replica *__restrict__ reps,
                                                    const uint16_t *__restrict__ blk_rep,
                                                    int shape, long long *force,
                                                    uint32_t *mask, typename C::R enc_s,
                                                    typename C::R dec_s, EnsClock *clock,
                                                    int vacf_on, uint32_t order) {
    const uint32_t b = sweep_block(order);
    const uint32_t rid = blk_rep[b];
    const Replica &rp = reps[rid];
    const uint32_t lane_cell = (b - rp.first_block[shape]) * BS + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the step's last reader of the clock has finished (previous kernel)
        clock->step += 1;
        if (vacf_on) clock->vacf_t += 1;
    }
    if (lane_cell >= rp.g.ncell / CPT) return;
    const ForceField ff{force + 3 * rp.cell_off, mask + rp.mask_off};
    double acc[4];
    using R = typename C::R;
    collide_lane<C, true, false, CPT, NTS>(A + rp.pop_off, B + rp.pop_off, rp.g, R(rp.omega),
                                           enc_s, dec_s, ff, R(0), R(0), R(0), lane_cell, acc);
}

// Streaming-only counterpart of k_ens_collide (same block -> box table, block
// order, lanes and store policy): the comparison kernel the ensemble
// stream-collide is measured against.
template <class C, int CPT, int BS, bool NTS>
__global__ __launch_bounds__(BS) void k_ens_stream_only(const typename C::T *__restrict__ A,
                                                        typename C::T *__restrict__ B,
                                                        const Replica *__restrict__ reps,
                                                        const uint16_t *__restrict__ blk_rep, int shape,
                                                        uint32_t order) {
    const uint32_t b = sweep_block(order);
    const Replica &rp = reps[blk_rep[b]];
    const uint32_t lane_cell = (b - rp.first_block[shape]) * BS + threadIdx.x;
    if (lane_cell >= rp.g.ncell / CPT) return;
    stream_only_lane<C, CPT, NTS>(A + rp.pop_off, B + rp.pop_off, rp.g, lane_cell);
}

template <class C>
__global__ __launch_bounds__(kParticleBlock) void k_ens_particle(
    const typename C::T *__restrict__ A, const Replica *__restrict__ reps,
    const uint16_t *__restrict__ part_rep, typename C::R dec_s, ParticleArgs pa,
    const EnsClock *__restrict__ clock, long long *force_cur, uint32_t *mask_cur,
    long long *force_old, uint32_t *mask_old) {
    const uint32_t gt = blockIdx.x * kParticleBlock + threadIdx.x;
    const int32_t i = int32_t(gt >> 3);
    const int p = int(gt & 7u);
    const bool valid = i < pa.n;
    const int32_t ii = valid ? i : pa.n - 1;
    // step-dependent values from the device clock
    pa.step = uint32_t(clock->step);
    if (pa.acc) {
        const int64_t t = clock->vacf_t;
        pa.t = t;
        pa.k_hi = t / pa.stride;
        pa.k_lo = t > pa.max_lag ? (t - pa.max_lag + pa.stride - 1) / pa.stride : 0;
        pa.slot_lo = int32_t(pa.k_lo % pa.nslot);
    }
    double r[3], V[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = pa.r[3 * ii + k];
        V[k] = pa.v[3 * ii + k];
    }
    const Replica &rp = reps[part_rep[ii]];
    const ParticleSite<C> site{A + rp.pop_off,
                               rp.g,
                               ForceField{force_cur + 3 * rp.cell_off, mask_cur + rp.mask_off},
                               ForceField{force_old + 3 * rp.cell_off, mask_old + rp.mask_off},
                               rp.seed,
                               rp.replica_id,
                               uint32_t(ii) - rp.part_off,
                               rp.R};
    particle_lane<C>(site, dec_s, pa, i, p, valid, r, V);
}

// ---------------------------------------------------------------------------
// Recorded observables: two fixed-order stages over the per-wavefront partials
// left by the stream-collide (rho~ - 1, u) and the per-block ones of the
// particle kernel (M V).
// ---------------------------------------------------------------------------
constexpr int kSeriesBlocks = 64;

__global__ __launch_bounds__(kBlock) void k_series_stage1(const double *__restrict__ fluid,
                                                          int32_t nfluid,
                                                          const double *__restrict__ part,
                                                          int32_t npart,
                                                          double *__restrict__ stage) {
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const int32_t stride = kSeriesBlocks * kBlock;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < nfluid; i += stride)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += fluid[4 * int64_t(i) + k];
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < npart; i += stride)
#pragma unroll
        for (int k = 0; k < 3; ++k) v[4 + k] += part[3 * int64_t(i) + k];
    block_sum<7, kBlock>(v, stage + 7 * blockIdx.x);
}

__global__ void k_series_stage2(const double *__restrict__ stage, double ncell, double step,
                                double *__restrict__ out) {
    if (threadIdx.x < 7) {
        double s = 0.0;
        for (int b = 0; b < kSeriesBlocks; ++b) s += stage[7 * b + threadIdx.x];
        out[1 + threadIdx.x] = threadIdx.x == 0 ? ncell + s : s;
    }
    if (threadIdx.x == 0) out[0] = step;
}

// ---------------------------------------------------------------------------
// Field access kernels (set-up and diagnostics, not on the stepping path).
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(kBlock) void k_get_populations(const typename C::T *__restrict__ A,
                                                            Grid g, typename C::R dec_s,
                                                            double *__restrict__ f) {
    using Vs = typename C::V;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    static_for<0, Vs::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[uint64_t(a) * g.ncell + cell] =
            double(C::dec(A[nb.template pop<Vs, a>(g)], dec_s)) + Vs::template w<double>(a);
    });
}

template <class C>
__global__ __launch_bounds__(kBlock) void k_get_moments(const typename C::T *__restrict__ A,
                                                        Grid g, typename C::R dec_s,
                                                        double *__restrict__ rho,
                                                        double *__restrict__ u) {
    using Vs = typename C::V;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    double dr = 0.0, m[3] = {0.0, 0.0, 0.0};
    static_for<0, Vs::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        const double gvl = double(C::dec(A[nb.template pop<Vs, a>(g)], dec_s));
        dr += gvl;
        m[0] += Vs::ex[a] * gvl;
        m[1] += Vs::ey[a] * gvl;
        m[2] += Vs::ez[a] * gvl;
    });
    if (rho) rho[cell] = 1.0 + dr;
    if (u) {
        u[cell] = m[0];
        u[uint64_t(g.ncell) + cell] = m[1];
        u[2 * uint64_t(g.ncell) + cell] = m[2];
    }
}

// A_a(y) = enc(f_a(y + e_a) - w_a): the post-streaming population at node x is
// the pulled value A_a(x - e_a).
template <class C>
__global__ __launch_bounds__(kBlock) void k_set_populations(const double *__restrict__ f,
                                                            typename C::T *__restrict__ A, Grid g,
                                                            typename C::R enc_s) {
    using Vs = typename C::V;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);  // nb.src of the opposite direction is y + e_a
    static_for<0, Vs::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int o = (a == 0) ? 0 : ((a & 1) ? a + 1 : a - 1);
        const double gvl = f[uint64_t(a) * g.ncell + nb.template src<Vs, o>(g)] - Vs::template w<double>(a);
        A[pop_index<Vs>(g, x, y, z, a)] = C::enc(typename C::R(gvl), enc_s);
    });
}

template <class C>
__global__ __launch_bounds__(kBlock) void k_set_equilibrium(const double *__restrict__ rho,
                                                            const double *__restrict__ u,
                                                            typename C::T *__restrict__ A, Grid g,
                                                            typename C::R enc_s) {
    using Vs = typename C::V;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    static_for<0, Vs::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int o = (a == 0) ? 0 : ((a & 1) ? a + 1 : a - 1);
        const uint32_t src = nb.template src<Vs, o>(g);  // node y + e_a
        const double dr = rho ? rho[src] - 1.0 : 0.0;
        double uc[3] = {0.0, 0.0, 0.0};
        if (u) {
            uc[0] = u[src];
            uc[1] = u[uint64_t(g.ncell) + src];
            uc[2] = u[2 * uint64_t(g.ncell) + src];
        }
        const double eu = Vs::ex[a] * uc[0] + Vs::ey[a] * uc[1] + Vs::ez[a] * uc[2];
        const double uu = uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2];
        const double geq = Vs::template w<double>(a) * (dr + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        A[pop_index<Vs>(g, x, y, z, a)] = C::enc(typename C::R(geq), enc_s);
    });
}

// The same populations in another row-group layout: B[in layout gb] =
// A[in layout ga], element for element (a permutation; no arithmetic).
template <class C>
__global__ __launch_bounds__(kBlock) void k_relayout(const typename C::T *__restrict__ A, Grid ga,
                                                     typename C::T *__restrict__ B, Grid gb) {
    using Vs = typename C::V;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ga.ncell) return;
    const uint32_t x = cell % ga.nx, t = cell / ga.nx, y = t % ga.ny, z = t / ga.ny;
    static_for<0, Vs::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        B[pop_index<Vs>(gb, x, y, z, a)] = A[pop_index<Vs>(ga, x, y, z, a)];
    });
}

// FP64 sums of (rho - 1, u) over all nodes: fixed grid, fixed tree order, so the
// result is deterministic.
template <class C>
__global__ __launch_bounds__(kBlock) void k_fluid_partials(const typename C::T *__restrict__ A,
                                                           Grid g, typename C::R dec_s,
                                                           double *__restrict__ partials) {
    using Vs = typename C::V;
    __shared__ double sh[4][kBlock];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t cell = blockIdx.x * kBlock + threadIdx.x; cell < g.ncell;
         cell += gridDim.x * kBlock) {
        const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
        const Neighbours nb(x, y, z, g);
        static_for<0, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            const double gvl = double(C::dec(A[nb.template pop<Vs, a>(g)], dec_s));
            acc[0] += gvl;
            acc[1] += Vs::ex[a] * gvl;
            acc[2] += Vs::ey[a] * gvl;
            acc[3] += Vs::ez[a] * gvl;
        });
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_final_sums(const double *__restrict__ partials,
                                                       int32_t nparts, double ncell,
                                                       const double *__restrict__ v, int32_t n,
                                                       double mass, double *__restrict__ out) {
    __shared__ double sh[7][kBlock];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int32_t b = threadIdx.x; b < nparts; b += kBlock)
        for (int k = 0; k < 4; ++k) acc[k] += partials[4 * b + k];
    for (int32_t i = threadIdx.x; i < n; i += kBlock)
        for (int k = 0; k < 3; ++k) acc[4 + k] += v[3 * i + k];
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h)
            for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ncell + sh[0][0];
        for (int k = 1; k < 4; ++k) out[k] = sh[k][0];
        for (int k = 0; k < 3; ++k) out[4 + k] = mass * sh[4 + k][0];
    }
}

}  // namespace lbmbp

// ===========================================================================
// Host side: the C ABI.
// ===========================================================================
using namespace lbmbp;

struct lbm_ctx {
    lbm_grid_desc desc;
    Grid g;
    int q;  // velocity set: 19 or 15
    size_t elem;
    void *pop[2];  // pop[cur] holds post-collision values of the last step
    int cur;
    hipStream_t stream;
    double omega;
    double enc_s, dec_s;
    double body[3];  // uniform body force on every node (lbm_set_body_force)
    // grid scratch
    uint32_t *mask[2];
    long long *force[2];  // [ncell][3] fixed-point node forces, alternating steps
    uint32_t mask_words;
    double *partials;
    double *result;
    uint32_t *err;
    // particles
    int32_t np;
    lbm_particle_desc pdesc;
    double R;
    double *r, *v;
    uint32_t *prev_cell;
    double *fh, *fr;
    const double *fext;  // given force on each particle (lbm_set_particle_force) or null
    uint32_t warnings;   // LBM_WARN_* of the attached particles
    // soft pair repulsion (lbm_set_pair_force)
    int pair_on;
    PairGrid pg;
    PairList plist;       // particle scratch: the cell list
    double *fpair;        // particle scratch: [n][3] pair forces of the last step
    // velocity autocorrelation
    int vacf_on;
    int32_t max_lag, stride, nslot;
    double *acc, *origins;
    int64_t vacf_t;
    int64_t step;
    // per-kernel event timing (host-side event objects)
    int prof_on;
    hipEvent_t *prof_ev;    // pairs: [2k] start, [2k+1] stop
    int32_t *prof_kind;     // per pair: 0 stream-collide, 1 particle phase
    int32_t prof_used, prof_cap;
    int shape;   // index into kShapes
    int order;   // block order of the sweep (kOrderLinear / kOrderXcdSlabs)
    int cap;     // residency cap of the sweep: index into kResidencyCaps
    int lds_cu, lds_block;  // LDS bytes per compute unit and per block (device limits)
    int device;  // device current at lbm_init (autotune cache key)
    // recorded observables (lbm_series_config)
    int32_t series_every;
    double *series;
    int64_t series_cap, series_count, series_t;
    double *fluid_partials;  // grid scratch: [collide wavefronts][4]
    double *series_stage;    // grid scratch: [kSeriesBlocks][7]
    double *part_partials;   // particle scratch: [particle blocks][3]
    // forward run kept for the adjoint (lbm_record)
    void *rec_tape;
    int64_t rec_n0;
    int32_t rec_nsteps, rec_every, rec_np;
    lbm_particle_desc rec_pdesc;
    double rec_R;
    const double *rec_fext;
    int rec_pair_on;
    PairGrid rec_pg;
    uint32_t rec_rows;  // layout (rows per group) of the recorded lattices
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t elem_size(int storage) {
    switch (storage) {
        case LBM_STORE_F64: return 8;
        case LBM_STORE_F32: return 4;
        case LBM_STORE_BF16:
        case LBM_STORE_F16: return 2;
        default: return 0;
    }
}

int velocity_count(const lbm_grid_desc *g) { return g->velocities == 15 ? 15 : 19; }

bool grid_ok(const lbm_grid_desc *g) {
    if (!g) return false;
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return false;
    const uint64_t nc = uint64_t(g->nx) * uint64_t(g->ny) * uint64_t(g->nz);
    if (nc >= (uint64_t(1) << 31)) return false;
    if (!(g->tau > 0.5) || !isfinite(g->tau)) return false;
    if (elem_size(g->storage) == 0) return false;
    if (g->storage == LBM_STORE_F16 && (g->f16_scale_log2 < 0 || g->f16_scale_log2 > 24)) return false;
    if (g->velocities != 0 && g->velocities != 19 && g->velocities != 15) return false;
    if (g->reserved != 0) return false;
    return true;
}

uint64_t ncell_of(const lbm_grid_desc *g) {
    return uint64_t(g->nx) * uint64_t(g->ny) * uint64_t(g->nz);
}

// Elements per population row: nx, unpadded.  (Padding rows to whole
// 128-byte lines left gaps between the rows of a row group and measured 4-14%
// slower at sizes that are not multiples of a line.)
uint32_t row_chunk(const lbm_grid_desc *g) { return uint32_t(g->nx); }

uint32_t mask_words(uint64_t ncell) { return uint32_t(align_up((ncell + 31) / 32, 64)); }

size_t force_field_bytes(const lbm_grid_desc *g) { return align_up(ncell_of(g) * 3 * 8, kAlign); }

// Blocks of the row-aligned stream-collide grid (configurations 8, 9).
uint32_t row_grid_blocks(uint32_t nx, uint32_t ny, uint32_t nz) {
    const uint32_t lpr = row_lanes(nx), nrows = ny * nz;
    if (lpr <= uint32_t(kRowBlock)) {
        const uint32_t rpb = uint32_t(kRowBlock) / lpr;  // rows per block
        return (nrows + rpb - 1) / rpb;
    }
    return nrows * ((lpr + kRowBlock - 1) / kRowBlock);
}

// Per-wavefront moment partials of the largest stream-collide grid: one node
// per lane in whole blocks of up to 512 lanes, or the row-aligned grid,
// whichever has more wavefronts.
size_t fluid_partials_bytes(const lbm_grid_desc *g) {
    const size_t flat = (ncell_of(g) / 512 + 1) * 8;
    const size_t row = row_grid_blocks(uint32_t(g->nx), uint32_t(g->ny), uint32_t(g->nz)) * (kRowBlock / 64);
    return align_up((flat > row ? flat : row) * 4 * 8, kAlign);
}

size_t grid_scratch_size(const lbm_grid_desc *g) {
    const size_t words = mask_words(ncell_of(g));
    size_t s = 0;
    s += 2 * align_up(words * 4, kAlign);            // two bitmasks
    s += 2 * force_field_bytes(g);                   // two node-force fields
    s += fluid_partials_bytes(g);                    // recorded-moment partials
    s += align_up(size_t(kSeriesBlocks) * 7 * 8, kAlign);
    s += align_up(size_t(kRedBlocks) * 4 * 8, kAlign);  // partials
    s += align_up(8 * 8, kAlign);                    // result
    s += kAlign;                                      // error flags
    return s;
}

size_t particle_blocks(int32_t n) { return (size_t(n) * 8 + kParticleBlock - 1) / kParticleBlock; }

// Advisory conditions of a particle set (section 2.2's parameter ranges and
// the sign of the fit's gain); see LBM_WARN_* in the header.
uint32_t coupling_warnings(int32_t friction, double R, int32_t n, double ncell) {
    uint32_t w = 0;
    const double s3 = sqrt(3.0);
    if (friction == LBM_FRICTION_STOKESLET || friction == LBM_FRICTION_STOKESLET_2DX ||
        friction == LBM_FRICTION_STOKESLET_CUBE) {
        const double span = friction == LBM_FRICTION_STOKESLET ? 1.0 : 2.0;  // cube edge
        if (R > s3 * span) w |= LBM_WARN_RADIUS_BOUND;
        if (R > 0.5 * s3 * span) w |= LBM_WARN_NEGATIVE_GAIN;
    }
    if (friction != LBM_FRICTION_BD && double(n) * (4.0 / 3.0) * M_PI * R * R * R > 0.1 * ncell)
        w |= LBM_WARN_VOLUME_FRACTION;
    return w;
}

// Buckets of the pair cell list: a power of two >= 2n.
uint32_t pair_buckets(int32_t n) {
    uint32_t T = 64;
    while (T < 2u * uint32_t(n)) T <<= 1;
    return T;
}

size_t pair_list_bytes(int32_t n) {
    const size_t T = pair_buckets(n);
    return align_up(size_t(n) * 8, kAlign) + 3 * align_up(size_t(n) * 4, kAlign) +
           align_up(T * 4, kAlign) + align_up((T + 1) * 4, kAlign);
}

// Carves the cell list out of pair_list_bytes(n) bytes at s.
PairList pair_list_at(char *s, int32_t n) {
    const size_t T = pair_buckets(n);
    PairList pl;
    pl.cell = reinterpret_cast<uint64_t *>(s);
    s += align_up(size_t(n) * 8, kAlign);
    pl.bucket = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(n) * 4, kAlign);
    pl.slot = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(n) * 4, kAlign);
    pl.list = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(n) * 4, kAlign);
    pl.count = reinterpret_cast<uint32_t *>(s);
    s += align_up(T * 4, kAlign);
    pl.start = reinterpret_cast<uint32_t *>(s);
    return pl;
}

size_t particle_scratch_size(int32_t n) {
    if (n <= 0) return 0;
    size_t s = 0;
    s += align_up(size_t(n) * 8 * 4, kAlign);  // prev cell
    s += align_up(particle_blocks(n) * 3 * 8, kAlign);  // momentum partials
    s += 2 * align_up(size_t(n) * 3 * 8, kAlign);  // fh, fr
    s += pair_list_bytes(n);                       // pair cell list
    s += align_up(size_t(n) * 3 * 8, kAlign);      // pair forces
    return s;
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

lbm_status launch_status() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

unsigned blocks_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }
// Launch configuration k of the stream-collide: CALL(nodes per lane, block,
// non-temporal stores, row-aligned mapping).  Ensembles take k < 8 only.
#define LBM_CONFIG_SWITCH(k, CALL)                  \
    switch (k) {                                    \
        case 1: CALL(1, 256, false, false); break;  \
        case 2: CALL(2, 512, false, false); break;  \
        case 3: CALL(2, 256, false, false); break;  \
        case 4: CALL(1, 512, true, false); break;   \
        case 5: CALL(1, 256, true, false); break;   \
        case 6: CALL(2, 512, true, false); break;   \
        case 7: CALL(2, 256, true, false); break;   \
        case 8: CALL(1, 256, false, true); break;   \
        case 9: CALL(1, 256, true, true); break;    \
        default: CALL(1, 512, false, false); break; \
    }

// The row-aligned mapping places lanes exactly as configurations 1 and 5 do
// when every 256-lane block holds whole rows that fill it (64 | nx and nx
// divides 256) or every row fills whole blocks (256 | nx).
bool row_mapping_is_flat(uint32_t nx) { return nx % 64 == 0 && (256 % nx == 0 || nx % 256 == 0); }

bool shape_ok(const lbm_ctx *c, int k) {
    return config_row(k) || c->g.ny % uint32_t(kShapes[k & 3].cpt) == 0;
}

uint32_t collide_grid(const lbm_ctx *c, int shape) {
    if (config_row(shape)) return row_grid_blocks(c->g.nx, c->g.ny, c->g.nz);
    const CollideShape &sh = kShapes[shape & 3];
    const uint64_t band = c->g.ncell / uint32_t(sh.cpt);
    return uint32_t((band + sh.bs - 1) / sh.bs);
}

// Dynamic LDS that caps the sweep at kResidencyCaps[cap] waves per SIMD for
// blocks of bs lanes (0: no cap); -1 if the device cannot impose that cap.
// The kernels never touch it: it only keeps further blocks off the unit.
// Up to 1 KiB of the unit is left for the kernels' own LDS.
long residency_lds(int lds_cu, int lds_block, int cap, int bs) {
    const int waves = kResidencyCaps[cap];
    if (waves == 0) return 0;
    // bs / 64 waves per block over the unit's four SIMDs: `blocks` resident
    // blocks give blocks * bs / 256 waves per SIMD
    const int blocks = waves * 256 / bs;
    if (blocks < 1 || lds_cu <= 0) return -1;
    const long per = (long(lds_cu) / blocks - 1024) / 512 * 512;
    if (per <= 0 || per + 1024 > lds_block) return -1;
    if (long(blocks + 1) * per <= lds_cu) return -1;  // would not cap
    return per;
}

long sweep_lds(const lbm_ctx *c, int cap, int bs) { return residency_lds(c->lds_cu, c->lds_block, cap, bs); }

// Addressing of the sweep (kAddr* in collide.hpp).  The row-aligned mapping
// always addresses by wavefront rows.  The flat mapping does so for 16-bit
// storage when rows are whole wavefronts: there the per-lane index arithmetic
// competes with the collision for the vector unit (FP16 step 1.8%, BF16 0.4%
// faster by rows, measured A/B on one device).  FP32 and FP64 sweeps are
// memory-bound, and per-lane indices measured as fast or faster (FP32 step
// 0.9%: its sum-carrying launches run longer by rows); those are in 32 bits
// unless the lattice holds 2^32 or more elements (Q nx ny nz; boxes beyond
// about 226M nodes).
int sweep_addr(const lbm_ctx *c, bool row_mapping) {
    if (row_mapping || (c->elem == 2 && c->g.nx % 64 == 0)) return kAddrRow;
    return uint64_t(c->q) * c->g.ncell >= (uint64_t(1) << 32) ? kAddrLane64 : kAddrLane32;
}

template <class C, bool FORCED, bool MOMENTS, int CPT, int BS, bool NTS, bool ROW, int ADDR>
void launch_collide_addr(lbm_ctx *c, const typename C::T *A, typename C::T *B, ForceField ff,
                         double *mom, unsigned grid, int order, size_t dyn) {
    using R = typename C::R;
    hipLaunchKernelGGL((k_stream_collide<C, FORCED, MOMENTS, CPT, BS, NTS, ROW, ADDR>), dim3(grid),
                       dim3(BS), dyn, c->stream, A, B, c->g, R(c->omega), R(c->enc_s), R(c->dec_s),
                       ff, R(c->body[0]), R(c->body[1]), R(c->body[2]), mom, uint32_t(order));
}

template <class C, bool FORCED, bool MOMENTS, int CPT, int BS, bool NTS, bool ROW>
void launch_collide_shape(lbm_ctx *c, const typename C::T *A, typename C::T *B, ForceField ff,
                          double *mom, unsigned grid, int order, int cap) {
    const long lds = sweep_lds(c, cap, BS);
    const size_t dyn = lds > 0 ? size_t(lds) : 0;
    const int addr = sweep_addr(c, ROW);
    if constexpr (ROW) {
        launch_collide_addr<C, FORCED, MOMENTS, CPT, BS, NTS, ROW, kAddrRow>(c, A, B, ff, mom, grid, order, dyn);
    } else {
        if (addr == kAddrRow)
            launch_collide_addr<C, FORCED, MOMENTS, CPT, BS, NTS, ROW, kAddrRow>(c, A, B, ff, mom, grid, order, dyn);
        else if (addr == kAddrLane64)
            launch_collide_addr<C, FORCED, MOMENTS, CPT, BS, NTS, ROW, kAddrLane64>(c, A, B, ff, mom, grid, order, dyn);
        else
            launch_collide_addr<C, FORCED, MOMENTS, CPT, BS, NTS, ROW, kAddrLane32>(c, A, B, ff, mom, grid, order, dyn);
    }
}

// mom != nullptr: also leave the per-wavefront FP64 moment sums there.  order,
// cap: block order and residency cap (-1: the context's).
template <class C, bool FORCED>
void launch_collide(lbm_ctx *c, const typename C::T *A, typename C::T *B, ForceField ff, int shape,
                    double *mom = nullptr, int order = -1, int cap = -1) {
    const unsigned grid = collide_grid(c, shape);
    if (order < 0) order = c->order;
    if (cap < 0) cap = c->cap;
#define LBM_SHAPE(CPT, BS, NTS, ROW)                                                           \
    do {                                                                                       \
        if (mom)                                                                               \
            launch_collide_shape<C, FORCED, true, CPT, BS, NTS, ROW>(c, A, B, ff, mom, grid,    \
                                                                     order, cap);              \
        else                                                                                   \
            launch_collide_shape<C, FORCED, false, CPT, BS, NTS, ROW>(c, A, B, ff, mom, grid,   \
                                                                      order, cap);             \
    } while (0)
    LBM_CONFIG_SWITCH(shape, LBM_SHAPE)
#undef LBM_SHAPE
}

ForceField field(lbm_ctx *c, int par) { return ForceField{c->force[par], c->mask[par]}; }

// Blocks for the neighbour sums: kPairLanes lanes per particle.
dim3 pair_group_blocks(int32_t n) {
    return dim3(unsigned((size_t(n) * kPairLanes + kPairBlock - 1) / kPairBlock));
}

// Pair forces of the positions r: build the cell list (its counts start and
// end at zero), then the neighbour sums.
void launch_pairs(hipStream_t st, const double *r, int32_t n, const PairGrid &pg, const PairList &pl,
                  double *F) {
    const dim3 pblocks(unsigned((n + kPairBlock - 1) / kPairBlock));
    hipLaunchKernelGGL(k_pair_count, pblocks, dim3(kPairBlock), 0, st, r, n, pg, pl);
    hipLaunchKernelGGL(k_pair_scan, dim3(1), dim3(kPairScanThreads), 0, st, pg, pl);
    hipLaunchKernelGGL(k_pair_scatter, pblocks, dim3(kPairBlock), 0, st, n, pl);
    hipLaunchKernelGGL(k_pair_bucket_sort, dim3((pg.T + kPairBlock - 1) / kPairBlock), dim3(kPairBlock), 0,
                       st, pg, pl);
    hipLaunchKernelGGL(k_pair_force, pair_group_blocks(n), dim3(kPairBlock), 0, st, r, n, pg, pl, F);
}

// Returns the start event of a new timing pair (or nullptr when profiling is
// off); the caller records it before the launch and prof_stop after.
bool prof_grow(lbm_ctx *c) {
    const int32_t cap = c->prof_cap ? 2 * c->prof_cap : 256;
    hipEvent_t *ev = static_cast<hipEvent_t *>(realloc(c->prof_ev, sizeof(hipEvent_t) * 2 * cap));
    if (!ev) return false;
    c->prof_ev = ev;
    int32_t *kind = static_cast<int32_t *>(realloc(c->prof_kind, sizeof(int32_t) * cap));
    if (!kind) return false;
    c->prof_kind = kind;
    for (int32_t k = 2 * c->prof_cap; k < 2 * cap; ++k)
        if (hipEventCreate(&c->prof_ev[k]) != hipSuccess) return false;
    c->prof_cap = cap;
    return true;
}

int32_t prof_start(lbm_ctx *c, int32_t kind) {
    if (!c->prof_on) return -1;
    if (c->prof_used == c->prof_cap && !prof_grow(c)) return -1;
    const int32_t k = c->prof_used++;
    c->prof_kind[k] = kind;
    (void)hipEventRecord(c->prof_ev[2 * k], c->stream);
    return k;
}

void prof_stop(lbm_ctx *c, int32_t k) {
    if (k >= 0) (void)hipEventRecord(c->prof_ev[2 * k + 1], c->stream);
}

template <class C>
void launch_step(lbm_ctx *c) {
    using T = typename C::T;
    using R = typename C::R;
    const T *A = static_cast<const T *>(c->pop[c->cur]);
    T *B = static_cast<T *>(c->pop[c->cur ^ 1]);
    const int par = int(c->step & 1);
    // Record the observables of the state at the start of this step?
    const bool sample = c->series_every > 0 && c->series_t % c->series_every == 0 &&
                        c->series_count < c->series_cap;
    if (c->series_every > 0) c->series_t += 1;
    double *mom = sample ? c->fluid_partials : nullptr;
    if (c->np > 0) {
        const int32_t pk = prof_start(c, 1);
        ParticleArgs pa;
        pa.pmom = sample ? c->part_partials : nullptr;
        pa.acc = nullptr;
        pa.origins = nullptr;
        pa.t = pa.k_lo = 0;
        pa.k_hi = -1;
        pa.nslot = pa.stride = 1;
        pa.max_lag = 0;
        pa.slot_lo = 0;
        if (c->vacf_on) {
            // active origins k*stride with t - max_lag <= k*stride <= t
            const int64_t t = c->vacf_t;
            pa.acc = c->acc;
            pa.origins = c->origins;
            pa.t = t;
            pa.k_hi = t / c->stride;
            pa.k_lo = t > c->max_lag ? (t - c->max_lag + c->stride - 1) / c->stride : 0;
            pa.nslot = c->nslot;
            pa.slot_lo = int32_t(pa.k_lo % c->nslot);
            pa.stride = c->stride;
            pa.max_lag = c->max_lag;
            c->vacf_t += 1;
        }
        pa.r = c->r;
        pa.v = c->v;
        pa.fh = c->fh;
        pa.fr = c->fr;
        pa.prev_cell = c->prev_cell;
        pa.err = c->err;
        pa.n = c->np;
        pa.friction = c->pdesc.friction;
        pa.mass = c->pdesc.mass;
        pa.gamma = c->pdesc.gamma;
        pa.sig = c->pdesc.kT > 0.0 ? sqrt(2.0 * c->pdesc.gamma * c->pdesc.kT) : 0.0;
        pa.R = c->R;
        pa.seed = c->pdesc.seed;
        pa.replica = c->pdesc.replica;
        pa.step = uint32_t(c->step);
        pa.fext = c->fext;
        pa.fpair = nullptr;
        if (c->pair_on) {
            launch_pairs(c->stream, c->r, c->np, c->pg, c->plist, c->fpair);
            pa.fpair = c->fpair;
        }
        hipLaunchKernelGGL(k_particle<C>, dim3(unsigned((uint64_t(c->np) * 8 + kParticleBlock - 1) / kParticleBlock)), dim3(kParticleBlock), 0,
                           c->stream, A, c->g, R(c->dec_s), pa, field(c, par), field(c, par ^ 1));
        prof_stop(c, pk);
        const int32_t ck = prof_start(c, 0);
        launch_collide<C, true>(c, A, B, field(c, par), c->shape, mom);
        prof_stop(c, ck);
    } else {
        const int32_t ck = prof_start(c, 0);
        launch_collide<C, false>(c, A, B, field(c, par), c->shape, mom);
        prof_stop(c, ck);
    }
    if (sample) {
        const int32_t np_blocks = c->np > 0 ? int32_t(particle_blocks(c->np)) : 0;
        hipLaunchKernelGGL(k_series_stage1, dim3(kSeriesBlocks), dim3(kBlock), 0, c->stream,
                           c->fluid_partials,
                           int32_t(collide_grid(c, c->shape) * (config_block(c->shape) / 64)),
                           c->part_partials,
                           np_blocks, c->series_stage);
        hipLaunchKernelGGL(k_series_stage2, dim3(1), dim3(64), 0, c->stream, c->series_stage,
                           double(c->g.ncell), double(c->step), c->series + 8 * c->series_count);
        c->series_count += 1;
    }
    c->cur ^= 1;
    c->step += 1;
}

// Times stream-collide launches on A -> B without swapping (the simulation
// state in A is untouched; B is the next step's output anyway): ms[j] for
// the launch (ks[j], orders[j], caps[j]), -1 where it does not apply.  With
// particles attached the forced variant is timed, reading the node forces of
// the last step (still in place until the next particle kernel).
template <class C>
void time_launches(lbm_ctx *c, int32_t iters, int n, const int *ks, const int *orders,
                   const int *caps, double *ms, hipError_t *err) {
    using T = typename C::T;
    const T *A = static_cast<const T *>(c->pop[c->cur]);
    T *B = static_cast<T *>(c->pop[c->cur ^ 1]);
    hipEvent_t e0, e1;
    *err = hipEventCreate(&e0);
    if (*err == hipSuccess) *err = hipEventCreate(&e1);
    if (*err != hipSuccess) return;
    const bool forced = c->np > 0;
    const ForceField last = field(c, int((c->step + 1) & 1));
    for (int j = 0; j < n && *err == hipSuccess; ++j) {
        const int k = ks[j], order = orders[j], cap = caps[j];
        ms[j] = -1.0;
        if (!shape_ok(c, k) || (config_row(k) && row_mapping_is_flat(c->g.nx))) continue;
        if (sweep_lds(c, cap, config_block(k)) < 0) continue;
        auto launch = [&]() {
            if (forced)
                launch_collide<C, true>(c, A, B, last, k, nullptr, order, cap);
            else
                launch_collide<C, false>(c, A, B, last, k, nullptr, order, cap);
        };
        for (int w = 0; w < 2; ++w) launch();
        (void)hipEventRecord(e0, c->stream);
        for (int it = 0; it < iters; ++it) launch();
        (void)hipEventRecord(e1, c->stream);
        *err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (*err == hipSuccess) *err = hipEventElapsedTime(&t, e0, e1);
        ms[j] = double(t) / iters;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

// Mean time per launch of the streaming-only kernel in configuration k with
// the context's block order and residency cap, over iters launches (A -> B,
// as the autotuner's trial launches).
template <class C, int CPT, int BS, bool NTS, bool ROW>
void stream_only_shape(lbm_ctx *c, const typename C::T *A, typename C::T *B, unsigned grid,
                       uint32_t order, size_t dyn) {
    const int addr = sweep_addr(c, ROW);
    if constexpr (ROW) {
        hipLaunchKernelGGL((k_stream_only<C, CPT, BS, NTS, ROW, kAddrRow>), dim3(grid), dim3(BS), dyn,
                           c->stream, A, B, c->g, order);
    } else {
        if (addr == kAddrRow)
            hipLaunchKernelGGL((k_stream_only<C, CPT, BS, NTS, ROW, kAddrRow>), dim3(grid), dim3(BS), dyn,
                               c->stream, A, B, c->g, order);
        else if (addr == kAddrLane64)
            hipLaunchKernelGGL((k_stream_only<C, CPT, BS, NTS, ROW, kAddrLane64>), dim3(grid), dim3(BS),
                               dyn, c->stream, A, B, c->g, order);
        else
            hipLaunchKernelGGL((k_stream_only<C, CPT, BS, NTS, ROW, kAddrLane32>), dim3(grid), dim3(BS),
                               dyn, c->stream, A, B, c->g, order);
    }
}

template <class C>
void time_stream_only(lbm_ctx *c, int k, int32_t iters, double *ms, hipError_t *err) {
    using T = typename C::T;
    const T *A = static_cast<const T *>(c->pop[c->cur]);
    T *B = static_cast<T *>(c->pop[c->cur ^ 1]);
    const unsigned grid = collide_grid(c, k);
    const long lds = sweep_lds(c, c->cap, config_block(k));
    const size_t dyn = lds > 0 ? size_t(lds) : 0;
    const uint32_t order = uint32_t(c->order);
    auto launch = [&]() {
#define LBM_STREAM_ONLY(CPT, BS, NTS, ROW) stream_only_shape<C, CPT, BS, NTS, ROW>(c, A, B, grid, order, dyn)
        LBM_CONFIG_SWITCH(k, LBM_STREAM_ONLY)
#undef LBM_STREAM_ONLY
    };
    hipEvent_t e0, e1;
    *err = hipEventCreate(&e0);
    if (*err == hipSuccess) *err = hipEventCreate(&e1);
    if (*err != hipSuccess) return;
    for (int w = 0; w < 2; ++w) launch();
    (void)hipEventRecord(e0, c->stream);
    for (int it = 0; it < iters; ++it) launch();
    (void)hipEventRecord(e1, c->stream);
    *err = hipEventSynchronize(e1);
    float t = 0.0f;
    if (*err == hipSuccess) *err = hipEventElapsedTime(&t, e0, e1);
    *ms = double(t) / iters;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

template <class C>
void launch_get_populations(lbm_ctx *c, double *f) {
    hipLaunchKernelGGL(k_get_populations<C>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0,
                       c->stream, static_cast<const typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->dec_s), f);
}

template <class C>
void launch_get_moments(lbm_ctx *c, double *rho, double *u) {
    hipLaunchKernelGGL(k_get_moments<C>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0,
                       c->stream, static_cast<const typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->dec_s), rho, u);
}

template <class C>
void launch_set_populations(lbm_ctx *c, const double *f) {
    hipLaunchKernelGGL(k_set_populations<C>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0,
                       c->stream, f, static_cast<typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->enc_s));
}

template <class C>
void launch_set_equilibrium(lbm_ctx *c, const double *rho, const double *u) {
    hipLaunchKernelGGL(k_set_equilibrium<C>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0,
                       c->stream, rho, u, static_cast<typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->enc_s));
}

template <class C>
void launch_partials(lbm_ctx *c, double *partials) {
    hipLaunchKernelGGL(k_fluid_partials<C>, dim3(kRedBlocks), dim3(kBlock), 0, c->stream,
                       static_cast<const typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->dec_s), partials);
}

// Moves the state into the layout with Y rows per group: the current lattice
// is permuted into the spare one and copied back, so the current populations
// stay in the same buffer.
template <class C>
void launch_relayout(lbm_ctx *c, uint32_t Y, hipError_t *err) {
    const Grid gn = with_rows_per_group(c->g, Y);
    hipLaunchKernelGGL(k_relayout<C>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0, c->stream,
                       static_cast<const typename C::T *>(c->pop[c->cur]), c->g,
                       static_cast<typename C::T *>(c->pop[c->cur ^ 1]), gn);
    size_t lat = 0;
    lbm_lattice_bytes(&c->desc, &lat);
    *err = hipMemcpyAsync(c->pop[c->cur], c->pop[c->cur ^ 1], lat, hipMemcpyDeviceToDevice,
                          c->stream);
    c->g = gn;
}

// The storage codec x velocity set combinations the library instantiates.
using F64Q19 = Cfg<CodecF64, D3Q19>;
using F32Q19 = Cfg<CodecF32, D3Q19>;
using BF16Q19 = Cfg<CodecBF16, D3Q19>;
using F16Q19 = Cfg<CodecF16, D3Q19>;
using F64Q15 = Cfg<CodecF64, D3Q15>;
using F32Q15 = Cfg<CodecF32, D3Q15>;
using BF16Q15 = Cfg<CodecBF16, D3Q15>;
using F16Q15 = Cfg<CodecF16, D3Q15>;

#define LBM_DISPATCH(ctx, FN, ...)                                                      \
    do {                                                                                \
        if ((ctx)->q == 15) {                                                           \
            switch ((ctx)->desc.storage) {                                              \
                case LBM_STORE_F64: FN<F64Q15>(ctx, ##__VA_ARGS__); break;              \
                case LBM_STORE_F32: FN<F32Q15>(ctx, ##__VA_ARGS__); break;              \
                case LBM_STORE_BF16: FN<BF16Q15>(ctx, ##__VA_ARGS__); break;            \
                case LBM_STORE_F16: FN<F16Q15>(ctx, ##__VA_ARGS__); break;              \
            }                                                                           \
        } else {                                                                        \
            switch ((ctx)->desc.storage) {                                              \
                case LBM_STORE_F64: FN<F64Q19>(ctx, ##__VA_ARGS__); break;              \
                case LBM_STORE_F32: FN<F32Q19>(ctx, ##__VA_ARGS__); break;              \
                case LBM_STORE_BF16: FN<BF16Q19>(ctx, ##__VA_ARGS__); break;            \
                case LBM_STORE_F16: FN<F16Q19>(ctx, ##__VA_ARGS__); break;              \
            }                                                                           \
        }                                                                               \
    } while (0)

}  // namespace

extern "C" {

lbm_status lbm_lattice_bytes(const lbm_grid_desc *grid, size_t *bytes) {
    if (!grid_ok(grid) || !bytes) return LBM_E_INVAL;
    *bytes = align_up(size_t(row_chunk(grid)) * size_t(velocity_count(grid)) * size_t(grid->ny) *
                          size_t(grid->nz) *
                          elem_size(grid->storage),
                      kAlign);
    return LBM_OK;
}

lbm_status lbm_grid_scratch_bytes(const lbm_grid_desc *grid, size_t *bytes) {
    if (!grid_ok(grid) || !bytes) return LBM_E_INVAL;
    *bytes = grid_scratch_size(grid);
    return LBM_OK;
}

lbm_status lbm_particle_scratch_bytes(const lbm_grid_desc *grid, int32_t n, size_t *bytes) {
    if (!grid_ok(grid) || !bytes || n < 0 || n > (1 << 24)) return LBM_E_INVAL;
    *bytes = particle_scratch_size(n);
    return LBM_OK;
}

lbm_status lbm_vacf_origin_bytes(int32_t n, int32_t max_lag, int32_t stride, size_t *bytes) {
    if (!bytes || n < 0 || max_lag < 0 || stride < 1) return LBM_E_INVAL;
    *bytes = size_t(max_lag / stride + 1) * size_t(n) * 3 * sizeof(double);
    return LBM_OK;
}

}  // extern "C"

// Device memory of lbm_observables_noalloc: the FP64 reduction partials
// ([kRedBlocks][4]) followed by the seven sums.  Every device the library runs
// on holds one copy until the process ends.  Host code never passes this name
// to a kernel or a copy (on the host it is only a stand-in for the symbol):
// it uses the device address that hipGetSymbolAddress returned for that
// device, kept in g_noalloc below.
constexpr size_t kNoAllocDoubles = size_t(kRedBlocks) * 4 + 8;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

// Device address of `scratch` per device, looked up once per device by
// lbm_init (with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
bool g_noalloc_done[kMaxDevices];
double *g_noalloc[kMaxDevices];

void noalloc_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_done[dev]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_noalloc[dev] = (e == hipSuccess) ? static_cast<double *>(p) : nullptr;
    g_noalloc_done[dev] = true;
}

double *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return g_noalloc[dev];
}

}  // namespace

namespace {

// Launch configurations the autotuners chose, kept for the life of the
// process and keyed by device, storage, velocity set and the sizes of every
// box: a context or ensemble created later with the same key starts from that
// choice instead of the size-based default.
struct TuneKey {
    int kind;  // 0 single box (its code holds configuration, order and cap), 1 ensemble
    int device, storage, q;
    std::vector<int32_t> dims;  // nx, ny, nz of each box
    bool operator<(const TuneKey &o) const {
        return std::tie(kind, device, storage, q, dims) <
               std::tie(o.kind, o.device, o.storage, o.q, o.dims);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

int current_device() {
    int d = 0;
    return hipGetDevice(&d) == hipSuccess ? d : -1;
}

int tune_lookup(const TuneKey &k, int fallback) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(k);
    return it == g_tune.end() ? fallback : it->second;
}

void tune_store(const TuneKey &k, int shape) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[k] = shape;
}

// A single-box choice is kept as one code: configuration, block order,
// residency cap and layout (log2 of the rows per group); an ensemble's code
// holds the same four, its layout being the rows per group requested of
// every box.
int tune_code(int shape, int order, int cap, int rows_log2) {
    return shape + kNumShapes * (order + int(kNumOrders) * (cap + kNumCaps * rows_log2));
}

int rows_log2(const Grid &g) {
    int k = 0;
    while ((1u << k) < g.ymask + 1u) ++k;
    return k;
}

// Layouts of the lattice: 1, 2, 4, ..., 64 rows per group, those that divide ny.
constexpr int kMaxRowsLog2 = 6;

int layout_candidates(const lbm_ctx *c, uint32_t *ys) {
    int n = 0;
    for (int k = 0; k <= kMaxRowsLog2; ++k)
        if (c->g.ny % (1u << k) == 0) ys[n++] = 1u << k;
    return n;
}

// Puts the state into the layout with Y rows per group (no change of value).
lbm_status set_layout(lbm_ctx *c, uint32_t Y) {
    if (Y == c->g.ymask + 1u) return LBM_OK;
    hipError_t err = hipSuccess;
    LBM_DISPATCH(c, launch_relayout, Y, &err);
    const lbm_status st = launch_status();
    return err != hipSuccess ? LBM_E_DEVICE : st;
}

TuneKey ctx_tune_key(const lbm_ctx *c) {
    return TuneKey{0, c->device, c->desc.storage, c->q, {c->desc.nx, c->desc.ny, c->desc.nz}};
}

}  // namespace

extern "C" {

lbm_status lbm_init(const lbm_grid_desc *grid, void *pop_a, void *pop_b, void *grid_scratch,
                    void *stream, lbm_ctx **out) {
    if (!grid_ok(grid) || !pop_a || !pop_b || !grid_scratch || !out) return LBM_E_INVAL;
    if (!aligned(pop_a) || !aligned(pop_b) || !aligned(grid_scratch) || pop_a == pop_b)
        return LBM_E_INVAL;
    lbm_ctx *c = static_cast<lbm_ctx *>(calloc(1, sizeof(lbm_ctx)));
    if (!c) return LBM_E_DEVICE;
    uint32_t init_rows = 1;
    c->desc = *grid;
    c->g.nx = uint32_t(grid->nx);
    c->g.ny = uint32_t(grid->ny);
    c->g.nz = uint32_t(grid->nz);
    c->g.ncell = uint32_t(ncell_of(grid));
    c->g.chunk = row_chunk(grid);
    c->g = with_rows_per_group(c->g, 1);
    c->q = velocity_count(grid);
    c->device = current_device();
    noalloc_setup(c->device);
    {
        size_t lat = 0;
        lbm_lattice_bytes(grid, &lat);
        // until lbm_autotune: the last choice for this key, else the row-aligned
        // mapping for rows that are not whole wavefronts (and long enough that
        // idle lanes are few), else by lattice size
        const int fallback = (grid->nx % 64 != 0 && grid->nx >= 96) ? kNumFlatShapes
                             : lat >= kStreamStoreBytes              ? kNumGeomShapes
                                                                     : 0;
        const int code = tune_lookup(ctx_tune_key(c), fallback);
        c->shape = code % kNumShapes;
        c->order = (code / kNumShapes) % int(kNumOrders);
        c->cap = (code / (kNumShapes * int(kNumOrders))) % kNumCaps;
        // the remembered layout, applied once the lattices are at rest below
        init_rows = uint32_t(1) << (code / (kNumShapes * int(kNumOrders) * kNumCaps));
        if (grid->ny % int32_t(init_rows) != 0) init_rows = 1;
        // LDS limits of the device, for the residency caps (none if unknown)
        int v = 0;
        c->lds_cu = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                           c->device) == hipSuccess) ? v : 0;
        c->lds_block = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                              c->device) == hipSuccess) ? v : 0;
        if (sweep_lds(c, c->cap, config_block(c->shape)) < 0) c->cap = 0;
    }
    c->elem = elem_size(grid->storage);
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->cur = 0;
    c->stream = static_cast<hipStream_t>(stream);
    c->omega = 1.0 / grid->tau;
    if (grid->storage == LBM_STORE_F16) {
        c->enc_s = ldexp(1.0, grid->f16_scale_log2);
        c->dec_s = ldexp(1.0, -grid->f16_scale_log2);
    } else {
        c->enc_s = c->dec_s = 1.0;
    }
    char *s = static_cast<char *>(grid_scratch);
    c->mask_words = mask_words(c->g.ncell);
    c->mask[0] = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(c->mask_words) * 4, kAlign);
    c->mask[1] = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(c->mask_words) * 4, kAlign);
    c->force[0] = reinterpret_cast<long long *>(s);
    s += force_field_bytes(grid);
    c->force[1] = reinterpret_cast<long long *>(s);
    s += force_field_bytes(grid);
    c->fluid_partials = reinterpret_cast<double *>(s);
    s += fluid_partials_bytes(grid);
    // every configuration's grid must fit the per-wavefront partials
    for (int k = 0; k < kNumShapes; ++k)
        if (shape_ok(c, k) &&
            size_t(collide_grid(c, k)) * (config_block(k) / 64) * 4 * 8 > fluid_partials_bytes(grid)) {
            free(c);
            return LBM_E_UNSUPPORTED;
        }
    c->series_stage = reinterpret_cast<double *>(s);
    s += align_up(size_t(kSeriesBlocks) * 7 * 8, kAlign);
    c->partials = reinterpret_cast<double *>(s);
    s += align_up(size_t(kRedBlocks) * 4 * 8, kAlign);
    c->result = reinterpret_cast<double *>(s);
    s += align_up(8 * 8, kAlign);
    c->err = reinterpret_cast<uint32_t *>(s);
    c->R = -1.0;

    size_t lat;
    lbm_lattice_bytes(grid, &lat);
    hipError_t e = hipMemsetAsync(pop_a, 0, lat, c->stream);  // g = 0 is the rest state
    if (e == hipSuccess) e = hipMemsetAsync(pop_b, 0, lat, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(grid_scratch, 0, grid_scratch_size(grid), c->stream);
    if (e != hipSuccess) {
        free(c);
        return LBM_E_DEVICE;
    }
    // the rest state is all zeros in every layout
    c->g = with_rows_per_group(c->g, init_rows);
    *out = c;
    return LBM_OK;
}

lbm_status lbm_set_equilibrium(lbm_ctx *ctx, const double *rho, const double *u) {
    if (!ctx) return LBM_E_INVAL;
    LBM_DISPATCH(ctx, launch_set_equilibrium, rho, u);
    return launch_status();
}

lbm_status lbm_set_populations(lbm_ctx *ctx, const double *f) {
    if (!ctx || !f) return LBM_E_INVAL;
    LBM_DISPATCH(ctx, launch_set_populations, f);
    return launch_status();
}

lbm_status lbm_set_body_force(lbm_ctx *ctx, const double *g) {
    if (!ctx) return LBM_E_INVAL;
    double v[3] = {0.0, 0.0, 0.0};
    if (g) {
        for (int k = 0; k < 3; ++k) {
            if (!isfinite(g[k])) return LBM_E_INVAL;
            v[k] = g[k];
        }
    }
    for (int k = 0; k < 3; ++k) ctx->body[k] = v[k];
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx *ctx, double *f) {
    if (!ctx || !f) return LBM_E_INVAL;
    LBM_DISPATCH(ctx, launch_get_populations, f);
    return launch_status();
}

lbm_status lbm_get_moments(lbm_ctx *ctx, double *rho, double *u) {
    if (!ctx || (!rho && !u)) return LBM_E_INVAL;
    LBM_DISPATCH(ctx, launch_get_moments, rho, u);
    return launch_status();
}

lbm_status particles_couple(lbm_ctx *ctx, const lbm_particle_desc *d, double *r, double *v,
                            void *particle_scratch) {
    if (!ctx || !d) return LBM_E_INVAL;
    if (d->n < 0 || d->n > (1 << 24) || d->reserved != 0) return LBM_E_INVAL;
    if (d->n > 0) {
        if (!r || !v || !particle_scratch || !aligned(particle_scratch)) return LBM_E_INVAL;
        if (!(d->mass > 0.0) || !isfinite(d->mass)) return LBM_E_INVAL;
        if (!(d->gamma >= 0.0) || !isfinite(d->gamma)) return LBM_E_INVAL;
        if (!(d->kT >= 0.0) || !isfinite(d->kT)) return LBM_E_INVAL;
        if (!isfinite(d->radius)) return LBM_E_INVAL;
        if (d->friction < LBM_FRICTION_STOKESLET || d->friction > LBM_FRICTION_STOKESLET_CUBE)
            return LBM_E_INVAL;
    }
    // Node forces left by any previous particle set are cleared.
    hipError_t e = hipMemsetAsync(ctx->mask[0], 0, size_t(ctx->mask_words) * 4, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->mask[1], 0, size_t(ctx->mask_words) * 4, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->force[0], 0, force_field_bytes(&ctx->desc), ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->force[1], 0, force_field_bytes(&ctx->desc), ctx->stream);
    if (e != hipSuccess) return LBM_E_DEVICE;
    ctx->vacf_on = 0;
    ctx->fext = nullptr;
    ctx->pair_on = 0;
    ctx->np = d->n;
    ctx->pdesc = *d;
    ctx->warnings = 0;
    if (d->n == 0) {
        ctx->R = -1.0;
        return LBM_OK;
    }
    // Stokes' law gamma = 6 pi eta R, eta = rho0 nu, nu = (tau - 1/2)/3.
    const double nu = (ctx->desc.tau - 0.5) / 3.0;
    ctx->R = d->radius > 0.0 ? d->radius : d->gamma / (6.0 * M_PI * nu);
    ctx->warnings = coupling_warnings(d->friction, ctx->R, d->n, double(ctx->g.ncell));
    ctx->r = r;
    ctx->v = v;
    char *s = static_cast<char *>(particle_scratch);
    ctx->prev_cell = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(d->n) * 8 * 4, kAlign);
    ctx->part_partials = reinterpret_cast<double *>(s);
    s += align_up(particle_blocks(d->n) * 3 * 8, kAlign);
    ctx->fh = reinterpret_cast<double *>(s);
    s += align_up(size_t(d->n) * 3 * 8, kAlign);
    ctx->fr = reinterpret_cast<double *>(s);
    s += align_up(size_t(d->n) * 3 * 8, kAlign);
    ctx->plist = pair_list_at(s, d->n);
    s += pair_list_bytes(d->n);
    ctx->fpair = reinterpret_cast<double *>(s);
    // prev_cell -> kNoNode (all ones); forces and bucket counts zero.
    e = hipMemsetAsync(ctx->prev_cell, 0xFF, size_t(d->n) * 8 * 4, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->plist.count, 0, size_t(pair_buckets(d->n)) * 4, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->fh, 0, size_t(d->n) * 3 * 8, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->fr, 0, size_t(d->n) * 3 * 8, ctx->stream);
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

lbm_status lbm_set_pair_force(lbm_ctx *ctx, double a_f, double r_c) {
    if (!ctx || !isfinite(a_f) || !isfinite(r_c)) return LBM_E_INVAL;
    if (a_f == 0.0) {
        ctx->pair_on = 0;
        return LBM_OK;
    }
    if (ctx->np == 0) return LBM_E_STATE;
    const uint32_t Ln[3] = {ctx->g.nx, ctx->g.ny, ctx->g.nz};
    const uint32_t lmin = Ln[0] < Ln[1] ? (Ln[0] < Ln[2] ? Ln[0] : Ln[2]) : (Ln[1] < Ln[2] ? Ln[1] : Ln[2]);
    if (!(r_c > 0.0) || r_c > 0.5 * double(lmin)) return LBM_E_INVAL;
    if (ctx->np > kPairMax) return LBM_E_UNSUPPORTED;
    PairGrid pg;
    for (int k = 0; k < 3; ++k) {
        const double cells = floor(double(Ln[k]) / r_c);
        pg.nc[k] = cells < 1.0 ? 1u : uint32_t(cells);
        pg.L[k] = double(Ln[k]);
    }
    pg.T = pair_buckets(ctx->np);
    pg.a = a_f;
    pg.rc = r_c;
    ctx->pg = pg;
    ctx->pair_on = 1;
    return LBM_OK;
}

lbm_status lbm_pair_forces(lbm_ctx *ctx, double *fc) {
    if (!ctx || !fc) return LBM_E_INVAL;
    if (ctx->np == 0) return LBM_E_STATE;
    const size_t bytes = size_t(ctx->np) * 3 * 8;
    const hipError_t e = ctx->pair_on
                             ? hipMemcpyAsync(fc, ctx->fpair, bytes, hipMemcpyDeviceToDevice, ctx->stream)
                             : hipMemsetAsync(fc, 0, bytes, ctx->stream);
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

lbm_status lbm_set_particle_force(lbm_ctx *ctx, const double *f) {
    if (!ctx) return LBM_E_INVAL;
    if (f && ctx->np == 0) return LBM_E_STATE;
    ctx->fext = f;
    return LBM_OK;
}

double lbm_particle_radius(const lbm_ctx *ctx) { return (ctx && ctx->np > 0) ? ctx->R : -1.0; }

lbm_status lbm_particle_forces(lbm_ctx *ctx, double *fh, double *fr) {
    if (!ctx) return LBM_E_INVAL;
    if (ctx->np == 0) return LBM_E_STATE;
    const size_t bytes = size_t(ctx->np) * 3 * 8;
    hipError_t e = hipSuccess;
    if (fh) e = hipMemcpyAsync(fh, ctx->fh, bytes, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess && fr)
        e = hipMemcpyAsync(fr, ctx->fr, bytes, hipMemcpyDeviceToDevice, ctx->stream);
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

lbm_status lbm_vacf_config(lbm_ctx *ctx, int32_t max_lag, int32_t stride, double *acc,
                           double *origins) {
    if (!ctx) return LBM_E_INVAL;
    if (max_lag == -1) {
        ctx->vacf_on = 0;
        return LBM_OK;
    }
    if (max_lag < 0 || stride < 1 || !acc || !origins) return LBM_E_INVAL;
    if (ctx->np == 0) return LBM_E_STATE;
    ctx->max_lag = max_lag;
    ctx->stride = stride;
    ctx->nslot = max_lag / stride + 1;
    ctx->acc = acc;
    ctx->origins = origins;
    ctx->vacf_t = 0;
    const hipError_t e = hipMemsetAsync(acc, 0, size_t(ctx->np) * size_t(max_lag + 1) * 8,
                                        ctx->stream);
    if (e != hipSuccess) return LBM_E_DEVICE;
    ctx->vacf_on = 1;
    return LBM_OK;
}

lbm_status lbm_vacf_counts(const lbm_ctx *ctx, int64_t *cnt) {
    if (!ctx || !cnt) return LBM_E_INVAL;
    if (!ctx->vacf_on) return LBM_E_STATE;
    // Samples t = 0 .. T-1; origins t0 = k * stride; lag l counts the origins
    // with t0 + l <= T - 1.
    const int64_t T = ctx->vacf_t;
    for (int32_t l = 0; l <= ctx->max_lag; ++l)
        cnt[l] = (T - 1 - l >= 0) ? (T - 1 - l) / ctx->stride + 1 : 0;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps) {
    if (!ctx || nsteps < 0) return LBM_E_INVAL;
    for (int32_t s = 0; s < nsteps; ++s) LBM_DISPATCH(ctx, launch_step);
    return launch_status();
}

}  // extern "C"

namespace {

// The sums of lbm_observables with the reduction partials ([kRedBlocks][4])
// and the result (7 doubles) in the given device buffers.
lbm_status observables_into(lbm_ctx *ctx, double *partials, double *result, double out[7]) {
    LBM_DISPATCH(ctx, launch_partials, partials);
    hipLaunchKernelGGL(k_final_sums, dim3(1), dim3(kBlock), 0, ctx->stream, partials,
                       kRedBlocks, double(ctx->g.ncell), ctx->np > 0 ? ctx->v : nullptr, ctx->np,
                       ctx->np > 0 ? ctx->pdesc.mass : 0.0, result);
    if (launch_status() != LBM_OK) return LBM_E_DEVICE;
    double host[7];
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(host, result, sizeof(host), hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&err, ctx->err, sizeof(err), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->err, 0, sizeof(uint32_t), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return LBM_E_DEVICE;
    bool finite = true;
    for (int k = 0; k < 7; ++k) {
        out[k] = host[k];
        finite = finite && isfinite(host[k]);
    }
    return (finite && err == 0) ? LBM_OK : LBM_E_NONFINITE;
}

}  // namespace

extern "C" {

lbm_status lbm_observables(lbm_ctx *ctx, double out[7]) {
    if (!ctx || !out) return LBM_E_INVAL;
    return observables_into(ctx, ctx->partials, ctx->result, out);
}

lbm_status lbm_observables_noalloc(lbm_ctx *ctx, double out[7]) {
    if (!ctx || !out) return LBM_E_INVAL;
    // the reduction runs over a fixed grid whatever the box or particle count,
    // so every context fits the array
    static_assert(kNoAllocDoubles >= size_t(kRedBlocks) * 4 + 7, "scratch too small");
    // the kernels run on the context's device, with that device's copy
    if (current_device() != ctx->device) return LBM_E_STATE;
    double *s = noalloc_scratch(ctx->device);
    if (!s) return LBM_E_DEVICE;
    return observables_into(ctx, s, s + size_t(kRedBlocks) * 4, out);
}

lbm_status lbm_profile_enable(lbm_ctx *ctx, int32_t enable) {
    if (!ctx || (enable != 0 && enable != 1)) return LBM_E_INVAL;
    ctx->prof_on = enable;
    return LBM_OK;
}

lbm_status lbm_profile_read(lbm_ctx *ctx, double out[4]) {
    if (!ctx || !out) return LBM_E_INVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return LBM_E_DEVICE;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t k = 0; k < ctx->prof_used; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->prof_ev[2 * k], ctx->prof_ev[2 * k + 1]) != hipSuccess)
            return LBM_E_DEVICE;
        const int kind = ctx->prof_kind[k];
        acc[2 * kind] += ms;
        acc[2 * kind + 1] += 1.0;
    }
    ctx->prof_used = 0;
    for (int k = 0; k < 4; ++k) out[k] = acc[k];
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *ctx, int32_t iters, double *ms, int32_t *chosen) {
    if (!ctx || iters < 1 || iters > 10000) return LBM_E_INVAL;
    uint32_t ys[kMaxRowsLog2 + 1];
    const int nl = layout_candidates(ctx, ys);
    constexpr int kMaxTrials = kNumShapes * kNumOrders * kNumCaps;
    int ks[kMaxTrials], os[kMaxTrials], cs[kMaxTrials];
    double t[kMaxTrials];
    hipError_t err = hipSuccess;
    double best_k[kNumShapes];
    for (int k = 0; k < kNumShapes; ++k) best_k[k] = -1.0;
    // every launch timed: configuration, order, cap, layout index, ms
    struct Trial {
        int k, o, c, l;
        double t;
    };
    std::vector<Trial> trials;
    auto note = [&](int k, int o, int c, int l, double v) {
        if (v <= 0.0) return;
        if (best_k[k] <= 0.0 || v < best_k[k]) best_k[k] = v;
        trials.push_back(Trial{k, o, c, l, v});
    };
    auto time_one_layout = [&](int l, int n) -> bool {
        if (set_layout(ctx, ys[l]) != LBM_OK) return false;
        LBM_DISPATCH(ctx, time_launches, iters, n, ks, os, cs, t, &err);
        return err == hipSuccess && launch_status() == LBM_OK;
    };
    // Stage 1: every configuration in linear order without a residency cap,
    // in every layout; keep the layout of the fastest launch.
    double t1[kMaxRowsLog2 + 1][kNumShapes];
    int bl = -1, first = -1;
    for (int l = 0; l < nl; ++l) {
        for (int k = 0; k < kNumShapes; ++k) ks[k] = k, os[k] = int(kOrderLinear), cs[k] = 0;
        if (!time_one_layout(l, kNumShapes)) return LBM_E_DEVICE;
        for (int k = 0; k < kNumShapes; ++k) {
            t1[l][k] = t[k];
            note(k, int(kOrderLinear), 0, l, t[k]);
            if (t[k] > 0.0 && (bl < 0 || t[k] < t1[bl][first])) bl = l, first = k;
        }
    }
    if (bl < 0) return LBM_E_DEVICE;
    // Stage 2: in that layout, its two fastest configurations with every block
    // order and cap.
    int second = -1;
    for (int k = 0; k < kNumShapes; ++k)
        if (k != first && t1[bl][k] > 0.0 && (second < 0 || t1[bl][k] < t1[bl][second])) second = k;
    int n = 0;
    for (int k : {first, second}) {
        if (k < 0) continue;
        for (int o = 0; o < int(kNumOrders); ++o)
            for (int cap = 0; cap < kNumCaps; ++cap) {
                if (o == int(kOrderLinear) && cap == 0) continue;  // timed in stage 1
                ks[n] = k, os[n] = o, cs[n] = cap;
                ++n;
            }
    }
    if (!time_one_layout(bl, n)) return LBM_E_DEVICE;
    Trial best{first, int(kOrderLinear), 0, bl, t1[bl][first]};
    for (int j = 0; j < n; ++j) {
        note(ks[j], os[j], cs[j], bl, t[j]);
        if (t[j] > 0.0 && t[j] < best.t) best = Trial{ks[j], os[j], cs[j], bl, t[j]};
    }
    // Stage 3: that launch in every other layout (a cap or order can change
    // which layout streams best).
    if (best.o != int(kOrderLinear) || best.c != 0) {
        const Trial b0 = best;
        for (int l = 0; l < nl; ++l) {
            if (l == b0.l) continue;
            ks[0] = b0.k, os[0] = b0.o, cs[0] = b0.c;
            if (!time_one_layout(l, 1)) return LBM_E_DEVICE;
            note(b0.k, b0.o, b0.c, l, t[0]);
        }
    }
    // Stage 4: single timings differ by a percent or two from run to run, so
    // the three fastest launches are timed again, in turn, twice each with
    // twice the iterations, and the lowest total wins.
    std::sort(trials.begin(), trials.end(), [](const Trial &x, const Trial &y) { return x.t < y.t; });
    const int m = int(std::min<size_t>(3, trials.size()));
    double total[3] = {0.0, 0.0, 0.0};
    for (int round = 0; round < 2; ++round)
        for (int j = 0; j < m; ++j) {
            ks[0] = trials[j].k, os[0] = trials[j].o, cs[0] = trials[j].c;
            if (set_layout(ctx, ys[trials[j].l]) != LBM_OK) return LBM_E_DEVICE;
            LBM_DISPATCH(ctx, time_launches, 2 * iters, 1, ks, os, cs, t, &err);
            if (err != hipSuccess || launch_status() != LBM_OK) return LBM_E_DEVICE;
            total[j] += t[0] > 0.0 ? t[0] : 1e30;
        }
    int jb = 0;
    for (int j = 1; j < m; ++j)
        if (total[j] < total[jb]) jb = j;
    best = trials[jb];
    if (set_layout(ctx, ys[best.l]) != LBM_OK) return LBM_E_DEVICE;
    ctx->shape = best.k;
    ctx->order = best.o;
    ctx->cap = best.c;
    tune_store(ctx_tune_key(ctx), tune_code(best.k, best.o, best.c, rows_log2(ctx->g)));
    if (ms)
        for (int k = 0; k < kNumShapes; ++k) ms[k] = best_k[k];
    if (chosen) *chosen = best.k;
    return LBM_OK;
}

lbm_status lbm_set_layout(lbm_ctx *ctx, int32_t rows_per_group) {
    if (!ctx || rows_per_group < 1 || rows_per_group > (1 << kMaxRowsLog2) ||
        (rows_per_group & (rows_per_group - 1)) != 0 || ctx->desc.ny % rows_per_group != 0)
        return LBM_E_INVAL;
    return set_layout(ctx, uint32_t(rows_per_group));
}

lbm_status lbm_get_layout(const lbm_ctx *ctx, int32_t *rows_per_group) {
    if (!ctx || !rows_per_group) return LBM_E_INVAL;
    *rows_per_group = int32_t(ctx->g.ymask + 1);
    return LBM_OK;
}

lbm_status lbm_set_sweep_launch(lbm_ctx *ctx, int32_t order, int32_t waves_per_simd) {
    if (!ctx || order < 0 || order >= int32_t(kNumOrders)) return LBM_E_INVAL;
    int cap = -1;
    for (int j = 0; j < kNumCaps; ++j)
        if (kResidencyCaps[j] == waves_per_simd) cap = j;
    if (cap < 0 || sweep_lds(ctx, cap, config_block(ctx->shape)) < 0) return LBM_E_INVAL;
    ctx->order = order;
    ctx->cap = cap;
    return LBM_OK;
}

lbm_status lbm_get_sweep_launch(const lbm_ctx *ctx, int32_t *order, int32_t *waves_per_simd) {
    if (!ctx || !order || !waves_per_simd) return LBM_E_INVAL;
    *order = ctx->order;
    *waves_per_simd = kResidencyCaps[ctx->cap];
    return LBM_OK;
}

lbm_status lbm_stream_ceiling(lbm_ctx *ctx, int32_t k, int32_t iters, double *ms) {
    if (!ctx || !ms || iters < 1 || iters > 10000) return LBM_E_INVAL;
    if (k < 0) k = ctx->shape;
    if (k >= kNumShapes || !shape_ok(ctx, k)) return LBM_E_INVAL;
    hipError_t err = hipSuccess;
    double t = 0.0;
    LBM_DISPATCH(ctx, time_stream_only, k, iters, &t, &err);
    if (err != hipSuccess || launch_status() != LBM_OK) return LBM_E_DEVICE;
    *ms = t;
    return LBM_OK;
}

lbm_status lbm_set_shape(lbm_ctx *ctx, int32_t k) {
    if (!ctx || k < 0 || k >= kNumShapes || !shape_ok(ctx, k)) return LBM_E_INVAL;
    ctx->shape = k;
    if (sweep_lds(ctx, ctx->cap, config_block(k)) < 0) ctx->cap = 0;  // cap not possible here
    return LBM_OK;
}

lbm_status lbm_warnings(const lbm_ctx *ctx, uint32_t *flags) {
    if (!ctx || !flags) return LBM_E_INVAL;
    *flags = ctx->warnings;
    return LBM_OK;
}

lbm_status lbm_get_shape(const lbm_ctx *ctx, int32_t *k) {
    if (!ctx || !k) return LBM_E_INVAL;
    *k = ctx->shape;
    return LBM_OK;
}

lbm_status lbm_series_config(lbm_ctx *ctx, int32_t every, double *series, int64_t capacity) {
    if (!ctx || every < 0) return LBM_E_INVAL;
    if (every > 0 && (!series || capacity < 1)) return LBM_E_INVAL;
    ctx->series_every = every;
    ctx->series = every > 0 ? series : nullptr;
    ctx->series_cap = every > 0 ? capacity : 0;
    ctx->series_count = 0;
    ctx->series_t = 0;
    return LBM_OK;
}

lbm_status lbm_series_count(const lbm_ctx *ctx, int64_t *count) {
    if (!ctx || !count) return LBM_E_INVAL;
    *count = ctx->series_count;
    return LBM_OK;
}

lbm_status lbm_get_step(const lbm_ctx *ctx, int64_t *step) {
    if (!ctx || !step) return LBM_E_INVAL;
    *step = ctx->step;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx *ctx) {
    if (!ctx) return LBM_E_INVAL;
    for (int32_t k = 0; k < 2 * ctx->prof_cap; ++k) (void)hipEventDestroy(ctx->prof_ev[k]);
    free(ctx->prof_ev);
    free(ctx->prof_kind);
    free(ctx);
    return LBM_OK;
}

const char *lbm_status_string(lbm_status status) {
    switch (status) {
        case LBM_OK: return "ok";
        case LBM_E_INVAL: return "invalid argument";
        case LBM_E_DEVICE: return "device error";
        case LBM_E_STATE: return "invalid state";
        case LBM_E_NONFINITE: return "non-finite value or node force out of range";
        case LBM_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

}  // extern "C"

// ===========================================================================
// Host side: ensembles of independent boxes.
// ===========================================================================
struct lbm_ens {
    lbm_ensemble_desc desc;
    int32_t nrep;
    lbm_replica_desc *host_reps;  // copy of the caller's descriptors
    Replica *host_table;          // device-side table, host copy
    size_t elem;
    void *pop[2];
    int cur;
    hipStream_t stream;
    double enc_s, dec_s;
    uint64_t total_cells, total_pop;
    uint32_t total_blocks[kNumGeomShapes];
    int32_t n;  // particles in all replicas
    // scratch
    Replica *reps;
    uint16_t *blk_rep[kNumGeomShapes];
    uint16_t *part_rep;
    uint32_t *mask[2];
    long long *force[2];
    uint64_t total_mask_words;
    uint32_t *prev_cell;
    double *fh, *fr;
    EnsClock *clock;
    uint32_t *err;
    double *partials, *result;
    double *r, *v;
    // velocity autocorrelation
    int vacf_on;
    int32_t max_lag, stride, nslot;
    double *acc, *origins;
    int64_t vacf_t;
    int64_t step;
    int shape;
    int order, cap;         // block order and residency cap of the stream-collide
    int lds_cu, lds_block;  // LDS bytes per compute unit and per block (device limits)
    int rows;    // requested rows per group: each box takes the largest power of two <= rows dividing its ny
    int device;  // device current at lbm_ens_init (autotune cache key)
    // graph of LBM_ENS_GRAPH_STEPS steps, captured on a private stream and
    // replayed on `stream`
    int use_graph;
    hipGraphExec_t graph;
    int graph_valid;
    hipStream_t cap_stream;
    int graph_replays;  // number of graph launches so far
};

namespace {

TuneKey ens_tune_key(const lbm_ens *e) {
    TuneKey k{1, e->device, e->desc.storage, int(D3Q19::Q), {}};
    k.dims.reserve(3 * size_t(e->nrep));
    for (int32_t q = 0; q < e->nrep; ++q) {
        k.dims.push_back(e->host_reps[q].nx);
        k.dims.push_back(e->host_reps[q].ny);
        k.dims.push_back(e->host_reps[q].nz);
    }
    return k;
}

uint32_t ens_chunk(int32_t nx) { return uint32_t(nx); }  // unpadded, as row_chunk

struct EnsLayout {
    uint64_t total_cells = 0, total_pop = 0, total_mask_words = 0;
    uint32_t total_blocks[kNumGeomShapes] = {0, 0, 0, 0};
    int32_t n = 0;
    size_t lattice_bytes = 0, scratch_bytes = 0;
    // scratch offsets
    size_t o_reps, o_blk[kNumGeomShapes], o_part, o_mask[2], o_force[2], o_prev, o_fh, o_fr, o_clock,
        o_err, o_partials, o_result;
};

bool ens_desc_ok(const lbm_ensemble_desc *d, const lbm_replica_desc *reps) {
    if (!d || !reps || d->nrep < 1 || d->nrep > 65535 || d->reserved != 0) return false;
    if (elem_size(d->storage) == 0) return false;
    if (d->storage == LBM_STORE_F16 && (d->f16_scale_log2 < 0 || d->f16_scale_log2 > 24)) return false;
    if (!(d->mass > 0.0) || !isfinite(d->mass) || !(d->gamma >= 0.0) || !isfinite(d->gamma)) return false;
    if (!(d->kT >= 0.0) || !isfinite(d->kT) || !isfinite(d->radius)) return false;
    if (d->friction < LBM_FRICTION_STOKESLET || d->friction > LBM_FRICTION_STOKESLET_CUBE) return false;
    uint64_t cells = 0, n = 0;
    for (int32_t k = 0; k < d->nrep; ++k) {
        const lbm_replica_desc &r = reps[k];
        if (r.nx < 2 || r.ny < 2 || r.nz < 2 || r.n < 1 || !(r.tau > 0.5) || !isfinite(r.tau))
            return false;
        if (r.reserved != 0) return false;
        // a box's sweep indexes within the box in 32 bits
        if (uint64_t(r.nx) * uint64_t(r.ny) * uint64_t(r.nz) * 19 >= (uint64_t(1) << 32)) return false;
        cells += uint64_t(r.nx) * uint64_t(r.ny) * uint64_t(r.nz);
        n += uint64_t(r.n);
    }
    return cells < (uint64_t(1) << 31) && n < (uint64_t(1) << 24);
}

EnsLayout ens_layout(const lbm_ensemble_desc *d, const lbm_replica_desc *reps) {
    EnsLayout L;
    const size_t elem = elem_size(d->storage);
    for (int32_t k = 0; k < d->nrep; ++k) {
        const lbm_replica_desc &r = reps[k];
        const uint64_t cells = uint64_t(r.nx) * r.ny * r.nz;
        L.total_cells += cells;
        L.total_pop += uint64_t(ens_chunk(r.nx)) * D3Q19::Q * r.ny * r.nz;
        L.total_mask_words += mask_words(cells);
        for (int s = 0; s < kNumGeomShapes; ++s) {
            const uint64_t band = (r.ny % kShapes[s].cpt == 0) ? cells / kShapes[s].cpt : 0;
            L.total_blocks[s] += uint32_t((band + kShapes[s].bs - 1) / kShapes[s].bs);
        }
        L.n += r.n;
    }
    L.lattice_bytes = align_up(L.total_pop * elem, kAlign);
    size_t o = 0;
    L.o_reps = o;
    o += align_up(sizeof(Replica) * size_t(d->nrep), kAlign);
    for (int s = 0; s < kNumGeomShapes; ++s) {
        L.o_blk[s] = o;
        o += align_up(size_t(L.total_blocks[s]) * 2 + 2, kAlign);
    }
    L.o_part = o;
    o += align_up(size_t(L.n) * 2, kAlign);
    for (int k = 0; k < 2; ++k) {
        L.o_mask[k] = o;
        o += align_up(L.total_mask_words * 4, kAlign);
    }
    for (int k = 0; k < 2; ++k) {
        L.o_force[k] = o;
        o += align_up(L.total_cells * 3 * 8, kAlign);
    }
    L.o_prev = o;
    o += align_up(size_t(L.n) * 8 * 4, kAlign);
    L.o_fh = o;
    o += align_up(size_t(L.n) * 3 * 8, kAlign);
    L.o_fr = o;
    o += align_up(size_t(L.n) * 3 * 8, kAlign);
    L.o_clock = o;
    o += kAlign;
    L.o_err = o;
    o += kAlign;
    L.o_partials = o;
    o += align_up(size_t(kRedBlocks) * 4 * 8, kAlign);
    L.o_result = o;
    o += kAlign;
    L.scratch_bytes = o;
    return L;
}

ParticleArgs ens_particle_args(lbm_ens *e) {
    ParticleArgs pa;
    memset(&pa, 0, sizeof(pa));
    pa.r = e->r;
    pa.v = e->v;
    pa.fh = e->fh;
    pa.fr = e->fr;
    pa.prev_cell = e->prev_cell;
    pa.err = e->err;
    pa.n = e->n;
    pa.friction = e->desc.friction;
    pa.mass = e->desc.mass;
    pa.gamma = e->desc.gamma;
    pa.sig = e->desc.kT > 0.0 ? sqrt(2.0 * e->desc.gamma * e->desc.kT) : 0.0;
    pa.acc = nullptr;
    pa.origins = nullptr;
    pa.k_hi = -1;
    pa.nslot = pa.stride = 1;
    pa.pmom = nullptr;
    if (e->vacf_on) {
        pa.acc = e->acc;
        pa.origins = e->origins;
        pa.nslot = e->nslot;
        pa.stride = e->stride;
        pa.max_lag = e->max_lag;
    }
    return pa;
}

// Dynamic LDS that caps the ensemble sweep at kResidencyCaps[cap] waves per
// SIMD for blocks of bs lanes (0: no cap; -1: not possible on this device).
long ens_sweep_lds(const lbm_ens *e, int cap, int bs) { return residency_lds(e->lds_cu, e->lds_block, cap, bs); }

template <class C, int CPT, int BS, bool NTS>
void ens_collide_shape(lbm_ens *e, const typename C::T *A, typename C::T *B, int par) {
    using R = typename C::R;
    const int sh = e->shape & 3;
    const long lds = ens_sweep_lds(e, e->cap, BS);
    hipLaunchKernelGGL((k_ens_collide<C, CPT, BS, NTS>), dim3(e->total_blocks[sh]), dim3(BS),
                       lds > 0 ? size_t(lds) : 0, e->stream, A, B, e->reps, e->blk_rep[sh], sh,
                       e->force[par], e->mask[par], R(e->enc_s), R(e->dec_s), e->clock, e->vacf_on,
                       uint32_t(e->order));
}

// One step of every replica; par = field parity of this step.
template <class C>
void ens_launch_step(lbm_ens *e, int cur, int par) {
    using T = typename C::T;
    using R = typename C::R;
    const T *A = static_cast<const T *>(e->pop[cur]);
    T *B = static_cast<T *>(e->pop[cur ^ 1]);
    const ParticleArgs pa = ens_particle_args(e);
    hipLaunchKernelGGL(k_ens_particle<C>,
                       dim3(unsigned((uint64_t(e->n) * 8 + kParticleBlock - 1) / kParticleBlock)),
                       dim3(kParticleBlock), 0, e->stream, A, e->reps, e->part_rep, R(e->dec_s), pa,
                       e->clock, e->force[par], e->mask[par], e->force[par ^ 1], e->mask[par ^ 1]);
#define LBM_ENS_CALL(CPT, BS, NTS, ROW) ens_collide_shape<C, CPT, BS, NTS>(e, A, B, par)
    LBM_CONFIG_SWITCH(e->shape, LBM_ENS_CALL)
#undef LBM_ENS_CALL
}

void ens_dispatch_step(lbm_ens *e, int cur, int par) {
    switch (e->desc.storage) {
        case LBM_STORE_F64: ens_launch_step<F64Q19>(e, cur, par); break;
        case LBM_STORE_F32: ens_launch_step<F32Q19>(e, cur, par); break;
        case LBM_STORE_BF16: ens_launch_step<BF16Q19>(e, cur, par); break;
        case LBM_STORE_F16: ens_launch_step<F16Q19>(e, cur, par); break;
    }
}

// Rows per group of a box with ny rows per plane when `rows` is requested: the
// largest power of two not above it that divides ny.
uint32_t ens_box_rows(int rows, int32_t ny) {
    uint32_t y = uint32_t(rows);
    while (y > 1 && ny % int32_t(y) != 0) y >>= 1;
    return y;
}

// Moves every box into the layout ens_box_rows(rows, ny): each box is permuted
// into the spare lattice, and the whole spare lattice is copied back, so the
// state stays in the current buffer; then the device table is updated.
template <class C>
void ens_relayout(lbm_ens *e, int rows, hipError_t *err) {
    using T = typename C::T;
    const T *A = static_cast<const T *>(e->pop[e->cur]);
    T *B = static_cast<T *>(e->pop[e->cur ^ 1]);
    for (int32_t k = 0; k < e->nrep; ++k) {
        Replica &t = e->host_table[k];
        const Grid gn = with_rows_per_group(t.g, ens_box_rows(rows, int32_t(t.g.ny)));
        hipLaunchKernelGGL(k_relayout<C>, dim3(blocks_for(t.g.ncell)), dim3(kBlock), 0, e->stream,
                           A + t.pop_off, t.g, B + t.pop_off, gn);
        t.g = gn;
    }
    *err = hipGetLastError();
    if (*err == hipSuccess)
        *err = hipMemcpyAsync(e->pop[e->cur], e->pop[e->cur ^ 1], e->total_pop * sizeof(T),
                              hipMemcpyDeviceToDevice, e->stream);
    if (*err == hipSuccess)
        *err = hipMemcpyAsync(e->reps, e->host_table, sizeof(Replica) * e->nrep,
                              hipMemcpyHostToDevice, e->stream);
    if (*err == hipSuccess) *err = hipStreamSynchronize(e->stream);  // host_table is reused
    e->rows = rows;
}

void ens_drop_graph(lbm_ens *e);

lbm_status ens_set_layout(lbm_ens *e, int rows) {
    if (rows == e->rows) return LBM_OK;
    ens_drop_graph(e);
    hipError_t err = hipSuccess;
    switch (e->desc.storage) {
        case LBM_STORE_F64: ens_relayout<F64Q19>(e, rows, &err); break;
        case LBM_STORE_F32: ens_relayout<F32Q19>(e, rows, &err); break;
        case LBM_STORE_BF16: ens_relayout<BF16Q19>(e, rows, &err); break;
        case LBM_STORE_F16: ens_relayout<F16Q19>(e, rows, &err); break;
    }
    return err == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

void ens_drop_graph(lbm_ens *e) {
    if (e->graph_valid) (void)hipGraphExecDestroy(e->graph);
    e->graph_valid = 0;
}

// Steps per graph replay: kGraphPairs pairs of steps (the lattice parity and
// the force-field parity both return to their start after every pair).  Two
// steps per graph cost about 1.5% over plain launches on the 64-box
// workload; sixteen amortise the graph launch.
constexpr int kGraphPairs = LBM_ENS_GRAPH_STEPS / 2;
static_assert(LBM_ENS_GRAPH_STEPS % 2 == 0, "whole pairs of steps");

// Capture kGraphPairs pairs of steps with parity (0, 1) starting from lattice
// e->cur into a graph.
// Capture runs on a private non-blocking stream (the caller's stream may be
// the null stream, which cannot be captured); the graph is then launched on
// the caller's stream.  Returns false when no graph could be made.
bool ens_capture(lbm_ens *e) {
    ens_drop_graph(e);
    if (!e->cap_stream && hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        e->cap_stream = nullptr;
        return false;
    }
    hipStream_t user = e->stream;
    if (hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return false;
    e->stream = e->cap_stream;
    for (int k = 0; k < kGraphPairs; ++k) {
        ens_dispatch_step(e, e->cur, 0);
        ens_dispatch_step(e, e->cur ^ 1, 1);
    }
    e->stream = user;
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(e->cap_stream, &g);
    if (end != hipSuccess || !g) {
        (void)hipGetLastError();
        return false;
    }
    const hipError_t err = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    e->graph_valid = 1;
    return true;
}

template <class C, int CPT, int BS, bool NTS>
void ens_time_shape(lbm_ens *e, int k, int o, int c) {
    // A -> B without swapping (the state in A is untouched); the caller
    // restores the device clock the launches advance.
    const int saved[3] = {e->shape, e->order, e->cap};
    e->shape = k;
    e->order = o;
    e->cap = c;
    ens_collide_shape<C, CPT, BS, NTS>(e, static_cast<const typename C::T *>(e->pop[e->cur]),
                                       static_cast<typename C::T *>(e->pop[e->cur ^ 1]),
                                       int((e->step + 1) & 1));  // last step's node forces
    e->shape = saved[0];
    e->order = saved[1];
    e->cap = saved[2];
}

template <class C>
void ens_time_dispatch(lbm_ens *e, int k, int o, int c) {
#define LBM_ENS_TIME(CPT, BS, NTS, ROW) ens_time_shape<C, CPT, BS, NTS>(e, k, o, c)
    LBM_CONFIG_SWITCH(k, LBM_ENS_TIME)
#undef LBM_ENS_TIME
}

template <class C>
void ens_stream_only(lbm_ens *e, int k) {
    using T = typename C::T;
    const int sh = k & 3;
    const T *A = static_cast<const T *>(e->pop[e->cur]);
    T *B = static_cast<T *>(e->pop[e->cur ^ 1]);
#define LBM_ENS_STREAM_ONLY(CPT, BS, NTS, ROW)                                                   \
    do {                                                                                          \
        const long lds = ens_sweep_lds(e, e->cap, BS);                                            \
        hipLaunchKernelGGL((k_ens_stream_only<C, CPT, BS, NTS>), dim3(e->total_blocks[sh]),       \
                           dim3(BS), lds > 0 ? size_t(lds) : 0, e->stream, A, B, e->reps,         \
                           e->blk_rep[sh], sh, uint32_t(e->order));                               \
    } while (0)
    LBM_CONFIG_SWITCH(k, LBM_ENS_STREAM_ONLY)
#undef LBM_ENS_STREAM_ONLY
}

void ens_stream_only_any(lbm_ens *e, int k) {
    switch (e->desc.storage) {
        case LBM_STORE_F64: ens_stream_only<F64Q19>(e, k); break;
        case LBM_STORE_F32: ens_stream_only<F32Q19>(e, k); break;
        case LBM_STORE_BF16: ens_stream_only<BF16Q19>(e, k); break;
        case LBM_STORE_F16: ens_stream_only<F16Q19>(e, k); break;
    }
}

void ens_time_any(lbm_ens *e, int k, int o, int c) {
    switch (e->desc.storage) {
        case LBM_STORE_F64: ens_time_dispatch<F64Q19>(e, k, o, c); break;
        case LBM_STORE_F32: ens_time_dispatch<F32Q19>(e, k, o, c); break;
        case LBM_STORE_BF16: ens_time_dispatch<BF16Q19>(e, k, o, c); break;
        case LBM_STORE_F16: ens_time_dispatch<F16Q19>(e, k, o, c); break;
    }
}

// Configuration k applies to every box (two-node shapes need an even ny) and
// cap c can be imposed on its blocks.
bool ens_launch_ok(const lbm_ens *e, int k, int c) {
    if (k < 0 || k >= kNumShapes || config_row(k) || e->total_blocks[k & 3] == 0) return false;
    for (int32_t q = 0; q < e->nrep; ++q)
        if (e->host_reps[q].ny % kShapes[k & 3].cpt != 0) return false;
    return ens_sweep_lds(e, c, config_block(k)) >= 0;
}

// Mean ms per launch of configuration k with block order o and cap c over
// iters launches (after two unrecorded ones); < 0 on a device error.
double ens_time_launch(lbm_ens *e, int k, int o, int c, int32_t iters, hipEvent_t e0, hipEvent_t e1) {
    for (int w = 0; w < 2; ++w) ens_time_any(e, k, o, c);
    (void)hipEventRecord(e0, e->stream);
    for (int32_t it = 0; it < iters; ++it) ens_time_any(e, k, o, c);
    (void)hipEventRecord(e1, e->stream);
    float f = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&f, e0, e1) != hipSuccess ||
        launch_status() != LBM_OK)
        return -1.0;
    return double(f) / iters;
}

}  // namespace

extern "C" {

lbm_status lbm_ens_bytes(const lbm_ensemble_desc *desc, const lbm_replica_desc *reps,
                         size_t *lattice_bytes, size_t *scratch_bytes) {
    if (!ens_desc_ok(desc, reps) || !lattice_bytes || !scratch_bytes) return LBM_E_INVAL;
    const EnsLayout L = ens_layout(desc, reps);
    *lattice_bytes = L.lattice_bytes;
    *scratch_bytes = L.scratch_bytes;
    return LBM_OK;
}

lbm_status lbm_ens_init(const lbm_ensemble_desc *desc, const lbm_replica_desc *reps, void *pop_a,
                        void *pop_b, void *scratch, double *r, double *v, void *stream,
                        lbm_ens **out) {
    if (!ens_desc_ok(desc, reps) || !pop_a || !pop_b || !scratch || !r || !v || !out)
        return LBM_E_INVAL;
    if (!aligned(pop_a) || !aligned(pop_b) || !aligned(scratch) || pop_a == pop_b) return LBM_E_INVAL;
    const EnsLayout L = ens_layout(desc, reps);
    lbm_ens *e = static_cast<lbm_ens *>(calloc(1, sizeof(lbm_ens)));
    if (!e) return LBM_E_DEVICE;
    e->desc = *desc;
    e->nrep = desc->nrep;
    e->host_reps = static_cast<lbm_replica_desc *>(malloc(sizeof(lbm_replica_desc) * e->nrep));
    e->host_table = static_cast<Replica *>(calloc(e->nrep, sizeof(Replica)));
    uint16_t *blk[kNumGeomShapes];
    for (int s = 0; s < kNumGeomShapes; ++s)
        blk[s] = static_cast<uint16_t *>(malloc(size_t(L.total_blocks[s]) * 2 + 2));
    uint16_t *prep = static_cast<uint16_t *>(malloc(size_t(L.n) * 2));
    bool ok = e->host_reps && e->host_table && prep;
    for (int s = 0; s < kNumGeomShapes; ++s) ok = ok && blk[s];
    if (!ok) {
        for (int s = 0; s < kNumGeomShapes; ++s) free(blk[s]);
        free(prep);
        free(e->host_reps);
        free(e->host_table);
        free(e);
        return LBM_E_DEVICE;
    }
    memcpy(e->host_reps, reps, sizeof(lbm_replica_desc) * e->nrep);
    e->elem = elem_size(desc->storage);
    e->pop[0] = pop_a;
    e->pop[1] = pop_b;
    e->stream = static_cast<hipStream_t>(stream);
    if (desc->storage == LBM_STORE_F16) {
        e->enc_s = ldexp(1.0, desc->f16_scale_log2);
        e->dec_s = ldexp(1.0, -desc->f16_scale_log2);
    } else {
        e->enc_s = e->dec_s = 1.0;
    }
    e->total_cells = L.total_cells;
    e->total_pop = L.total_pop;
    e->total_mask_words = L.total_mask_words;
    e->device = current_device();
    // until lbm_ens_autotune: the last choice for this key, else by lattice size
    {
        const int code = tune_lookup(ens_tune_key(e), L.lattice_bytes >= kStreamStoreBytes ? kNumGeomShapes : 0);
        e->shape = code % kNumShapes;
        e->order = (code / kNumShapes) % int(kNumOrders);
        e->cap = (code / (kNumShapes * int(kNumOrders))) % kNumCaps;
        // applied to every box below (the rest state is all zeros)
        e->rows = 1 << (code / (kNumShapes * int(kNumOrders) * kNumCaps));
        int v = 0;
        e->lds_cu = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                           e->device) == hipSuccess) ? v : 0;
        e->lds_block = (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                              e->device) == hipSuccess) ? v : 0;
        if (ens_sweep_lds(e, e->cap, config_block(e->shape)) < 0) e->cap = 0;
    }
    for (int s = 0; s < kNumGeomShapes; ++s) e->total_blocks[s] = L.total_blocks[s];
    e->n = L.n;
    char *base = static_cast<char *>(scratch);
    e->reps = reinterpret_cast<Replica *>(base + L.o_reps);
    for (int s = 0; s < kNumGeomShapes; ++s) e->blk_rep[s] = reinterpret_cast<uint16_t *>(base + L.o_blk[s]);
    e->part_rep = reinterpret_cast<uint16_t *>(base + L.o_part);
    for (int k = 0; k < 2; ++k) {
        e->mask[k] = reinterpret_cast<uint32_t *>(base + L.o_mask[k]);
        e->force[k] = reinterpret_cast<long long *>(base + L.o_force[k]);
    }
    e->prev_cell = reinterpret_cast<uint32_t *>(base + L.o_prev);
    e->fh = reinterpret_cast<double *>(base + L.o_fh);
    e->fr = reinterpret_cast<double *>(base + L.o_fr);
    e->clock = reinterpret_cast<EnsClock *>(base + L.o_clock);
    e->err = reinterpret_cast<uint32_t *>(base + L.o_err);
    e->partials = reinterpret_cast<double *>(base + L.o_partials);
    e->result = reinterpret_cast<double *>(base + L.o_result);
    e->r = r;
    e->v = v;
    e->use_graph = 1;
    // replica table, block and particle maps
    uint64_t pop_off = 0, cell_off = 0, mask_off = 0;
    uint32_t first[kNumGeomShapes] = {0, 0, 0, 0};
    uint32_t part_off = 0;
    for (int32_t k = 0; k < e->nrep; ++k) {
        const lbm_replica_desc &rd = reps[k];
        Replica &t = e->host_table[k];
        t.g.nx = uint32_t(rd.nx);
        t.g.ny = uint32_t(rd.ny);
        t.g.nz = uint32_t(rd.nz);
        t.g.ncell = uint32_t(uint64_t(rd.nx) * rd.ny * rd.nz);
        t.g.chunk = ens_chunk(rd.nx);
        t.g = with_rows_per_group(t.g, ens_box_rows(e->rows, rd.ny));
        t.pop_off = pop_off;
        t.cell_off = cell_off;
        t.mask_off = uint32_t(mask_off);
        t.part_off = part_off;
        t.npart = uint32_t(rd.n);
        t.replica_id = rd.replica;
        t.seed = rd.seed;
        t.omega = 1.0 / rd.tau;
        const double nu = (rd.tau - 0.5) / 3.0;
        t.R = desc->radius > 0.0 ? desc->radius : desc->gamma / (6.0 * M_PI * nu);
        for (int s = 0; s < kNumGeomShapes; ++s) {
            t.first_block[s] = first[s];
            const uint64_t band = (rd.ny % kShapes[s].cpt == 0) ? t.g.ncell / kShapes[s].cpt : 0;
            const uint32_t nb = uint32_t((band + kShapes[s].bs - 1) / kShapes[s].bs);
            for (uint32_t b = 0; b < nb; ++b) blk[s][first[s] + b] = uint16_t(k);
            first[s] += nb;
        }
        for (int32_t q = 0; q < rd.n; ++q) prep[part_off + q] = uint16_t(k);
        pop_off += uint64_t(t.g.chunk) * D3Q19::Q * rd.ny * rd.nz;
        cell_off += t.g.ncell;
        mask_off += mask_words(t.g.ncell);
        part_off += uint32_t(rd.n);
    }
    hipError_t err = hipMemsetAsync(pop_a, 0, L.lattice_bytes, e->stream);
    if (err == hipSuccess) err = hipMemsetAsync(pop_b, 0, L.lattice_bytes, e->stream);
    if (err == hipSuccess) err = hipMemsetAsync(scratch, 0, L.scratch_bytes, e->stream);
    if (err == hipSuccess)
        err = hipMemsetAsync(e->prev_cell, 0xFF, size_t(L.n) * 8 * 4, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->reps, e->host_table, sizeof(Replica) * e->nrep,
                             hipMemcpyHostToDevice, e->stream);
    for (int s = 0; s < kNumGeomShapes && err == hipSuccess; ++s)
        if (L.total_blocks[s] > 0)
            err = hipMemcpyAsync(e->blk_rep[s], blk[s], size_t(L.total_blocks[s]) * 2,
                                 hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->part_rep, prep, size_t(L.n) * 2, hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);  // host staging is freed below
    for (int s = 0; s < kNumGeomShapes; ++s) free(blk[s]);
    free(prep);
    if (err != hipSuccess) {
        free(e->host_reps);
        free(e->host_table);
        free(e);
        return LBM_E_DEVICE;
    }
    *out = e;
    return LBM_OK;
}

lbm_status lbm_ens_use_graph(lbm_ens *e, int32_t use) {
    if (!e || (use != 0 && use != 1)) return LBM_E_INVAL;
    e->use_graph = use;
    if (!use) ens_drop_graph(e);
    return LBM_OK;
}

lbm_status lbm_ens_vacf_config(lbm_ens *e, int32_t max_lag, int32_t stride, double *acc,
                               double *origins) {
    if (!e) return LBM_E_INVAL;
    ens_drop_graph(e);
    if (max_lag == -1) {
        e->vacf_on = 0;
        return LBM_OK;
    }
    if (max_lag < 0 || stride < 1 || !acc || !origins) return LBM_E_INVAL;
    e->max_lag = max_lag;
    e->stride = stride;
    e->nslot = max_lag / stride + 1;
    e->acc = acc;
    e->origins = origins;
    e->vacf_t = 0;
    const EnsClock clk{e->step, 0};
    hipError_t err = hipMemsetAsync(acc, 0, size_t(e->n) * size_t(max_lag + 1) * 8, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->clock, &clk, sizeof(clk), hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) return LBM_E_DEVICE;
    e->vacf_on = 1;
    return LBM_OK;
}

lbm_status lbm_ens_vacf_counts(const lbm_ens *e, int64_t *cnt) {
    if (!e || !cnt) return LBM_E_INVAL;
    if (!e->vacf_on) return LBM_E_STATE;
    const int64_t T = e->vacf_t;
    for (int32_t l = 0; l <= e->max_lag; ++l)
        cnt[l] = (T - 1 - l >= 0) ? (T - 1 - l) / e->stride + 1 : 0;
    return LBM_OK;
}

lbm_status lbm_ens_step(lbm_ens *e, int32_t nsteps) {
    if (!e || nsteps < 0) return LBM_E_INVAL;
    int32_t left = nsteps;
    auto eager = [&]() {
        ens_dispatch_step(e, e->cur, int(e->step & 1));
        e->cur ^= 1;
        e->step += 1;
        if (e->vacf_on) e->vacf_t += 1;
        --left;
    };
    if (e->use_graph) {
        if (left > 0 && (e->step & 1)) eager();
        constexpr int32_t per = 2 * kGraphPairs;
        if (left >= per && !e->graph_valid && !ens_capture(e)) e->use_graph = 0;  // plain launches
        if (left >= per && e->graph_valid) {
            // the graph was captured from lattice parity cur at an even step;
            // cur and the step parity change together, so they still match
            while (left >= per) {
                if (hipGraphLaunch(e->graph, e->stream) != hipSuccess) return LBM_E_DEVICE;
                e->graph_replays += 1;
                e->step += per;
                if (e->vacf_on) e->vacf_t += per;
                left -= per;
            }
        }
    }
    while (left > 0) eager();
    return launch_status();
}

lbm_status lbm_ens_autotune(lbm_ens *e, int32_t iters, double *ms, int32_t *chosen) {
    if (!e || iters < 1 || iters > 10000) return LBM_E_INVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_E_DEVICE;
    }
    // the timing launches advance the device clock; restore it afterwards
    EnsClock saved;
    hipError_t err = hipMemcpyAsync(&saved, e->clock, sizeof(saved), hipMemcpyDeviceToHost, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    double best_k[kNumShapes];
    for (int k = 0; k < kNumShapes; ++k) best_k[k] = -1.0;
    // every launch timed: configuration, order, cap, layout (log2 of the rows
    // per group requested of all boxes), ms
    struct Trial {
        int k, o, c, l;
        double t;
    };
    std::vector<Trial> trials;
    bool ok = err == hipSuccess;
    auto time_in = [&](int l, int k, int o, int c, int32_t n) -> double {
        if (!ok) return -1.0;
        if (ens_set_layout(e, 1 << l) != LBM_OK) {
            ok = false;
            return -1.0;
        }
        const double v = ens_time_launch(e, k, o, c, n, e0, e1);
        if (v < 0.0) ok = false;
        return v;
    };
    auto note = [&](int k, int o, int c, int l, double v) {
        if (v <= 0.0) return;
        if (best_k[k] <= 0.0 || v < best_k[k]) best_k[k] = v;
        trials.push_back(Trial{k, o, c, l, v});
    };
    // Stage 1: every configuration in linear order without a residency cap,
    // in every layout; keep the layout of the fastest launch.
    double t1[kMaxRowsLog2 + 1][kNumShapes];
    int bl = -1, first = -1;
    for (int l = 0; l <= kMaxRowsLog2 && ok; ++l)
        for (int k = 0; k < kNumShapes && ok; ++k) {
            t1[l][k] = ens_launch_ok(e, k, 0) ? time_in(l, k, int(kOrderLinear), 0, iters) : -1.0;
            note(k, int(kOrderLinear), 0, l, t1[l][k]);
            if (t1[l][k] > 0.0 && (bl < 0 || t1[l][k] < t1[bl][first])) bl = l, first = k;
        }
    if (bl < 0) ok = false;
    // Stage 2: in that layout, its two fastest configurations with every block
    // order and cap.
    Trial best{first, int(kOrderLinear), 0, bl, ok ? t1[bl][first] : 0.0};
    if (ok) {
        int second = -1;
        for (int k = 0; k < kNumShapes; ++k)
            if (k != first && t1[bl][k] > 0.0 && (second < 0 || t1[bl][k] < t1[bl][second])) second = k;
        for (int k : {first, second}) {
            if (k < 0) continue;
            for (int o = 0; o < int(kNumOrders) && ok; ++o)
                for (int c = 0; c < kNumCaps && ok; ++c) {
                    if ((o == int(kOrderLinear) && c == 0) || !ens_launch_ok(e, k, c)) continue;
                    const double v = time_in(bl, k, o, c, iters);
                    note(k, o, c, bl, v);
                    if (v > 0.0 && v < best.t) best = Trial{k, o, c, bl, v};
                }
        }
    }
    // Stage 3: that launch in every other layout (a cap or order can change
    // which layout streams best).
    if (ok && (best.o != int(kOrderLinear) || best.c != 0)) {
        const Trial b0 = best;
        for (int l = 0; l <= kMaxRowsLog2 && ok; ++l)
            if (l != b0.l) note(b0.k, b0.o, b0.c, l, time_in(l, b0.k, b0.o, b0.c, iters));
    }
    // Stage 4: the three fastest launches timed again, in turn, twice each
    // with twice the iterations; the lowest total wins.
    if (ok) {
        std::sort(trials.begin(), trials.end(), [](const Trial &x, const Trial &y) { return x.t < y.t; });
        const int m = int(std::min<size_t>(3, trials.size()));
        double total[3] = {0.0, 0.0, 0.0};
        for (int round = 0; round < 2 && ok; ++round)
            for (int j = 0; j < m && ok; ++j) {
                const double v = time_in(trials[j].l, trials[j].k, trials[j].o, trials[j].c, 2 * iters);
                total[j] += v > 0.0 ? v : 1e30;
            }
        int jb = 0;
        for (int j = 1; j < m; ++j)
            if (total[j] < total[jb]) jb = j;
        if (m > 0) best = trials[jb];
    }
    if (ok && ens_set_layout(e, 1 << best.l) != LBM_OK) ok = false;
    if (ok) {
        err = hipMemcpyAsync(e->clock, &saved, sizeof(saved), hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
        ok = err == hipSuccess;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return LBM_E_DEVICE;
    if (best.k != e->shape || best.o != e->order || best.c != e->cap) ens_drop_graph(e);
    e->shape = best.k;
    e->order = best.o;
    e->cap = best.c;
    tune_store(ens_tune_key(e), tune_code(best.k, best.o, best.c, best.l));
    if (ms)
        for (int k = 0; k < kNumShapes; ++k) ms[k] = best_k[k];
    if (chosen) *chosen = best.k;
    return LBM_OK;
}

lbm_status lbm_ens_set_sweep_launch(lbm_ens *e, int32_t order, int32_t waves_per_simd) {
    if (!e || order < 0 || order >= int32_t(kNumOrders)) return LBM_E_INVAL;
    int cap = -1;
    for (int j = 0; j < kNumCaps; ++j)
        if (kResidencyCaps[j] == waves_per_simd) cap = j;
    if (cap < 0 || ens_sweep_lds(e, cap, config_block(e->shape)) < 0) return LBM_E_INVAL;
    if (order != e->order || cap != e->cap) ens_drop_graph(e);
    e->order = order;
    e->cap = cap;
    return LBM_OK;
}

lbm_status lbm_ens_get_sweep_launch(const lbm_ens *e, int32_t *order, int32_t *waves_per_simd) {
    if (!e || !order || !waves_per_simd) return LBM_E_INVAL;
    *order = e->order;
    *waves_per_simd = kResidencyCaps[e->cap];
    return LBM_OK;
}

lbm_status lbm_ens_set_layout(lbm_ens *e, int32_t rows_per_group) {
    if (!e || rows_per_group < 1 || rows_per_group > (1 << kMaxRowsLog2) ||
        (rows_per_group & (rows_per_group - 1)) != 0)
        return LBM_E_INVAL;
    return ens_set_layout(e, rows_per_group);
}

lbm_status lbm_ens_get_layout(const lbm_ens *e, int32_t replica, int32_t *rows_per_group) {
    if (!e || !rows_per_group || replica < 0 || replica >= e->nrep) return LBM_E_INVAL;
    *rows_per_group = int32_t(e->host_table[replica].g.ymask + 1);
    return LBM_OK;
}

lbm_status lbm_ens_stream_ceiling(lbm_ens *e, int32_t k, int32_t iters, double *ms) {
    if (!e || !ms || iters < 1 || iters > 10000) return LBM_E_INVAL;
    if (k < 0) k = e->shape;
    if (k >= kNumShapes || config_row(k) || e->total_blocks[k & 3] == 0) return LBM_E_INVAL;
    for (int32_t q = 0; q < e->nrep; ++q)
        if (e->host_reps[q].ny % kShapes[k & 3].cpt != 0) return LBM_E_INVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_E_DEVICE;
    }
    for (int w = 0; w < 2; ++w) ens_stream_only_any(e, k);
    (void)hipEventRecord(e0, e->stream);
    for (int32_t it = 0; it < iters; ++it) ens_stream_only_any(e, k);
    (void)hipEventRecord(e1, e->stream);
    hipError_t err = hipEventSynchronize(e1);
    float f = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&f, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess || launch_status() != LBM_OK) return LBM_E_DEVICE;
    *ms = double(f) / iters;
    return LBM_OK;
}

lbm_status lbm_ens_observables(lbm_ens *e, int32_t replica, double out[7]) {
    if (!e || !out || replica < 0 || replica >= e->nrep) return LBM_E_INVAL;
    const Replica &t = e->host_table[replica];
    const char *A = static_cast<const char *>(e->pop[e->cur]) + t.pop_off * e->elem;
    switch (e->desc.storage) {
#define LBM_ENS_PARTIALS(CODEC)                                                                 \
    hipLaunchKernelGGL(k_fluid_partials<CODEC>, dim3(kRedBlocks), dim3(kBlock), 0, e->stream, \
                       reinterpret_cast<const CODEC::T *>(A), t.g, CODEC::R(e->dec_s),          \
                       e->partials)
        case LBM_STORE_F64: LBM_ENS_PARTIALS(F64Q19); break;
        case LBM_STORE_F32: LBM_ENS_PARTIALS(F32Q19); break;
        case LBM_STORE_BF16: LBM_ENS_PARTIALS(BF16Q19); break;
        case LBM_STORE_F16: LBM_ENS_PARTIALS(F16Q19); break;
#undef LBM_ENS_PARTIALS
    }
    hipLaunchKernelGGL(k_final_sums, dim3(1), dim3(kBlock), 0, e->stream, e->partials, kRedBlocks,
                       double(t.g.ncell), e->v + 3 * uint64_t(t.part_off), int32_t(t.npart),
                       e->desc.mass, e->result);
    if (launch_status() != LBM_OK) return LBM_E_DEVICE;
    double host[7];
    uint32_t flag = 0;
    hipError_t err = hipMemcpyAsync(host, e->result, sizeof(host), hipMemcpyDeviceToHost, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(&flag, e->err, sizeof(flag), hipMemcpyDeviceToHost, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) return LBM_E_DEVICE;
    bool finite = true;
    for (int k = 0; k < 7; ++k) {
        out[k] = host[k];
        finite = finite && isfinite(host[k]);
    }
    return (finite && flag == 0) ? LBM_OK : LBM_E_NONFINITE;
}

lbm_status lbm_ens_get_populations(lbm_ens *e, int32_t replica, double *f) {
    if (!e || !f || replica < 0 || replica >= e->nrep) return LBM_E_INVAL;
    const Replica &t = e->host_table[replica];
    const char *A = static_cast<const char *>(e->pop[e->cur]) + t.pop_off * e->elem;
    switch (e->desc.storage) {
#define LBM_ENS_POPS(CODEC)                                                                      \
    hipLaunchKernelGGL(k_get_populations<CODEC>, dim3(blocks_for(t.g.ncell)), dim3(kBlock), 0, \
                       e->stream, reinterpret_cast<const CODEC::T *>(A), t.g, CODEC::R(e->dec_s), f)
        case LBM_STORE_F64: LBM_ENS_POPS(F64Q19); break;
        case LBM_STORE_F32: LBM_ENS_POPS(F32Q19); break;
        case LBM_STORE_BF16: LBM_ENS_POPS(BF16Q19); break;
        case LBM_STORE_F16: LBM_ENS_POPS(F16Q19); break;
#undef LBM_ENS_POPS
    }
    return launch_status();
}

lbm_status lbm_ens_set_shape(lbm_ens *e, int32_t k) {
    if (!e || !ens_launch_ok(e, k, 0)) return LBM_E_INVAL;
    const int cap = ens_sweep_lds(e, e->cap, config_block(k)) < 0 ? 0 : e->cap;  // cap not possible here
    if (k != e->shape || cap != e->cap) ens_drop_graph(e);
    e->shape = k;
    e->cap = cap;
    return LBM_OK;
}

lbm_status lbm_ens_get_shape(const lbm_ens *e, int32_t *k) {
    if (!e || !k) return LBM_E_INVAL;
    *k = e->shape;
    return LBM_OK;
}

lbm_status lbm_ens_get_step(const lbm_ens *e, int64_t *step) {
    if (!e || !step) return LBM_E_INVAL;
    *step = e->step;
    return LBM_OK;
}

lbm_status lbm_ens_graph_replays(const lbm_ens *e, int64_t *replays) {
    if (!e || !replays) return LBM_E_INVAL;
    *replays = e->graph_replays;
    return LBM_OK;
}

lbm_status lbm_ens_destroy(lbm_ens *e) {
    if (!e) return LBM_E_INVAL;
    ens_drop_graph(e);
    if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
    free(e->host_reps);
    free(e->host_table);
    free(e);
    return LBM_OK;
}

}  // extern "C"

// ===========================================================================
// Reverse mode: recorded forward runs and their adjoint.
// ===========================================================================
namespace {

// One checkpoint: the lattice as stored (post-collision values at their
// source node) and the particle state r[n][3], v[n][3].
struct TapeLayout {
    size_t lat, part, slot;
};

TapeLayout tape_layout(const lbm_ctx *c, int32_t np) {
    TapeLayout t;
    lbm_lattice_bytes(&c->desc, &t.lat);
    t.part = align_up(size_t(np) * 6 * 8, kAlign);
    t.slot = t.lat + t.part;
    return t;
}

// The FP64 adjoint lattice: interleaved rows of 128-byte-aligned doubles, one
// row per group whatever the forward lattice's layout.
Grid adj_grid(const lbm_ctx *c) {
    Grid gd = c->g;
    gd.chunk = uint32_t(align_up(c->g.nx, 16));
    return with_rows_per_group(gd, 1);
}

size_t adj_lattice_bytes(const lbm_ctx *c) {
    const Grid gd = adj_grid(c);
    return align_up(size_t(gd.chunk) * size_t(c->q) * gd.ny * gd.nz * 8, kAlign);
}

struct AdjLayout {
    size_t seg_lat, seg_part;  // `every` lattice / particle states of one segment
    size_t abar[2];            // adjoint lattices
    size_t uf[2], um[2];       // adjoint node fields and their flags
    size_t ff[2], fm[2];       // node-force fields of the forward recompute
    size_t prev_fwd, prev_adj, fh, fr, pgrad, wacc;
    size_t plist, fpair, fcbar;  // pair forces (when recorded with them)
    size_t total;
};

AdjLayout adj_layout(const lbm_ctx *c, int32_t np, int32_t every) {
    AdjLayout L;
    const TapeLayout t = tape_layout(c, np);
    const size_t field = force_field_bytes(&c->desc);
    const size_t mask = align_up(size_t(c->mask_words) * 4, kAlign);
    const size_t pcell = align_up(size_t(np) * 8 * 4, kAlign);
    size_t o = 0;
    L.seg_lat = o;
    o += size_t(every) * t.lat;
    L.seg_part = o;
    o += size_t(every) * t.part;
    for (int k = 0; k < 2; ++k) {
        L.abar[k] = o;
        o += adj_lattice_bytes(c);
    }
    for (int k = 0; k < 2; ++k) {
        L.uf[k] = o;
        o += field;
        L.um[k] = o;
        o += mask;
    }
    for (int k = 0; k < 2; ++k) {
        L.ff[k] = o;
        o += field;
        L.fm[k] = o;
        o += mask;
    }
    L.prev_fwd = o;
    o += pcell;
    L.prev_adj = o;
    o += pcell;
    L.fh = o;
    o += align_up(size_t(np) * 3 * 8, kAlign);
    L.fr = o;
    o += align_up(size_t(np) * 3 * 8, kAlign);
    L.pgrad = o;
    o += align_up(size_t(np) * 4 * 8, kAlign);
    L.wacc = o;
    o += align_up(size_t(blocks_for(c->g.ncell)) * 8, kAlign);
    L.plist = o;
    o += pair_list_bytes(np);
    L.fpair = o;
    o += align_up(size_t(np) * 3 * 8, kAlign);
    L.fcbar = o;
    o += align_up(size_t(np) * 3 * 8, kAlign);
    L.total = o;
    return L;
}

bool adjoint_storage(const lbm_ctx *c) {
    return c->desc.storage == LBM_STORE_F64 || c->desc.storage == LBM_STORE_F32;
}

// The adjoint stream-collide, addressing by wavefront rows where every
// wavefront lies in one lattice row (64 | nx), by per-lane 64-bit indices
// otherwise.
template <class C, bool FORCED, bool NTS>
void launch_adj_collide(hipStream_t st, unsigned cgrid, const typename C::T *A, const Grid &g,
                        typename C::R dec_s, const double *Abar, double *Bbar, const Grid &gd,
                        double omega, AdjField uf, double *wacc) {
    if (g.nx % 64 == 0)
        hipLaunchKernelGGL((k_adj_collide<C, FORCED, NTS, true>), dim3(cgrid), dim3(kBlock), 0, st, A, g,
                           dec_s, Abar, Bbar, gd, omega, uf, wacc);
    else
        hipLaunchKernelGGL((k_adj_collide<C, FORCED, NTS, false>), dim3(cgrid), dim3(kBlock), 0, st, A, g,
                           dec_s, Abar, Bbar, gd, omega, uf, wacc);
}

template <class C>
hipError_t adjoint_run(lbm_ctx *c, char *tape, char *work, double *adj_pop, double *adj_r,
                       double *adj_v, double *adj_param) {
    using T = typename C::T;
    using R = typename C::R;
    const int32_t np = c->rec_np, N = c->rec_nsteps, K = c->rec_every;
    const lbm_particle_desc &pd = c->rec_pdesc;
    const TapeLayout t = tape_layout(c, np);
    const AdjLayout L = adj_layout(c, np, K);
    const Grid gd = adj_grid(c);
    hipStream_t st = c->stream;
    const size_t field = force_field_bytes(&c->desc);
    const size_t mask = size_t(c->mask_words) * 4;
    const size_t pbytes = size_t(np) * 3 * 8;
    auto at = [&](size_t off) { return work + off; };
    auto seg = [&](int32_t k) { return reinterpret_cast<T *>(at(L.seg_lat + size_t(k) * t.lat)); };
    auto seg_r = [&](int32_t k) { return reinterpret_cast<double *>(at(L.seg_part + size_t(k) * t.part)); };
    auto seg_v = [&](int32_t k) { return seg_r(k) + 3 * size_t(np); };
    double *abar[2] = {reinterpret_cast<double *>(at(L.abar[0])),
                       reinterpret_cast<double *>(at(L.abar[1]))};
    AdjField uf[2], ff_unused{nullptr, nullptr};
    ForceField ff[2];
    for (int k = 0; k < 2; ++k) {
        uf[k] = AdjField{reinterpret_cast<double *>(at(L.uf[k])), reinterpret_cast<uint32_t *>(at(L.um[k]))};
        ff[k] = ForceField{reinterpret_cast<long long *>(at(L.ff[k])), reinterpret_cast<uint32_t *>(at(L.fm[k]))};
    }
    double *pgrad = reinterpret_cast<double *>(at(L.pgrad));
    double *wacc = reinterpret_cast<double *>(at(L.wacc));
    const PairList plist = pair_list_at(at(L.plist), np);
    double *fpair = reinterpret_cast<double *>(at(L.fpair));
    double *fcbar = reinterpret_cast<double *>(at(L.fcbar));
    const bool pairs = c->rec_pair_on && np > 0;
    uint32_t *prev_fwd = reinterpret_cast<uint32_t *>(at(L.prev_fwd));
    uint32_t *prev_adj = reinterpret_cast<uint32_t *>(at(L.prev_adj));

    hipError_t e = hipSuccess;
    auto memset_ = [&](void *p, int v, size_t n) {
        if (e == hipSuccess && n) e = hipMemsetAsync(p, v, n, st);
    };
    auto copy_ = [&](void *dst, const void *src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st);
    };
    for (int k = 0; k < 2; ++k) {
        memset_(uf[k].u, 0, field);
        memset_(uf[k].mask, 0, mask);
    }
    memset_(prev_adj, 0xFF, size_t(np) * 8 * 4);
    memset_(pgrad, 0, size_t(np) * 4 * 8);
    memset_(wacc, 0, size_t(blocks_for(c->g.ncell)) * 8);
    if (pairs) memset_(plist.count, 0, size_t(c->rec_pg.T) * 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_import<typename C::V>, dim3(blocks_for(c->g.ncell)), dim3(kBlock), 0, st, adj_pop,
                       abar[0], gd);

    // Forward recompute: the particle kernel without VACF or sums.
    ParticleArgs pa{};
    pa.fh = reinterpret_cast<double *>(at(L.fh));
    pa.fr = reinterpret_cast<double *>(at(L.fr));
    pa.prev_cell = prev_fwd;
    pa.err = c->err;
    pa.n = np;
    pa.friction = pd.friction;
    pa.mass = pd.mass;
    pa.gamma = pd.gamma;
    pa.sig = pd.kT > 0.0 ? sqrt(2.0 * pd.gamma * pd.kT) : 0.0;
    pa.R = c->rec_R;
    pa.seed = pd.seed;
    pa.replica = pd.replica;
    pa.acc = nullptr;
    pa.origins = nullptr;
    pa.pmom = nullptr;
    pa.fext = c->rec_fext;
    pa.k_hi = -1;
    pa.nslot = pa.stride = 1;
    pa.slot_lo = 0;

    AdjParticleArgs ap{};
    ap.rbar = adj_r;
    ap.vbar = adj_v;
    ap.pgrad = pgrad;
    ap.fext = c->rec_fext;
    ap.prev_cell = prev_adj;
    ap.n = np;
    ap.friction = pd.friction;
    ap.mass = pd.mass;
    ap.gamma = pd.gamma;
    ap.kT = pd.kT;
    ap.sig = pa.sig;
    ap.R = c->rec_R;
    if (pd.radius > 0.0) {
        ap.dR_dgamma = ap.dR_dtau = 0.0;
    } else {
        const double nu = (c->desc.tau - 0.5) / 3.0;
        ap.dR_dgamma = 1.0 / (6.0 * M_PI * nu);
        ap.dR_dtau = -c->rec_R / (3.0 * nu);
    }
    ap.seed = pd.seed;
    ap.replica = pd.replica;
    const unsigned pgrid = np > 0 ? unsigned(particle_blocks(np)) : 0;
    const unsigned cgrid = blocks_for(c->g.ncell);
    // the adjoint lattice is FP64: stream its stores once it outgrows the cache
    const bool stream_stores = adj_lattice_bytes(c) >= kStreamStoreBytes;

    int cur = 0;
    const int32_t nseg = (N + K - 1) / K;
    for (int32_t j = nseg - 1; j >= 0 && e == hipSuccess; --j) {
        const int32_t len = (N - j * K) < K ? (N - j * K) : K;
        const char *slot = tape + size_t(j) * t.slot;
        copy_(seg(0), slot, t.lat);
        copy_(seg_r(0), slot + t.lat, 2 * pbytes);
        if (np > 0 && len > 1) {
            for (int k = 0; k < 2; ++k) {
                memset_(ff[k].f, 0, field);
                memset_(ff[k].mask, 0, mask);
            }
            memset_(prev_fwd, 0xFF, size_t(np) * 8 * 4);
        }
        for (int32_t k = 0; k + 1 < len && e == hipSuccess; ++k) {
            const int64_t n = c->rec_n0 + int64_t(j) * K + k;
            const int par = int(n & 1);
            if (np > 0) {
                copy_(seg_r(k + 1), seg_r(k), 2 * pbytes);
                pa.r = seg_r(k + 1);
                pa.v = seg_v(k + 1);
                pa.step = uint32_t(n);
                pa.fpair = nullptr;
                if (pairs) {
                    launch_pairs(st, seg_r(k), np, c->rec_pg, plist, fpair);
                    pa.fpair = fpair;
                }
                hipLaunchKernelGGL(k_particle<C>, dim3(pgrid), dim3(kParticleBlock), 0, st, seg(k),
                                   c->g, R(c->dec_s), pa, ff[par], ff[par ^ 1]);
                launch_collide<C, true>(c, seg(k), seg(k + 1), ff[par], c->shape);
            } else {
                launch_collide<C, false>(c, seg(k), seg(k + 1), ff[0], c->shape);
            }
        }
        for (int32_t k = len - 1; k >= 0 && e == hipSuccess; --k) {
            const int64_t n = c->rec_n0 + int64_t(j) * K + k;
            const int par = int(n & 1);
            if (np > 0) {
                ap.r = seg_r(k);
                ap.v = seg_v(k);
                ap.step = uint32_t(n);
                ap.fpair = ap.fcbar = nullptr;
                if (pairs) {
                    launch_pairs(st, seg_r(k), np, c->rec_pg, plist, fpair);
                    ap.fpair = fpair;
                    ap.fcbar = fcbar;
                }
                hipLaunchKernelGGL(k_adj_particle<C>, dim3(pgrid), dim3(kParticleBlock), 0, st,
                                   seg(k), c->g, R(c->dec_s), abar[cur], gd, ap, uf[par],
                                   uf[par ^ 1]);
                if (pairs)
                    hipLaunchKernelGGL(k_adj_pair, pair_group_blocks(np), dim3(kPairBlock), 0, st,
                                       seg_r(k), np, c->rec_pg, plist, fcbar, adj_r);
                if (stream_stores)
                    launch_adj_collide<C, true, true>(st, cgrid, seg(k), c->g, R(c->dec_s), abar[cur], abar[cur ^ 1], gd,
                                       1.0 / c->desc.tau, uf[par], wacc);
                else
                    launch_adj_collide<C, true, false>(st, cgrid, seg(k), c->g, R(c->dec_s), abar[cur], abar[cur ^ 1], gd,
                                       1.0 / c->desc.tau, uf[par], wacc);
            } else if (stream_stores) {
                launch_adj_collide<C, false, true>(st, cgrid,
                                   seg(k), c->g, R(c->dec_s), abar[cur], abar[cur ^ 1], gd,
                                   1.0 / c->desc.tau, ff_unused, wacc);
            } else {
                launch_adj_collide<C, false, false>(st, cgrid,
                                   seg(k), c->g, R(c->dec_s), abar[cur], abar[cur ^ 1], gd,
                                   1.0 / c->desc.tau, ff_unused, wacc);
            }
            cur ^= 1;
            const hipError_t le = hipGetLastError();
            if (le != hipSuccess) e = le;
        }
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_export<typename C::V>, dim3(cgrid), dim3(kBlock), 0, st, abar[cur], adj_pop, gd);
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(kBlock), 0, st, pgrad, np, wacc,
                       int32_t(cgrid), c->desc.tau, adj_param);
    return hipGetLastError();
}

template <class C>
void adjoint_dispatch(lbm_ctx *c, char *tape, char *work, double *adj_pop, double *adj_r,
                      double *adj_v, double *adj_param, hipError_t *e) {
    *e = adjoint_run<C>(c, tape, work, adj_pop, adj_r, adj_v, adj_param);
}

}  // namespace

extern "C" {

lbm_status lbm_tape_bytes(const lbm_ctx *ctx, int32_t nsteps, int32_t every, size_t *bytes) {
    if (!ctx || !bytes || nsteps < 1 || every < 1) return LBM_E_INVAL;
    const TapeLayout t = tape_layout(ctx, ctx->np);
    *bytes = size_t((nsteps + every - 1) / every) * t.slot;
    return LBM_OK;
}

lbm_status lbm_record(lbm_ctx *ctx, int32_t nsteps, int32_t every, void *tape) {
    if (!ctx || nsteps < 1 || every < 1 || !tape || !aligned(tape)) return LBM_E_INVAL;
    if (!adjoint_storage(ctx)) return LBM_E_UNSUPPORTED;
    // the reverse sweep spreads on the unit cell (the cube spreading has no adjoint here)
    if (ctx->np > 0 && ctx->pdesc.friction == LBM_FRICTION_STOKESLET_CUBE) return LBM_E_UNSUPPORTED;
    const TapeLayout t = tape_layout(ctx, ctx->np);
    ctx->rec_tape = tape;
    ctx->rec_n0 = ctx->step;
    ctx->rec_nsteps = nsteps;
    ctx->rec_every = every;
    ctx->rec_np = ctx->np;
    ctx->rec_pdesc = ctx->pdesc;
    ctx->rec_R = ctx->R;
    ctx->rec_fext = ctx->fext;
    ctx->rec_pair_on = ctx->pair_on;
    ctx->rec_pg = ctx->pg;
    ctx->rec_rows = ctx->g.ymask + 1;
    const size_t pbytes = size_t(ctx->np) * 3 * 8;
    char *tp = static_cast<char *>(tape);
    for (int32_t s = 0; s < nsteps; ++s) {
        if (s % every == 0) {
            char *slot = tp + size_t(s / every) * t.slot;
            hipError_t e = hipMemcpyAsync(slot, ctx->pop[ctx->cur], t.lat,
                                          hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess && pbytes)
                e = hipMemcpyAsync(slot + t.lat, ctx->r, pbytes, hipMemcpyDeviceToDevice,
                                   ctx->stream);
            if (e == hipSuccess && pbytes)
                e = hipMemcpyAsync(slot + t.lat + pbytes, ctx->v, pbytes,
                                   hipMemcpyDeviceToDevice, ctx->stream);
            if (e != hipSuccess) {
                ctx->rec_tape = nullptr;
                return LBM_E_DEVICE;
            }
        }
        LBM_DISPATCH(ctx, launch_step);
    }
    return launch_status();
}

lbm_status lbm_adjoint_work_bytes(const lbm_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return LBM_E_INVAL;
    if (!ctx->rec_tape) return LBM_E_STATE;
    *bytes = adj_layout(ctx, ctx->rec_np, ctx->rec_every).total;
    return LBM_OK;
}

lbm_status lbm_adjoint(lbm_ctx *ctx, const void *tape, void *work, double *adj_pop,
                       double *adj_r, double *adj_v, double *adj_param) {
    if (!ctx || !tape || !work || !aligned(work) || !adj_pop || !adj_param) return LBM_E_INVAL;
    if (!adjoint_storage(ctx)) return LBM_E_UNSUPPORTED;
    if (ctx->rec_np > 0 && ctx->rec_pdesc.friction == LBM_FRICTION_STOKESLET_CUBE)
        return LBM_E_UNSUPPORTED;
    if (!ctx->rec_tape || tape != ctx->rec_tape) return LBM_E_STATE;
    // the checkpoints hold lattices in the layout they were recorded in
    if (ctx->g.ymask + 1 != ctx->rec_rows) return LBM_E_STATE;
    if (ctx->rec_np > 0 && (!adj_r || !adj_v)) return LBM_E_INVAL;
    hipError_t e = hipSuccess;
    LBM_DISPATCH(ctx, adjoint_dispatch, static_cast<char *>(const_cast<void *>(tape)),
                 static_cast<char *>(work), adj_pop, adj_r, adj_v, adj_param, &e);
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

}  // extern "C"
