// Particle side of one coupled step (section 2.1): eight lanes per particle,
// one per neighbour node.  Gather of the nodal velocity (Eq. s2-fv), friction
// (Eq. s2-slet-v, or Eqs. s2-dis1 / s2-dis0), Brownian force (Eqs. s2-rf1,
// s2-rf2), spreading of the reaction force (first Eq. s2-force) and the
// Langevin update (Eqs. s2-langevin, s2-langevin2), plus the VACF sample.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbmbp.h"
#include "codec.hpp"
#include "collide.hpp"
#include "velocities.hpp"
#include "philox.hpp"

namespace lbmbp {

constexpr int kVacfBatch = 4;  // VACF origins per lane whose loads are in flight together
constexpr int kParticleBlock = 64;  // eight particles per block: spread over every CU
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Particle coupling: eight lanes per particle, lane p owns neighbour node
// floor(s) + (p & 1, p >> 1 & 1, p >> 2 & 1).
// ---------------------------------------------------------------------------
struct ParticleArgs {
    double *r, *v;
    double *fh, *fr;
    uint32_t *prev_cell;  // [n][8] node each lane spread to last step, or kNoNode
    uint32_t *err;
    int32_t n;
    int32_t friction;
    double mass, gamma, sig, R;
    uint64_t seed;
    uint32_t replica;
    uint32_t step;
    // velocity autocorrelation (acc == nullptr: off).  Origins k*stride with
    // k in [k_lo, k_hi] are active at sample time t; origin k lives in slot
    // k % nslot.
    double *acc;      // [n][max_lag+1]
    double *origins;  // [nslot][n][3]
    int64_t t, k_lo, k_hi;
    int32_t nslot, stride, max_lag;
    int32_t slot_lo;  // slot of origin k_lo (k_lo % nslot)
    // per-block FP64 sums of M V^n (nullptr: off), [blocks][3]
    double *pmom;
    // given force on each particle, [n][3] (nullptr: none)
    const double *fext;
    // pair forces of this step, [n][3] (nullptr: none); F_C = fext + fpair
    const double *fpair;
};

__device__ inline double sum8(double v) {
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}

// Intermediates of the Stokeslet fit that its adjoint reuses.
struct FitTrace {
    double w[3];        // u_p - V at this lane's node
    double eN[3], mn;   // direction and length of the mean relative velocity
    double rp, de;      // |d_p| and d_p . e^N
    double ca, cb;      // g_p = ca e^N - cb d_p
    double g[3];
    double num, den, U; // U^inf = num / den
    bool has_dir, use, ok;
};

// Friction force on one particle from its eight lanes (lane p holds node p:
// velocity u, offset d = node - particle, trilinear weight W); every lane of
// the group calls it and receives the same F_H.
//   LBM_FRICTION_STOKESLET (Eq. s2-slet-v): e^N from the mean relative
//     velocity, least-squares amplitude U^inf of the Stokeslet shape g_p,
//     F_H = gamma U^inf e^N; LBM_FRICTION_STOKESLET_2DX and _CUBE are the
//     same fit with u and d taken at the corners of the (2 dx)^3 cube;
//   LBM_FRICTION_POINTWISE (Eq. s2-dis1): F_H = -gamma (V - u(r)) with u(r)
//     interpolated trilinearly;
//   LBM_FRICTION_BD (Eq. s2-dis0): F_H = -gamma V.
__device__ inline void friction_lanes(int32_t mode, double gamma, double R, double W,
                                      const double (&u)[3], const double (&V)[3],
                                      const double (&d)[3], double (&FH)[3], FitTrace &t) {
    FH[0] = FH[1] = FH[2] = 0.0;
    if (mode == LBM_FRICTION_BD) {
#pragma unroll
        for (int k = 0; k < 3; ++k) FH[k] = -gamma * V[k];
        return;
    }
    if (mode == LBM_FRICTION_POINTWISE) {
#pragma unroll
        for (int k = 0; k < 3; ++k) FH[k] = -gamma * (V[k] - sum8(W * u[k]));
        return;
    }
    double m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t.w[k] = u[k] - V[k];
        m[k] = sum8(t.w[k]) / 8.0;
    }
    t.mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    t.has_dir = t.mn > 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) t.eN[k] = t.has_dir ? m[k] / t.mn : 0.0;
    t.rp = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    t.use = t.rp > 1e-12;
    double num = 0.0, den = 0.0;
    t.de = t.ca = t.cb = 0.0;
    t.g[0] = t.g[1] = t.g[2] = 0.0;
    if (t.use) {
        t.de = d[0] * t.eN[0] + d[1] * t.eN[1] + d[2] * t.eN[2];
        t.ca = 1.0 - 3.0 * R / (4.0 * t.rp);
        t.cb = 3.0 * R * t.de / (4.0 * t.rp * t.rp * t.rp);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            t.g[k] = t.ca * t.eN[k] - t.cb * d[k];
            num += t.w[k] * t.g[k];
            den += t.g[k] * t.g[k];
        }
    }
    t.num = sum8(num);
    t.den = sum8(den);
    t.ok = t.has_dir && t.den != 0.0;
    t.U = t.ok ? t.num / t.den : 0.0;
    if (t.ok) {
#pragma unroll
        for (int k = 0; k < 3; ++k) FH[k] = gamma * t.U * t.eN[k];
    }
}

// Periodic node coordinate c + off for a corner offset off in [0, 2] and c
// in [lo, hi] (lo >= -1, hi + 2 <= L + 1), as the floor of a wrapped finite
// position gives it; the clamp keeps a non-finite position (converted to an
// arbitrary integer) in the box.  One conditional add or subtract of L in
// place of an integer division (L >= 2).
__device__ inline uint32_t wrap_node(int32_t c, int32_t lo, int32_t hi, int32_t off, int32_t L) {
    int32_t ci = min(max(c, lo), hi) + off;
    ci = ci < 0 ? ci + L : ci;
    ci = ci >= L ? ci - L : ci;
    return uint32_t(ci);
}

// Node p of the (2 dx)^3 fitting cube of the wide Stokeslet fit: per axis the
// corners c0 and c0 + 2 with c0 = floor(s + 1/2) - 1, s the wrapped position,
// so that the particle sits in the middle half of the cube.  q: the node
// (periodic), dq: node minus particle (unwrapped).
__device__ inline void wide_corner(const double (&r)[3], const uint32_t (&Ln)[3], const int (&b)[3],
                                   uint32_t (&q)[3], double (&dq)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = double(Ln[k]);
        const double s = r[k] - L * floor(r[k] / L);
        const double c0 = floor(s + 0.5) - 1.0;
        dq[k] = (c0 + 2.0 * double(b[k])) - s;
        // c0 in [-1, L - 1] for s in [-eps, L]
        q[k] = wrap_node(int32_t(c0), -1, int32_t(Ln[k]) - 1, 2 * b[k], int32_t(Ln[k]));
    }
}

// Where a particle lives: its box, lattice and node-force fields, and the
// Philox key and counter words of its Brownian force.
template <class C>
struct ParticleSite {
    const typename C::T *A;
    Grid g;
    ForceField cur, old;
    uint64_t seed;
    uint32_t replica;  // third counter word
    uint32_t index;    // second counter word: particle index within its box
    double R;          // particle radius used by the fit
};

// One lane (node p of particle i) of the coupled particle update.  r, V are
// the particle's position and velocity at the start of the step; the whole
// 8-lane group must call this together (it shuffles within the group).
template <class C>
__device__ inline void particle_lane(const ParticleSite<C> &site, typename C::R dec_s,
                                     const ParticleArgs &pa, int32_t i, int p, bool valid,
                                     const double (&r)[3], const double (&V)[3]) {
    using Vs = typename C::V;
    const typename C::T *__restrict__ A = site.A;
    const Grid &g = site.g;
    const ForceField &cur = site.cur;
    const ForceField &old = site.old;
    // Release this lane's node from the field used one step ago (that step's
    // stream-collide has consumed it).  Issued first, so that its stores are
    // in flight together with the gather below.
    const uint32_t pc = valid ? pa.prev_cell[8 * i + p] : kNoNode;
    if (pc != kNoNode) {
        old.f[3 * uint64_t(pc) + 0] = 0;
        old.f[3 * uint64_t(pc) + 1] = 0;
        old.f[3 * uint64_t(pc) + 2] = 0;
        atomicAnd(&old.mask[pc >> 5], ~(1u << (pc & 31)));
    }
    const uint32_t Ln[3] = {g.nx, g.ny, g.nz};
    const int b[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
    double d[3];
    uint32_t node[3];
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = double(Ln[k]);
        const double s = r[k] - L * floor(r[k] / L);  // wrapped position, in [-eps, L]
        const double c = floor(s);
        d[k] = (c + double(b[k])) - s;                // node minus particle, unwrapped
        // Rounding can leave c at -1 or L; the periodic wrap handles both.
        node[k] = wrap_node(int32_t(c), -1, int32_t(Ln[k]), b[k], int32_t(Ln[k]));
        W *= 1.0 - fabs(d[k]);
    }
    const uint32_t cell = (node[2] * g.ny + node[1]) * g.nx + node[0];
    const bool coupled = pa.friction != LBM_FRICTION_BD;
    // The fit reads the same eight nodes, or those of the (2 dx)^3 cube.
    uint32_t fnode[3] = {node[0], node[1], node[2]};
    double dfit[3] = {d[0], d[1], d[2]};
    const bool cube = pa.friction == LBM_FRICTION_STOKESLET_CUBE;
    if (pa.friction == LBM_FRICTION_STOKESLET_2DX || cube) wide_corner(r, Ln, b, fnode, dfit);
    // The reaction force goes to the unit cell's corner with its trilinear
    // weight, or with the cube fit to this lane's cube corner with the cube's
    // weight prod_k (1 - |d_k| / 2).
    uint32_t scell = cell;
    double sW = W;
    if (cube) {
        scell = (fnode[2] * g.ny + fnode[1]) * g.nx + fnode[0];
        sW = (1.0 - 0.5 * fabs(dfit[0])) * (1.0 - 0.5 * fabs(dfit[1])) * (1.0 - 0.5 * fabs(dfit[2]));
    }

    // Issue the gather of f^n at this lane's fitting node (pull from node -
    // e_a); the values are consumed only after the VACF sample and the
    // Brownian force, which overlap the load latency.  Plain loads: the
    // following sweep reads these lines again, and non-temporal ones, though
    // 1.2 us faster here, cost the sweep as much or more.
    typename C::T raw[Vs::Q];
    if (coupled) {
        const Neighbours nb(fnode[0], fnode[1], fnode[2], g);
        static_for<1, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            raw[a] = A[nb.template pop<Vs, a>(g)];
        });
    }

    // Loads whose results are needed only at the end: the given and pair forces.
    double fc[3] = {0.0, 0.0, 0.0};
    if (valid && p == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (pa.fext) fc[k] = pa.fext[3 * i + k];
            if (pa.fpair) fc[k] += pa.fpair[3 * i + k];
        }
    }

    // C_v(t) = <V(0).V(t)> (section 2.1): V^n against every active origin;
    // lane p takes the origins k = k_lo + p, k_lo + p + 8, ...  The newest
    // origin (lag 0) is stored by the lane that owns it.  Origins go in
    // batches of kVacfBatch: all loads of a batch before any of its stores.
    if (valid && pa.acc) {
        // accumulators are lag-major (acc[lag][n]): the same lane of the eight
        // particles of a wavefront updates eight consecutive doubles
        double *acc_i = pa.acc + i;
        const int64_t n = pa.n;
        // origin k lives in slot k % nslot; this lane's origins k_lo + p,
        // k_lo + p + 8, ... step through the slots by 8 (mod nslot)
        const int32_t ns = pa.nslot;
        const int32_t d8 = 8 % ns;
        int32_t slot = pa.slot_lo + p % ns;
        slot = slot >= ns ? slot - ns : slot;
        for (int64_t k0 = pa.k_lo + p; k0 <= pa.k_hi; k0 += 8 * kVacfBatch) {
            double ov[kVacfBatch][3], av[kVacfBatch];
            int32_t sl[kVacfBatch];
#pragma unroll
            for (int c = 0; c < kVacfBatch; ++c) {
                sl[c] = slot;
                slot += d8;
                slot = slot >= ns ? slot - ns : slot;
            }
#pragma unroll
            for (int c = 0; c < kVacfBatch; ++c) {
                const int64_t k = k0 + 8 * c;
                const int64_t lag = pa.t - k * pa.stride;
                ov[c][0] = ov[c][1] = ov[c][2] = av[c] = 0.0;
                if (k <= pa.k_hi && lag != 0) {
                    const double *o = pa.origins + (int64_t(sl[c]) * pa.n + i) * 3;
                    ov[c][0] = o[0];
                    ov[c][1] = o[1];
                    ov[c][2] = o[2];
                    av[c] = acc_i[lag * n];
                }
            }
#pragma unroll
            for (int c = 0; c < kVacfBatch; ++c) {
                const int64_t k = k0 + 8 * c;
                if (k > pa.k_hi) break;
                const int64_t lag = pa.t - k * pa.stride;
                if (lag == 0) {
                    double *o = pa.origins + (int64_t(sl[c]) * pa.n + i) * 3;
                    o[0] = V[0];
                    o[1] = V[1];
                    o[2] = V[2];
                    acc_i[0] += V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
                } else {
                    acc_i[lag * n] = av[c] + (ov[c][0] * V[0] + ov[c][1] * V[1] + ov[c][2] * V[2]);
                }
            }
        }
    }

    // Eqs. s2-rf1, s2-rf2: white noise of variance 2 gamma kT per step.  The
    // three Box-Muller outputs are computed by lanes 0, 1, 2 of the group
    // (one logarithm, square root and sine/cosine each) and gathered.
    double FR[3] = {0.0, 0.0, 0.0};
    if (pa.sig > 0.0) {
        const Philox4x32 x = philox4x32_10(pa.step, site.index, site.replica, 0u,
                                           uint32_t(site.seed), uint32_t(site.seed >> 32));
        const int q = p < 3 ? p : 0;
        const uint32_t wa = q == 2 ? x.v[2] : x.v[0];
        const uint32_t wb = q == 2 ? x.v[3] : x.v[1];
        double zq;
        box_muller_one(wa, wb, q == 1, &zq);
#pragma unroll
        for (int k = 0; k < 3; ++k) FR[k] = pa.sig * __shfl(zq, k, 8);
    }

    double FH[3];
    double u[3] = {0.0, 0.0, 0.0};
    if (coupled) {
        // u^n at this lane's node: u = sum_a e_a f_a = sum_a e_a g_a (Eq. s2-fv).
        static_for<1, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            const double gvl = double(C::dec(raw[a], dec_s));
            if constexpr (Vs::ex[a] != 0) u[0] += Vs::ex[a] > 0 ? gvl : -gvl;
            if constexpr (Vs::ey[a] != 0) u[1] += Vs::ey[a] > 0 ? gvl : -gvl;
            if constexpr (Vs::ez[a] != 0) u[2] += Vs::ez[a] > 0 ? gvl : -gvl;
        });
    }
    FitTrace tr;
    friction_lanes(pa.friction, pa.gamma, site.R, W, u, V, dfit, FH, tr);
    if (!valid) return;

    // First Eq. s2-force: the node receives -F_H W_p (unit cell volume).
    uint32_t my_cell = kNoNode;
    if (coupled) {
        long long q[3];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double c = -FH[k] * sW;
            ok = ok && (fabs(c) < kFixLimit);
            q[k] = __double2ll_rn(c * kFixScale);
        }
        if (!ok) {
            atomicOr(pa.err, kErrFixRange);
            q[0] = q[1] = q[2] = 0;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            atomicAdd(reinterpret_cast<unsigned long long *>(&cur.f[3 * uint64_t(scell) + k]),
                      static_cast<unsigned long long>(q[k]));
        atomicOr(&cur.mask[scell >> 5], 1u << (scell & 31));
        my_cell = scell;
    }
    pa.prev_cell[8 * i + p] = my_cell;

    if (p != 0) return;
    // Eqs. s2-langevin, s2-langevin2 with dt = 1; F_C is the given force (or 0).
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vn = V[k] + (fc[k] + FH[k] + FR[k]) / pa.mass;
        pa.v[3 * i + k] = vn;
        pa.r[3 * i + k] = r[k] + vn;
        pa.fh[3 * i + k] = FH[k];
        pa.fr[3 * i + k] = FR[k];
    }
}

template <class C>
__global__ __launch_bounds__(kParticleBlock) void k_particle(const typename C::T *__restrict__ A,
                                                             Grid g, typename C::R dec_s,
                                                             ParticleArgs pa, ForceField cur,
                                                             ForceField old) {
    const uint32_t gt = blockIdx.x * kParticleBlock + threadIdx.x;
    const int32_t i = int32_t(gt >> 3);
    const int p = int(gt & 7u);
    const bool valid = i < pa.n;
    const int32_t ii = valid ? i : pa.n - 1;  // whole 8-lane groups are valid or not

    double r[3], V[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = pa.r[3 * ii + k];
        V[k] = pa.v[3 * ii + k];
    }
    if (pa.pmom) {
        // particle momentum M V^n of the state at the start of the step
        double pm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) pm[k] = (valid && p == 0) ? pa.mass * V[k] : 0.0;
        block_sum<3, kParticleBlock>(pm, pa.pmom + 3 * uint64_t(blockIdx.x));
    }
    const ParticleSite<C> site{A, g, cur, old, pa.seed, pa.replica, uint32_t(i), pa.R};
    particle_lane<C>(site, dec_s, pa, i, p, valid, r, V);
}

}  // namespace lbmbp
