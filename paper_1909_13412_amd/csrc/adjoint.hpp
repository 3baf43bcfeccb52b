// Reverse mode of the coupled step: the adjoint (vector-Jacobian product) of
//   f^{n+1}, r^{n+1}, V^{n+1} = S(f^n, r^n, V^n; gamma, tau, M, kT)
// for one step S as the forward kernels compute it (section 2: Eqs. s2-fv,
// s2-slet-v / s2-dis1 / s2-dis0, s2-rf1, s2-rf2, first and second Eq.
// s2-force, s2-collision, s2-eq, s2-coll, s2-trans, s2-langevin,
// s2-langevin2).  Derivatives are those of the exact-arithmetic map taken at
// the stored forward trajectory; a given particle force F_C is a constant, and
// the corner cell floor(s) and the fit's branch tests are piecewise constant.
// Adjoint arithmetic is FP64 throughout.
//
// Adjoint populations fb^n_a(x) = dJ/df^n_a(x) (post-streaming populations at
// node x) live in an FP64 lattice of the interleaved-row layout, at their own
// node (no shift).  One reverse step n, given fb^{n+1}, rb^{n+1}, Vb^{n+1}:
//   k_adj_particle  per particle (eight lanes): recompute u at the nodes, the
//                   fit, F_R; node-force adjoint Fb(x_p) = 3 sum_a w_a e_a
//                   fb^{n+1}_a(x_p + e_a); back through the Langevin update,
//                   the spreading weights and the fit; push ub_p (the adjoint
//                   of the nodal velocity) into a flagged FP64 node field.
//   k_adj_collide   every node: fs_a = fb^{n+1}_a(x + e_a) (streaming
//                   transposed), then the transposed BGK Jacobian
//                   fb^n_b = (1 - w) fs_b + w [P + 3 e_b.Q + 9 e_b.T - 3 P u.e_b]
//                   with P = sum_a w_a fs_a, Q = sum_a w_a fs_a e_a,
//                   T = sum_a w_a fs_a (e_a.u) e_a (from
//                   d feq_a / d f_b = w_a [1 + 3 e_a.e_b + 9 (e_a.u)(e_a.e_b) - 3 u.e_b]),
//                   plus e_b.ub(x) at flagged nodes; dJ/domega partial
//                   sum_a fs_a (feq_a - f_a).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbmbp.h"
#include "codec.hpp"
#include "collide.hpp"
#include "velocities.hpp"
#include "particle.hpp"
#include "philox.hpp"

namespace lbmbp {

// FP64 adjoint of the nodal velocity, written only at the nodes around the
// particles and flagged one bit per node; two alternate between reverse steps
// and each particle lane clears the node it wrote one reverse step earlier.
struct AdjField {
    double *u;       // [ncell][3]
    uint32_t *mask;  // one bit per node
};

struct AdjParticleArgs {
    const double *r, *v;   // state at step n, [n][3]
    double *rbar, *vbar;   // in: dJ/dr^{n+1}, dJ/dV^{n+1}; out: dJ/dr^n, dJ/dV^n
    double *pgrad;         // [n][4] running dJ/d(gamma, tau, M, kT)
    const double *fext;    // given force on each particle, [n][3] (nullptr: none)
    const double *fpair;   // pair forces of step n, [n][3] (nullptr: none)
    double *fcbar;         // out: dJ/dF_C of step n, [n][3] (nullptr: not needed)
    uint32_t *prev_cell;   // [n][8] node each lane wrote one reverse step ago
    int32_t n;
    int32_t friction;
    double mass, gamma, kT, sig, R;
    double dR_dgamma, dR_dtau;  // zero when the radius is given
    uint64_t seed;
    uint32_t replica;
    uint32_t step;
};

// Storage index of population a at node x + e_a (the streaming target of x).
template <class Vs, int a>
__device__ inline uint64_t push_index(const Neighbours &nb, const Grid &g) {
    return pop_index<Vs>(g, nb.sx[1 - Vs::ex[a]], nb.sy[1 - Vs::ey[a]], nb.sz[1 - Vs::ez[a]], a);
}

template <class C>
__global__ __launch_bounds__(kParticleBlock) void k_adj_particle(
    const typename C::T *__restrict__ A, Grid g, typename C::R dec_s,
    const double *__restrict__ Abar, Grid gd, AdjParticleArgs pa, AdjField cur, AdjField old) {
    using Vs = typename C::V;
    const uint32_t gt = blockIdx.x * kParticleBlock + threadIdx.x;
    const int32_t i = int32_t(gt >> 3);
    const int p = int(gt & 7u);
    const bool valid = i < pa.n;
    const int32_t ii = valid ? i : pa.n - 1;  // whole 8-lane groups are valid or not

    double r[3], V[3], rb[3], vb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = pa.r[3 * ii + k];
        V[k] = pa.v[3 * ii + k];
        rb[k] = pa.rbar[3 * ii + k];
        vb[k] = pa.vbar[3 * ii + k];
    }
    // Geometry of this lane's node, exactly as the forward step.
    const uint32_t Ln[3] = {g.nx, g.ny, g.nz};
    const int b[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
    double d[3], tf[3];
    uint32_t node[3];
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = double(Ln[k]);
        const double s = r[k] - L * floor(r[k] / L);
        const double c = floor(s);
        d[k] = (c + double(b[k])) - s;
        node[k] = wrap_node(int32_t(c), -1, int32_t(Ln[k]), b[k], int32_t(Ln[k]));
        tf[k] = 1.0 - fabs(d[k]);
        W *= tf[k];
    }
    const bool coupled = pa.friction != LBM_FRICTION_BD;
    // Fitting node: the same, or the corner of the (2 dx)^3 cube.
    uint32_t fnode[3] = {node[0], node[1], node[2]};
    double dfit[3] = {d[0], d[1], d[2]};
    if (pa.friction == LBM_FRICTION_STOKESLET_2DX) wide_corner(r, Ln, b, fnode, dfit);
    const uint32_t fcell = (fnode[2] * g.ny + fnode[1]) * g.nx + fnode[0];

    // Nodal velocity u^n at the fitting node and the node-force adjoint
    // Fb = 3 sum_a w_a e_a fs_a at the spreading node.
    double u[3] = {0.0, 0.0, 0.0};
    double Fb[3] = {0.0, 0.0, 0.0};
    if (coupled) {
        const Neighbours nf(fnode[0], fnode[1], fnode[2], g);
        const Neighbours nb(node[0], node[1], node[2], g);
        static_for<1, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            const double gvl = double(C::dec(A[nf.template pop<Vs, a>(g)], dec_s));
            const double fs = Abar[push_index<Vs, a>(nb, gd)];
            const double w3 = 3.0 * Vs::template w<double>(a);
            if constexpr (Vs::ex[a] != 0) {
                u[0] += Vs::ex[a] > 0 ? gvl : -gvl;
                Fb[0] += Vs::ex[a] > 0 ? w3 * fs : -w3 * fs;
            }
            if constexpr (Vs::ey[a] != 0) {
                u[1] += Vs::ey[a] > 0 ? gvl : -gvl;
                Fb[1] += Vs::ey[a] > 0 ? w3 * fs : -w3 * fs;
            }
            if constexpr (Vs::ez[a] != 0) {
                u[2] += Vs::ez[a] > 0 ? gvl : -gvl;
                Fb[2] += Vs::ez[a] > 0 ? w3 * fs : -w3 * fs;
            }
        });
    }

    // The normals of the Brownian force, as the forward step draws them.
    double xi[3] = {0.0, 0.0, 0.0};
    if (pa.sig > 0.0) {
        const Philox4x32 x = philox4x32_10(pa.step, uint32_t(i), pa.replica, 0u,
                                           uint32_t(pa.seed), uint32_t(pa.seed >> 32));
        const int q = p < 3 ? p : 0;
        const uint32_t wa = q == 2 ? x.v[2] : x.v[0];
        const uint32_t wb = q == 2 ? x.v[3] : x.v[1];
        double zq;
        box_muller_one(wa, wb, q == 1, &zq);
#pragma unroll
        for (int k = 0; k < 3; ++k) xi[k] = __shfl(zq, k, 8);
    }
    double FH[3];
    FitTrace tr;
    friction_lanes(pa.friction, pa.gamma, pa.R, W, u, V, dfit, FH, tr);

    // Langevin update: V' = V + (F_C + F_H + F_R)/M, r' = r + V'.
    double Vt[3], FHb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Vt[k] = vb[k] + rb[k];
        FHb[k] = Vt[k] / pa.mass;
    }
    // Spreading: node p receives -F_H W_p.
    double Wb = 0.0;
    if (coupled) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            FHb[k] -= sum8(W * Fb[k]);
            Wb -= FH[k] * Fb[k];
        }
    }

    // Back through the friction.
    double ub[3] = {0.0, 0.0, 0.0};  // this lane's node velocity
    double Vbf[3] = {0.0, 0.0, 0.0}; // particle velocity, whole-particle value
    double db[3] = {0.0, 0.0, 0.0};  // this lane's fitting offset
    double gam_b = 0.0, R_b = 0.0;   // whole-particle values
    if (pa.friction == LBM_FRICTION_BD) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            gam_b -= FHb[k] * V[k];
            Vbf[k] = -pa.gamma * FHb[k];
        }
    } else if (pa.friction == LBM_FRICTION_POINTWISE) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double ur = sum8(W * u[k]);
            gam_b -= FHb[k] * (V[k] - ur);
            Vbf[k] = -pa.gamma * FHb[k];
            ub[k] = pa.gamma * FHb[k] * W;
            Wb += pa.gamma * FHb[k] * u[k];
        }
    } else if (tr.ok) {
        double Ub = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            gam_b += FHb[k] * tr.U * tr.eN[k];
            Ub += pa.gamma * FHb[k] * tr.eN[k];
        }
        const double numb = Ub / tr.den;
        const double denb = -Ub * tr.U / tr.den;
        double wb[3] = {0.0, 0.0, 0.0}, eNb[3] = {0.0, 0.0, 0.0}, Rb = 0.0;
        if (tr.use) {
            const double rp = tr.rp;
            const double rp3 = rp * rp * rp;
            double gb[3], cab = 0.0, cbb = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                wb[k] = numb * tr.g[k];
                gb[k] = numb * tr.w[k] + 2.0 * denb * tr.g[k];
                cab += gb[k] * tr.eN[k];
                cbb -= gb[k] * dfit[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                eNb[k] += tr.ca * gb[k];
                db[k] -= tr.cb * gb[k];
            }
            // ca = 1 - 3R/(4 rp), cb = 3R de/(4 rp^3)
            Rb = cbb * 3.0 * tr.de / (4.0 * rp3) - cab * 3.0 / (4.0 * rp);
            const double deb = cbb * 3.0 * pa.R / (4.0 * rp3);
            const double rpb = -cbb * 3.0 * tr.cb / rp + cab * 3.0 * pa.R / (4.0 * rp * rp);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                db[k] += deb * tr.eN[k] + rpb * dfit[k] / rp;
                eNb[k] += deb * dfit[k];
            }
        }
        // e^N = m / |m| with m the mean of w over the eight nodes.
        double eNt[3], proj = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            eNt[k] = pa.gamma * tr.U * FHb[k] + sum8(eNb[k]);
            proj += tr.eN[k] * eNt[k];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double mb = (eNt[k] - tr.eN[k] * proj) / tr.mn;
            wb[k] += mb / 8.0;
            ub[k] = wb[k];
            Vbf[k] = -sum8(wb[k]);
        }
        R_b = sum8(Rb);
    }
    // Wrapped position s = r - L floor(r/L) (slope 1); both offsets are a
    // fixed node minus s, and the weight factors are 1 + d (b = 0) or 1 - d
    // (b = 1) inside the corner cell.
    double sb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double others = tf[(k + 1) % 3] * tf[(k + 2) % 3];
        sb[k] = sum8(-db[k] + Wb * others * (b[k] ? 1.0 : -1.0));
    }
    if (!valid) return;

    // Release this lane's node from the field of the previous reverse step.
    const uint32_t pc = pa.prev_cell[8 * i + p];
    if (pc != kNoNode) {
        old.u[3 * uint64_t(pc) + 0] = 0.0;
        old.u[3 * uint64_t(pc) + 1] = 0.0;
        old.u[3 * uint64_t(pc) + 2] = 0.0;
        atomicAnd(&old.mask[pc >> 5], ~(1u << (pc & 31)));
    }
    uint32_t my_cell = kNoNode;
    if (coupled) {
#pragma unroll
        for (int k = 0; k < 3; ++k) atomicAdd(&cur.u[3 * uint64_t(fcell) + k], ub[k]);
        atomicOr(&cur.mask[fcell >> 5], 1u << (fcell & 31));
        my_cell = fcell;
    }
    pa.prev_cell[8 * i + p] = my_cell;

    if (p != 0) return;
    // Parameters: R(gamma, tau) when the radius follows Stokes' law; F_R =
    // sqrt(2 gamma kT) xi; the Langevin division by M.
    double FRb_xi = 0.0, dM = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        FRb_xi += (Vt[k] / pa.mass) * xi[k];
        double fc = pa.fext ? pa.fext[3 * i + k] : 0.0;
        if (pa.fpair) fc += pa.fpair[3 * i + k];
        dM -= Vt[k] * (fc + FH[k] + pa.sig * xi[k]) / (pa.mass * pa.mass);
        if (pa.fcbar) pa.fcbar[3 * i + k] = Vt[k] / pa.mass;
    }
    double *pg = pa.pgrad + 4 * int64_t(i);
    pg[0] += gam_b + R_b * pa.dR_dgamma + (pa.sig > 0.0 ? FRb_xi * pa.kT / pa.sig : 0.0);
    pg[1] += R_b * pa.dR_dtau;
    pg[2] += dM;
    pg[3] += pa.sig > 0.0 ? FRb_xi * pa.gamma / pa.sig : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pa.rbar[3 * i + k] = rb[k] + sb[k];
        pa.vbar[3 * i + k] = Vt[k] + Vbf[k];
    }
}

template <class C, bool FORCED, bool NTS, bool ROWS>
__global__ __launch_bounds__(kBlock) void k_adj_collide(const typename C::T *__restrict__ A, Grid g,
                                                        typename C::R dec_s,
                                                        const double *__restrict__ Abar,
                                                        double *__restrict__ Bbar, Grid gd,
                                                        double omega, AdjField uf,
                                                        double *__restrict__ wacc) {
    using Vs = typename C::V;
    using T = typename C::T;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    double wsum = 0.0;
    if (cell < g.ncell) {
        // ROWS: every wavefront lies in one row (64 | nx), addresses from the
        // wavefront's row offsets as in the forward sweep (kAddrRow)
        uint32_t x, y, z;
        lane_coords<ROWS ? kAddrRow : kAddrLane64>(g, cell, g.ny, x, y, z);
        const uint32_t popA = g.pstride * uint32_t(sizeof(T));
        const uint32_t popD = gd.pstride * uint32_t(sizeof(double));
        [[maybe_unused]] const RowOffsets roA(x, y, z, g, Vs::Q, sizeof(T));
        [[maybe_unused]] const RowOffsets roD(x, y, z, gd, Vs::Q, sizeof(double));
        const Neighbours nb(x, y, z, g);
        double gv[Vs::Q], fs[Vs::Q];
        static_for<0, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            if constexpr (ROWS) {
                gv[a] = double(C::dec(*roA.template pull<Vs, a>(A, popA), dec_s));
                fs[a] = *roD.template push<Vs, a>(Abar, popD);
            } else {
                gv[a] = double(C::dec(A[nb.template pop<Vs, a>(g)], dec_s));
                fs[a] = Abar[push_index<Vs, a>(nb, gd)];
            }
        });
        bool flagged = false;
        if constexpr (FORCED) flagged = (uf.mask[cell >> 5] >> (cell & 31)) & 1u;
        double drho = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
        static_for<0, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            drho += gv[a];
            if constexpr (Vs::ex[a] != 0) ux += Vs::ex[a] > 0 ? gv[a] : -gv[a];
            if constexpr (Vs::ey[a] != 0) uy += Vs::ey[a] > 0 ? gv[a] : -gv[a];
            if constexpr (Vs::ez[a] != 0) uz += Vs::ez[a] > 0 ? gv[a] : -gv[a];
        });
        const double uu = ux * ux + uy * uy + uz * uz;
        double P = 0.0, Qx = 0.0, Qy = 0.0, Qz = 0.0, Tx = 0.0, Ty = 0.0, Tz = 0.0;
        static_for<0, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int cx = Vs::ex[a], cy = Vs::ey[a], cz = Vs::ez[a];
            const double w = Vs::template w<double>(a);
            const double eu = double(cx) * ux + double(cy) * uy + double(cz) * uz;
            const double geq = w * (drho + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
            wsum += fs[a] * (geq - gv[a]);
            const double wf = w * fs[a];
            P += wf;
            Qx += double(cx) * wf;
            Qy += double(cy) * wf;
            Qz += double(cz) * wf;
            Tx += double(cx) * eu * wf;
            Ty += double(cy) * eu * wf;
            Tz += double(cz) * eu * wf;
        });
        double Ux = 0.0, Uy = 0.0, Uz = 0.0;
        if constexpr (FORCED) {
            if (flagged) {
                Ux = uf.u[3 * uint64_t(cell) + 0];
                Uy = uf.u[3 * uint64_t(cell) + 1];
                Uz = uf.u[3 * uint64_t(cell) + 2];
            }
        }
        const double Gx = 3.0 * Qx + 9.0 * Tx - 3.0 * P * ux;
        const double Gy = 3.0 * Qy + 9.0 * Ty - 3.0 * P * uy;
        const double Gz = 3.0 * Qz + 9.0 * Tz - 3.0 * P * uz;
        const uint64_t row_base = row_index<Vs>(gd, y, z) + x;
        static_for<0, Vs::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            constexpr int cx = Vs::ex[a], cy = Vs::ey[a], cz = Vs::ez[a];
            double out = (1.0 - omega) * fs[a] +
                         omega * (P + double(cx) * Gx + double(cy) * Gy + double(cz) * Gz);
            if constexpr (FORCED) out += double(cx) * Ux + double(cy) * Uy + double(cz) * Uz;
            double *dst = ROWS ? roD.own(Bbar, a, popD) : &Bbar[row_base + uint64_t(a) * gd.pstride];
            if constexpr (NTS)
                __builtin_nontemporal_store(out, dst);
            else
                *dst = out;
        });
    }
    // dJ/domega of this block, added to its own running slot (fixed order).
    __shared__ double sh[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
        wacc[blockIdx.x] += s;
    }
}

// Canonical FP64 [19][nz][ny][nx] <-> adjoint lattice (interleaved rows).
template <class Vs>
__global__ __launch_bounds__(kBlock) void k_adj_import(const double *__restrict__ canon,
                                                       double *__restrict__ Abar, Grid gd) {
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= gd.ncell) return;
    const uint32_t x = cell % gd.nx, t = cell / gd.nx, y = t % gd.ny, z = t / gd.ny;
    for (int a = 0; a < Vs::Q; ++a)
        Abar[pop_index<Vs>(gd, x, y, z, a)] = canon[uint64_t(a) * gd.ncell + cell];
}

template <class Vs>
__global__ __launch_bounds__(kBlock) void k_adj_export(const double *__restrict__ Abar,
                                                       double *__restrict__ canon, Grid gd) {
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= gd.ncell) return;
    const uint32_t x = cell % gd.nx, t = cell / gd.nx, y = t % gd.ny, z = t / gd.ny;
    for (int a = 0; a < Vs::Q; ++a)
        canon[uint64_t(a) * gd.ncell + cell] = Abar[pop_index<Vs>(gd, x, y, z, a)];
}

// dJ/d(gamma, tau, M, kT): per-particle running sums plus the collision's
// dJ/domega (omega = 1/tau), summed in a fixed order by one block.
__global__ __launch_bounds__(kBlock) void k_adj_params(const double *__restrict__ pgrad, int32_t n,
                                                       const double *__restrict__ wacc,
                                                       int32_t nblk, double tau,
                                                       double *__restrict__ out) {
    __shared__ double sh[5][kBlock];
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t i = threadIdx.x; i < n; i += kBlock)
        for (int k = 0; k < 4; ++k) s[k] += pgrad[4 * int64_t(i) + k];
    for (int32_t j = threadIdx.x; j < nblk; j += kBlock) s[4] += wacc[j];
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w)
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0] - sh[4][0] / (tau * tau);
        out[2] = sh[2][0];
        out[3] = sh[3][0];
    }
}

}  // namespace lbmbp
