// lbmbp: lattice-Boltzmann fluid two-way coupled to Brownian point particles
// (Yoshida, Kinjo & Washizu, arXiv:1909.13412), hand-written HIP for gfx950.
//
// One coupled step n (section 2):
//   [k_vacf]          C_i(l) += V_i(t0) . V_i(n)                    (section 2.1)
//   k_particle        per particle, eight lanes = eight neighbour nodes:
//                     gather u^n at the nodes (Eq. s2-fv), Stokeslet fit
//                     (Eq. s2-slet-v) -> F_H, Philox Brownian force
//                     (Eqs. s2-rf1, s2-rf2), spread -F_H into the forced-node
//                     table (first Eq. s2-force), Langevin update (Eqs.
//                     s2-langevin, s2-langevin2)
//   k_stream_collide  every node: pull f^n_a(x) = A_a(x - e_a) (Eq. s2-trans of
//                     the previous step), moments (Eqs. s2-density, s2-fv),
//                     BGK (Eqs. s2-collision, s2-eq) plus forcing (second
//                     Eq. s2-force) where the node is flagged, write B_a(x)
//                     (Eq. s2-coll); A and B swap.
//
// Layout: structure of arrays, one plane of nx*ny*nz values per velocity,
// x fastest.  Lattice A holds post-collision values at their source node, so
// the post-streaming population is read by pulling from x - e_a.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <type_traits>

#include "lbmbp.h"
#include "codec.hpp"
#include "d3q19.hpp"
#include "philox.hpp"

namespace lbmbp {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
// Node forces are accumulated as 64-bit fixed point (2^-48 resolution) so that
// the sum over particles sharing a node is exact and order independent: runs
// are bitwise reproducible.  |contribution| must stay below 2^14.
constexpr double kFixScale = 281474976710656.0;        // 2^48
constexpr double kFixInv = 1.0 / 281474976710656.0;
constexpr double kFixLimit = 16384.0;
constexpr uint32_t kErrFixRange = 1u;

struct Grid {
    uint32_t nx, ny, nz;
    uint32_t ncell;
    uint64_t pstride;  // elements between velocity planes
};

struct ForceTable {
    uint32_t *keys;    // [cap] node index or kEmpty
    long long *vals;   // [cap][3] fixed-point force
    uint32_t *mask;    // one bit per node: node carries a force this step
    uint32_t capmask;  // cap - 1 (cap is a power of two)
    uint32_t shift;    // 32 - log2(cap)
};

__device__ inline uint32_t hash_slot(uint32_t cell, uint32_t shift) {
    return (cell * 2654435769u) >> shift;  // Fibonacci hashing
}

// Source node of direction a for a pull at (x, y, z): x - e_a, periodic.
struct Neighbours {
    uint32_t sx[3], sy[3], sz[3];  // index [e + 1]: coordinate - e
    __device__ inline Neighbours(uint32_t x, uint32_t y, uint32_t z, const Grid &g) {
        sx[0] = (x + 1 == g.nx) ? 0 : x + 1;
        sx[1] = x;
        sx[2] = (x == 0) ? g.nx - 1 : x - 1;
        sy[0] = (y + 1 == g.ny) ? 0 : y + 1;
        sy[1] = y;
        sy[2] = (y == 0) ? g.ny - 1 : y - 1;
        sz[0] = (z + 1 == g.nz) ? 0 : z + 1;
        sz[1] = z;
        sz[2] = (z == 0) ? g.nz - 1 : z - 1;
    }
    template <int a>
    __device__ inline uint32_t src(const Grid &g) const {
        return (sz[D3Q19::ez[a] + 1] * g.ny + sy[D3Q19::ey[a] + 1]) * g.nx + sx[D3Q19::ex[a] + 1];
    }
};

template <int a, int Q, typename F>
__device__ inline void static_for(F &&f) {
    if constexpr (a < Q) {
        f(std::integral_constant<int, a>{});
        static_for<a + 1, Q>(f);
    }
}

// ---------------------------------------------------------------------------
// Fused pull stream-collide with sparse forcing.
// ---------------------------------------------------------------------------
template <class C, bool FORCED>
__global__ __launch_bounds__(kBlock) void k_stream_collide(const typename C::T *__restrict__ A,
                                                           typename C::T *__restrict__ B, Grid g,
                                                           typename C::R omega,
                                                           typename C::R enc_s,
                                                           typename C::R dec_s, ForceTable ft) {
    using T = typename C::T;
    using R = typename C::R;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx;
    const uint32_t t = cell / g.nx;
    const uint32_t y = t % g.ny;
    const uint32_t z = t / g.ny;
    const Neighbours nb(x, y, z, g);

    R gv[D3Q19::Q];
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        gv[a] = C::dec(A[a * g.pstride + nb.src<a>(g)], dec_s);
    });
    R drho = R(0), ux = R(0), uy = R(0), uz = R(0);
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        drho += gv[a];
        if constexpr (D3Q19::ex[a] != 0) ux += D3Q19::ex[a] > 0 ? gv[a] : -gv[a];
        if constexpr (D3Q19::ey[a] != 0) uy += D3Q19::ey[a] > 0 ? gv[a] : -gv[a];
        if constexpr (D3Q19::ez[a] != 0) uz += D3Q19::ez[a] > 0 ? gv[a] : -gv[a];
    });
    const R uu = ux * ux + uy * uy + uz * uz;
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if constexpr (FORCED) {
        const uint32_t word = ft.mask[cell >> 5];
        if ((word >> (cell & 31)) & 1u) {
            uint32_t slot = hash_slot(cell, ft.shift);
            for (uint32_t probe = 0; probe <= ft.capmask; ++probe) {
                if (ft.keys[slot] == cell) break;
                slot = (slot + 1) & ft.capmask;
            }
            Fx = R(double(ft.vals[3 * slot + 0]) * kFixInv);
            Fy = R(double(ft.vals[3 * slot + 1]) * kFixInv);
            Fz = R(double(ft.vals[3 * slot + 2]) * kFixInv);
        }
    }
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int cx = D3Q19::ex[a], cy = D3Q19::ey[a], cz = D3Q19::ez[a];
        const R w = D3Q19::w<R>(a);
        const R eu = R(cx) * ux + R(cy) * uy + R(cz) * uz;
        const R geq = w * (drho + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
        R gn = gv[a] + omega * (geq - gv[a]);
        if constexpr (FORCED) gn += R(3) * w * (R(cx) * Fx + R(cy) * Fy + R(cz) * Fz);
        B[a * g.pstride + cell] = C::enc(gn, enc_s);
    });
}

// ---------------------------------------------------------------------------
// Particle coupling: eight lanes per particle, lane p owns neighbour node
// floor(s) + (p & 1, p >> 1 & 1, p >> 2 & 1).
// ---------------------------------------------------------------------------
struct ParticleArgs {
    double *r, *v;
    double *fh, *fr;
    int32_t *prev_slot;
    uint32_t *prev_cell;
    uint32_t *err;
    int32_t n;
    int32_t friction;
    double mass, gamma, sig, R;
    uint64_t seed;
    uint32_t replica;
    uint32_t step;
};

__device__ inline double sum8(double v) {
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}

template <class C>
__global__ __launch_bounds__(kBlock) void k_particle(const typename C::T *__restrict__ A, Grid g,
                                                     typename C::R dec_s, ParticleArgs pa,
                                                     ForceTable cur, ForceTable old) {
    const uint32_t gt = blockIdx.x * kBlock + threadIdx.x;
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
    const uint32_t Ln[3] = {g.nx, g.ny, g.nz};
    const int b[3] = {p & 1, (p >> 1) & 1, (p >> 2) & 1};
    double d[3];
    uint32_t node[3];
    double W = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double L = double(Ln[k]);
        const double s = r[k] - L * floor(r[k] / L);  // wrapped position, in [0, L]
        const double c = floor(s);
        d[k] = (c + double(b[k])) - s;                // node minus particle, unwrapped
        // c may equal L after rounding; the modulo also keeps a non-finite
        // position (converted with saturation) inside the box
        node[k] = (uint32_t(c) + uint32_t(b[k])) % Ln[k];
        W *= 1.0 - fabs(d[k]);
    }
    const uint32_t cell = (node[2] * g.ny + node[1]) * g.nx + node[0];

    double FH[3] = {0.0, 0.0, 0.0};
    if (pa.friction == LBM_FRICTION_BD) {
#pragma unroll
        for (int k = 0; k < 3; ++k) FH[k] = -pa.gamma * V[k];
    } else {
        // u^n at this lane's node: u = sum_a e_a f_a = sum_a e_a g_a (Eq. s2-fv).
        const Neighbours nb(node[0], node[1], node[2], g);
        double u[3] = {0.0, 0.0, 0.0};
        static_for<0, D3Q19::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            if constexpr (a != 0) {
                const double gvl = double(C::dec(A[a * g.pstride + nb.src<a>(g)], dec_s));
                if constexpr (D3Q19::ex[a] != 0) u[0] += D3Q19::ex[a] > 0 ? gvl : -gvl;
                if constexpr (D3Q19::ey[a] != 0) u[1] += D3Q19::ey[a] > 0 ? gvl : -gvl;
                if constexpr (D3Q19::ez[a] != 0) u[2] += D3Q19::ez[a] > 0 ? gvl : -gvl;
            }
        });
        if (pa.friction == LBM_FRICTION_POINTWISE) {
            // Eq. s2-dis1 with u(r) interpolated trilinearly.
#pragma unroll
            for (int k = 0; k < 3; ++k) FH[k] = -pa.gamma * (V[k] - sum8(W * u[k]));
        } else {
            // Eq. s2-slet-v: e^N from the mean relative velocity, least-squares
            // amplitude of the Stokeslet shape, F_H = gamma U^inf e^N.
            double w[3], m[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] = u[k] - V[k];
                m[k] = sum8(w[k]) / 8.0;
            }
            const double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            const bool has_dir = mn > 0.0;
            double eN[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) eN[k] = has_dir ? m[k] / mn : 0.0;
            const double rp = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double num = 0.0, den = 0.0;
            if (rp > 1e-12) {
                const double de = d[0] * eN[0] + d[1] * eN[1] + d[2] * eN[2];
                const double ca = 1.0 - 3.0 * pa.R / (4.0 * rp);
                const double cb = 3.0 * pa.R * de / (4.0 * rp * rp * rp);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double gk = ca * eN[k] - cb * d[k];
                    num += w[k] * gk;
                    den += gk * gk;
                }
            }
            num = sum8(num);
            den = sum8(den);
            if (has_dir && den != 0.0) {
                const double Uinf = num / den;
#pragma unroll
                for (int k = 0; k < 3; ++k) FH[k] = pa.gamma * Uinf * eN[k];
            }
        }
    }
    if (!valid) return;

    // Release this lane's node from the table used one step ago (its entries
    // were consumed by that step's stream-collide).
    const int32_t ps = pa.prev_slot[8 * i + p];
    if (ps >= 0) {
        const uint32_t pc = pa.prev_cell[8 * i + p];
        old.keys[ps] = kEmpty;
        old.vals[3 * ps + 0] = 0;
        old.vals[3 * ps + 1] = 0;
        old.vals[3 * ps + 2] = 0;
        atomicAnd(&old.mask[pc >> 5], ~(1u << (pc & 31)));
    }
    // First Eq. s2-force: the node receives -F_H W_p (unit cell volume).
    int32_t my_slot = -1;
    if (pa.friction != LBM_FRICTION_BD) {
        long long q[3];
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double c = -FH[k] * W;
            ok = ok && (fabs(c) < kFixLimit);
            q[k] = __double2ll_rn(c * kFixScale);
        }
        if (!ok) {
            atomicOr(pa.err, kErrFixRange);
            q[0] = q[1] = q[2] = 0;
        }
        uint32_t slot = hash_slot(cell, cur.shift);
        for (uint32_t probe = 0; probe <= cur.capmask; ++probe) {
            const uint32_t prev = atomicCAS(&cur.keys[slot], kEmpty, cell);
            if (prev == kEmpty || prev == cell) break;
            slot = (slot + 1) & cur.capmask;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            atomicAdd(reinterpret_cast<unsigned long long *>(&cur.vals[3 * slot + k]),
                      static_cast<unsigned long long>(q[k]));
        atomicOr(&cur.mask[cell >> 5], 1u << (cell & 31));
        my_slot = int32_t(slot);
    }
    pa.prev_slot[8 * i + p] = my_slot;
    pa.prev_cell[8 * i + p] = cell;

    if (p != 0) return;
    // Eqs. s2-rf1, s2-rf2: white noise of variance 2 gamma kT per step.
    double FR[3] = {0.0, 0.0, 0.0};
    if (pa.sig > 0.0) {
        double z[3];
        gauss3(pa.seed, pa.step, uint32_t(i), pa.replica, 0u, z);
#pragma unroll
        for (int k = 0; k < 3; ++k) FR[k] = pa.sig * z[k];
    }
    // Eqs. s2-langevin, s2-langevin2 with dt = 1 (F_C = 0).
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vn = V[k] + (FH[k] + FR[k]) / pa.mass;
        pa.v[3 * i + k] = vn;
        pa.r[3 * i + k] = r[k] + vn;
        pa.fh[3 * i + k] = FH[k];
        pa.fr[3 * i + k] = FR[k];
    }
}

// ---------------------------------------------------------------------------
// Velocity autocorrelation, one thread per (origin slot, particle).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_vacf(const double *__restrict__ v, int32_t n,
                                                 int32_t nslot, int32_t stride, int32_t max_lag,
                                                 int64_t t, double *__restrict__ origins,
                                                 double *__restrict__ acc) {
    const int64_t gt = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (gt >= int64_t(n) * nslot) return;
    const int32_t i = int32_t(gt % n);
    const int32_t s = int32_t(gt / n);
    const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
    const int64_t kn = t / stride;
    double *o = origins + (int64_t(s) * n + i) * 3;
    if (t % stride == 0 && s == int32_t(kn % nslot)) {
        o[0] = vx;
        o[1] = vy;
        o[2] = vz;
        acc[int64_t(i) * (max_lag + 1)] += vx * vx + vy * vy + vz * vz;
        return;
    }
    const int64_t back = ((kn - s) % nslot + nslot) % nslot;
    const int64_t k = kn - back;
    if (k < 0) return;
    const int64_t lag = t - k * stride;
    if (lag > max_lag) return;
    acc[int64_t(i) * (max_lag + 1) + lag] += o[0] * vx + o[1] * vy + o[2] * vz;
}

// ---------------------------------------------------------------------------
// Field access kernels (set-up and diagnostics, not on the stepping path).
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(kBlock) void k_get_populations(const typename C::T *__restrict__ A,
                                                            Grid g, typename C::R dec_s,
                                                            double *__restrict__ f) {
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        f[uint64_t(a) * g.ncell + cell] =
            double(C::dec(A[a * g.pstride + nb.src<a>(g)], dec_s)) + D3Q19::w<double>(a);
    });
}

template <class C>
__global__ __launch_bounds__(kBlock) void k_get_moments(const typename C::T *__restrict__ A,
                                                        Grid g, typename C::R dec_s,
                                                        double *__restrict__ rho,
                                                        double *__restrict__ u) {
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    double dr = 0.0, m[3] = {0.0, 0.0, 0.0};
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        const double gvl = double(C::dec(A[a * g.pstride + nb.src<a>(g)], dec_s));
        dr += gvl;
        m[0] += D3Q19::ex[a] * gvl;
        m[1] += D3Q19::ey[a] * gvl;
        m[2] += D3Q19::ez[a] * gvl;
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
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);  // nb.src of the opposite direction is y + e_a
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int o = (a == 0) ? 0 : ((a & 1) ? a + 1 : a - 1);
        const double gvl = f[uint64_t(a) * g.ncell + nb.src<o>(g)] - D3Q19::w<double>(a);
        A[a * g.pstride + cell] = C::enc(typename C::R(gvl), enc_s);
    });
}

template <class C>
__global__ __launch_bounds__(kBlock) void k_set_equilibrium(const double *__restrict__ rho,
                                                            const double *__restrict__ u,
                                                            typename C::T *__restrict__ A, Grid g,
                                                            typename C::R enc_s) {
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= g.ncell) return;
    const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
    const Neighbours nb(x, y, z, g);
    static_for<0, D3Q19::Q>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int o = (a == 0) ? 0 : ((a & 1) ? a + 1 : a - 1);
        const uint32_t src = nb.src<o>(g);  // node y + e_a
        const double dr = rho ? rho[src] - 1.0 : 0.0;
        double uc[3] = {0.0, 0.0, 0.0};
        if (u) {
            uc[0] = u[src];
            uc[1] = u[uint64_t(g.ncell) + src];
            uc[2] = u[2 * uint64_t(g.ncell) + src];
        }
        const double eu = D3Q19::ex[a] * uc[0] + D3Q19::ey[a] * uc[1] + D3Q19::ez[a] * uc[2];
        const double uu = uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2];
        const double geq = D3Q19::w<double>(a) * (dr + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        A[a * g.pstride + cell] = C::enc(typename C::R(geq), enc_s);
    });
}

// FP64 sums of (rho - 1, u) over all nodes: fixed grid, fixed tree order, so the
// result is deterministic.
template <class C>
__global__ __launch_bounds__(kBlock) void k_fluid_partials(const typename C::T *__restrict__ A,
                                                           Grid g, typename C::R dec_s,
                                                           double *__restrict__ partials) {
    __shared__ double sh[4][kBlock];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t cell = blockIdx.x * kBlock + threadIdx.x; cell < g.ncell;
         cell += gridDim.x * kBlock) {
        const uint32_t x = cell % g.nx, t = cell / g.nx, y = t % g.ny, z = t / g.ny;
        const Neighbours nb(x, y, z, g);
        static_for<0, D3Q19::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            const double gvl = double(C::dec(A[a * g.pstride + nb.src<a>(g)], dec_s));
            acc[0] += gvl;
            acc[1] += D3Q19::ex[a] * gvl;
            acc[2] += D3Q19::ey[a] * gvl;
            acc[3] += D3Q19::ez[a] * gvl;
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
    size_t elem;
    void *pop[2];  // pop[cur] holds post-collision values of the last step
    int cur;
    hipStream_t stream;
    double omega;
    double enc_s, dec_s;
    // grid scratch
    uint32_t *mask[2];
    uint32_t mask_words;
    double *partials;
    double *result;
    uint32_t *err;
    // particles
    int32_t np;
    lbm_particle_desc pdesc;
    double R;
    double *r, *v;
    uint32_t *keys[2];
    long long *vals[2];
    uint32_t cap, shift;
    int32_t *prev_slot;
    uint32_t *prev_cell;
    double *fh, *fr;
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

bool grid_ok(const lbm_grid_desc *g) {
    if (!g) return false;
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return false;
    const uint64_t nc = uint64_t(g->nx) * uint64_t(g->ny) * uint64_t(g->nz);
    if (nc >= (uint64_t(1) << 31)) return false;
    if (!(g->tau > 0.5) || !isfinite(g->tau)) return false;
    if (elem_size(g->storage) == 0) return false;
    if (g->storage == LBM_STORE_F16 && (g->f16_scale_log2 < 0 || g->f16_scale_log2 > 24)) return false;
    return true;
}

uint64_t ncell_of(const lbm_grid_desc *g) {
    return uint64_t(g->nx) * uint64_t(g->ny) * uint64_t(g->nz);
}

// Elements between velocity planes: whole 256-byte lines.
uint64_t plane_stride(const lbm_grid_desc *g) {
    const uint64_t per_line = kAlign / elem_size(g->storage);
    return align_up(ncell_of(g), per_line);
}

uint32_t mask_words(uint64_t ncell) { return uint32_t(align_up((ncell + 31) / 32, 64)); }

size_t grid_scratch_size(const lbm_grid_desc *g) {
    const size_t words = mask_words(ncell_of(g));
    size_t s = 0;
    s += 2 * align_up(words * 4, kAlign);            // two bitmasks
    s += align_up(size_t(kRedBlocks) * 4 * 8, kAlign);  // partials
    s += align_up(8 * 8, kAlign);                    // result
    s += kAlign;                                      // error flags
    return s;
}

uint32_t table_cap(int32_t n) {
    uint32_t cap = 64;
    while (cap < uint32_t(16) * uint32_t(n)) cap <<= 1;
    return cap;
}

size_t particle_scratch_size(int32_t n) {
    if (n <= 0) return 0;
    const size_t cap = table_cap(n);
    size_t s = 0;
    s += 2 * align_up(cap * 4, kAlign);        // keys
    s += 2 * align_up(cap * 3 * 8, kAlign);    // values
    s += align_up(size_t(n) * 8 * 4, kAlign);  // prev slot
    s += align_up(size_t(n) * 8 * 4, kAlign);  // prev cell
    s += 2 * align_up(size_t(n) * 3 * 8, kAlign);  // fh, fr
    return s;
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

lbm_status launch_status() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

unsigned blocks_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

ForceTable table(lbm_ctx *c, int par) {
    ForceTable t;
    t.keys = c->np > 0 ? c->keys[par] : nullptr;
    t.vals = c->np > 0 ? c->vals[par] : nullptr;
    t.mask = c->mask[par];
    t.capmask = c->np > 0 ? c->cap - 1 : 0;
    t.shift = c->np > 0 ? c->shift : 31;
    return t;
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
    hipEventRecord(c->prof_ev[2 * k], c->stream);
    return k;
}

void prof_stop(lbm_ctx *c, int32_t k) {
    if (k >= 0) hipEventRecord(c->prof_ev[2 * k + 1], c->stream);
}

template <class C>
void launch_step(lbm_ctx *c) {
    using T = typename C::T;
    using R = typename C::R;
    const T *A = static_cast<const T *>(c->pop[c->cur]);
    T *B = static_cast<T *>(c->pop[c->cur ^ 1]);
    const int par = int(c->step & 1);
    if (c->np > 0) {
        const int32_t pk = prof_start(c, 1);
        if (c->vacf_on) {
            const int64_t work = int64_t(c->np) * c->nslot;
            hipLaunchKernelGGL(k_vacf, dim3(blocks_for(work)), dim3(kBlock), 0, c->stream, c->v,
                               c->np, c->nslot, c->stride, c->max_lag, c->vacf_t, c->origins,
                               c->acc);
            c->vacf_t += 1;
        }
        ParticleArgs pa;
        pa.r = c->r;
        pa.v = c->v;
        pa.fh = c->fh;
        pa.fr = c->fr;
        pa.prev_slot = c->prev_slot;
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
        hipLaunchKernelGGL(k_particle<C>, dim3(blocks_for(uint64_t(c->np) * 8)), dim3(kBlock), 0,
                           c->stream, A, c->g, R(c->dec_s), pa, table(c, par), table(c, par ^ 1));
        prof_stop(c, pk);
        const int32_t ck = prof_start(c, 0);
        hipLaunchKernelGGL((k_stream_collide<C, true>), dim3(blocks_for(c->g.ncell)), dim3(kBlock),
                           0, c->stream, A, B, c->g, R(c->omega), R(c->enc_s), R(c->dec_s),
                           table(c, par));
        prof_stop(c, ck);
    } else {
        const int32_t ck = prof_start(c, 0);
        hipLaunchKernelGGL((k_stream_collide<C, false>), dim3(blocks_for(c->g.ncell)),
                           dim3(kBlock), 0, c->stream, A, B, c->g, R(c->omega), R(c->enc_s),
                           R(c->dec_s), table(c, par));
        prof_stop(c, ck);
    }
    c->cur ^= 1;
    c->step += 1;
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
void launch_partials(lbm_ctx *c) {
    hipLaunchKernelGGL(k_fluid_partials<C>, dim3(kRedBlocks), dim3(kBlock), 0, c->stream,
                       static_cast<const typename C::T *>(c->pop[c->cur]), c->g,
                       typename C::R(c->dec_s), c->partials);
}

#define LBM_DISPATCH(ctx, FN, ...)                                            \
    do {                                                                      \
        switch ((ctx)->desc.storage) {                                        \
            case LBM_STORE_F64: FN<CodecF64>(ctx, ##__VA_ARGS__); break;      \
            case LBM_STORE_F32: FN<CodecF32>(ctx, ##__VA_ARGS__); break;      \
            case LBM_STORE_BF16: FN<CodecBF16>(ctx, ##__VA_ARGS__); break;    \
            case LBM_STORE_F16: FN<CodecF16>(ctx, ##__VA_ARGS__); break;      \
        }                                                                     \
    } while (0)

}  // namespace

extern "C" {

lbm_status lbm_lattice_bytes(const lbm_grid_desc *grid, size_t *bytes) {
    if (!grid_ok(grid) || !bytes) return LBM_E_INVAL;
    *bytes = size_t(plane_stride(grid)) * LBM_Q * elem_size(grid->storage);
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

lbm_status lbm_init(const lbm_grid_desc *grid, void *pop_a, void *pop_b, void *grid_scratch,
                    void *stream, lbm_ctx **out) {
    if (!grid_ok(grid) || !pop_a || !pop_b || !grid_scratch || !out) return LBM_E_INVAL;
    if (!aligned(pop_a) || !aligned(pop_b) || !aligned(grid_scratch) || pop_a == pop_b)
        return LBM_E_INVAL;
    lbm_ctx *c = static_cast<lbm_ctx *>(calloc(1, sizeof(lbm_ctx)));
    if (!c) return LBM_E_DEVICE;
    c->desc = *grid;
    c->g.nx = uint32_t(grid->nx);
    c->g.ny = uint32_t(grid->ny);
    c->g.nz = uint32_t(grid->nz);
    c->g.ncell = uint32_t(ncell_of(grid));
    c->g.pstride = plane_stride(grid);
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
        if (d->friction < LBM_FRICTION_STOKESLET || d->friction > LBM_FRICTION_BD)
            return LBM_E_INVAL;
    }
    // Forced-node state from any previous particle set is cleared.
    hipError_t e = hipMemsetAsync(ctx->mask[0], 0, size_t(ctx->mask_words) * 4, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->mask[1], 0, size_t(ctx->mask_words) * 4, ctx->stream);
    if (e != hipSuccess) return LBM_E_DEVICE;
    ctx->vacf_on = 0;
    ctx->np = d->n;
    ctx->pdesc = *d;
    if (d->n == 0) {
        ctx->R = -1.0;
        return LBM_OK;
    }
    // Stokes' law gamma = 6 pi eta R, eta = rho0 nu, nu = (tau - 1/2)/3.
    const double nu = (ctx->desc.tau - 0.5) / 3.0;
    ctx->R = d->radius > 0.0 ? d->radius : d->gamma / (6.0 * M_PI * nu);
    ctx->r = r;
    ctx->v = v;
    ctx->cap = table_cap(d->n);
    int lg = 0;
    while ((1u << lg) < ctx->cap) ++lg;
    ctx->shift = uint32_t(32 - lg);
    char *s = static_cast<char *>(particle_scratch);
    ctx->keys[0] = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(ctx->cap) * 4, kAlign);
    ctx->keys[1] = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(ctx->cap) * 4, kAlign);
    ctx->vals[0] = reinterpret_cast<long long *>(s);
    s += align_up(size_t(ctx->cap) * 3 * 8, kAlign);
    ctx->vals[1] = reinterpret_cast<long long *>(s);
    s += align_up(size_t(ctx->cap) * 3 * 8, kAlign);
    ctx->prev_slot = reinterpret_cast<int32_t *>(s);
    s += align_up(size_t(d->n) * 8 * 4, kAlign);
    ctx->prev_cell = reinterpret_cast<uint32_t *>(s);
    s += align_up(size_t(d->n) * 8 * 4, kAlign);
    ctx->fh = reinterpret_cast<double *>(s);
    s += align_up(size_t(d->n) * 3 * 8, kAlign);
    ctx->fr = reinterpret_cast<double *>(s);
    // keys -> kEmpty (all ones), prev_slot -> -1 (all ones), the rest zero.
    e = hipMemsetAsync(ctx->keys[0], 0xFF, size_t(ctx->cap) * 4, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->keys[1], 0xFF, size_t(ctx->cap) * 4, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->vals[0], 0, size_t(ctx->cap) * 3 * 8, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->vals[1], 0, size_t(ctx->cap) * 3 * 8, ctx->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->prev_slot, 0xFF, size_t(d->n) * 8 * 4, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->fh, 0, size_t(d->n) * 3 * 8 * 2, ctx->stream);
    return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
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

lbm_status lbm_observables(lbm_ctx *ctx, double out[7]) {
    if (!ctx || !out) return LBM_E_INVAL;
    LBM_DISPATCH(ctx, launch_partials);
    hipLaunchKernelGGL(k_final_sums, dim3(1), dim3(kBlock), 0, ctx->stream, ctx->partials,
                       kRedBlocks, double(ctx->g.ncell), ctx->np > 0 ? ctx->v : nullptr, ctx->np,
                       ctx->np > 0 ? ctx->pdesc.mass : 0.0, ctx->result);
    if (launch_status() != LBM_OK) return LBM_E_DEVICE;
    double host[7];
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(host, ctx->result, sizeof(host), hipMemcpyDeviceToHost,
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

lbm_status lbm_get_step(const lbm_ctx *ctx, int64_t *step) {
    if (!ctx || !step) return LBM_E_INVAL;
    *step = ctx->step;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx *ctx) {
    if (!ctx) return LBM_E_INVAL;
    for (int32_t k = 0; k < 2 * ctx->prof_cap; ++k) hipEventDestroy(ctx->prof_ev[k]);
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
