// Fused pull stream-collide of the BGK lattice with sparse node forcing
// (section 2.2: Eqs. s2-lbe, s2-collision, s2-eq, s2-coll, s2-trans and the
// second Eq. s2-force), and the data layout it streams.
//
// Layout: the lattice rows (y, z) are taken Y at a time (Y = 1, 2, 4, ..., 64,
// a divisor of ny: rows y with the same y / Y and z form a group); a group
// stores, for each population a in turn, its Y rows one after another, x
// fastest.  Element (a, x, y, z) sits at
// ((z*ny + Y*(y/Y))*Q + (y mod Y))*chunk + a*Y*chunk + x with chunk = nx (no
// padding).  A block streams whole rows, so each wave reads from nine row
// groups and writes into one; with Y > 1 a population's rows of a group are
// one run of Y*nx elements, so the pulls of consecutive rows continue the same
// runs (fewer, longer streams).  Y = 1 puts the 19 population rows of each
// lattice row back to back; one plane per velocity (38 far-apart streams) is
// slower than either.  Y is a property of the context, chosen by the
// autotuner (same bits in every layout).
// Lattice A holds post-collision values at their source node, so the
// post-streaming population is read by pulling from x - e_a.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "codec.hpp"
#include "velocities.hpp"

namespace lbmbp {

constexpr int kBlock = 256;
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
    uint32_t chunk;    // elements per population row (nx)
    uint32_t ymask;    // rows per group minus one (Y - 1; Y a power of two dividing ny)
    uint32_t pstride;  // elements from one population of a node to the next (Y * chunk)
};

// A Grid with Y rows per group (Y a power of two that divides ny).
__host__ __device__ inline Grid with_rows_per_group(Grid g, uint32_t Y) {
    g.ymask = Y - 1u;
    g.pstride = Y * g.chunk;
    return g;
}

// Storage index of population 0 of node (0, y, z): the start of its group
// plus its row within the group.  I is the index arithmetic's type: 32 bits
// suffice (and save the sweep its 64-bit multiplies) while Q nx ny nz < 2^32.
template <class V, class I = uint64_t>
__device__ inline I row_index(const Grid &g, uint32_t y, uint32_t z) {
    return (I(z * g.ny + (y & ~g.ymask)) * V::Q + (y & g.ymask)) * g.chunk;
}

// Storage index of population a at node (x, y, z) for velocity set V.
template <class V, class I = uint64_t>
__device__ inline I pop_index(const Grid &g, uint32_t x, uint32_t y, uint32_t z, int a) {
    return row_index<V, I>(g, y, z) + I(a) * g.pstride + x;
}

// Addressing of the sweep's loads and stores.
//   kAddrLane32, kAddrLane64: every lane decodes its own node and computes each
//     element index itself, in 32 bits (lattices below 2^32 elements) or 64.
//   kAddrRow: every wavefront lies in one lattice row (nx a multiple of 64, or
//     the row-aligned mapping), so y and z are the same in all its lanes: the
//     base addresses of the nine source rows and of the node's own row are
//     computed once per wavefront in scalar registers, and an access adds only
//     the lane's 32-bit byte offset (x, x + 1 or x - 1, plus the population's
//     offset).  Any lattice size.
constexpr int kAddrLane32 = 0;
constexpr int kAddrLane64 = 1;
constexpr int kAddrRow = 2;

// Index type of the per-lane modes.
template <int ADDR>
using SweepIndex = typename std::conditional<ADDR == kAddrLane64, uint64_t, uint32_t>::type;

// Lane byte offset plus a population's offset, added in the vector unit: left
// to itself the compiler folds the (wavefront-uniform) population offset into
// a 64-bit scalar address per access, two scalar instructions each.
__device__ inline uint32_t lane_offset(uint32_t xo, uint32_t pop_bytes) {
    uint32_t r;
    asm("v_add_u32 %0, %1, %2" : "=v"(r) : "s"(pop_bytes), "v"(xo));
    return r;
}

// Rows of one wavefront in the kAddrRow mode: the byte offsets of row y and of
// its neighbours y -/+ 1 (periodic) within a z-plane, of plane z and its
// neighbours, and the lane's byte offsets of x - e_x.  Every member but xo is
// the same in all lanes of the wavefront.
struct RowOffsets {
    uint64_t yb[3], zb[3];  // index e + 1: coordinate - e
    uint32_t xo[3];
    __device__ inline RowOffsets(uint32_t x, uint32_t y, uint32_t z, const Grid &g, uint32_t q,
                                 uint32_t elem) {
        const uint32_t ys[3] = {y + 1 == g.ny ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
        const uint32_t zs[3] = {z + 1 == g.nz ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
        const uint64_t row_bytes = uint64_t(g.chunk) * elem;
        const uint64_t plane_bytes = uint64_t(g.ny) * q * row_bytes;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // row_index(y, z) = z ny Q chunk + ((y & ~ymask) Q + (y & ymask)) chunk
            yb[k] = uint64_t((ys[k] & ~g.ymask) * q + (ys[k] & g.ymask)) * row_bytes;
            zb[k] = uint64_t(zs[k]) * plane_bytes;
        }
        xo[0] = (x + 1 == g.nx ? 0u : x + 1) * elem;
        xo[1] = x * elem;
        xo[2] = (x == 0 ? g.nx - 1 : x - 1) * elem;
    }
    // population a of the node (x, y, z) - e_a, pulled
    template <class V, int a, class T>
    __device__ inline const T *pull(const T *A, uint32_t pop_bytes) const {
        const char *row = reinterpret_cast<const char *>(A) + (zb[V::ez[a] + 1] + yb[V::ey[a] + 1]);
        const uint32_t off = a == 0 ? xo[V::ex[a] + 1] : lane_offset(xo[V::ex[a] + 1], uint32_t(a) * pop_bytes);
        return reinterpret_cast<const T *>(row + off);
    }
    // population a of the node (x, y, z) + e_a, the streaming target
    template <class V, int a, class T>
    __device__ inline const T *push(const T *A, uint32_t pop_bytes) const {
        const char *row = reinterpret_cast<const char *>(A) + (zb[1 - V::ez[a]] + yb[1 - V::ey[a]]);
        const uint32_t off = a == 0 ? xo[1 - V::ex[a]] : lane_offset(xo[1 - V::ex[a]], uint32_t(a) * pop_bytes);
        return reinterpret_cast<const T *>(row + off);
    }
    // population a of the node (x, y, z) itself
    template <class T>
    __device__ inline T *own(T *B, int a, uint32_t pop_bytes) const {
        char *row = reinterpret_cast<char *>(B) + (zb[1] + yb[1]);
        const uint32_t off = a == 0 ? xo[1] : lane_offset(xo[1], uint32_t(a) * pop_bytes);
        return reinterpret_cast<T *>(row + off);
    }
};

// The node coordinates of a lane: x, the first band's row y0 and the plane z
// of lane_cell (< ncell / CPT; rows = ny / CPT rows per band).  In the kAddrRow
// mode the row is decoded from the wavefront's first node (lane_cell minus the
// lane index is the same in every lane: blocks and rows start at whole
// wavefronts), so y0 and z are wavefront-uniform.
template <int ADDR>
__device__ inline void lane_coords(const Grid &g, uint32_t lane_cell, uint32_t rows, uint32_t &x,
                                   uint32_t &y0, uint32_t &z) {
    if constexpr (ADDR == kAddrRow) {
        const uint32_t first = __builtin_amdgcn_readfirstlane(lane_cell - (threadIdx.x & 63u));
        const uint32_t t = first / g.nx;
        x = lane_cell - t * g.nx;
        y0 = t % rows;
        z = t / rows;
    } else {
        x = lane_cell % g.nx;
        const uint32_t t = lane_cell / g.nx;
        y0 = t % rows;
        z = t / rows;
    }
}

// Node forces of one step: a dense fixed-point field, written only at the
// (at most 8 per particle) nodes that receive a reaction force and read only
// where the one-bit flag is set, so the stream-collide pays 1/8 byte per node.
// Two of them alternate between steps; each is cleared node by node by the
// particles that wrote it.
struct ForceField {
    long long *f;    // [ncell][3] fixed-point force
    uint32_t *mask;  // one bit per node: node carries a force this step
};

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
    // linear node index of x - e_a (canonical [z][y][x] order)
    template <class V, int a>
    __device__ inline uint32_t src(const Grid &g) const {
        return (sz[V::ez[a] + 1] * g.ny + sy[V::ey[a] + 1]) * g.nx + sx[V::ex[a] + 1];
    }
    // storage index of population a at x - e_a
    template <class V, int a, class I = uint64_t>
    __device__ inline I pop(const Grid &g) const {
        return pop_index<V, I>(g, sx[V::ex[a] + 1], sy[V::ey[a] + 1], sz[V::ez[a] + 1], a);
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
//
// Each lane updates CPT nodes with the same x in rows y, y + ny/CPT, ...: all
// 19 x CPT population loads (and the forcing flags) are issued before any of
// them is consumed, which keeps more bytes in flight per wave.  BS lanes per
// block.  Lattice A -> B; F is the node-force field of this step.
// ---------------------------------------------------------------------------
// Deterministic block sum of N doubles (fixed butterfly and wave order);
// thread k < N writes out[k].  Every thread of the block must call it.
// Sums of four doubles over the lanes of one wavefront, written to out[0..3].
// Every lane of the wavefront must call it.  A reduce-scatter butterfly: at
// offset 32 each lane keeps two of the four values (the half its partner
// does not) and receives the partner's copy of them, at offset 16 it keeps
// one, and offsets 8..1 sum that one; seven FP64 exchanges instead of 24 for
// four full butterflies.  Each addition pairs the same two partials as the
// full butterfly over offsets 32, 16, ..., 1 (a + b = b + a exactly), so the
// sums are those of that order bit for bit.  Lanes 0, 16, 32, 48 hold sums 0,
// 1, 2, 3 and write them.
__device__ inline void wave_sum4(const double (&v)[4], double *__restrict__ out) {
    const uint32_t lane = threadIdx.x & 63u;
    const bool h32 = (lane & 32u) != 0;
    double k0 = h32 ? v[2] : v[0];
    double k1 = h32 ? v[3] : v[1];
    const double s0 = h32 ? v[0] : v[2];
    const double s1 = h32 ? v[1] : v[3];
    k0 += __shfl_xor(s0, 32);
    k1 += __shfl_xor(s1, 32);
    const bool h16 = (lane & 16u) != 0;
    double k = h16 ? k1 : k0;
    k += __shfl_xor(h16 ? k0 : k1, 16);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) k += __shfl_xor(k, off);
    if ((lane & 15u) == 0) out[lane >> 4] = k;
}

template <int N, int BS>
__device__ inline void block_sum(double (&v)[N], double *__restrict__ out) {
    __shared__ double sh[BS / 64][N];
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) sh[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int w = 0; w < BS / 64; ++w) s += sh[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// The nodes of one lane: lane_cell < ncell / CPT indexes the first band of
// ny/CPT rows; the lane also takes the same (x, z) in the CPT - 1 bands below.
// With MOMENTS the FP64 sums of (rho~ - 1, u) over these nodes are added to acc.
// The force at a node is the uniform body force G plus, where the node is
// flagged (FORCED), the particles' reaction force.
// NTS: write the populations with non-temporal stores (streamed past the
// caches); pays off once the lattice no longer fits in the last-level cache.
template <class C, bool FORCED, bool MOMENTS, int CPT, bool NTS, int ADDR = kAddrLane32>
__device__ inline void collide_lane(const typename C::T *__restrict__ A,
                                    typename C::T *__restrict__ B, const Grid &g,
                                    typename C::R omega, typename C::R enc_s, typename C::R dec_s,
                                    const ForceField &ff, typename C::R Gx, typename C::R Gy,
                                    typename C::R Gz, uint32_t lane_cell, double (&acc)[4]) {
    // Multiply-adds fuse only within one expression: fusion across statements
    // depends on how the compiler lays out the blocks, which differs between
    // launch configurations, and every configuration must round each node the
    // same way.
#pragma clang fp contract(on)
    using T = typename C::T;
    using R = typename C::R;
    using V = typename C::V;
    using I = SweepIndex<ADDR>;
    const uint32_t rows = g.ny / CPT;
    uint32_t x, y0, z;
    lane_coords<ADDR>(g, lane_cell, rows, x, y0, z);
    const uint32_t pop_bytes = g.pstride * uint32_t(sizeof(T));

    T raw[CPT][V::Q];
    uint32_t flags[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const uint32_t y = y0 + uint32_t(c) * rows;
        if constexpr (ADDR == kAddrRow) {
            const RowOffsets ro(x, y, z, g, V::Q, sizeof(T));
            static_for<0, V::Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                raw[c][a] = *ro.template pull<V, a>(A, pop_bytes);
            });
        } else {
            const Neighbours nb(x, y, z, g);
            static_for<0, V::Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                raw[c][a] = A[nb.template pop<V, a, I>(g)];
            });
        }
        if constexpr (FORCED) {
            const uint32_t cell = (z * g.ny + y) * g.nx + x;
            flags[c] = (ff.mask[cell >> 5] >> (cell & 31)) & 1u;
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const uint32_t y = y0 + uint32_t(c) * rows;
        R gv[V::Q];
        static_for<0, V::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            gv[a] = C::dec(raw[c][a], dec_s);
        });
        R drho = R(0), ux = R(0), uy = R(0), uz = R(0);
        static_for<0, V::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            drho += gv[a];
            if constexpr (V::ex[a] != 0) ux += V::ex[a] > 0 ? gv[a] : -gv[a];
            if constexpr (V::ey[a] != 0) uy += V::ey[a] > 0 ? gv[a] : -gv[a];
            if constexpr (V::ez[a] != 0) uz += V::ez[a] > 0 ? gv[a] : -gv[a];
        });
        const R uu = ux * ux + uy * uy + uz * uz;
        if constexpr (MOMENTS) {
            acc[0] += double(drho);
            acc[1] += double(ux);
            acc[2] += double(uy);
            acc[3] += double(uz);
        }
        R Fx = Gx, Fy = Gy, Fz = Gz;
        if constexpr (FORCED) {
            if (flags[c]) {
                const uint64_t cell = (z * g.ny + y) * g.nx + x;
                Fx += R(double(ff.f[3 * cell + 0]) * kFixInv);
                Fy += R(double(ff.f[3 * cell + 1]) * kFixInv);
                Fz += R(double(ff.f[3 * cell + 2]) * kFixInv);
            }
        }
        // written once and read only by the next step
        [[maybe_unused]] const RowOffsets ro(x, y, z, g, V::Q, sizeof(T));  // kAddrRow only
        auto put = [&](int a, R gn) {
            T *p;
            if constexpr (ADDR == kAddrRow)
                p = ro.own(B, a, pop_bytes);
            else
                p = &B[row_index<V, I>(g, y, z) + x + I(a) * g.pstride];
            if constexpr (NTS)
                __builtin_nontemporal_store(C::enc(gn, enc_s), p);
            else
                *p = C::enc(gn, enc_s);
        };
        // BGK relaxation to the equilibrium of Eq. s2-eq plus the forcing term
        // 3 w e.F, one opposite pair (a, a + 1) at a time: e_{a+1} = -e_a, so
        // the even part of the equilibrium, w (drho + 4.5 (e.u)^2 - 1.5 u.u),
        // is shared, and its odd part 3 w e.u and the forcing change sign.
        const R base = drho - R(1.5) * uu;
        put(0, gv[0] + omega * (V::template w<R>(0) * base - gv[0]));
        static_for<0, (V::Q - 1) / 2>([&](auto pc) {
            constexpr int a = 1 + 2 * decltype(pc)::value;
            constexpr int cx = V::ex[a], cy = V::ey[a], cz = V::ez[a];
            static_assert(V::ex[a + 1] == -cx && V::ey[a + 1] == -cy && V::ez[a + 1] == -cz,
                          "opposite velocities are adjacent");
            constexpr R w = V::template w<R>(a);
            constexpr R w3 = R(3) * w;
            R eu = R(0), eF = R(0);
            if constexpr (cx != 0) eu += cx > 0 ? ux : -ux;
            if constexpr (cy != 0) eu += cy > 0 ? uy : -uy;
            if constexpr (cz != 0) eu += cz > 0 ? uz : -uz;
            if constexpr (cx != 0) eF += cx > 0 ? Fx : -Fx;
            if constexpr (cy != 0) eF += cy > 0 ? Fy : -Fy;
            if constexpr (cz != 0) eF += cz > 0 ? Fz : -Fz;
            const R sym = w * (base + R(4.5) * eu * eu);
            const R anti = w3 * eu;
            const R fa = w3 * eF;
            put(a, gv[a] + omega * ((sym + anti) - gv[a]) + fa);
            put(a + 1, gv[a + 1] + omega * ((sym - anti) - gv[a + 1]) - fa);
        });
    }
}

// Lanes per row of the row-aligned mapping: nx rounded up to whole wavefronts.
__host__ __device__ inline uint32_t row_lanes(uint32_t nx) { return (nx + 63u) & ~63u; }

// Block orders of the sweep.  The hardware hands consecutive workgroups to
// the eight XCDs in turn (workgroup b to XCD b mod 8).  Order 0 maps block b
// to the b-th block of nodes, so every XCD works across the whole front of
// the sweep; order 1 gives XCD k the k-th contiguous eighth of the blocks (a
// slab of z-planes), so the eight XCDs sweep eight separate regions at once.
// Both are permutations of the blocks (the last gridDim.x mod 8 blocks keep
// their place), so the nodes updated and the results are the same.
constexpr uint32_t kOrderLinear = 0;
constexpr uint32_t kOrderXcdSlabs = 1;
constexpr uint32_t kNumOrders = 2;
constexpr uint32_t kXcds = 8;

__device__ inline uint32_t sweep_block(uint32_t order) {
    const uint32_t b = blockIdx.x;
    if (order != kOrderXcdSlabs) return b;
    const uint32_t per = gridDim.x / kXcds;
    return b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
}

// The node of this lane (in the first row band when CPT = 2); false for lanes
// without one.  ROW: lanes map to whole rows (every row starts a wavefront: a
// block of BS lanes holds BS / row_lanes rows, or a row spans several blocks),
// so no wave straddles two rows when nx is not a multiple of 64; otherwise
// lanes map to consecutive nodes (rows y and y + ny/CPT for CPT = 2).
template <int CPT, int BS, bool ROW>
__device__ inline bool lane_node(const Grid &g, uint32_t blk, uint32_t &lane_cell) {
    if constexpr (ROW) {
        static_assert(CPT == 1, "the row-aligned mapping takes one node per lane");
        const uint32_t lpr = row_lanes(g.nx);
        uint32_t row, x;
        bool in_rows = true;  // lanes past the block's last whole row stay idle
        if (lpr <= uint32_t(BS)) {
            const uint32_t rpb = uint32_t(BS) / lpr;  // rows per block
            const uint32_t slot = threadIdx.x / lpr;
            in_rows = slot < rpb;
            row = blk * rpb + slot;
            x = threadIdx.x % lpr;
        } else {
            const uint32_t bpr = (lpr + BS - 1) / BS;  // blocks per row
            row = blk / bpr;
            x = (blk % bpr) * BS + threadIdx.x;
        }
        lane_cell = row * g.nx + x;
        return in_rows && x < g.nx && row < g.ny * g.nz;
    } else {
        lane_cell = blk * BS + threadIdx.x;
        return lane_cell < g.ncell / CPT;
    }
}

template <class C, bool FORCED, bool MOMENTS, int CPT, int BS, bool NTS, bool ROW, int ADDR>
__global__ __launch_bounds__(BS) void k_stream_collide(const typename C::T *__restrict__ A,
                                                       typename C::T *__restrict__ B, Grid g,
                                                       typename C::R omega, typename C::R enc_s,
                                                       typename C::R dec_s, ForceField ff,
                                                       typename C::R Gx, typename C::R Gy,
                                                       typename C::R Gz, double *__restrict__ mom,
                                                       uint32_t order) {
    const uint32_t blk = sweep_block(order);
    uint32_t lane_cell;
    const bool active = lane_node<CPT, BS, ROW>(g, blk, lane_cell);
    if constexpr (!MOMENTS) {
        if (!active) return;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (active)
        collide_lane<C, FORCED, MOMENTS, CPT, NTS, ADDR>(A, B, g, omega, enc_s, dec_s, ff, Gx, Gy,
                                                         Gz, lane_cell, acc);
    // partials by wavefront of the node block (no barrier), so that every
    // block order gives the same sums
    if constexpr (MOMENTS)
        wave_sum4(acc, mom + 4 * (uint64_t(blk) * (BS / 64) + threadIdx.x / 64));
}

// The stream-collide's data movement alone, for the nodes of one lane (as in
// collide_lane): every population is pulled from x - e_a and stored
// unchanged at x (no moments, collision or forcing), with the same layout and
// store policy.  Its duration bounds what the stream-collide can reach with
// this access pattern; B does not hold a lattice update.
template <class C, int CPT, bool NTS, int ADDR = kAddrLane32>
__device__ inline void stream_only_lane(const typename C::T *__restrict__ A,
                                        typename C::T *__restrict__ B, const Grid &g,
                                        uint32_t lane_cell) {
    using T = typename C::T;
    using V = typename C::V;
    using I = SweepIndex<ADDR>;
    const uint32_t rows = g.ny / CPT;
    uint32_t x, y0, z;
    lane_coords<ADDR>(g, lane_cell, rows, x, y0, z);
    const uint32_t pop_bytes = g.pstride * uint32_t(sizeof(T));
    T raw[CPT][V::Q];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const uint32_t y = y0 + uint32_t(c) * rows;
        if constexpr (ADDR == kAddrRow) {
            const RowOffsets ro(x, y, z, g, V::Q, sizeof(T));
            static_for<0, V::Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                raw[c][a] = *ro.template pull<V, a>(A, pop_bytes);
            });
        } else {
            const Neighbours nb(x, y, z, g);
            static_for<0, V::Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                raw[c][a] = A[nb.template pop<V, a, I>(g)];
            });
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const uint32_t y = y0 + uint32_t(c) * rows;
        [[maybe_unused]] const RowOffsets ro(x, y, z, g, V::Q, sizeof(T));  // kAddrRow only
        static_for<0, V::Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            T *p;
            if constexpr (ADDR == kAddrRow)
                p = ro.own(B, a, pop_bytes);
            else
                p = &B[row_index<V, I>(g, y, z) + x + I(a) * g.pstride];
            if constexpr (NTS)
                __builtin_nontemporal_store(raw[c][a], p);
            else
                *p = raw[c][a];
        });
    }
}

// Streaming-only counterpart of k_stream_collide in configuration <CPT, BS,
// NTS, ROW> (same lanes).
template <class C, int CPT, int BS, bool NTS, bool ROW, int ADDR>
__global__ __launch_bounds__(BS) void k_stream_only(const typename C::T *__restrict__ A,
                                                    typename C::T *__restrict__ B, Grid g,
                                                    uint32_t order) {
    uint32_t lane_cell;
    if (!lane_node<CPT, BS, ROW>(g, sweep_block(order), lane_cell)) return;
    stream_only_lane<C, CPT, NTS, ADDR>(A, B, g, lane_cell);
}

// Launch configurations of the stream-collide, chosen per context
// (lbm_autotune): configurations 0-7 map lanes to consecutive nodes with the
// geometric shape kShapes[k & 3], non-temporal stores when k >= 4;
// configurations 8 and 9 use the row-aligned mapping (one node per lane,
// 256-lane blocks) with plain and non-temporal stores.  Ensembles use 0-7.
struct CollideShape {
    int cpt, bs;
};
constexpr CollideShape kShapes[] = {{1, 512}, {1, 256}, {2, 512}, {2, 256}};
constexpr int kNumGeomShapes = 4;
constexpr int kNumFlatShapes = 2 * kNumGeomShapes;
constexpr int kNumShapes = kNumFlatShapes + 2;
constexpr int kRowBlock = 256;
constexpr bool config_row(int k) { return k >= kNumFlatShapes; }
// Lanes per block of configuration k.
constexpr int config_block(int k) { return config_row(k) ? kRowBlock : kShapes[k & 3].bs; }
// Lattices of at least this many bytes default to non-temporal stores.
constexpr size_t kStreamStoreBytes = size_t(256) << 20;

// Residency caps of the sweep, in waves per SIMD (0: none, the kernel's own
// limit).  A cap is imposed by reserving LDS the kernel never touches, so
// that only cap * 256 / BS blocks fit on a compute unit; fewer concurrent
// blocks means fewer concurrent row streams per memory channel.
constexpr int kResidencyCaps[] = {0, 6, 5, 4, 3, 2};
constexpr int kNumCaps = 6;

}  // namespace lbmbp
