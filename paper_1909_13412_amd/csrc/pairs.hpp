// Soft repulsion between particles: the conservative force F_C of Eq.
// s2-langevin with the potential of Eq. s2-softpot, read as the conservative
// force of dissipative particle dynamics: a pair closer than the cutoff r_c
// pushes apart with a_f (1 - r/r_c) along the line of centres (nearest
// periodic image).
//
// Neighbours come from a cell list: the box is cut into nc cells per axis
// of edge L/nc >= r_c and the cells are hashed into T buckets (T a power of
// two >= 2n).  Four short passes build it: count the particles of every
// bucket, scan the counts into bucket offsets, scatter the particle indices,
// and sort each bucket by particle index.  Every particle then walks the (up
// to) 27 cells around its own in a fixed order, each cell's particles in
// ascending index (entries of other cells hashed to the same bucket are
// skipped); the 27 cells go to 27 lanes and their sums are combined in a
// fixed order: the result is bitwise reproducible.  The adjoint kernel uses
// the same walk.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lbmbp {

constexpr int kPairScanThreads = 1024;
constexpr int kPairMax = 65536;  // particles the single-block bucket scan is sized for
constexpr int kPairBlock = 256;

struct PairGrid {
    uint32_t nc[3];  // cells per axis
    uint32_t T;      // buckets (power of two)
    double L[3];     // box edges
    double a, rc;    // a_f and the cutoff
};

// The cell list: particles grouped by bucket, ascending index within one.
struct PairList {
    uint64_t *cell;    // [n] cell of each particle
    uint32_t *bucket;  // [n] its bucket
    uint32_t *slot;    // [n] its arrival slot in the bucket
    uint32_t *count;   // [T] particles per bucket (kept zero between builds)
    uint32_t *start;   // [T + 1] bucket offsets into list
    uint32_t *list;    // [n] particle indices
};

__device__ inline uint32_t pair_cell_coord(double r, double L, uint32_t nc) {
    const double s = r - L * floor(r / L);  // wrapped position
    int32_t c = int32_t(floor(s * double(nc) / L));
    c = c < 0 ? 0 : (c >= int32_t(nc) ? int32_t(nc) - 1 : c);
    return uint32_t(c);
}

__device__ inline uint64_t pair_cell(const PairGrid &pg, uint32_t cx, uint32_t cy, uint32_t cz) {
    return (uint64_t(cz) * pg.nc[1] + cy) * pg.nc[0] + cx;
}

// Fibonacci hashing of the cell index into the T buckets.
__device__ inline uint32_t pair_bucket(uint64_t cell, uint32_t T) {
    return uint32_t((cell * 0x9E3779B97F4A7C15ull) >> 32) & (T - 1u);
}

__global__ __launch_bounds__(kPairBlock) void k_pair_count(const double *__restrict__ r, int32_t n,
                                                           PairGrid pg, PairList pl) {
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    const uint32_t cx = pair_cell_coord(r[3 * i + 0], pg.L[0], pg.nc[0]);
    const uint32_t cy = pair_cell_coord(r[3 * i + 1], pg.L[1], pg.nc[1]);
    const uint32_t cz = pair_cell_coord(r[3 * i + 2], pg.L[2], pg.nc[2]);
    const uint64_t cell = pair_cell(pg, cx, cy, cz);
    const uint32_t b = pair_bucket(cell, pg.T);
    pl.cell[i] = cell;
    pl.bucket[i] = b;
    pl.slot[i] = atomicAdd(&pl.count[b], 1u);
}

// Sum of the counts of buckets [b0, b0 + per) (per a power of two; groups of
// four as 16-byte loads, four loads in flight at a time).
__device__ inline uint32_t pair_count_sum(const uint32_t *__restrict__ count, uint32_t b0, uint32_t per) {
    if (per < 4) {
        uint32_t s = 0;
        for (uint32_t k = 0; k < per; ++k) s += count[b0 + k];
        return s;
    }
    const uint4 *c4 = reinterpret_cast<const uint4 *>(count + b0);
    const uint32_t nv = per / 4;
    uint32_t s = 0;
    for (uint32_t k = 0; k < nv; k += 4) {
        uint4 v[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) v[u] = k + u < nv ? c4[k + u] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    return s;
}

// One block: start = exclusive scan of count (start[T] = n); the counts are
// cleared for the next build.  Each thread owns T/1024 consecutive buckets
// (one when T <= 1024); the per-thread totals are scanned within each
// wavefront by shuffles, then across the sixteen wavefronts.
__global__ __launch_bounds__(kPairScanThreads) void k_pair_scan(PairGrid pg, PairList pl) {
    constexpr int kWaves = kPairScanThreads / 64;
    __shared__ uint32_t wsum[kWaves];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t per = pg.T / kPairScanThreads > 0 ? pg.T / kPairScanThreads : 1u;
    const uint32_t b0 = threadIdx.x * per;
    const bool mine = b0 < pg.T;
    const uint32_t local = mine ? pair_count_sum(pl.count, b0, per) : 0u;
    uint32_t x = local;  // inclusive scan within the wavefront
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= uint32_t(off)) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
        uint32_t w = lane < uint32_t(kWaves) ? wsum[lane] : 0u;
        for (int off = 1; off < kWaves; off <<= 1) {
            const uint32_t y = __shfl_up(w, off, 64);
            if (lane >= uint32_t(off)) w += y;
        }
        if (lane < uint32_t(kWaves)) wsum[lane] = w;
    }
    __syncthreads();
    if (mine) {
        uint32_t run = x - local + (wave > 0 ? wsum[wave - 1] : 0u);
        if (per < 4) {
            for (uint32_t k = 0; k < per; ++k) {
                const uint32_t c = pl.count[b0 + k];
                pl.start[b0 + k] = run;
                pl.count[b0 + k] = 0u;
                run += c;
            }
        } else {
            uint4 *c4 = reinterpret_cast<uint4 *>(pl.count + b0);
            uint4 *s4 = reinterpret_cast<uint4 *>(pl.start + b0);
            const uint32_t nv = per / 4;
            for (uint32_t k = 0; k < nv; k += 4) {
                uint4 v[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) v[u] = k + u < nv ? c4[k + u] : make_uint4(0, 0, 0, 0);
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    if (k + u >= nv) break;
                    uint4 o;
                    o.x = run;
                    o.y = o.x + v[u].x;
                    o.z = o.y + v[u].y;
                    o.w = o.z + v[u].z;
                    run = o.w + v[u].w;
                    s4[k + u] = o;
                    c4[k + u] = make_uint4(0, 0, 0, 0);
                }
            }
        }
    }
    if (threadIdx.x == kPairScanThreads - 1) pl.start[pg.T] = wsum[kWaves - 1];
}

__global__ __launch_bounds__(kPairBlock) void k_pair_scatter(int32_t n, PairList pl) {
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    pl.list[pl.start[pl.bucket[i]] + pl.slot[i]] = uint32_t(i);
}

// Each bucket's entries into ascending particle order (insertion sort; a
// bucket holds ~0.5 particles on average).
__global__ __launch_bounds__(kPairBlock) void k_pair_bucket_sort(PairGrid pg, PairList pl) {
    const uint32_t b = blockIdx.x * kPairBlock + threadIdx.x;
    if (b >= pg.T) return;
    const uint32_t lo = pl.start[b], hi = pl.start[b + 1];
    for (uint32_t p = lo + 1; p < hi; ++p) {
        const uint32_t v = pl.list[p];
        uint32_t q = p;
        while (q > lo && pl.list[q - 1] > v) {
            pl.list[q] = pl.list[q - 1];
            --q;
        }
        pl.list[q] = v;
    }
}

// A group of kPairLanes lanes serves one particle: lane l visits the l-th of
// its (up to) 27 neighbour cells (offsets in x fastest, then y, z) and calls
// fn(j, d, |d|^2) for every particle j != i of that cell within the cutoff,
// d = r_i - r_j at the nearest image, in ascending j.
constexpr int kPairLanes = 32;

template <typename Fn>
__device__ inline void pair_cell_visit(const double *__restrict__ r, const PairGrid &pg,
                                       const PairList &pl, int32_t i, uint32_t l, Fn &&fn) {
    const double ri[3] = {r[3 * i + 0], r[3 * i + 1], r[3 * i + 2]};
    const uint32_t o[3] = {l % 3u, (l / 3u) % 3u, l / 9u};
    uint32_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // one, two or three distinct cells per axis
        const uint32_t cnt = pg.nc[k] >= 3 ? 3u : pg.nc[k];
        if (o[k] >= cnt) return;
        const uint32_t c = pair_cell_coord(ri[k], pg.L[k], pg.nc[k]);
        q[k] = pg.nc[k] >= 3 ? (c + o[k] + pg.nc[k] - 1u) % pg.nc[k] : (c + o[k]) % pg.nc[k];
    }
    const double rc2 = pg.rc * pg.rc;
    const uint64_t cell = pair_cell(pg, q[0], q[1], q[2]);
    const uint32_t b = pair_bucket(cell, pg.T);
    const uint32_t hi = pl.start[b + 1];
    for (uint32_t p = pl.start[b]; p < hi; ++p) {
        const int32_t j = int32_t(pl.list[p]);
        if (j == i || pl.cell[j] != cell) continue;
        double d[3], rr = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            d[k] = ri[k] - r[3 * j + k];
            d[k] -= pg.L[k] * rint(d[k] / pg.L[k]);
            rr += d[k] * d[k];
        }
        if (rr > 0.0 && rr < rc2) fn(j, d, rr);
    }
}

// Sum of v over the kPairLanes lanes of a group, in a fixed butterfly order
// (every lane receives it).
__device__ inline double pair_group_sum(double v) {
#pragma unroll
    for (int m = kPairLanes / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kPairLanes);
    return v;
}

// F[i] = sum over neighbours of a_f (1 - |d|/r_c) d/|d|.
__global__ __launch_bounds__(kPairBlock) void k_pair_force(const double *__restrict__ r, int32_t n,
                                                           PairGrid pg, PairList pl,
                                                           double *__restrict__ F) {
    const int32_t i = int32_t((blockIdx.x * kPairBlock + threadIdx.x) / kPairLanes);
    const uint32_t l = threadIdx.x % kPairLanes;
    if (i >= n) return;  // whole groups leave together
    double f[3] = {0.0, 0.0, 0.0};
    if (l < 27)
        pair_cell_visit(r, pg, pl, i, l, [&](int32_t, const double (&d)[3], double rr) {
            const double dist = sqrt(rr);
            const double mag = pg.a * (1.0 - dist / pg.rc) / dist;
#pragma unroll
            for (int k = 0; k < 3; ++k) f[k] += mag * d[k];
        });
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = pair_group_sum(f[k]);
    if (l == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) F[3 * i + k] = f[k];
}

// Adjoint: with Fb = dJ/dF_C of every particle, rbar[i] += sum over
// neighbours of Jac(d) (Fb[i] - Fb[j]), Jac(d) = a_f [(1/|d| - 1/r_c) I -
// d d^T / |d|^3] (the force of a pair is odd in d, its Jacobian even and
// symmetric).
__global__ __launch_bounds__(kPairBlock) void k_adj_pair(const double *__restrict__ r, int32_t n,
                                                         PairGrid pg, PairList pl,
                                                         const double *__restrict__ Fb,
                                                         double *__restrict__ rbar) {
    const int32_t i = int32_t((blockIdx.x * kPairBlock + threadIdx.x) / kPairLanes);
    const uint32_t l = threadIdx.x % kPairLanes;
    if (i >= n) return;
    const double fi[3] = {Fb[3 * i + 0], Fb[3 * i + 1], Fb[3 * i + 2]};
    double g[3] = {0.0, 0.0, 0.0};
    if (l < 27)
        pair_cell_visit(r, pg, pl, i, l, [&](int32_t j, const double (&d)[3], double rr) {
            const double dist = sqrt(rr);
            const double diag = pg.a * (1.0 / dist - 1.0 / pg.rc);
            const double outer = pg.a / (rr * dist);
            double w[3], dw = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] = fi[k] - Fb[3 * j + k];
                dw += d[k] * w[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) g[k] += diag * w[k] - outer * d[k] * dw;
        });
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = pair_group_sum(g[k]);
    if (l == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) rbar[3 * i + k] += g[k];
}

}  // namespace lbmbp
