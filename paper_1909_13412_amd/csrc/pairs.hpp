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
// skipped): the sums are bitwise reproducible.  The adjoint kernel uses the
// same walk.
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

// One block: start = exclusive scan of count (start[T] = n); the counts are
// cleared for the next build.
__global__ __launch_bounds__(kPairScanThreads) void k_pair_scan(PairGrid pg, PairList pl) {
    __shared__ uint32_t part[kPairScanThreads];
    const uint32_t per = pg.T / kPairScanThreads > 0 ? pg.T / kPairScanThreads : 1u;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < pg.T) local += pl.count[b0 + k];
    part[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < kPairScanThreads; off <<= 1) {  // inclusive scan of the partials
        const uint32_t v = threadIdx.x >= uint32_t(off) ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - local;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < pg.T) {
            pl.start[b0 + k] = run;
            run += pl.count[b0 + k];
            pl.count[b0 + k] = 0u;
        }
    if (threadIdx.x == kPairScanThreads - 1) pl.start[pg.T] = part[threadIdx.x];
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

// Visit every neighbour j != i within the cutoff: fn(j, d) with d = r_i - r_j
// (nearest image) and |d| < r_c.
template <typename Fn>
__device__ inline void pair_neighbours(const double *__restrict__ r, const PairGrid &pg,
                                       const PairList &pl, int32_t i, Fn &&fn) {
    const double ri[3] = {r[3 * i + 0], r[3 * i + 1], r[3 * i + 2]};
    uint32_t c[3];
    int32_t lo[3], cnt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c[k] = pair_cell_coord(ri[k], pg.L[k], pg.nc[k]);
        // one, two or three distinct cells per axis
        cnt[k] = pg.nc[k] >= 3 ? 3 : int32_t(pg.nc[k]);
        lo[k] = pg.nc[k] >= 3 ? -1 : 0;
    }
    const double rc2 = pg.rc * pg.rc;
    for (int32_t oz = 0; oz < cnt[2]; ++oz)
        for (int32_t oy = 0; oy < cnt[1]; ++oy)
            for (int32_t ox = 0; ox < cnt[0]; ++ox) {
                const int32_t o[3] = {lo[0] + ox, lo[1] + oy, lo[2] + oz};
                uint32_t q[3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    q[k] = uint32_t((int32_t(c[k]) + o[k] + int32_t(pg.nc[k])) % int32_t(pg.nc[k]));
                const uint64_t cell = pair_cell(pg, q[0], q[1], q[2]);
                const uint32_t b = pair_bucket(cell, pg.T);
                for (uint32_t p = pl.start[b]; p < pl.start[b + 1]; ++p) {
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
}

// F[i] = sum over neighbours of a_f (1 - |d|/r_c) d/|d|.
__global__ __launch_bounds__(kPairBlock) void k_pair_force(const double *__restrict__ r, int32_t n,
                                                           PairGrid pg, PairList pl,
                                                           double *__restrict__ F) {
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    double f[3] = {0.0, 0.0, 0.0};
    pair_neighbours(r, pg, pl, i, [&](int32_t, const double (&d)[3], double rr) {
        const double dist = sqrt(rr);
        const double mag = pg.a * (1.0 - dist / pg.rc) / dist;
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k] += mag * d[k];
    });
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
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    const double fi[3] = {Fb[3 * i + 0], Fb[3 * i + 1], Fb[3 * i + 2]};
    double g[3] = {0.0, 0.0, 0.0};
    pair_neighbours(r, pg, pl, i, [&](int32_t j, const double (&d)[3], double rr) {
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
    for (int k = 0; k < 3; ++k) rbar[3 * i + k] += g[k];
}

}  // namespace lbmbp
