// Soft repulsion between particles: the conservative force F_C of Eq.
// s2-langevin with the potential of Eq. s2-softpot, read as the conservative
// force of dissipative particle dynamics: a pair closer than the cutoff r_c
// pushes apart with a_f (1 - r/r_c) along the line of centres (nearest
// periodic image).
//
// Neighbours come from a cell list: the box is cut into nc cells per axis of
// edge L/nc >= r_c, one block sorts the keys (cell << 24 | particle) in LDS
// (bitonic network), and every particle walks the (up to) 27 cells around
// its own in a fixed order, each cell's particles in ascending index: the
// sums are bitwise reproducible.  The adjoint kernel uses the same search.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lbmbp {

constexpr int kPairSortThreads = 1024;
constexpr int kPairMax = 8192;  // keys of at most this many particles fit the sort's 64 KB of LDS
constexpr int kPairBlock = 256;

struct PairGrid {
    uint32_t nc[3];  // cells per axis
    double L[3];     // box edges
    double a, rc;    // a_f and the cutoff
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

// One block of kPairSortThreads: keys[0..n) = sorted (cell << 24 | i).
// npad = n rounded up to a power of two (>= 2); dynamic LDS of npad * 8 bytes.
__global__ __launch_bounds__(kPairSortThreads) void k_pair_sort(const double *__restrict__ r,
                                                                int32_t n, int32_t npad,
                                                                PairGrid pg,
                                                                uint64_t *__restrict__ keys) {
    extern __shared__ uint64_t sk[];
    for (int32_t i = threadIdx.x; i < npad; i += kPairSortThreads) {
        uint64_t key = ~uint64_t(0);
        if (i < n) {
            const uint32_t cx = pair_cell_coord(r[3 * i + 0], pg.L[0], pg.nc[0]);
            const uint32_t cy = pair_cell_coord(r[3 * i + 1], pg.L[1], pg.nc[1]);
            const uint32_t cz = pair_cell_coord(r[3 * i + 2], pg.L[2], pg.nc[2]);
            key = (pair_cell(pg, cx, cy, cz) << 24) | uint64_t(i);
        }
        sk[i] = key;
    }
    __syncthreads();
    for (int32_t size = 2; size <= npad; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t t = threadIdx.x; t < npad / 2; t += kPairSortThreads) {
                const int32_t i = 2 * t - (t & (stride - 1));  // stride bit clear
                const int32_t j = i + stride;
                const bool ascending = (i & size) == 0;
                const uint64_t x = sk[i], y = sk[j];
                if ((x > y) == ascending) {
                    sk[i] = y;
                    sk[j] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int32_t i = threadIdx.x; i < n; i += kPairSortThreads) keys[i] = sk[i];
}

// First position in keys[0, n) whose cell is >= cell.
__device__ inline int32_t pair_lower_bound(const uint64_t *__restrict__ keys, int32_t n,
                                           uint64_t cell) {
    const uint64_t target = cell << 24;
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (keys[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Visit every neighbour j != i within the cutoff: fn(j, d) with d = r_i - r_j
// (nearest image) and |d| < r_c.
template <typename Fn>
__device__ inline void pair_neighbours(const double *__restrict__ r, int32_t n, const PairGrid &pg,
                                       const uint64_t *__restrict__ keys, int32_t i, Fn &&fn) {
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
                for (int32_t p = pair_lower_bound(keys, n, cell); p < n && (keys[p] >> 24) == cell;
                     ++p) {
                    const int32_t j = int32_t(keys[p] & 0xFFFFFFu);
                    if (j == i) continue;
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
                                                           PairGrid pg,
                                                           const uint64_t *__restrict__ keys,
                                                           double *__restrict__ F) {
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    double f[3] = {0.0, 0.0, 0.0};
    pair_neighbours(r, n, pg, keys, i, [&](int32_t, const double (&d)[3], double rr) {
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
                                                         PairGrid pg,
                                                         const uint64_t *__restrict__ keys,
                                                         const double *__restrict__ Fb,
                                                         double *__restrict__ rbar) {
    const int32_t i = int32_t(blockIdx.x * kPairBlock + threadIdx.x);
    if (i >= n) return;
    const double fi[3] = {Fb[3 * i + 0], Fb[3 * i + 1], Fb[3 * i + 2]};
    double g[3] = {0.0, 0.0, 0.0};
    pair_neighbours(r, n, pg, keys, i, [&](int32_t j, const double (&d)[3], double rr) {
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
