// Counter-based random numbers for the Brownian force (Eqs. s2-rf1, s2-rf2).
// Philox4x32-10 as defined by Salmon, Moraes, Dror & Shaw ("Parallel random
// numbers: as easy as 1, 2, 3", SC'11): a ten-round Feistel-like bijection of a
// 128-bit counter under a 64-bit key, two 32x32->64 multiplies per round, key
// bumped by the golden-ratio and sqrt(3)-derived Weyl increments.  Gaussians by
// the Box-Muller transform (Box & Muller, 1958).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmbp {

struct Philox4x32 {
    uint32_t v[4];
};

__device__ inline Philox4x32 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t hiA = __umulhi(MA, c0), loA = MA * c0;
        const uint32_t hiB = __umulhi(MB, c2), loB = MB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += WA;
        k1 += WB;
    }
    return Philox4x32{{c0, c1, c2, c3}};
}

// Maps a 32-bit word to the open unit interval: (x + 1/2) 2^-32.
__device__ inline double unit_open(uint32_t x) {
    return (double(x) + 0.5) * 2.3283064365386962890625e-10;
}

// One Box-Muller output from two words: sqrt(-2 ln u_a) times cos(2 pi u_b)
// (or sin when `sine`), the same numbers gauss3 produces.
__device__ inline void box_muller_one(uint32_t wa, uint32_t wb, bool sine, double *z) {
    constexpr double two_pi = 6.283185307179586476925286766559;
    const double rad = sqrt(-2.0 * log(unit_open(wa)));
    double sn, cs;
    sincos(two_pi * unit_open(wb), &sn, &cs);
    *z = rad * (sine ? sn : cs);
}

// Three standard normals for (step, particle, replica, stream) under `seed`.
// Words map to the open unit interval as (x + 1/2) 2^-32; (u0, u1) give two
// normals, (u2, u3) the third.
__device__ inline void gauss3(uint64_t seed, uint32_t step, uint32_t particle, uint32_t replica,
                              uint32_t stream, double z[3]) {
    const Philox4x32 x = philox4x32_10(step, particle, replica, stream, uint32_t(seed),
                                       uint32_t(seed >> 32));
    constexpr double twopow32inv = 2.3283064365386962890625e-10;
    constexpr double two_pi = 6.283185307179586476925286766559;
    const double u0 = (double(x.v[0]) + 0.5) * twopow32inv;
    const double u1 = (double(x.v[1]) + 0.5) * twopow32inv;
    const double u2 = (double(x.v[2]) + 0.5) * twopow32inv;
    const double u3 = (double(x.v[3]) + 0.5) * twopow32inv;
    const double a = sqrt(-2.0 * log(u0));
    const double b = sqrt(-2.0 * log(u2));
    z[0] = a * cos(two_pi * u1);
    z[1] = a * sin(two_pi * u1);
    z[2] = b * cos(two_pi * u3);
}

}  // namespace lbmbp
