// Discrete velocity sets of the cubic lattice (c_s^2 = 1/3), lattice units
// dx = dt = 1.  The equilibrium, forcing and viscosity relations (Eqs. s2-eq,
// second s2-force, s2-ident3) hold unchanged for both sets.  Velocity order is
// part of the C ABI (opposites adjacent).
//   D3Q19: rest, +-x, +-y, +-z, then the twelve edge diagonals; weights 1/3,
//          1/18, 1/36.
//   D3Q15: the set section 2.2 uses -- rest, +-x, +-y, +-z, then the eight
//          body diagonals (+-1, +-1, +-1); weights 2/9, 1/9, 1/72.
#pragma once

namespace lbmbp {

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int ex[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    // weight class: 0 rest (1/3), 1 axis (1/18), 2 diagonal (1/36)
    static constexpr int wclass[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};

    template <typename R>
    __host__ __device__ static constexpr R w(int a) {
        return wclass[a] == 0 ? R(1) / R(3) : (wclass[a] == 1 ? R(1) / R(18) : R(1) / R(36));
    }
};

struct D3Q15 {
    static constexpr int Q = 15;
    static constexpr int ex[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int ey[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
    // weight class: 0 rest (2/9), 1 axis (1/9), 2 body diagonal (1/72)
    static constexpr int wclass[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2};

    template <typename R>
    __host__ __device__ static constexpr R w(int a) {
        return wclass[a] == 0 ? R(2) / R(9) : (wclass[a] == 1 ? R(1) / R(9) : R(1) / R(72));
    }
};

// A storage codec together with the velocity set of the lattice it stores.
template <class Codec, class Vel>
struct Cfg : Codec {
    using V = Vel;
};

}  // namespace lbmbp
