// Nineteen-velocity cubic lattice (c_s^2 = 1/3), lattice units dx = dt = 1.
// The paper uses the fifteen-velocity member of the same family (section 2.2);
// the equilibrium, forcing and viscosity relations (Eqs. s2-eq, second s2-force,
// s2-ident3) hold unchanged for this set.  Velocity order is part of the C ABI
// (opposites adjacent): rest, +-x, +-y, +-z, then the twelve edge diagonals.
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

}  // namespace lbmbp
