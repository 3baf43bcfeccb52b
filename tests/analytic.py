"""Closed-form references for the validation tests (section 3), independent of
both the oracle and the GPU path.

Velocity relaxation of a point particle of mass M with Stokes friction gamma and
the Basset history force of a sphere of radius R in a fluid of density rho and
kinematic viscosity nu (the hydrodynamic memory behind the long-time tail the
paper compares against in Fig. 2; Hinch, J. Fluid Mech. 72, 1975; Paul & Pusey,
J. Phys. A 14, 1981).  No added mass: the coupled particles are points.

The particle starts at rest in a fluid at rest and receives an impulse M V0 at
t = 0; the history force -6 R^2 sqrt(pi rho eta) int V'(s') / sqrt(t - s') ds'
then sees the whole jump, its transform is -b sqrt(s) V(s), and

    V(s) / V0 = M / (M s + b sqrt(s) + gamma),    b = 6 pi R^2 sqrt(rho eta).

With x1, x2 the roots of M x^2 + b x + gamma = 0 (complex for small b) the
partial fractions in sqrt(s) invert term by term,
L^-1[1 / (sqrt(s) - x)] = 1 / sqrt(pi t) + x exp(x^2 t) erfc(-x sqrt(t)):

    phi(t) = [x1 E(x1, t) - x2 E(x2, t)] / (x1 - x2),  E(x, t) = exp(x^2 t) erfc(-x sqrt t),

with E(x, t) = w(-i x sqrt t) in terms of the Faddeeva function w.  Near s = 0
the transform is (M/gamma)(1 - (b/gamma) sqrt(s) + ...), so for large t
phi ~ B t^(-3/2) with B = M b / (2 sqrt(pi) gamma^2); under Stokes' law
gamma = 6 pi eta R that is M / [12 rho (pi nu)^(3/2)], the amplitude the paper
quotes.  For b -> 0, phi -> exp(-gamma t / M).
"""
import math

import numpy as np
from scipy.special import wofz


def basset_b(R: float, nu: float, rho: float = 1.0) -> float:
    """History-force coefficient b = 6 pi R^2 sqrt(rho eta), eta = rho nu."""
    return 6.0 * math.pi * R * R * math.sqrt(rho * rho * nu)


def velocity_relaxation(t, M: float, gamma: float, R: float, nu: float, rho: float = 1.0):
    """phi(t) = V(t) / V(0) after a kick, for t >= 0 (array or scalar)."""
    b = basset_b(R, nu, rho)
    disc = np.sqrt(complex(b * b - 4.0 * M * gamma))
    x1 = (-b + disc) / (2.0 * M)
    x2 = (-b - disc) / (2.0 * M)
    st = np.sqrt(np.asarray(t, dtype=np.float64))

    def E(x):
        return wofz(-1j * x * st)

    return ((x1 * E(x1) - x2 * E(x2)) / (x1 - x2)).real


def tail_amplitude(M: float, gamma: float, R: float, nu: float, rho: float = 1.0) -> float:
    """B of phi ~ B t^(-3/2): M b / (2 sqrt(pi) gamma^2)."""
    return M * basset_b(R, nu, rho) / (2.0 * math.sqrt(math.pi) * gamma * gamma)


def particle_noise_vacf(phi, gamma: float, M: float, kT: float, lags: int):
    """Stationary VACF of a particle whose random force acts on it alone
    (Eqs. s2-rf1, s2-rf2: independent normals of variance 2 gamma kT per
    component and step, nothing acting on the fluid), for a coupled system
    that responds linearly.

    phi[p, d, j, c] is component c of the particle velocity j steps after a
    kick of unit velocity along axis d, with the fluid at rest before the
    kick, measured at the particle position p (p indexes positions over which
    the result is averaged).  The random force F^k of step k changes V^(k+1)
    by F^k / M (Eq. s2-langevin), so by superposition
    V^n = sum_k phi(n - 1 - k) F^k / M, and with independent F^k

        C(t) = sum_c <V_c^n V_c^(n+t)> = (2 gamma kT / M^2) sum_{j,d,c} phi_cd(j) phi_cd(j + t).

    Only when phi is a single exponential (Brownian dynamics) is this
    proportional to phi itself; the fluctuation-dissipation form
    C(t) = (kT / M) phi(t) needs random stresses in the fluid as well.
    Returns C(t) for t = 0..lags, averaged over p; the sums run over the
    recorded lags j + t <= J."""
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim != 4 or phi.shape[1] != 3 or phi.shape[3] != 3:
        raise ValueError("phi must be [positions, 3 kick axes, J + 1 lags, 3 components]")
    J1 = phi.shape[2]
    C = np.empty(lags + 1)
    for t in range(lags + 1):
        C[t] = np.sum(phi[:, :, : J1 - t, :] * phi[:, :, t:, :]) / phi.shape[0]
    return 2.0 * gamma * kT / (M * M) * C
