"""Pins of the closed-form references in analytic.py against facts that do not
depend on the formula's derivation: its Laplace transform computed by
quadrature, the limit without history force, the long-time amplitude and the
initial value; and of the VACF under noise on the particle alone against the
closed autocovariances of first- and second-order autoregressions."""
import math

import numpy as np
from scipy.integrate import quad

from analytic import particle_noise_vacf, tail_amplitude, velocity_relaxation

CASES = [  # (M, gamma, R, nu): complex roots, real roots, the paper's Fig. 2 point
    (16.0, 6 * math.pi * 0.0178 * 1.0, 1.0, 0.0178),
    (0.2, 1.0, 0.8, 0.1),
    (2.0, 0.17, 0.5, 0.0178),
]


def test_initial_value_is_one():
    for M, g, R, nu in CASES:
        assert abs(velocity_relaxation(0.0, M, g, R, nu) - 1.0) < 1e-14


def test_laplace_transform_by_quadrature():
    # int_0^inf phi(t) exp(-s t) dt = M / (M s + b sqrt(s) + gamma)
    for M, g, R, nu in CASES:
        b = 6.0 * math.pi * R * R * math.sqrt(nu)
        for s in (0.01, 0.1, 1.0):
            val, err = quad(lambda t: velocity_relaxation(t, M, g, R, nu) * math.exp(-s * t),
                            0.0, np.inf, limit=400)
            ref = M / (M * s + b * math.sqrt(s) + g)
            assert abs(val / ref - 1.0) < 1e-7, (M, g, R, nu, s, val, ref)


def test_no_history_force_is_exponential():
    t = np.linspace(0.0, 200.0, 41)
    phi = velocity_relaxation(t, 10.0, 0.3, 1e-9, 0.1)
    assert np.allclose(phi, np.exp(-0.03 * t), rtol=1e-7, atol=1e-12)


def test_long_time_tail_amplitude():
    for M, g, R, nu in CASES:
        B = tail_amplitude(M, g, R, nu)
        t = 1e9
        assert abs(velocity_relaxation(t, M, g, R, nu) * t**1.5 / B - 1.0) < 1e-3
    # under Stokes' law (the first case) B = M / [12 rho (pi nu)^(3/2)]
    M, g, R, nu = CASES[0]
    assert abs(tail_amplitude(M, g, R, nu) * 12.0 * (math.pi * nu) ** 1.5 / M - 1.0) < 1e-12


def _isotropic(phi1):
    """[1, 3, J + 1, 3] response: a kick along axis d moves only component d."""
    phi = np.zeros((1, 3, phi1.size, 3))
    for d in range(3):
        phi[0, d, :, d] = phi1
    return phi


def test_particle_noise_vacf_first_order():
    # Brownian dynamics: V' = (1 - gamma/M) V + F/M is an AR(1) process whose
    # stationary variance per component is s2 / (1 - a^2), s2 = 2 gamma kT / M^2,
    # and whose autocorrelation is a^t: M <V^2> / kT = 6 M / (2 M - gamma).
    M, g, kT = 10.0, 1.0, 1e-4
    a = 1.0 - g / M
    C = particle_noise_vacf(_isotropic(a ** np.arange(4000)), g, M, kT, 30)
    assert abs(M * C[0] / kT - 6.0 * M / (2.0 * M - g)) < 1e-12
    assert np.allclose(C / C[0], a ** np.arange(31), rtol=1e-12, atol=0.0)


def test_particle_noise_vacf_second_order():
    # x_n = a1 x_(n-1) + a2 x_(n-2) + e_n (a response that is not one
    # exponential): Yule-Walker gives rho_1 = a1 / (1 - a2),
    # rho_k = a1 rho_(k-1) + a2 rho_(k-2) and
    # var = s2 (1 - a2) / [(1 + a2) ((1 - a2)^2 - a1^2)].
    M, g, kT = 4.0, 0.7, 2e-3
    s2 = 2.0 * g * kT / (M * M)
    for a1, a2 in ((1.2, -0.5), (0.5, 0.3), (-0.4, 0.2)):
        phi1 = np.zeros(6000)
        phi1[0], phi1[1] = 1.0, a1
        for j in range(2, phi1.size):
            phi1[j] = a1 * phi1[j - 1] + a2 * phi1[j - 2]
        C = particle_noise_vacf(_isotropic(phi1), g, M, kT, 20)
        var = s2 * (1.0 - a2) / ((1.0 + a2) * ((1.0 - a2) ** 2 - a1 * a1))
        rho = [1.0, a1 / (1.0 - a2)]
        for k in range(2, 21):
            rho.append(a1 * rho[-1] + a2 * rho[-2])
        assert abs(C[0] / (3.0 * var) - 1.0) < 1e-12, (a1, a2)
        assert np.allclose(C / C[0], rho, rtol=0.0, atol=1e-12), (a1, a2)
        # and the regression relation C / C(0) = phi fails for it
        assert np.max(np.abs(C / C[0] - phi1[:21])) > 0.05
