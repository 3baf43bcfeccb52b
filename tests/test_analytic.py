"""Pins of the closed-form references in analytic.py against facts that do not
depend on the formula's derivation: its Laplace transform computed by
quadrature, the limit without history force, the long-time amplitude and the
initial value."""
import math

import numpy as np
from scipy.integrate import quad

from analytic import tail_amplitude, velocity_relaxation

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
