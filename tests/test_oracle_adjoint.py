"""Pins of the reference derivatives in oracle/adjoint.py.

* its float forward reproduces the C oracle's steps (so it differentiates the
  same map);
* its complex-step directional derivative matches central finite differences
  of the C oracle (an independent evaluation of the same derivative);
* its reverse sweep satisfies <vjp(c), d> = <c, jvp(d)> for random c, d;
* closed forms: Brownian-dynamics friction decouples the particles
  (V^N = (1 - gamma/M)^N V^0 at kT = 0), and mass and total momentum are
  conserved by the coupled step, which fixes the gradients of those
  functionals exactly.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as A

E, W = oracle.lattice()


def _setup(L=8, n=3, seed=1, tau=0.8, amp=0.02, q=19):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal((L, L, L))
    u = amp * rng.standard_normal((3, L, L, L))
    o = oracle.Sim(L, L, L, tau, q=q)
    o.set_equilibrium(rho, u)
    f0 = o.populations()
    r0 = rng.uniform(0.0, L, (n, 3))
    v0 = 0.01 * rng.standard_normal((n, 3))
    return rng, f0, r0, v0


def _oracle_run(f0, r0, v0, theta, nsteps, friction, radius=0.0, seed=5, fc=None):
    gamma, tau, M, kT = theta
    L = f0.shape[1]
    o = oracle.Sim(L, L, L, tau, q=f0.shape[0])
    o.set_populations(f0)
    o.set_particles(r0, v0, mass=M, gamma=gamma, kT=kT, radius=radius, seed=seed,
                    friction=friction)
    if fc is not None:
        o.set_particle_force(fc)
    o.step(nsteps)
    r, v = o.particles()
    return o.populations(), r, v


@pytest.mark.parametrize("friction,kT,radius,force", [("stokeslet", 1e-4, 0.0, False),
                                                      ("stokeslet", 0.0, 0.4, True),
                                                      ("pointwise", 1e-4, 0.0, False),
                                                      ("bd", 1e-4, 0.0, True),
                                                      ("stokeslet2dx", 1e-4, 1.2, False)])
def test_forward_matches_c_oracle(friction, kT, radius, force):
    _, f0, r0, v0 = _setup()
    theta = np.array([1.0, 0.8, 10.0, kT])
    N = 8
    fc = np.array([[1e-3, 0.0, -5e-4], [0.0, 2e-3, 0.0], [1e-4, 1e-4, 1e-4]]) if force else None
    fr, rr, vr = _oracle_run(f0, r0, v0, theta, N, friction, radius, fc=fc)
    f, r, v = A.run(f0, r0, v0, theta, A.noise(3, N, 5), friction, radius, fc=fc)
    assert np.max(np.abs(f - fr)) < 1e-14
    assert np.max(np.abs(r - rr)) < 1e-13
    assert np.max(np.abs(v - vr)) < 1e-15


@pytest.mark.parametrize("friction", ["stokeslet", "stokeslet2dx"])
def test_fifteen_velocities_forward_and_transpose(friction):
    rng, f0, r0, v0 = _setup(seed=8, q=15)
    theta = np.array([1.0, 0.8, 10.0, 1e-4])
    N = 6
    fr, rr, vr = _oracle_run(f0, r0, v0, theta, N, friction, 1.0)
    xi = A.noise(3, N, 5)
    f, r, v = A.run(f0, r0, v0, theta, xi, friction, 1.0)
    assert f.shape[0] == 15
    assert np.max(np.abs(f - fr)) < 1e-14 and np.max(np.abs(v - vr)) < 1e-15
    cf = rng.standard_normal(f0.shape)
    cr = rng.standard_normal(r0.shape)
    cv = rng.standard_normal(v0.shape)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, xi, cf, cr, cv, friction, 1.0)
    df = rng.standard_normal(f0.shape)
    dr = rng.standard_normal(r0.shape)
    dv = rng.standard_normal(v0.shape)
    dth = rng.standard_normal(4)
    jf, jr, jv = A.jvp(f0, r0, v0, theta, xi, df, dr, dv, dth, friction, 1.0)
    lhs = (gf * df).sum() + (gr * dr).sum() + (gv * dv).sum() + (gth * dth).sum()
    rhs = (cf * jf).sum() + (cr * jr).sum() + (cv * jv).sum()
    assert abs(lhs - rhs) < 1e-11 * (abs(rhs) + 1.0)


def test_forward_with_body_force_matches_c_oracle():
    _, f0, r0, v0 = _setup(seed=7)
    theta = np.array([1.0, 0.8, 10.0, 1e-4])
    G = np.array([2e-5, -1e-5, 4e-6])
    L = f0.shape[1]
    o = oracle.Sim(L, L, L, theta[1])
    o.set_populations(f0)
    o.set_particles(r0, v0, mass=10.0, gamma=1.0, kT=1e-4, seed=5)
    o.set_body_force(np.broadcast_to(G.reshape(3, 1, 1, 1), (3, L, L, L)).copy())
    o.step(6)
    f, r, v = A.run(f0, r0, v0, theta, A.noise(3, 6, 5), body=G)
    assert np.max(np.abs(f - o.populations())) < 1e-14
    assert np.max(np.abs(v - o.particles()[1])) < 1e-15


@pytest.mark.parametrize("friction", ["stokeslet", "pointwise", "bd", "stokeslet2dx"])
def test_complex_step_matches_finite_differences_of_c_oracle(friction):
    rng, f0, r0, v0 = _setup(seed=2)
    theta = np.array([1.0, 0.8, 10.0, 1e-4])
    N = 6
    cf = rng.standard_normal(f0.shape)
    cr = rng.standard_normal(r0.shape)
    cv = rng.standard_normal(v0.shape)
    df = 1e-3 * rng.standard_normal(f0.shape)
    dr = 0.1 * rng.standard_normal(r0.shape)
    dv = 0.01 * rng.standard_normal(v0.shape)
    dth = np.array([0.3, 0.1, 2.0, 1e-4])
    jf, jr, jv = A.jvp(f0, r0, v0, theta, A.noise(3, N, 5), df, dr, dv, dth, friction)
    dj = (cf * jf).sum() + (cr * jr).sum() + (cv * jv).sum()

    def J(h):
        f, r, v = _oracle_run(f0 + h * df, r0 + h * dr, v0 + h * dv, theta + h * dth, N, friction)
        return (cf * f).sum() + (cr * r).sum() + (cv * v).sum()

    h = 1e-5
    fd = (J(h) - J(-h)) / (2 * h)
    assert abs(fd - dj) < 1e-7 * abs(dj)
    # a plausible slip (a parameter left out) would be far outside that band
    jf2, jr2, jv2 = A.jvp(f0, r0, v0, theta, A.noise(3, N, 5), df, dr, dv, dth * [1, 0, 1, 1],
                          friction)
    dj2 = (cf * jf2).sum() + (cr * jr2).sum() + (cv * jv2).sum()
    assert abs(dj2 - dj) > 1e-4 * abs(dj)


@pytest.mark.parametrize("friction,kT,radius,force", [("stokeslet", 1e-4, 0.0, False),
                                                      ("stokeslet", 0.0, 0.4, True),
                                                      ("pointwise", 1e-4, 0.0, False),
                                                      ("bd", 1e-4, 0.0, True),
                                                      ("stokeslet2dx", 1e-4, 1.2, True)])
def test_reverse_sweep_is_the_transpose_of_the_complex_step(friction, kT, radius, force):
    rng, f0, r0, v0 = _setup(seed=3)
    theta = np.array([1.0, 0.8, 10.0, kT])
    N = 7
    xi = A.noise(3, N, 5)
    cf = rng.standard_normal(f0.shape)
    cr = rng.standard_normal(r0.shape)
    cv = rng.standard_normal(v0.shape)
    fc = 1e-3 * rng.standard_normal(r0.shape) if force else None
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, xi, cf, cr, cv, friction, radius, fc=fc)
    for trial in range(2):
        df = rng.standard_normal(f0.shape)
        dr = rng.standard_normal(r0.shape)
        dv = rng.standard_normal(v0.shape)
        dth = rng.standard_normal(4)
        if kT == 0.0:
            dth[3] = 0.0
        jf, jr, jv = A.jvp(f0, r0, v0, theta, xi, df, dr, dv, dth, friction, radius, fc=fc)
        lhs = (gf * df).sum() + (gr * dr).sum() + (gv * dv).sum() + (gth * dth).sum()
        rhs = (cf * jf).sum() + (cr * jr).sum() + (cv * jv).sum()
        assert abs(lhs - rhs) < 1e-11 * (abs(rhs) + 1.0)


def test_brownian_dynamics_closed_form():
    rng, f0, r0, v0 = _setup(seed=4)
    gamma, M, N = 1.0, 10.0, 9
    theta = np.array([gamma, 0.8, M, 0.0])
    a = 1.0 - gamma / M
    cv = rng.standard_normal(v0.shape)
    cr = rng.standard_normal(r0.shape)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, A.noise(3, N, 5), 0 * f0, cr, cv, "bd")
    # V^N = a^N V^0, r^N = r^0 + V^0 sum_{k=1..N} a^k
    S = sum(a ** k for k in range(1, N + 1))
    dS = sum(k * a ** (k - 1) for k in range(1, N + 1))  # dS/da
    assert np.allclose(gv, a ** N * cv + S * cr, rtol=1e-13, atol=0)
    assert np.allclose(gr, cr, rtol=1e-15, atol=0)
    assert np.max(np.abs(gf)) == 0.0
    dJ_da = N * a ** (N - 1) * (cv * v0).sum() + dS * (cr * v0).sum()
    assert gth[0] == pytest.approx(dJ_da * (-1.0 / M), rel=1e-12)
    assert gth[2] == pytest.approx(dJ_da * (gamma / M ** 2), rel=1e-12)
    assert gth[1] == 0.0 and gth[3] == 0.0


def test_mass_and_momentum_gradients_are_exact():
    _, f0, r0, v0 = _setup(seed=5, n=4)
    M = 10.0
    theta = np.array([1.0, 0.8, M, 0.0])
    N = 6
    xi = A.noise(4, N, 5)
    # J = total mass: dJ/df0 = 1, nothing else
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, xi, np.ones_like(f0), 0 * r0, 0 * v0)
    assert np.max(np.abs(gf - 1.0)) < 1e-13
    assert np.max(np.abs(gr)) < 1e-13 and np.max(np.abs(gv)) < 1e-13
    assert np.max(np.abs(gth)) < 1e-11
    # J = total x momentum (fluid + M V) at kT = 0: conserved by the step
    cf = np.broadcast_to(E[:, 0].reshape(19, 1, 1, 1), f0.shape).astype(float)
    cv = np.zeros_like(v0)
    cv[:, 0] = M
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, xi, cf, 0 * r0, cv)
    _, _, vN = A.run(f0, r0, v0, theta, xi)
    assert np.max(np.abs(gf - cf)) < 1e-12
    assert np.max(np.abs(gv - cv)) < 1e-11
    assert np.max(np.abs(gr)) < 1e-11
    assert abs(gth[0]) < 1e-11 and abs(gth[1]) < 1e-11
    assert gth[2] == pytest.approx(v0[:, 0].sum() - vN[:, 0].sum(), abs=1e-12)


def test_pair_force_forward_and_transpose():
    # The soft pair repulsion couples the particles through their positions.
    rng, f0, r0, v0 = _setup(seed=9, n=5)
    r0 = 3.0 + rng.uniform(0, 1.2, (5, 3))  # close enough to interact
    theta = np.array([1.0, 0.8, 10.0, 1e-4])
    N, pair = 6, (0.02, 1.0)
    L = f0.shape[1]
    o = oracle.Sim(L, L, L, theta[1])
    o.set_populations(f0)
    o.set_particles(r0, v0, mass=10.0, gamma=1.0, kT=1e-4, seed=5)
    o.set_pair_force(*pair)
    o.step(N)
    xi = A.noise(5, N, 5)
    f, r, v = A.run(f0, r0, v0, theta, xi, pair=pair)
    assert np.max(np.abs(o.pair_forces())) > 0.0
    assert np.max(np.abs(f - o.populations())) < 1e-14
    assert np.max(np.abs(v - o.particles()[1])) < 1e-15
    cf = rng.standard_normal(f0.shape)
    cr = rng.standard_normal(r0.shape)
    cv = rng.standard_normal(v0.shape)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, theta, xi, cf, cr, cv, pair=pair)
    df = rng.standard_normal(f0.shape)
    dr = rng.standard_normal(r0.shape)
    dv = rng.standard_normal(v0.shape)
    dth = rng.standard_normal(4)
    jf, jr, jv = A.jvp(f0, r0, v0, theta, xi, df, dr, dv, dth, pair=pair)
    lhs = (gf * df).sum() + (gr * dr).sum() + (gv * dv).sum() + (gth * dth).sum()
    rhs = (cf * jf).sum() + (cr * jr).sum() + (cv * jv).sum()
    assert abs(lhs - rhs) < 1e-11 * (abs(rhs) + 1.0)
    # and the pair term matters: dropping it changes the position gradient
    gf2, gr2, gv2, _ = A.vjp(f0, r0, v0, theta, xi, cf, cr, cv)
    assert np.max(np.abs(gr2 - gr)) > 1e-6 * np.max(np.abs(gr))
