"""GPU reverse mode (lbm_record / lbm_adjoint through the C ABI) against the
oracle's derivatives, plus exact identities and finite differences at the
64^3 / 16-particle / 2000-step size.

Tolerances: FP64 storage is the exact-arithmetic map up to rounding, so the
gradients agree with the oracle's complex-step reverse sweep to 1e-10 of their
largest entry.  FP32 storage linearises the same map along the FP32 trajectory,
which departs from the FP64 one by about 1e-7 per step relative; the bound used
for it (2e-4) is that drift carried through the reverse sweep, with margin.
"""
import numpy as np
import pytest

from helpers import announce, nmax_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


BOX = (12, 10, 9)  # nx, ny, nz: unequal sides catch axis mix-ups


def _case(oracle_mod, seed, n=5, tau=0.8, box=BOX, amp=0.02, q=19):
    rng = np.random.default_rng(seed)
    nx, ny, nz = box
    o = oracle_mod.Sim(nx, ny, nz, tau, q=q)
    o.set_equilibrium(1.0 + 0.01 * rng.standard_normal((nz, ny, nx)),
                      amp * rng.standard_normal((3, nz, ny, nx)))
    f0 = o.populations()
    r0 = rng.uniform(0.0, 1.0, (n, 3)) * np.array([nx, ny, nz])
    v0 = 0.01 * rng.standard_normal((n, 3))
    cf = rng.standard_normal(f0.shape)
    cr = rng.standard_normal((n, 3))
    cv = rng.standard_normal((n, 3))
    return f0, r0, v0, cf, cr, cv


def _gpu_grad(storage, f0, r0, v0, theta, cf, cr, cv, nsteps, every, friction, radius, seed,
              box=BOX):
    from paper_1909_13412_amd import Lattice

    gamma, tau, M, kT = theta
    nx, ny, nz = box
    lat = Lattice(nx, ny, nz, tau, storage=storage, velocities=f0.shape[0])
    lat.set_populations(f0)
    lat.particles_couple(r0, v0, mass=M, gamma=gamma, kT=kT, radius=radius, seed=seed,
                         friction=friction)
    tape = lat.record(nsteps, every)
    g = lat.adjoint(tape, cf, cr, cv)
    return lat, tape, {k: t.cpu().numpy() for k, t in g.items()}


CASES = [("stokeslet", 1e-4, 0.0), ("stokeslet", 0.0, 0.4), ("pointwise", 1e-4, 0.0),
         ("bd", 1e-4, 0.0), ("stokeslet2dx", 1e-4, 1.2)]


@pytest.mark.parametrize("friction,kT,radius", CASES)
def test_adjoint_f64_matches_oracle(oracle_mod, friction, kT, radius):
    from oracle import adjoint as A

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 11)
    theta = (1.0, 0.8, 10.0, kT)
    N, every, seed = 23, 5, 31  # segments 5, 5, 5, 5, 3
    announce(f"adjoint f64 {friction} kT={kT} R={radius} box={BOX} N={N} every={every}")
    _, _, g = _gpu_grad("f64", f0, r0, v0, theta, cf, cr, cv, N, every, friction, radius, seed)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, np.array(theta), A.noise(len(r0), N, seed), cf, cr, cv,
                            friction, radius)
    errs = (nmax_err(g["pop"], gf), nmax_err(g["r"], gr), nmax_err(g["v"], gv))
    announce(f"  pop {errs[0]:.2e} r {errs[1]:.2e} v {errs[2]:.2e} params {g['params']} vs {gth}")
    assert max(errs) < 1e-10
    for k in range(4):
        assert abs(g["params"][k] - gth[k]) <= 1e-10 * max(1.0, abs(gth[k])), k


@pytest.mark.parametrize("friction", ["stokeslet", "stokeslet2dx"])
def test_adjoint_fifteen_velocities_matches_oracle(oracle_mod, friction):
    from oracle import adjoint as A

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 17, q=15)
    theta = (1.0, 0.8, 10.0, 1e-4)
    N, every, seed = 19, 7, 33
    announce(f"adjoint D3Q15 f64 {friction} box={BOX} N={N}")
    _, _, g = _gpu_grad("f64", f0, r0, v0, theta, cf, cr, cv, N, every, friction, 0.9, seed)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, np.array(theta), A.noise(len(r0), N, seed), cf, cr, cv,
                            friction, 0.9)
    errs = (nmax_err(g["pop"], gf), nmax_err(g["r"], gr), nmax_err(g["v"], gv),
            nmax_err(g["params"], gth))
    announce(f"  {errs}")
    assert g["pop"].shape[0] == 15 and max(errs) < 1e-10


def test_adjoint_f32_close_to_oracle(oracle_mod):
    from oracle import adjoint as A

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 12)
    theta = (1.0, 0.8, 10.0, 1e-4)
    N, every, seed = 40, 16, 32
    announce(f"adjoint f32 stokeslet box={BOX} N={N} every={every}")
    _, _, g = _gpu_grad("f32", f0, r0, v0, theta, cf, cr, cv, N, every, "stokeslet", 0.0, seed)
    gf, gr, gv, gth = A.vjp(f0, r0, v0, np.array(theta), A.noise(len(r0), N, seed), cf, cr, cv)
    errs = (nmax_err(g["pop"], gf), nmax_err(g["r"], gr), nmax_err(g["v"], gv),
            nmax_err(g["params"], gth))
    announce(f"  pop {errs[0]:.2e} r {errs[1]:.2e} v {errs[2]:.2e} params {errs[3]:.2e}")
    assert max(errs) < 2e-4


def test_adjoint_without_particles_and_single_segment(oracle_mod):
    from oracle import adjoint as A
    from paper_1909_13412_amd import Lattice

    f0, _, _, cf, _, _ = _case(oracle_mod, 13, n=0)
    N = 9
    lat = Lattice(*BOX, 0.7, storage="f64")
    lat.set_populations(f0)
    tape = lat.record(N, 50)  # one segment longer than the run
    g = lat.adjoint(tape, cf)
    e = np.zeros((0, 3))
    gf, _, _, gth = A.vjp(f0, e, e, np.array([1.0, 0.7, 10.0, 0.0]), np.zeros((N, 0, 3)), cf, e, e)
    assert nmax_err(g["pop"].cpu().numpy(), gf) < 1e-11
    assert abs(g["params"][1].item() - gth[1]) < 1e-10 * abs(gth[1])


def test_adjoint_repeatable_and_leaves_state_alone(oracle_mod):
    import torch

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 14)
    lat, tape, g1 = _gpu_grad("f64", f0, r0, v0, (1.0, 0.8, 10.0, 1e-4), cf, cr, cv, 12, 4,
                              "stokeslet", 0.0, 7)
    before = lat.populations().clone()
    r_before = lat.r.clone()
    g2 = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, cr, cv).items()}
    torch.cuda.synchronize()
    assert torch.equal(before, lat.populations()) and torch.equal(r_before, lat.r)
    for k in g1:
        assert np.allclose(g1[k], g2[k], rtol=1e-14, atol=1e-300), k


def test_adjoint_in_another_layout_and_after_a_layout_change(oracle_mod):
    # A run recorded with two rows per group gives the gradients of the
    # default layout (to the rounding of the FP64 atomics at shared nodes);
    # switching the layout after the recording
    # makes the adjoint refuse until the recorded layout is set back.
    from paper_1909_13412_amd import Lattice, _abi

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 15)
    theta = (1.0, 0.8, 10.0, 1e-4)
    _, _, g1 = _gpu_grad("f64", f0, r0, v0, theta, cf, cr, cv, 12, 5, "stokeslet", 0.0, 9)
    gamma, tau, M, kT = theta
    lat = Lattice(*BOX, tau, storage="f64")
    lat.set_layout(2)
    lat.set_populations(f0)
    lat.particles_couple(r0, v0, mass=M, gamma=gamma, kT=kT, seed=9)
    tape = lat.record(12, 5)
    g2 = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, cr, cv).items()}
    for k in g1:
        assert np.allclose(g1[k], g2[k], rtol=1e-14, atol=1e-300), k
    lat.set_layout(1)
    with pytest.raises(_abi.LbmError):
        lat.adjoint(tape, cf, cr, cv)
    lat.set_layout(2)
    g3 = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, cr, cv).items()}
    for k in g1:
        assert np.allclose(g1[k], g3[k], rtol=1e-14, atol=1e-300), k


def test_adjoint_rejects_unsupported_and_stale(oracle_mod):
    from paper_1909_13412_amd import Lattice, _abi

    lat = Lattice(8, 8, 8, 0.8, storage="bf16")
    with pytest.raises(_abi.LbmError):
        lat.record(4, 2)
    lat = Lattice(8, 8, 8, 0.8, storage="f64")
    t1 = lat.record(4, 2)
    lat.record(4, 2)
    with pytest.raises(ValueError):
        lat.adjoint(t1)


def test_autograd_function_matches_oracle(oracle_mod):
    import torch

    from oracle import adjoint as A
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.autograd import coupled_steps

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 15, n=4)
    theta = (1.0, 0.8, 10.0, 1e-4)
    N, seed = 15, 9
    lat = Lattice(*BOX, theta[1], storage="f64")
    lat.particles_couple(r0, v0, mass=theta[2], gamma=theta[0], kT=theta[3], seed=seed)
    dev = lat.device
    tf0 = torch.tensor(f0, device=dev, requires_grad=True)
    tr0 = torch.tensor(r0, device=dev, requires_grad=True)
    tv0 = torch.tensor(v0, device=dev, requires_grad=True)
    tth = torch.tensor(theta, dtype=torch.float64, device=dev, requires_grad=True)
    fN, rN, vN = coupled_steps(lat, tf0, tr0, tv0, tth, N, every=4)
    loss = (fN * torch.tensor(cf, device=dev)).sum() + (rN * torch.tensor(cr, device=dev)).sum() + \
        (vN * torch.tensor(cv, device=dev)).sum()
    gf, gr, gv, gth = torch.autograd.grad(loss, (tf0, tr0, tv0, tth))
    rf, rr, rv, rth = A.vjp(f0, r0, v0, np.array(theta), A.noise(4, N, seed), cf, cr, cv)
    assert nmax_err(gf.cpu().numpy(), rf) < 1e-10
    assert nmax_err(gr.cpu().numpy(), rr) < 1e-10
    assert nmax_err(gv.cpu().numpy(), rv) < 1e-10
    assert nmax_err(gth.cpu().numpy(), rth) < 1e-10


# ---- 64^3, tau 0.8, 16 particles, 2000 steps, checkpoints every 100 --------------

def _c4(storage, kT=1e-4, gamma=1.0, tau=0.8, M=10.0, seed=404):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L, n = 64, 16
    lat = Lattice(L, L, L, tau, storage=storage)
    r0 = particle_positions(n, L, seed)
    v0 = particle_velocities(n, 1e-5, seed)  # fixed: the parameters must not move V0
    lat.particles_couple(r0, v0, mass=M, gamma=gamma, kT=kT, seed=seed)
    return lat, r0, v0


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_adjoint_conservation_identities_64(oracle_mod, storage):
    """Mass is conserved and total momentum changes only by the Brownian
    forces, so the gradients of those functionals are known exactly."""
    import torch

    E, _ = oracle_mod.lattice()
    N, every, M, gamma, kT, seed = 2000, 100, 10.0, 1.0, 1e-4, 404
    announce(f"adjoint identities 64^3 {storage} N={N} every={every}")
    lat, r0, v0 = _c4(storage, kT=kT, gamma=gamma, M=M, seed=seed)
    tape = lat.record(N, every)
    vN = lat.v.cpu().numpy()
    g = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, torch.ones((19, 64, 64, 64),
                                                                     dtype=torch.float64)).items()}
    announce(f"  mass: pop dev {np.max(np.abs(g['pop'] - 1)):.2e} r {np.max(np.abs(g['r'])):.2e} "
             f"v {np.max(np.abs(g['v'])):.2e} params {g['params']}")
    assert np.max(np.abs(g["pop"] - 1.0)) < 1e-9
    assert np.max(np.abs(g["r"])) < 1e-9 and np.max(np.abs(g["v"])) < 1e-9
    assert np.max(np.abs(g["params"][[0, 2, 3]])) < 1e-9 and abs(g["params"][1]) < 1e-5
    # J = sum_a e_ax f_a + M sum_i V_ix after N steps
    cf = np.broadcast_to(E[:, 0].reshape(19, 1, 1, 1), (19, 64, 64, 64)).astype(float)
    cv = np.zeros((16, 3))
    cv[:, 0] = M
    g = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, None, cv).items()}
    FRx = np.sum([oracle_mod.gauss3(seed, s, i)[0] for s in range(N) for i in range(16)])
    FRx *= np.sqrt(2.0 * gamma * kT)
    want = [FRx / (2 * gamma), 0.0, v0[:, 0].sum() - vN[:, 0].sum(), FRx / (2 * kT)]
    announce(f"  momentum: pop dev {np.max(np.abs(g['pop'] - cf)):.2e} v dev "
             f"{np.max(np.abs(g['v'] - cv)):.2e} params {g['params']} want {want}")
    assert np.max(np.abs(g["pop"] - cf)) < 1e-9
    assert np.max(np.abs(g["v"] - cv)) < 1e-8 and np.max(np.abs(g["r"])) < 1e-8
    assert abs(g["params"][0] - want[0]) < 1e-8 * abs(want[0])
    assert abs(g["params"][1]) < 1e-5
    assert abs(g["params"][2] - want[2]) < 1e-8 * max(abs(want[2]), 1e-3)
    assert abs(g["params"][3] - want[3]) < 1e-8 * abs(want[3])


def test_adjoint_finite_differences_64(oracle_mod):
    """<grad J, d> against central differences of the FP64 forward along a
    direction d in (V0, gamma, tau, M, kT); J weighs the final particle state."""
    import torch

    N, every, seed = 2000, 100, 405
    base = dict(gamma=1.0, tau=0.8, M=10.0, kT=1e-4)
    rng = np.random.default_rng(6)
    cr = rng.standard_normal((16, 3))
    cv = rng.standard_normal((16, 3)) * 100.0
    dv = rng.standard_normal((16, 3)) * 1e-3
    dth = np.array([0.2, 0.05, 1.5, 0.5e-4])
    announce(f"adjoint finite differences 64^3 f64 N={N}")

    def J(h):
        p = {k: base[k] + h * dth[i] for i, k in enumerate(("gamma", "tau", "M", "kT"))}
        lat, r0, v0 = _c4("f64", kT=p["kT"], gamma=p["gamma"], tau=p["tau"], M=p["M"], seed=seed)
        lat.v.add_(torch.tensor(h * dv, device=lat.device))
        if h == 0.0:
            tape = lat.record(N, every)
            g = lat.adjoint(tape, None, cr, cv)
        else:
            lat.step(N)
            g = None
        rN, vN = lat.r.cpu().numpy(), lat.v.cpu().numpy()
        return (cr * rN).sum() + (cv * vN).sum(), g

    _, g = J(0.0)
    dj = float((g["v"].cpu().numpy() * dv).sum() + (g["params"].cpu().numpy() * dth).sum())
    h = 1e-7
    fd = (J(h)[0] - J(-h)[0]) / (2 * h)
    announce(f"  adjoint {dj:.10e}  central difference {fd:.10e}")
    assert abs(fd - dj) < 1e-5 * abs(dj)


def test_adjoint_with_body_force_and_particle_force(oracle_mod):
    """The recorded forward and the segment recompute include a body force and
    a given particle force; both are constants of the map (F_C enters the M
    derivative)."""
    from oracle import adjoint as A
    from paper_1909_13412_amd import Lattice

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 16)
    theta = (1.0, 0.8, 10.0, 1e-4)
    N, every, seed = 17, 6, 12
    G = np.array([3e-6, 0.0, -2e-6])
    fc = np.random.default_rng(16).standard_normal(r0.shape) * 1e-3
    nx, ny, nz = BOX
    lat = Lattice(nx, ny, nz, theta[1], storage="f64")
    lat.set_populations(f0)
    lat.particles_couple(r0, v0, mass=theta[2], gamma=theta[0], kT=theta[3], seed=seed)
    lat.set_body_force(G)
    lat.set_particle_force(fc)
    tape = lat.record(N, every)
    g = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, cr, cv).items()}
    gf, gr, gv, gth = A.vjp(f0, r0, v0, np.array(theta), A.noise(len(r0), N, seed), cf, cr, cv,
                            fc=fc, body=G)
    errs = (nmax_err(g["pop"], gf), nmax_err(g["r"], gr), nmax_err(g["v"], gv),
            nmax_err(g["params"], gth))
    announce(f"adjoint with body force and F_C: {errs}")
    assert max(errs) < 1e-10


# ---- the 64^3 workload's own loss: mean squared displacement after 2000 steps ----

def _msd_run(storage, friction, gamma, tau, vshift, grad):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import ADJOINT64, particle_positions, particle_velocities

    w = ADJOINT64
    L, n = w["L"], w["n"]
    r0 = particle_positions(n, L, w["seed"])
    v0 = particle_velocities(n, w["kT"] / w["mass"], w["seed"])
    lat = Lattice(L, L, L, tau, storage=storage)
    lat.particles_couple(r0, v0 + vshift, mass=w["mass"], gamma=gamma, kT=w["kT"], seed=w["seed"],
                         friction=friction)
    if grad:
        tape = lat.record(w["steps"], w["every"])
    else:
        lat.step(w["steps"])
    rN = lat.r.cpu().numpy()
    J = float(np.mean(np.sum((rN - r0) ** 2, axis=1)))
    if not grad:
        return J, None
    g = lat.adjoint(tape, None, 2.0 * (rN - r0) / n, None)
    return J, (g["params"].cpu().numpy(), g["v"].cpu().numpy())


def _msd_fd(storage, friction, h, dv):
    from paper_1909_13412_amd.inputs import ADJOINT64 as w

    def J(dg=0.0, dt=0.0, s=0.0):
        return _msd_run(storage, friction, w["gamma"] + dg, w["tau"] + dt, s * dv, False)[0]

    return ((J(dg=h) - J(dg=-h)) / (2 * h), (J(dt=h) - J(dt=-h)) / (2 * h),
            (J(s=h) - J(s=-h)) / (2 * h))


def _dv():
    from paper_1909_13412_amd.inputs import ADJOINT64 as w

    return np.random.default_rng(1).standard_normal((w["n"], 3)) * np.sqrt(w["kT"] / w["mass"])


def test_msd_gradient_fp64_finite_differences_64():
    """Loss = mean |r^N - r^0|^2 of the 16 particles after 2000 steps.  The
    Stokeslet fit changes its node set when a particle crosses a cell face, so
    the loss is only piecewise smooth; h = 1e-6 keeps every crossing on the
    same step on both sides (measured: FD converges there and is off by tens
    of percent at h >= 1e-5 for tau)."""
    dv = _dv()
    _, (gp, gv) = _msd_run("f64", "stokeslet", 1.0, 0.8, 0.0, True)
    adj = (gp[0], gp[1], float(np.sum(gv * dv)))
    fd = _msd_fd("f64", "stokeslet", 1e-6, dv)
    announce(f"MSD 64^3 f64: adjoint {adj} fd(h=1e-6) {fd}")
    for a, f in zip(adj, fd):
        assert abs(f - a) < 1e-4 * abs(a)


def test_msd_gradient_fp32_equals_fp64_adjoint_64():
    dv = _dv()
    _, (g64, v64) = _msd_run("f64", "stokeslet", 1.0, 0.8, 0.0, True)
    _, (g32, v32) = _msd_run("f32", "stokeslet", 1.0, 0.8, 0.0, True)
    announce(f"MSD 64^3 adjoint f32 {g32[:2]} {np.sum(v32 * dv):.6e} vs f64 {g64[:2]} {np.sum(v64 * dv):.6e}")
    assert np.max(np.abs(g32 - g64)) < 1e-3 * np.max(np.abs(g64))
    assert nmax_err(v32, v64) < 1e-3


def test_msd_gradient_fp32_pointwise_h1e3_64():
    """With the pointwise friction (trilinear interpolation, continuous across
    cell faces) the map is smooth and central differences with h = 1e-3 on the
    FP32 run agree with the adjoint."""
    dv = _dv()
    _, (gp, gv) = _msd_run("f32", "pointwise", 1.0, 0.8, 0.0, True)
    adj = (gp[0], gp[1], float(np.sum(gv * dv)))
    fd = _msd_fd("f32", "pointwise", 1e-3, dv)
    announce(f"MSD 64^3 f32 pointwise: adjoint {adj} fd(h=1e-3) {fd}")
    for a, f in zip(adj, fd):
        assert abs(f - a) < 2e-2 * abs(a)


def test_adjoint_with_pair_repulsion_matches_oracle(oracle_mod):
    from oracle import adjoint as A
    from paper_1909_13412_amd import Lattice

    f0, r0, v0, cf, cr, cv = _case(oracle_mod, 18, n=6)
    r0 = 3.0 + np.random.default_rng(18).uniform(0.0, 2.0, (6, 3))  # interacting cluster
    theta = (1.0, 0.8, 10.0, 1e-4)
    N, every, seed, pair = 16, 5, 14, (0.02, 1.2)
    nx, ny, nz = BOX
    lat = Lattice(nx, ny, nz, theta[1], storage="f64")
    lat.set_populations(f0)
    lat.particles_couple(r0, v0, mass=theta[2], gamma=theta[0], kT=theta[3], seed=seed)
    lat.set_pair_force(*pair)
    tape = lat.record(N, every)
    g = {k: t.cpu().numpy() for k, t in lat.adjoint(tape, cf, cr, cv).items()}
    gf, gr, gv, gth = A.vjp(f0, r0, v0, np.array(theta), A.noise(6, N, seed), cf, cr, cv,
                            pair=pair)
    errs = (nmax_err(g["pop"], gf), nmax_err(g["r"], gr), nmax_err(g["v"], gv),
            nmax_err(g["params"], gth))
    announce(f"adjoint with pair repulsion: {errs}")
    assert max(errs) < 1e-10


def test_reverse_mode_refuses_cube_spreading():
    # the reverse sweep spreads on the unit cell; a run with the reaction force
    # spread on the fitting cube is refused rather than differentiated wrongly
    from paper_1909_13412_amd import LbmError, Lattice

    lat = Lattice(12, 10, 8, 0.8, storage="f64")
    lat.particles_couple(np.array([[3.3, 4.2, 5.7]]), np.array([[1e-3, 0.0, 0.0]]),
                         friction="stokeslet_cube", radius=0.8)
    with pytest.raises(LbmError):
        lat.record(5, 5)
    lat.step(3)  # stepping itself is supported
