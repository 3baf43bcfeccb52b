"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (normalised max error max|x - x_ref| / max|x_ref|, per output array):
FP64 storage 1e-10, FP32 storage 1e-5.  Fields are compared as shifted
populations g = f - w and as moments (rho - 1, u); particles as velocities and
positions.
"""
import numpy as np
import pytest

from helpers import announce, nmax_err, pulled, raw_rows, rounding_pin, run_pair

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _w(q=19):
    import oracle

    _, w = oracle.lattice(q)
    return w


def _compare_fields(gpu, ref, tol, what="", flow_scale=0.0):
    """Shifted populations g = f - w, rho - 1 and u.  Errors are normalised by
    the largest reference value, or by `flow_scale` (a velocity scale of the
    run) when that is larger: once a flow has decayed, the oracle's unshifted
    FP64 populations carry a rounding floor of ~1e-16 x steps absolute."""
    fg = gpu.populations().cpu().numpy()
    fr = ref.populations()
    w = _w(fg.shape[0])
    gg = fg - w[:, None, None, None]
    gr = fr - w[:, None, None, None]
    g_scale = max(np.max(np.abs(gr)), flow_scale / 6.0)  # |g| ~ 3 w |u|, w <= 1/18
    e_g = float(np.max(np.abs(gg - gr)) / g_scale) if g_scale > 0 else 0.0
    rho_g, u_g = gpu.moments()
    rho_r, u_r = ref.moments()
    # density deviations can be pure rounding (shear waves): scale them by the
    # larger of the density and velocity deviations
    drho_r = rho_r - 1.0
    scale = max(np.max(np.abs(drho_r)), np.max(np.abs(u_r)), flow_scale)
    e_rho = float(np.max(np.abs(rho_g.cpu().numpy() - 1.0 - drho_r)) / scale) if scale > 0 else 0.0
    u_scale = max(np.max(np.abs(u_r)), flow_scale)
    e_u = float(np.max(np.abs(u_g.cpu().numpy() - u_r)) / u_scale) if u_scale > 0 else 0.0
    announce(f"  {what} fields: g {e_g:.2e}  rho-1 {e_rho:.2e}  u {e_u:.2e}")
    assert e_g < tol and e_u < tol and e_rho < tol, (e_g, e_u, e_rho)


def _compare_particles(gpu, ref, tol, what=""):
    rr, vr = ref.particles()
    vg = gpu.v.cpu().numpy()
    rg = gpu.r.cpu().numpy()
    e_v = nmax_err(vg, vr)
    e_r = np.max(np.abs(rg - rr))
    announce(f"  {what} particles: v {e_v:.2e}  r abs {e_r:.2e}")
    assert e_v < tol, e_v
    assert e_r < tol * max(1.0, np.max(np.abs(rr))), e_r


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_rest_state_is_exact(oracle_mod, storage):
    from paper_1909_13412_amd import Lattice

    g = Lattice(12, 10, 8, 0.8, storage=storage)
    g.particles_couple(np.array([[3.3, 4.2, 5.7], [0.0, 0.0, 0.0]]), np.zeros((2, 3)))
    g.step(50)
    f = g.populations().cpu().numpy()
    w = _w()
    assert np.array_equal(f, np.broadcast_to(w[:, None, None, None], f.shape))
    assert np.array_equal(g.v.cpu().numpy(), np.zeros((2, 3)))
    obs = g.observables()
    assert obs[0] == 12 * 10 * 8 and np.all(obs[1:] == 0.0)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_population_roundtrip(oracle_mod, storage):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import perturbed_fields

    L = (13, 7, 5)
    ref = oracle_mod.Sim(*L, 0.7)
    rho, u = perturbed_fields(L[::-1], seed=5, amp_rho=1e-2, amp_u=1e-2)
    ref.set_equilibrium(rho, u)
    ref.step(3)
    f = ref.populations()
    g = Lattice(*L, 0.7, storage=storage)
    g.set_populations(f)
    back = g.populations().cpu().numpy()
    w = _w()[:, None, None, None]
    if storage == "f64":
        assert np.max(np.abs(back - f)) <= 1e-17
    else:
        assert nmax_err(back - w, f - w) < 1e-7


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_equilibrium_initialisation(oracle_mod, storage):
    from paper_1909_13412_amd.inputs import perturbed_fields

    L = (9, 11, 6)
    rho, u = perturbed_fields(L[::-1], seed=8, amp_rho=1e-3, amp_u=1e-3)
    out = run_pair(oracle_mod, L, 0.9, storage, None, None, 0, rho=rho, u=u)
    _compare_fields(out["gpu"], out["ref"], TOL[storage] / 10, "equilibrium")


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_shear_wave_no_particles(oracle_mod, storage, tau):
    L = 24
    z = np.arange(L)
    u = np.zeros((3, L, 4, 4))
    u[0] = 1e-2 * np.sin(2 * np.pi * z / L)[:, None, None]
    u[2] = 3e-3 * np.cos(4 * np.pi * z / L)[:, None, None]
    out = run_pair(oracle_mod, (4, 4, L), tau, storage, None, None, 40, u=u)
    _compare_fields(out["gpu"], out["ref"], TOL[storage], f"shear tau={tau}")


def test_relaxation32_full_trace(oracle_mod):
    # The kicked-particle relaxation at 32^3, tau 1, FP64: every step's
    # particle velocity, fluid mass, fluid and particle momentum.
    from paper_1909_13412_amd.inputs import WORKLOADS, workload_particles

    w = WORKLOADS["relaxation32"]
    r, v = workload_particles("relaxation32")
    announce(f"relaxation32: r0 = {r[0]}")
    out = run_pair(oracle_mod, (w["L"],) * 3, w["tau"], "f64", r, v, w["steps"], mass=w["mass"],
                   gamma=w["gamma"], kT=w["kT"], seed=w["seed"], trace=True)
    tv_g = np.array(out["gpu_trace_v"])
    tv_r = np.array(out["ref_trace_v"])
    e_v = nmax_err(tv_g, tv_r)
    og = np.array(out["gpu_obs"])
    orf = np.array(out["ref_obs"])
    e_mass = nmax_err(og[:, 0], orf[:, 0])
    e_pf = nmax_err(og[:, 1:4], orf[:, 1:4])
    e_pp = nmax_err(og[:, 4:7], orf[:, 4:7])
    # The late window on its own scale: by then V has relaxed to ~1e-6.  Node
    # forces are 64-bit fixed point with 2^-48 resolution, so each of the 8
    # node forces of a step is off by at most 2^-49 per component: the fluid
    # momentum by at most 8 x 2^-49 per step, 1.4e-11 over 1000 steps, and
    # (total momentum is conserved on both sides) the particle's velocity by
    # at most 1.4e-11 / M.  Against V ~ 3e-6 at the end that bounds the
    # window's relative error by about 5e-7 (a random walk of the roundings,
    # 1.5e-8).
    late = slice(w["steps"] - 500, w["steps"])
    e_late = nmax_err(tv_g[late], tv_r[late])
    bound = 8 * 2.0**-49 * w["steps"] / w["mass"] / np.max(np.abs(tv_r[late]))
    announce(f"  V trace {e_v:.2e}  mass {e_mass:.2e}  P_fluid {e_pf:.2e}  P_particle {e_pp:.2e}  "
             f"last 500 steps on their own scale {e_late:.2e} (fixed-point bound {bound:.1e})")
    assert e_v < 1e-10 and e_mass < 1e-10 and e_pf < 1e-10 and e_pp < 1e-10
    assert e_late < bound
    # exact bookkeeping on the GPU side too: total momentum conserved (kT = 0)
    tot = og[:, 1:4] + og[:, 4:7]
    assert np.max(np.abs(tot - tot[0])) < 1e-11 * np.abs(tot[0]).max()
    # by step 1000 the flow has decayed ~100-fold: normalise by the kick speed
    _compare_fields(out["gpu"], out["ref"], 1e-10, "relaxation32 final", flow_scale=w["kick"])


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("friction", ["stokeslet", "pointwise", "bd", "stokeslet2dx", "stokeslet_cube"])
def test_ragged_suspension(oracle_mod, storage, friction):
    # Box sizes that are not multiples of the block, several blocks, noise on.
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (37, 23, 19)
    r = particle_positions(7, L, seed=12)
    v = particle_velocities(7, 1e-4 / 10.0, seed=12)
    out = run_pair(oracle_mod, L, 0.7, storage, r, v, 60, kT=1e-4, seed=4242, friction=friction)
    tol = TOL[storage]
    _compare_particles(out["gpu"], out["ref"], tol, f"{storage}/{friction}")
    if friction != "bd":
        _compare_fields(out["gpu"], out["ref"], tol, f"{storage}/{friction}")
    fh_g, fr_g = out["gpu"].particle_forces()
    fh_r, fr_r = out["ref"].particle_forces()
    assert nmax_err(fr_g.cpu().numpy(), fr_r) < 1e-12
    assert nmax_err(fh_g.cpu().numpy(), fh_r) < tol


def test_shared_nodes_and_edge_positions(oracle_mod):
    # Several particles in one cell (all eight nodes shared), a particle exactly
    # on a node, at the periodic seam, at negative unwrapped coordinates and at
    # coordinates beyond the box.
    L = (10, 9, 8)
    r = np.array([
        [4.2, 4.3, 4.1], [4.7, 4.6, 4.9], [4.5, 4.5, 4.5],
        [2.0, 3.0, 5.0],
        [9.999999, 8.9999999, 7.5], [0.0, 0.0, 0.0],
        [-0.3, -12.4, -1e-9],
        [31.2, 18.05, 16.5],
    ])
    v = np.array([[1e-2, 0, 0], [-1e-2, 5e-3, 0], [0, 0, 1e-2], [3e-3, -2e-3, 1e-3],
                  [2e-3, 2e-3, 2e-3], [-1e-3, 0, 4e-3], [5e-3, -5e-3, 0], [0, 1e-3, -1e-3]])
    out = run_pair(oracle_mod, L, 0.8, "f64", r, v, 40, kT=1e-4, seed=7)
    _compare_particles(out["gpu"], out["ref"], 1e-10, "edges")
    _compare_fields(out["gpu"], out["ref"], 1e-10, "edges")


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_particle_set_replaced_then_detached(oracle_mod, storage):
    # particles_couple in mid-run (section 2.1): a new, smaller set replaces
    # the old one and couples from its next step, the nodes the old set forced
    # are released (its reaction force reaches no later step, first Eq.
    # s2-force), and n = 0 leaves the plain fluid update (Eq. s2-coll).  Noise
    # on, a ragged box, against the oracle doing the same.
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (21, 18, 13)
    gpu = Lattice(*L, 0.7, storage=storage)
    ref = oracle_mod.Sim(*L, 0.7)
    kw = dict(mass=10.0, gamma=1.0, kT=1e-4, seed=77)
    sets = [(particle_positions(5, L, seed=31), particle_velocities(5, 1e-5, seed=31), 20),
            (particle_positions(3, L, seed=32), particle_velocities(3, 1e-5, seed=32), 15),
            (np.zeros((0, 3)), np.zeros((0, 3)), 12)]
    for k, (r, v, steps) in enumerate(sets):
        gpu.particles_couple(r, v, **kw)
        ref.set_particles(r, v, **kw)
        gpu.step(steps)
        ref.step(steps)
        if len(r):
            _compare_particles(gpu, ref, TOL[storage], f"{storage} set {k}")
        _compare_fields(gpu, ref, TOL[storage], f"{storage} set {k}")
    assert gpu.n == 0


@pytest.mark.parametrize("n,L,steps", [(1 << 20, (48, 40, 36), 2), (1 << 24, (128, 128, 96), 1)])
def test_maximum_particle_count(oracle_mod, n, L, steps):
    # The particle count's documented maximum, 2^24 (and 2^20), with far more
    # particles than nodes (11 to 15 per node): up to 134M particle lanes, and
    # every node's reaction force summed from about a hundred fixed-point
    # contributions (first Eq. s2-force).  Noise on, FP64, one or two steps
    # (the oracle takes about 25 s per step at 2^24): every particle and
    # every node against the oracle.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    r = particle_positions(n, L, seed=41)
    v = particle_velocities(n, 1e-5, seed=41)
    kw = dict(mass=10.0, gamma=1.0, kT=1e-4, seed=9)
    gpu = Lattice(*L, 0.8, storage="f64")
    gpu.particles_couple(r, v, **kw)
    ref = oracle_mod.Sim(*L, 0.8)
    ref.set_particles(r, v, **kw)
    del r, v
    gpu.step(steps)
    ref.step(steps)
    torch.cuda.synchronize()
    _compare_particles(gpu, ref, TOL["f64"], f"{n} particles")
    _compare_fields(gpu, ref, TOL["f64"], f"{n} particles")
    del gpu
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("friction", ["stokeslet", "pointwise", "stokeslet_cube"])
def test_zero_friction_is_ballistic(oracle_mod, storage, friction):
    # gamma = 0 (Eq. s2-langevin): no friction, no noise (its variance is
    # 2 gamma kT, Eqs. s2-rf1, s2-rf2) and no reaction force, so each particle
    # keeps V^0 and moves by V^0 per step while the fluid stays exactly at
    # rest; the oracle does the same.
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L, n, steps = (19, 14, 11), 6, 25
    r0 = particle_positions(n, L, seed=51)
    v0 = particle_velocities(n, 1e-4, seed=51)
    kw = dict(mass=10.0, gamma=0.0, kT=1e-4, radius=0.5, seed=3, friction=friction)
    gpu = Lattice(*L, 0.7, storage=storage)
    gpu.particles_couple(r0, v0, **kw)
    ref = oracle_mod.Sim(*L, 0.7)
    ref.set_particles(r0, v0, **kw)
    r = r0.copy()
    for _ in range(steps):
        r = r + v0
    gpu.step(steps)
    ref.step(steps)
    assert np.array_equal(gpu.v.cpu().numpy(), v0)
    assert np.array_equal(gpu.r.cpu().numpy(), r)
    rr, vr = ref.particles()
    assert np.array_equal(vr, v0) and np.array_equal(rr, r)
    fh, fr = gpu.particle_forces()
    assert not fh.cpu().numpy().any() and not fr.cpu().numpy().any()
    f = gpu.populations().cpu().numpy()
    assert np.array_equal(f, np.broadcast_to(_w()[:, None, None, None], f.shape))
    obs = gpu.observables()
    assert obs[0] == float(np.prod(L)) and not np.any(obs[1:4])


def test_bitwise_reproducible(oracle_mod):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = 16
    r = particle_positions(40, 4.0, seed=3) + 6.0  # crowded: many shared nodes
    v = particle_velocities(40, 1e-5, seed=3)
    runs = []
    for _ in range(2):
        g = Lattice(L, L, L, 0.8, storage="f32")
        g.particles_couple(r, v, kT=1e-4, seed=11)
        g.step(30)
        runs.append((g.populations().cpu().numpy(), g.v.cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_vacf_accumulation(oracle_mod):
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (12, 12, 12)
    r = particle_positions(9, L, seed=19)
    v = particle_velocities(9, 1e-5, seed=19)
    out = run_pair(oracle_mod, L, 0.8, "f64", r, v, 57, kT=1e-4, seed=5, vacf=(13, 4))
    acc_g, cnt_g = out["gpu"].vacf()
    acc_r, cnt_r = out["ref"].vacf()
    assert np.array_equal(cnt_g, cnt_r)
    e = nmax_err(acc_g.cpu().numpy(), acc_r)
    announce(f"  vacf acc {e:.2e}")
    assert e < 1e-10


def test_vacf128_truncated(oracle_mod):
    # The 128^3 / 64-particle / FP32 workload, first 500 steps.
    from paper_1909_13412_amd.inputs import WORKLOADS, workload_particles

    w = WORKLOADS["vacf128"]
    r, v = workload_particles("vacf128")
    announce("vacf128: 128^3 FP32, 64 particles, 500 steps")
    out = run_pair(oracle_mod, (w["L"],) * 3, w["tau"], "f32", r, v, 500, mass=w["mass"],
                   gamma=w["gamma"], kT=w["kT"], seed=w["seed"], vacf=(w["max_lag"], w["stride"]))
    _compare_particles(out["gpu"], out["ref"], 1e-5, "vacf128")
    acc_g, cnt_g = out["gpu"].vacf()
    acc_r, cnt_r = out["ref"].vacf()
    assert np.array_equal(cnt_g, cnt_r)
    e = nmax_err(acc_g.cpu().numpy()[:, :500], acc_r[:, :500])
    announce(f"  vacf acc {e:.2e}")
    assert e < 1e-5
    _compare_fields(out["gpu"], out["ref"], 1e-5, "vacf128")


def test_suspension256_bench_configuration(oracle_mod):
    # The benchmark workload (256^3, 4096 particles, tau 0.6, FP32, kT 1e-4)
    # in the launch configuration the benchmark times, 3 steps, all particles
    # and all nodes compared.
    from paper_1909_13412_amd.inputs import WORKLOADS, workload_particles

    w = WORKLOADS["suspension256"]
    r, v = workload_particles("suspension256")
    announce("suspension256: 256^3 FP32, 4096 particles, 3 steps")
    out = run_pair(oracle_mod, (w["L"],) * 3, w["tau"], "f32", r, v, 3, mass=w["mass"],
                   gamma=w["gamma"], kT=w["kT"], radius=w["radius"], seed=w["seed"],
                   vacf=(w["max_lag"], w["stride"]), autotune=True)
    _compare_particles(out["gpu"], out["ref"], 1e-5, "suspension256")
    rho_g, u_g = out["gpu"].moments()
    rho_r, u_r = out["ref"].moments()
    e_u = nmax_err(u_g.cpu().numpy(), u_r)
    e_rho = nmax_err(rho_g.cpu().numpy() - 1.0, rho_r - 1.0)
    announce(f"  suspension256 fields: u {e_u:.2e}  rho-1 {e_rho:.2e}")
    assert e_u < 1e-5 and e_rho < 1e-5


def test_suspension512_conservation():
    # 512^3 (19 x 512^3 > 2^31 elements) for a few steps: FP64 sums show mass
    # conserved and momentum changed exactly by the random forces.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import WORKLOADS, workload_particles

    w = WORKLOADS["suspension512"]
    r, v = workload_particles("suspension512")
    announce("suspension512: 512^3 FP32, 4096 particles, 4 steps")
    g = Lattice(w["L"], w["L"], w["L"], w["tau"], storage="f32")
    g.particles_couple(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                       seed=w["seed"])
    o = g.observables()
    for _ in range(4):
        g.step(1)
        fh, fr = g.particle_forces()
        o1 = g.observables()
        dp = (o1[1:4] + o1[4:7]) - (o[1:4] + o[4:7])
        scale = np.abs(o1[4:7]).max() + np.abs(fr.sum(0).cpu().numpy()).max()
        # FP32 populations: momentum bookkeeping holds to FP32 rounding of the
        # node sums
        assert np.allclose(dp, fr.sum(0).cpu().numpy(), rtol=0, atol=1e-4 * scale)
        assert abs(o1[0] - o[0]) < 1e-6 * o[0]
        o = o1
    del g
    torch.cuda.empty_cache()


def test_suspension512_tiled_against_oracle(oracle_mod):
    # Full size, every node: a 32^3 state (perturbed fields, one particle,
    # kT = 0) tiled 16 x 16 x 16 times into the 512^3 box, 4096 particles at
    # the same place in every tile.  The 512^3 run is then the 32^3 run
    # repeated: every tile, including those whose population offsets lie
    # beyond 2^31 elements, must hold the same moments, in every non-temporal
    # launch configuration (row-aligned included), and tile
    # 0 must match the oracle's 32^3 run.  The start positions are dyadic, so
    # the first step is the same in every tile bit for bit; later positions
    # r + V round differently at different magnitudes (FP64, ~1e-14
    # relative), so tiles may differ by that much.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import WORKLOADS, perturbed_fields

    w = WORKLOADS["suspension512"]
    T, K, steps = 32, 16, 5
    rho_t, u_t = perturbed_fields((T, T, T), seed=51, amp_rho=1e-3, amp_u=1e-3)
    p0 = np.array([13.25, 7.8125, 21.625])
    v0 = np.array([[2e-4, -1e-4, 5e-5]])
    kw = dict(mass=w["mass"], gamma=w["gamma"], kT=0.0, radius=w["radius"], seed=w["seed"])
    ref = oracle_mod.Sim(T, T, T, w["tau"])
    ref.set_equilibrium(rho_t, u_t)
    ref.set_particles(p0[None, :], v0, **kw)
    ref.step(steps)
    rho_r, u_r = ref.moments()
    v_r = ref.particles()[1][0]

    idx = np.stack(np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij"), -1).reshape(-1, 3)
    r = (T * idx + p0).astype(np.float64)
    v = np.repeat(v0, len(r), axis=0)
    L = T * K
    announce(f"suspension512 tiled: {L}^3 FP32 of {T}^3 tiles, {len(r)} particles, {steps} steps")
    dev = torch.device("cuda")
    rho_d = torch.from_numpy(rho_t).to(dev).repeat(K, K, K)
    u_d = torch.from_numpy(u_t).to(dev).repeat(1, K, K, K)
    g = Lattice(L, L, L, w["tau"], storage="f32")
    first = None
    # the non-temporal configurations with one row per group, and two of them
    # in the row-group layouts the benchmark's autotuner keeps at this size
    for shape, rows in ((4, 1), (5, 1), (6, 1), (7, 1), (9, 1), (5, 16), (4, 32)):
        g.set_layout(rows)
        g.set_shape(shape)
        g.set_equilibrium(rho_d, u_d)
        g.particles_couple(r, v, **kw)
        g.step(steps)
        rho_g, u_g = g.moments()
        rv = rho_g.view(K, T, K, T, K, T)
        uv = u_g.view(3, K, T, K, T, K, T)
        d_rho = (rv - rv[:1, :, :1, :, :1, :]).abs().max().item()
        d_u = (uv - uv[:, :1, :, :1, :, :1, :]).abs().max().item()
        vg = g.v.cpu().numpy()
        d_v = np.abs(vg - vg[:1]).max()
        tile_rho = rho_g[:T, :T, :T].cpu().numpy()
        tile_u = u_g[:, :T, :T, :T].cpu().numpy()
        e_rho = nmax_err(tile_rho - 1.0, rho_r - 1.0)
        e_u = nmax_err(tile_u, u_r)
        e_v = nmax_err(vg[0], v_r)
        announce(f"  shape {shape}, {rows} rows per group: tiles differ by rho {d_rho:.1e} u {d_u:.1e} v {d_v:.1e}; "
                 f"tile 0 vs oracle rho-1 {e_rho:.2e} u {e_u:.2e} v {e_v:.2e}")
        assert d_rho <= 1e-9 and d_u <= 1e-9 and d_v <= 1e-10 * np.abs(v0).max()
        assert e_rho < 1e-5 and e_u < 1e-5 and e_v < 1e-5
        # the launch configuration does not change the result
        if first is None:
            first = (tile_rho, tile_u, vg[0].copy())
        else:
            assert np.array_equal(first[0], tile_rho) and np.array_equal(first[1], tile_u)
            assert np.array_equal(first[2], vg[0])
        del rho_g, u_g, rv, uv
    del g, rho_d, u_d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tiles_x", [32, 31])
def test_beyond_32bit_lattice_index_tiled_against_oracle(oracle_mod, tiles_x):
    # Lattices of 19 x nx x 512 x 448 >= 2^32 population elements, nx = 1024
    # and 992: per-lane 64-bit indices in the flat configurations (FP32), and
    # 64-bit row offsets per wavefront in the row-aligned one.  A 32^3 state (perturbed fields, one particle,
    # kT = 0) tiled tiles_x x 16 x 14 times, a particle at the same place in
    # every tile, 3 steps in FP32, with one and with 16 rows per group.
    # Every tile must hold the same moments and tile 0 must match the
    # oracle's 32^3 run.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import perturbed_fields

    T, steps = 32, 3
    K = (tiles_x, 16, 14)  # tiles along x, y, z
    dims = (T * K[0], T * K[1], T * K[2])
    assert 19 * dims[0] * dims[1] * dims[2] >= 2**32
    tau = 0.6
    rho_t, u_t = perturbed_fields((T, T, T), seed=53, amp_rho=1e-3, amp_u=1e-3)
    p0 = np.array([13.25, 7.8125, 21.625])
    v0 = np.array([[2e-4, -1e-4, 5e-5]])
    kw = dict(mass=10.0, gamma=1.0, kT=0.0, radius=0.5, seed=77)
    ref = oracle_mod.Sim(T, T, T, tau)
    ref.set_equilibrium(rho_t, u_t)
    ref.set_particles(p0[None, :], v0, **kw)
    ref.step(steps)
    rho_r, u_r = ref.moments()
    v_r = ref.particles()[1][0]
    idx = np.stack(np.meshgrid(np.arange(K[0]), np.arange(K[1]), np.arange(K[2]), indexing="ij"),
                   -1).reshape(-1, 3)
    r = (T * idx + p0).astype(np.float64)
    v = np.repeat(v0, len(r), axis=0)
    announce(f"64-bit lattice index: {dims} FP32 of {T}^3 tiles, {len(r)} particles, {steps} steps")
    dev = torch.device("cuda")
    rho_d = torch.from_numpy(rho_t).to(dev).repeat(K[2], K[1], K[0])
    u_d = torch.from_numpy(u_t).to(dev).repeat(1, K[2], K[1], K[0])
    g = Lattice(*dims, tau, storage="f32")
    first = None
    runs = ((5, 1), (4, 16), (9, 1))
    for shape, rows in runs:
        g.set_layout(rows)
        g.set_shape(shape)
        g.set_equilibrium(rho_d, u_d)
        g.particles_couple(r, v, **kw)
        g.step(steps)
        rho_g, u_g = g.moments()
        rv = rho_g.view(K[2], T, K[1], T, K[0], T)
        uv = u_g.view(3, K[2], T, K[1], T, K[0], T)
        d_rho = (rv - rv[:1, :, :1, :, :1, :]).abs().max().item()
        d_u = (uv - uv[:, :1, :, :1, :, :1, :]).abs().max().item()
        vg = g.v.cpu().numpy()
        tile_rho = rho_g[:T, :T, :T].cpu().numpy()
        tile_u = u_g[:, :T, :T, :T].cpu().numpy()
        e_rho = nmax_err(tile_rho - 1.0, rho_r - 1.0)
        e_u = nmax_err(tile_u, u_r)
        e_v = nmax_err(vg[0], v_r)
        announce(f"  shape {shape}, {rows} rows per group: tiles differ by rho {d_rho:.1e} u {d_u:.1e}; "
                 f"tile 0 vs oracle rho-1 {e_rho:.2e} u {e_u:.2e} v {e_v:.2e}")
        assert d_rho <= 1e-9 and d_u <= 1e-9
        assert np.abs(vg - vg[:1]).max() <= 1e-10 * np.abs(v0).max()
        assert e_rho < 1e-5 and e_u < 1e-5 and e_v < 1e-5
        if first is None:
            first = (tile_rho, tile_u)
        else:
            assert np.array_equal(first[0], tile_rho) and np.array_equal(first[1], tile_u)
        del rho_g, u_g, rv, uv
    del g, rho_d, u_d
    torch.cuda.empty_cache()


def test_suspension512_tiled_bf16_one_step_pinned_to_rounding(oracle_mod):
    # The BF16 instance at full size (19 x 512^3 elements), every node: a 32^3
    # perturbed state whose shifted populations are rounded to BF16 (so the
    # storage holds it exactly) is tiled 16^3 times, with one particle at the
    # same dyadic place in every tile (4096 in all).  After one step every
    # tile must hold the same bits, and tile 0's stored post-collision values
    # must be BF16 roundings (to nearest, ties to even) of values within the
    # FP32 arithmetic's error bound of the oracle's FP64 step on the 32^3
    # tile, all but a fraction 2e-3 the rounding of the oracle's value
    # itself; in every non-temporal launch configuration, and in row-group
    # layouts.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import WORKLOADS, perturbed_fields

    w = WORKLOADS["suspension512"]
    T, K = 32, 16
    L = T * K
    e, wts = oracle_mod.lattice(19)
    wq = wts[:, None, None, None]
    rho_t, u_t = perturbed_fields((T, T, T), seed=52, amp_rho=1e-3, amp_u=1e-3)
    p0 = np.array([13.25, 7.8125, 21.625])
    v0 = np.array([[2e-4, -1e-4, 5e-5]])
    kw = dict(mass=w["mass"], gamma=w["gamma"], kT=0.0, radius=w["radius"], seed=w["seed"])
    ref = oracle_mod.Sim(T, T, T, w["tau"])
    ref.set_equilibrium(rho_t, u_t)
    f0 = wq + _bf16_nearest_even(ref.populations() - wq)
    ref.set_populations(f0)
    ref.set_particles(p0[None, :], v0, **kw)
    ref.step(1)
    g1 = ref.populations() - wq
    # the stored lattice holds post-collision values at their own node: the
    # value the oracle streams to x + e_a
    g_exact = np.stack([np.roll(g1[a], shift=(-e[a, 2], -e[a, 1], -e[a, 0]), axis=(0, 1, 2))
                        for a in range(19)])
    # FP32 arithmetic error bound: 64 units in the last place of FP32 at the
    # largest population
    delta = 64 * 2.0**-24 * float(np.max(np.abs(g_exact)))
    v_r = ref.particles()[1][0]

    idx = np.stack(np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij"), -1).reshape(-1, 3)
    r = (T * idx + p0).astype(np.float64)
    v = np.repeat(v0, len(r), axis=0)
    announce(f"suspension512 tiled BF16: {L}^3 of {T}^3 tiles, {len(r)} particles, one step")
    dev = torch.device("cuda")
    f_d = torch.from_numpy(f0).to(dev).repeat(1, K, K, K)
    live = g_exact != 0.0
    for shape, rows in ((4, 1), (5, 1), (6, 1), (7, 1), (9, 1), (4, 8), (5, 32)):
        g = Lattice(L, L, L, w["tau"], storage="bf16")
        g.set_layout(rows)
        g.set_shape(shape)
        g.set_populations(f_d)
        g.particles_couple(r, v, **kw)
        g.step(1)  # the state moves from the first lattice to the second
        torch.cuda.synchronize()
        # raw layout [z][y / R][a][y mod R][x] with R rows per group (R divides T)
        R = g.layout
        raw = g.pop_b[: 19 * L**3 * 2].view(torch.int16).view(K, T, K, T // R, 19, R, K, T)
        same = bool(torch.equal(raw, raw[:1, :, :1, :, :, :, :1, :].expand_as(raw)))
        tile = raw[0, :, 0, :, :, :, 0, :].permute(2, 0, 1, 3, 4).reshape(19, T, T, T)
        g_gpu = tile.contiguous().view(torch.bfloat16).double().cpu().numpy()  # [a][z][y][x]
        frac, outside = rounding_pin(g_gpu, g_exact, _bf16_nearest_even, delta)
        vg = g.v.cpu().numpy()
        e_v = nmax_err(vg[0], v_r)
        announce(f"  shape {shape}, {R} rows per group: tiles identical {same}; tile 0: a fraction {frac:.1e} of the "
                 f"populations differ from the rounded oracle, {outside} outside the FP32 "
                 f"bracket; v {e_v:.2e}")
        assert same
        assert live.sum() > 0.9 * g_exact.size
        assert frac < 2e-3 and outside == 0
        assert e_v < 1e-10 and np.array_equal(vg, np.repeat(vg[:1], len(vg), axis=0))
        del raw, g
        torch.cuda.empty_cache()
    del f_d
    torch.cuda.empty_cache()


def test_autotune_choice_is_remembered():
    # lbm_autotune's choice is kept for the process, per device, storage,
    # velocity set and box size: a later context of the same key starts from
    # it, any other key from the size-based default.
    from paper_1909_13412_amd import Lattice

    for dims in ((40, 30, 22), (33, 17, 12)):
        a = Lattice(*dims, 0.8, storage="f32")
        k, ms = a.autotune(3)
        assert a.launch_config == k and ms[k] > 0.0
        b = Lattice(*dims, 0.8, storage="f32")
        assert b.launch_config == k
        # the launch options and the storage layout are remembered too
        assert b.sweep_launch == a.sweep_launch and b.layout == a.layout
        assert dims[1] % a.layout == 0
        assert Lattice(*dims, 0.8, storage="f32", velocities=15).launch_config == 0
        assert Lattice(dims[0], dims[1], dims[2] + 1, 0.8, storage="f32").launch_config == 0
    # a lattice beyond the last-level cache defaults to non-temporal stores;
    # rows that are not whole wavefronts to the row-aligned mapping
    # (a box size no other test autotunes, or the remembered choice would apply)
    assert Lattice(256, 256, 160, 0.6, storage="f32").launch_config == 4
    assert Lattice(250, 20, 10, 0.6, storage="f32").launch_config == 8
    assert Lattice(48, 20, 10, 0.6, storage="f32").launch_config == 0


def test_fixed_point_range_flagged():
    # A reaction force beyond the fixed-point node fields' range (|F W| >=
    # 16384) is not spread: the node receives nothing, the error is flagged and
    # the next observables call reports it (then clears it).
    from paper_1909_13412_amd import LbmError, Lattice

    lat = Lattice(8, 8, 8, 0.8, storage="f64")
    lat.particles_couple(np.array([[3.5, 3.5, 3.5]]), np.array([[1e6, 0.0, 0.0]]), mass=1.0, gamma=1.0)
    lat.step(1)
    with pytest.raises(LbmError):
        lat.observables()
    obs = lat.observables()  # the flag was cleared; nothing reached the fluid
    assert obs[0] == 512.0 and np.all(obs[1:4] == 0.0)


def test_coupling_warnings():
    # Advisory bits of section 2.2's parameter ranges, raised as warnings by
    # the binding; never errors.
    import warnings

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions

    lat = Lattice(24, 24, 24, 0.6)
    r = particle_positions(4, 24.0, seed=1)
    v = np.zeros((4, 3))
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        lat.particles_couple(r, v, radius=0.5)
        assert lat.warnings == 0
        lat.particles_couple(r, v, radius=1.59, friction="stokeslet2dx")  # within the cube's range
        assert lat.warnings == 0
        lat.particles_couple(r, v, radius=3.0, friction="bd")  # no fit, no fluid coupling
        assert lat.warnings == 0
    with pytest.warns(UserWarning, match="negative"):
        lat.particles_couple(r, v, gamma=1.0)  # Stokes' law at tau 0.6: R = 1.59
    assert lat.warnings == 2 and abs(lat.radius - 1.0 / (6 * np.pi * 0.1 / 3)) < 1e-12
    with pytest.warns(UserWarning, match="covers"):
        lat.particles_couple(r, v, radius=1.8)
    assert lat.warnings == 3
    with pytest.warns(UserWarning, match="volume fraction"):
        lat.particles_couple(particle_positions(4096, 24.0, seed=2), np.zeros((4096, 3)), radius=0.5)
    assert lat.warnings == 4
    lat.particles_couple(np.zeros((0, 3)), np.zeros((0, 3)))
    assert lat.warnings == 0
    lat.step(2)


def test_nonfinite_detected(oracle_mod):
    from paper_1909_13412_amd import LbmError, Lattice

    g = Lattice(8, 8, 8, 0.8, storage="f32")
    f = np.broadcast_to(_w()[:, None, None, None], (19, 8, 8, 8)).copy()
    f[3, 2, 2, 2] = np.nan
    g.set_populations(f)
    with pytest.raises(LbmError):
        g.observables()
    out = g.observables(allow_nonfinite=True)
    assert not np.isfinite(out[0])


@pytest.mark.parametrize("storage,tol", [("bf16", 3e-2), ("f16", 3e-3)])
def test_reduced_precision_storage_error(oracle_mod, storage, tol):
    # Shifted 16-bit storage with FP32 arithmetic: the error against the FP64
    # oracle is reported and bounded (no exact pin exists for rounded storage).
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (32, 32, 32)
    r = particle_positions(16, L, seed=23)
    v = particle_velocities(16, 1e-5, seed=23)
    out = run_pair(oracle_mod, L, 0.6, storage, r, v, 200, kT=1e-4, radius=0.5, seed=9)
    rr, vr = out["ref"].particles()
    e_v = nmax_err(out["gpu"].v.cpu().numpy(), vr)
    _, u_g = out["gpu"].moments()
    _, u_r = out["ref"].moments()
    e_u = nmax_err(u_g.cpu().numpy(), u_r)
    announce(f"  {storage}: particle v {e_v:.2e}  u {e_u:.2e}")
    assert e_v < tol and e_u < 10 * tol


def _bf16_nearest_even(x, toward_zero=False):
    # bfloat16 keeps 8 significant bits: x = m 2^e with 0.5 <= |m| < 1, so
    # the kept significand is m 2^8 rounded to an integer (ties to even, as
    # np.rint does), or cut toward zero for the comparison below
    m, e = np.frexp(x)
    k = np.trunc(m * 256.0) if toward_zero else np.rint(m * 256.0)
    return np.ldexp(k, e - 8)


def _f16_scaled(x, toward_zero=False):
    # binary16 of x 2^16 (11 significant bits, subnormal below 2^-14), back in units of x
    y = x * 65536.0
    if toward_zero:
        h = y.astype(np.float16).astype(np.float64)
        over = np.abs(h) > np.abs(y)
        h[over] = np.nextafter(h[over].astype(np.float16), np.float16(0)).astype(np.float64)
        return h / 65536.0
    return y.astype(np.float16).astype(np.float64) / 65536.0


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_sixteen_bit_storage_one_step_pinned_to_rounding(oracle_mod, storage):
    # One step from a state every storage holds exactly: the oracle steps in
    # FP64 and the shifted populations g = f - w are rounded to the storage
    # (to nearest, ties to even; FP16 scaled by 2^16) by the format's own
    # definition.  The GPU (FP32 arithmetic, then the same rounding) must
    # store exactly those values, except where its FP32 arithmetic lands on
    # the other side of a rounding boundary: rare, and then one unit in the
    # last place.  Rounding toward zero instead would miss about half.
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    rnd = _bf16_nearest_even if storage == "bf16" else _f16_scaled
    L = (14, 12, 10)
    w = _w()[:, None, None, None]
    r = particle_positions(6, L, seed=71)
    v = particle_velocities(6, 2e-3, seed=71)
    warm = oracle_mod.Sim(*L, 0.7)
    warm.set_particles(r, v, kT=1e-4, radius=0.5, seed=5)
    warm.step(25)
    r0, v0 = warm.particles()
    g0 = rnd(warm.populations() - w)
    f0 = w + g0  # exact: g0 has at most 11 significant bits
    ref = oracle_mod.Sim(*L, 0.7)
    ref.set_populations(f0)
    ref.set_particles(r0, v0, kT=1e-4, radius=0.5, seed=5)
    gpu = Lattice(*L, 0.7, storage=storage)
    gpu.set_populations(f0)
    gpu.particles_couple(r0, v0, kT=1e-4, radius=0.5, seed=5)
    assert np.array_equal(gpu.populations().cpu().numpy() - w, g0)
    ref.step(1)
    gpu.step(1)
    g_exact = ref.populations() - w
    g_want = rnd(g_exact)
    g_gpu = gpu.populations().cpu().numpy() - w
    live = g_exact != 0.0
    miss = g_gpu != g_want
    frac = miss.sum() / live.sum()
    # where they differ, the GPU holds the other neighbour of the exact value
    lo, hi = np.minimum(g_want, g_gpu), np.maximum(g_want, g_gpu)
    between = (lo <= g_exact) & (g_exact <= hi)
    frac_rtz = (g_gpu != rnd(g_exact, toward_zero=True)).sum() / live.sum()
    announce(f"  {storage}: {live.sum()} nonzero populations, {miss.sum()} differ from the "
             f"rounded oracle ({frac:.1e}); rounding toward zero would differ in {frac_rtz:.2f}")
    assert live.sum() > 0.9 * g_exact.size
    assert frac < 2e-3 and np.all(between[miss])
    assert frac_rtz > 0.3
    # ... and its neighbour: one unit in the last place apart at most
    big = np.maximum(np.abs(g_want), np.abs(g_gpu))[miss]
    _, e = np.frexp(big)
    if storage == "bf16":
        ulp = np.ldexp(1.0, e - 8)
    else:
        _, e16 = np.frexp(big * 65536.0)
        ulp = np.maximum(np.ldexp(1.0, e16 - 11), 2.0 ** -24) / 65536.0
    assert np.all(np.abs(g_gpu[miss] - g_want[miss]) <= ulp)
    _, vr = ref.particles()
    assert nmax_err(gpu.v.cpu().numpy(), vr) < 1e-10


def test_two_contexts_on_two_streams():
    # Two contexts on two caller streams (default priority), their steps
    # enqueued in turn and running concurrently, give the same bits as each
    # run alone on the default stream: no state is shared between contexts.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    boxes = [((40, 24, 16), 11), ((33, 20, 12), 7)]

    def make(L, n, stream=None):
        lat = Lattice(*L, 0.7, storage="f32", stream=stream)
        lat.particles_couple(particle_positions(n, L, seed=n), particle_velocities(n, 1e-4, seed=n),
                             kT=1e-4, radius=0.5, seed=n)
        lat.vacf_config(20, 2)
        return lat

    def state(lat):
        f = lat.populations()
        acc, cnt = lat.vacf()
        torch.cuda.synchronize()
        return f.cpu().numpy(), lat.v.cpu().numpy(), acc.cpu().numpy(), cnt

    alone = []
    for L, n in boxes:
        lat = make(L, n)
        lat.step(60)
        alone.append(state(lat))
        lat.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    lats = [make(L, n, s) for (L, n), s in zip(boxes, streams)]
    for _ in range(12):
        for lat in lats:
            lat.step(5)
    for lat, ref in zip(lats, alone):
        got = state(lat)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("storage,every,steps", [("f64", 1, 150), ("f32", 3, 61)])
def test_recorded_series_matches_oracle(oracle_mod, storage, every, steps):
    # Observables recorded inside the step kernels (fused FP64 sums) against the
    # oracle's per-step sums of the same state.
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (37, 23, 19)
    r = particle_positions(7, L, seed=12)
    v = particle_velocities(7, 1e-5, seed=12)
    gpu = Lattice(*L, 0.7, storage=storage)
    gpu.particles_couple(r, v, kT=1e-4, seed=4242)
    gpu.series_config(every, capacity=steps)
    ref = oracle_mod.Sim(*L, 0.7)
    ref.set_particles(r, v, kT=1e-4, seed=4242)
    want = []
    for n in range(steps):
        if n % every == 0:
            want.append(np.concatenate([[n], ref.observables()]))
        ref.step(1)
    gpu.step(steps)
    got = gpu.series()
    want = np.array(want)
    assert got.shape == want.shape
    assert np.array_equal(got[:, 0], want[:, 0])
    tol = TOL[storage]
    e_mass = np.max(np.abs(got[:, 1] - want[:, 1])) / want[0, 1]
    e_pf = nmax_err(got[:, 2:5], want[:, 2:5])
    e_pp = nmax_err(got[:, 5:8], want[:, 5:8])
    announce(f"  series {storage}: mass {e_mass:.2e}  P_fluid {e_pf:.2e}  P_particle {e_pp:.2e}")
    assert e_mass < tol * 1e-3 and e_pf < tol and e_pp < tol
    # and against the separate reduction of the final state
    gpu2 = Lattice(*L, 0.7, storage=storage)
    gpu2.particles_couple(r, v, kT=1e-4, seed=4242)
    gpu2.series_config(1, capacity=1)
    obs = gpu2.observables()
    gpu2.step(1)
    s = gpu2.series()[0]
    assert np.allclose(s[1:], obs, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("friction", ["stokeslet", "pointwise"])
def test_body_force_and_particle_force(oracle_mod, storage, friction):
    # Uniform body force on every node plus a given force F_C on each particle
    # (second Eq. s2-force, Eq. s2-langevin), noise on, ragged box.
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    nx, ny, nz = (21, 13, 11)
    n, steps, tau = 6, 45, 0.75
    G = np.array([2e-6, -1e-6, 5e-7])
    r = particle_positions(n, (nx, ny, nz), seed=21)
    v = particle_velocities(n, 1e-5, seed=21)
    F = np.random.default_rng(21).standard_normal((n, 3)) * 1e-3
    announce(f"body + particle force {storage} {friction} box=({nx},{ny},{nz}) n={n}")
    gpu = Lattice(nx, ny, nz, tau, storage=storage)
    ref = oracle_mod.Sim(nx, ny, nz, tau)
    kw = dict(mass=10.0, gamma=1.0, kT=1e-4, seed=77, friction=friction)
    gpu.particles_couple(r, v, **kw)
    ref.set_particles(r, v, **kw)
    gpu.set_body_force(G)
    ref.set_body_force(np.broadcast_to(G.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy())
    gpu.set_particle_force(F)
    ref.set_particle_force(F)
    gpu.step(steps)
    ref.step(steps)
    tol = TOL[storage]
    _compare_particles(gpu, ref, tol, f"{storage}/{friction}")
    _compare_fields(gpu, ref, tol, f"{storage}/{friction}")
    # fluid momentum gains G per node per step and the particles' reaction
    o_g, o_r = gpu.observables(), ref.observables()
    assert np.max(np.abs(o_g[1:7] - o_r[1:7])) < tol * np.max(np.abs(o_r[1:7]))


def test_body_force_alone_is_exact_momentum_input():
    from paper_1909_13412_amd import Lattice

    lat = Lattice(16, 12, 10, 0.9, storage="f64")
    G = np.array([1e-5, -2e-5, 3e-6])
    lat.set_body_force(G)
    lat.step(25)
    o = lat.observables()
    assert np.allclose(o[1:4], 25 * G * 1920, rtol=1e-12, atol=0)
    lat.set_body_force(None)
    lat.step(5)
    assert np.allclose(lat.observables()[1:4], o[1:4], rtol=1e-13, atol=0)


@pytest.mark.parametrize("friction", ["stokeslet2dx", "stokeslet_cube"])
def test_wide_fit_at_seams_and_shared_nodes(oracle_mod, friction):
    # The (2 dx)^3 fitting cube reaches one node beyond the unit cell on each
    # side: positions within half a node of the seams (c0 = -1 or c0 + 2 = L)
    # and beyond the box, with particles sharing fitting nodes (and, with the
    # cube spreading, the nodes their reaction forces go to).
    nx, ny, nz = (11, 9, 8)
    r = np.array([[0.2, 0.3, 0.1], [10.8, 8.7, 7.6], [-0.4, 4.5, 9.9], [5.5, 4.5, 3.5],
                  [5.9, 4.1, 3.2], [21.3, -8.6, 15.8]])
    v = np.random.default_rng(5).standard_normal((6, 3)) * 1e-3
    out = run_pair(oracle_mod, (nx, ny, nz), 0.8, "f64", r, v, 30, kT=1e-4, seed=9,
                   friction=friction, radius=1.2)
    _compare_particles(out["gpu"], out["ref"], 1e-10, f"{friction} seams")
    _compare_fields(out["gpu"], out["ref"], 1e-10, f"{friction} seams")


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("friction", ["stokeslet", "pointwise", "stokeslet2dx", "stokeslet_cube"])
def test_fifteen_velocity_suspension(oracle_mod, storage, friction):
    # The paper's own velocity set: ragged box, noise, body force, three
    # friction models.
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (29, 17, 13)
    r = particle_positions(7, L, seed=15)
    v = particle_velocities(7, 1e-5, seed=15)
    announce(f"D3Q15 {storage} {friction} box={L}")
    out = run_pair(oracle_mod, L, 0.7, storage, r, v, 1, kT=1e-4, seed=515, friction=friction,
                   radius=0.9 if friction == "stokeslet2dx" else 0.0, q=15)
    G = np.array([1e-6, 2e-6, -1e-6])
    out["gpu"].set_body_force(G)
    out["ref"].set_body_force(np.broadcast_to(G.reshape(3, 1, 1, 1), (3, L[2], L[1], L[0])).copy())
    out["gpu"].step(50)
    out["ref"].step(50)
    tol = TOL[storage]
    _compare_particles(out["gpu"], out["ref"], tol, f"D3Q15 {storage}/{friction}")
    _compare_fields(out["gpu"], out["ref"], tol, f"D3Q15 {storage}/{friction}")


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_fifteen_velocity_shear_wave(oracle_mod, tau):
    L = (4, 6, 24)
    nz = L[2]
    z = np.arange(nz)
    u = np.zeros((3, nz, L[1], L[0]))
    u[0] = 1e-2 * np.sin(2 * np.pi * z / nz)[:, None, None]
    out = run_pair(oracle_mod, L, tau, "f64", None, None, 80, u=u, q=15)
    _compare_fields(out["gpu"], out["ref"], 1e-10, f"D3Q15 shear tau={tau}")


def test_every_launch_configuration_is_bit_identical():
    # Four geometric shapes x plain / non-temporal stores, and the row-aligned
    # mapping x plain / non-temporal, with either block order and residency
    # cap, in every storage layout (rows per group), also with the layout
    # switched between steps: the same step, the same bits, also with the
    # FP64 sums fused in.  Boxes whose row-aligned mapping puts four rows in
    # a block, a row of three wavefronts with 62 idle lanes, rows longer than
    # a block, 64 short rows per plane (row groups up to 64 rows), and rows of
    # two whole wavefronts (64 | nx: the 16-bit storages address by wavefront
    # rows in every configuration, FP32 and FP64 by per-lane indices in the
    # flat ones; the row-aligned mapping always by rows).
    import torch

    from paper_1909_13412_amd import Lattice, _abi
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    for L in ((40, 24, 16), (130, 6, 8), (300, 6, 5), (24, 64, 5), (128, 10, 6)):
        r = particle_positions(9, L, seed=31)
        v = particle_velocities(9, 1e-5, seed=31)
        # every storage x velocity-set instance the library builds and the
        # benchmark times
        for storage, q in (("f32", 19), ("bf16", 19), ("f64", 19), ("f16", 19), ("f32", 15),
                           ("bf16", 15)):
            ref, sums = None, {}
            # every configuration in node order without a residency cap, and
            # three of them with the per-XCD block order and residency caps
            runs = [(k, 0, 0, 1, 1) for k in range(_abi.LBM_NUM_SHAPES)]
            runs += [(k, o, w, 1, 1) for k in (1, 5, 8) for o in (0, 1) for w in (0, 6, 4, 2)
                     if (o, w) != (0, 0)]
            # layouts: from the start, and switched after five steps
            ys = [y for y in (2, 4, 8, 16, 32, 64) if L[1] % y == 0]
            runs += [(k, 0, 0, y, y) for k in (1, 4, 7, 9) for y in ys]
            runs += [(5, 1, 4, ys[-1], 1), (5, 0, 0, 1, ys[-1])]
            for k, order, cap, y0, y1 in runs:
                lat = Lattice(*L, 0.7, storage=storage, velocities=q)
                lat.set_layout(y0)
                assert lat.layout == y0
                lat.particles_couple(r, v, kT=1e-4, seed=8)
                lat.series_config(3, 8)
                lat.set_shape(k)
                try:
                    lat.set_sweep_launch(order, cap)
                except _abi.LbmError:
                    assert cap == 2  # the device's LDS per block may not allow two blocks
                    continue
                assert lat.sweep_launch == (order, cap)
                lat.step(5)
                lat.set_layout(y1)
                assert lat.layout == y1
                lat.step(8)
                f = lat.populations()
                torch.cuda.synchronize()
                ser = lat.series()
                if ref is None:
                    ref = (f.clone(), lat.v.clone(), ser)
                else:
                    assert torch.equal(f, ref[0]), (L, storage, q, k, order, cap, y0, y1)
                    assert torch.equal(lat.v, ref[1]), (L, storage, q, k, order, cap, y0, y1)
                    # FP64 sums: per-block partials follow the lane mapping, so
                    # only the same mapping reproduces them bit for bit (block
                    # order and cap do not change it)
                    assert np.allclose(ser, ref[2], rtol=1e-12, atol=1e-15), (L, storage, q, k)
                key = "row" if k >= 8 else k & 3
                if key in sums:
                    assert np.array_equal(ser, sums[key]), (L, storage, q, k, order, cap)
                sums[key] = ser
    lat = Lattice(9, 7, 5, 0.7)
    with pytest.raises(Exception):
        lat.set_shape(2)  # two rows per lane need an even ny
    for y in (0, 2, 3, 7, 128):  # not a power of two up to 64 dividing ny = 7
        with pytest.raises(_abi.LbmError):
            lat.set_layout(y)
    assert lat.layout == 1


@pytest.mark.parametrize("storage", ["f32", "bf16", "f64"])
def test_stream_ceiling_kernel_pulls_every_population(storage):
    # The streaming-only kernel that bounds the stream-collide (lbm_stream_ceiling)
    # must move exactly the stream-collide's bytes: the spare lattice holds every
    # population pulled from x - e_a, unchanged, in every launch configuration,
    # and the simulation state is left as it was.
    import torch

    from paper_1909_13412_amd import Lattice, _abi
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    dt = {"f32": torch.float32, "bf16": torch.int16, "f64": torch.float64}[storage]
    for L in ((40, 24, 16), (130, 6, 8), (24, 64, 5)):
        nx, ny, nz = L
        lat = Lattice(*L, 0.7, storage=storage)
        lat.particles_couple(particle_positions(9, L, seed=33), particle_velocities(9, 1e-4, seed=33),
                             kT=1e-4, seed=8)
        lat.step(6)  # even: the current populations are back in the first buffer
        torch.cuda.synchronize()
        f0 = lat.populations().clone()
        n = 19 * nx * ny * nz

        def raw(buf):
            # [nz, ny, 19, nx] whatever the layout's rows per group
            return raw_rows(buf[: n * buf.new_empty(0, dtype=dt).element_size()].view(dt).cpu().numpy(),
                            nx, ny, nz, lat.layout)

        a0 = raw(lat.pop_a)
        expect = pulled(a0, nx, ny, nz)
        for k in range(_abi.LBM_NUM_SHAPES):
            lat.pop_b.zero_()
            torch.cuda.synchronize()
            ms = lat.stream_ceiling(1, config=k)
            assert ms > 0.0
            assert np.array_equal(raw(lat.pop_b), expect), (L, storage, k)
        # every layout moves the same values (the state is permuted into it
        # and stays in the first buffer)
        for y in (2, 4, 8, 16, 32, 64):
            if ny % y:
                continue
            lat.set_layout(y)
            lat.pop_b.zero_()
            torch.cuda.synchronize()
            assert np.array_equal(raw(lat.pop_a), a0), (L, storage, "layout", y)
            assert lat.stream_ceiling(1, config=5) > 0.0
            assert np.array_equal(raw(lat.pop_b), expect), (L, storage, "layout", y)
        lat.set_layout(1)
        # the per-XCD block order with a residency cap moves the same values
        lat.set_shape(1)
        lat.set_sweep_launch(1, 4)
        lat.pop_b.zero_()
        torch.cuda.synchronize()
        assert lat.stream_ceiling(1) > 0.0
        assert np.array_equal(raw(lat.pop_b), expect), (L, storage, "order 1, cap 4")
        assert np.array_equal(raw(lat.pop_a), a0)
        assert torch.equal(lat.populations(), f0)
        with pytest.raises(Exception):
            lat.stream_ceiling(0)
        with pytest.raises(Exception):
            lat.stream_ceiling(1, config=_abi.LBM_NUM_SHAPES)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("box,r_c", [((21, 13, 11), 1.3), ((6, 9, 13), 2.9)])
def test_pair_repulsion(oracle_mod, storage, box, r_c):
    # Soft pair repulsion (Eq. s2-softpot, DPD reading) on a crowded cluster:
    # cell lists with three or more cells per axis, and with two (6 / 2.9).
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    n = 14
    r = particle_positions(n, (4.0, 4.0, 4.0), seed=61) + 1.0
    r[-3:] = particle_positions(3, box, seed=62)  # a few far away, one near a seam
    r[-1] = [box[0] - 0.2, 0.3, box[2] - 0.4]
    v = particle_velocities(n, 1e-5, seed=61)
    announce(f"pair repulsion {storage} box={box} r_c={r_c} n={n}")
    out = run_pair(oracle_mod, box, 0.8, storage, r, v, 0, kT=1e-4, seed=3)
    out["gpu"].set_pair_force(0.02, r_c)
    out["ref"].set_pair_force(0.02, r_c)
    out["gpu"].step(1)
    out["ref"].step(1)
    fp_g, fp_r = out["gpu"].pair_forces().cpu().numpy(), out["ref"].pair_forces()
    announce(f"  first-step pair forces {nmax_err(fp_g, fp_r):.2e} (max |F| {np.max(np.abs(fp_r)):.3e})")
    assert np.max(np.abs(fp_r)) > 0.0
    assert nmax_err(fp_g, fp_r) < 1e-12
    out["gpu"].step(40)
    out["ref"].step(40)
    tol = TOL[storage]
    _compare_particles(out["gpu"], out["ref"], tol, f"pairs {storage}")
    _compare_fields(out["gpu"], out["ref"], tol, f"pairs {storage}")


@pytest.mark.parametrize("n,box,r_c", [(12000, (64, 48, 40), 1.0), (3000, (24, 24, 24), 1.2),
                                       (700, (16, 12, 20), 1.5)])
def test_pair_repulsion_many(oracle_mod, n, box, r_c):
    # Many particles: more cells than buckets (several cells share a bucket and
    # are told apart by their cell index), crowded buckets, all against the
    # oracle's all-pairs sum.  The bucket counts (32768, 8192, 2048) give the
    # one-block scan 32, 8 and 2 buckets per thread.
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    r = particle_positions(n, box, seed=71)
    v = particle_velocities(n, 1e-5, seed=71)
    announce(f"pair repulsion many n={n} box={box} r_c={r_c}")
    out = run_pair(oracle_mod, box, 0.8, "f64", r, v, 0, kT=1e-4, seed=5)
    out["gpu"].set_pair_force(0.03, r_c)
    out["ref"].set_pair_force(0.03, r_c)
    out["gpu"].step(1)
    out["ref"].step(1)
    fp_g, fp_r = out["gpu"].pair_forces().cpu().numpy(), out["ref"].pair_forces()
    touched = int(np.count_nonzero(np.any(fp_r != 0.0, axis=1)))
    announce(f"  pair forces {nmax_err(fp_g, fp_r):.2e}, {touched} particles with neighbours")
    assert touched > n // 10
    assert np.array_equal(fp_g == 0.0, fp_r == 0.0)
    assert nmax_err(fp_g, fp_r) < 1e-12


def test_pair_repulsion_reproducible_and_validated():
    import torch

    from paper_1909_13412_amd import Lattice, _abi
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    r = particle_positions(40, (5.0, 5.0, 5.0), seed=8) + 2.0
    v = particle_velocities(40, 1e-5, seed=8)
    runs = []
    for _ in range(2):
        lat = Lattice(16, 16, 16, 0.8, storage="f32")
        lat.particles_couple(r, v, kT=1e-4, seed=4)
        lat.set_pair_force(0.05, 1.5)
        lat.step(25)
        torch.cuda.synchronize()
        runs.append((lat.r.clone(), lat.populations()))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    lat = Lattice(8, 8, 8, 0.8)
    with pytest.raises(_abi.LbmError):
        lat.set_pair_force(0.1, 1.0)  # no particles
    lat.particles_couple(r[:2] % 8, v[:2])
    with pytest.raises(_abi.LbmError):
        lat.set_pair_force(0.1, 4.5)  # beyond half the box
    lat.set_pair_force(0.0, 0.0)  # off
    big = Lattice(32, 32, 32, 0.8)
    n_big = 65537  # one above the cell list's limit
    big.particles_couple(particle_positions(n_big, 32.0, seed=9), np.zeros((n_big, 3)))
    with pytest.raises(_abi.LbmError):
        big.set_pair_force(0.1, 1.0)
