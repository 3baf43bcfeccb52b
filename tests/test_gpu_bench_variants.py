"""Every kernel instance the benchmark times, against the FP64 oracle at the
benchmark's size and in the launch configuration its autotuner picks: the
256^3 suspension (tau 0.6, 4096 particles, R 0.5, kT 1e-4, VACF on) for each
storage x velocity set of the benchmark line (FP64, FP32, BF16, FP16 with
D3Q19; FP32, BF16 with D3Q15).

The fluid starts from a perturbed equilibrium (density and velocity noise of
1e-3 at every node, so every node's update is exercised) whose shifted
populations g = f - w are first rounded to the storage, so that both sides
start from the same state.  FP64 and FP32 storage then take three steps and
are compared with the normalised tolerances 1e-10 and 1e-5 (section 2.2,
Eqs. s2-coll, s2-trans; section 2.1 for the particles).  The 16-bit storages
take one step: every stored population must be the format's rounding (to
nearest, ties to even; FP16 scaled by 2^16) of a value within the FP32
arithmetic's error bound of the oracle's FP64 step, and all but a fraction
2e-3 must equal the rounding of the oracle's value itself (the rest lie on
the other side of a rounding boundary).
"""
import numpy as np
import pytest

from helpers import announce, nmax_err, rounding_pin

pytestmark = pytest.mark.gpu

VARIANTS = ["f64", "f32", "bf16", "f16", "f32q15", "bf16q15"]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _bf16(x):
    # bfloat16 keeps 8 significant bits: x = m 2^e with 0.5 <= |m| < 1; the
    # kept significand m 2^8 is rounded to an integer, ties to even
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def _f16_scaled(x):
    # binary16 of x 2^16 (numpy's conversion rounds to nearest even), in units of x
    return (x * 65536.0).astype(np.float16).astype(np.float64) / 65536.0


def _f32(x):
    return x.astype(np.float32).astype(np.float64)


ROUND = {"f64": lambda x: x, "f32": _f32, "bf16": _bf16, "f16": _f16_scaled}


@pytest.mark.parametrize("variant", VARIANTS)
def test_benchmark_instance_against_oracle(oracle_mod, variant):
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import WORKLOADS, perturbed_fields, workload_particles

    storage, q = (variant[:-3], 15) if variant.endswith("q15") else (variant, 19)
    w = WORKLOADS["suspension256"]
    L, tau = w["L"], w["tau"]
    steps = 3 if storage in ("f64", "f32") else 1
    announce(f"benchmark instance {variant}: {L}^3, {w['n']} particles, {steps} step(s)")
    _, wq = oracle_mod.lattice(q)
    wq = wq[:, None, None, None]
    rho, u = perturbed_fields((L, L, L), seed=256, amp_rho=1e-3, amp_u=1e-3)
    ref = oracle_mod.Sim(L, L, L, tau, q=q)
    ref.set_equilibrium(rho, u)
    del rho, u
    g0 = ROUND[storage](ref.populations() - wq)
    f0 = wq + g0
    ref.set_populations(f0)
    r, v = workload_particles("suspension256")
    kw = dict(mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"], seed=w["seed"])
    ref.set_particles(r, v, **kw)
    ref.vacf_config(w["max_lag"], w["stride"])

    gpu = Lattice(L, L, L, tau, storage=storage, velocities=q)
    gpu.set_populations(f0)
    gpu.particles_couple(r, v, **kw)
    gpu.vacf_config(w["max_lag"], w["stride"])
    shape, _ = gpu.autotune(10)
    announce(f"  autotuned launch configuration {shape}")
    # the start state is the same on both sides (the storage holds g0 exactly,
    # so w + g comes back as f0)
    assert np.array_equal(gpu.populations().cpu().numpy(), f0)
    del f0, g0

    ref.step(steps)
    gpu.step(steps)
    torch.cuda.synchronize()
    rr, vr = ref.particles()
    e_v = nmax_err(gpu.v.cpu().numpy(), vr)
    e_r = float(np.max(np.abs(gpu.r.cpu().numpy() - rr)))
    g_exact = ref.populations() - wq
    g_gpu = gpu.populations().cpu().numpy() - wq
    if storage in ("f64", "f32"):
        tol = 1e-10 if storage == "f64" else 1e-5
        e_g = nmax_err(g_gpu, g_exact)
        del g_gpu, g_exact
        rho_g, u_g = gpu.moments()
        rho_r, u_r = ref.moments()
        e_u = nmax_err(u_g.cpu().numpy(), u_r)
        e_rho = nmax_err(rho_g.cpu().numpy() - 1.0, rho_r - 1.0)
        announce(f"  {variant}: v {e_v:.2e}  r abs {e_r:.2e}  g {e_g:.2e}  u {e_u:.2e}  "
                 f"rho-1 {e_rho:.2e}")
        assert e_v < tol and e_r < tol * L
        assert e_g < tol and e_u < tol and e_rho < tol
    else:
        # FP32 arithmetic error bound: 64 units in the last place of FP32 at
        # the largest population
        delta = 64 * 2.0**-24 * float(np.max(np.abs(g_exact)))
        frac, outside = rounding_pin(g_gpu, g_exact, ROUND[storage], delta)
        live = int(np.count_nonzero(g_exact))
        announce(f"  {variant}: {live} nonzero populations, a fraction {frac:.1e} differ from "
                 f"the rounded oracle, {outside} outside the FP32 bracket; v {e_v:.2e}")
        assert live > 0.9 * g_exact.size
        assert frac < 2e-3 and outside == 0
        # the particle update reads the start state, which both sides hold exactly
        assert e_v < 1e-10 and e_r < 1e-10 * L
    del gpu, ref
    torch.cuda.empty_cache()
