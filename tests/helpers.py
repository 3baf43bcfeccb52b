"""Shared helpers for the GPU parity tests: run the same seeded case through the
HIP path (via the C ABI) and through the FP64 oracle, and compare."""
import sys

import numpy as np


def nmax_err(x, ref) -> float:
    """Normalised max error max|x - ref| / max|ref| (0/0 -> 0)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    diff = np.max(np.abs(x - ref)) if x.size else 0.0
    if scale == 0.0:
        return float(diff)
    return float(diff / scale)


def announce(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pair(oracle_mod, L, tau, storage, r, v, steps, *, mass=10.0, gamma=1.0, kT=0.0, seed=0,
             friction="stokeslet", radius=0.0, rho=None, u=None, trace=False, vacf=None,
             f16_scale_log2=16, q=19, autotune=False):
    """Run the oracle and the GPU side by side.  L is (nx, ny, nz).
    Returns dict with final fields/particles of both, and per-step traces."""
    import torch

    from paper_1909_13412_amd import Lattice

    nx, ny, nz = L
    gpu = Lattice(nx, ny, nz, tau, storage=storage, f16_scale_log2=f16_scale_log2, velocities=q)
    ref = oracle_mod.Sim(nx, ny, nz, tau, q=q)
    if rho is not None or u is not None:
        gpu.set_equilibrium(rho, u)
        ref.set_equilibrium(rho, u)
    n = 0 if r is None else len(r)
    if n:
        kw = dict(mass=mass, gamma=gamma, kT=kT, radius=radius, seed=seed, friction=friction)
        gpu.particles_couple(r, v, **kw)
        ref.set_particles(r, v, **kw)
        if vacf:
            gpu.vacf_config(*vacf)
            ref.vacf_config(*vacf)
    if autotune:  # the launch configuration the benchmark would time
        out_shape, _ = gpu.autotune(10)
        announce(f"  autotuned launch configuration {out_shape}")
    out = {"gpu_trace_v": [], "ref_trace_v": [], "gpu_obs": [], "ref_obs": []}
    if trace:
        for _ in range(steps):
            gpu.step(1)
            ref.step(1)
            if n:
                out["gpu_trace_v"].append(gpu.v.cpu().numpy().copy())
                out["ref_trace_v"].append(ref.particles()[1])
            out["gpu_obs"].append(gpu.observables())
            out["ref_obs"].append(ref.observables())
    else:
        gpu.step(steps)
        ref.step(steps)
    torch.cuda.synchronize()
    out["gpu"] = gpu
    out["ref"] = ref
    return out


# D3Q19 velocity order of the C ABI (the convention its header documents).
E19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
       (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]


def raw_rows(a, nx, ny, nz, rows_per_group=1, q=19):
    """A raw lattice buffer of the C ABI layout with the given rows per group R
    (element (a, x, y, z) at ((z ny + R (y / R)) q + y mod R) nx + a R nx + x)
    as an array [nz, ny, q, nx]."""
    R = rows_per_group
    a = np.asarray(a).reshape(nz, ny // R, q, R, nx)
    return a.transpose(0, 1, 3, 2, 4).reshape(nz, ny, q, nx)


def pulled(a, nx, ny, nz):
    """The stream-collide's pull applied to one lattice as [nz, ny, 19, nx]
    (the layout with one row per group, ((z * ny + y) * 19 + a) * nx + x):
    plane a of node x taken from x - e_a."""
    a = a.reshape(nz, ny, 19, nx)
    out = np.empty_like(a)
    for k, (ex, ey, ez) in enumerate(E19):
        out[:, :, k, :] = np.roll(a[:, :, k, :], shift=(ez, ey, ex), axis=(0, 1, 2))
    return out


def rounding_pin(g_gpu, g_exact, rnd, delta):
    """One step of a 16-bit storage against the oracle's exact step.

    The GPU computes g in FP32 and rounds it to the storage with `rnd`
    (to nearest, ties to even), so what it stores is rnd(x) for some x with
    |x - g_exact| <= delta, delta bounding the FP32 arithmetic's error.
    Rounding is monotonic, so every stored value must lie in
    [rnd(g_exact - delta), rnd(g_exact + delta)]: the rounded oracle value,
    or, where the FP32 result falls on the other side of a rounding boundary,
    its neighbour (near zero, where the format's spacing is finer than delta,
    possibly a few neighbours).  Returns (fraction of stored values that differ
    from rnd(g_exact), number outside the bracket)."""
    g_want = rnd(g_exact)
    miss = g_gpu != g_want
    lo = rnd(g_exact[miss] - delta)
    hi = rnd(g_exact[miss] + delta)
    outside = int(np.sum((g_gpu[miss] < lo) | (g_gpu[miss] > hi)))
    return float(miss.sum() / max(g_exact.size, 1)), outside
