"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the benchmark.

This module only draws initial conditions; it holds none of the method's
arithmetic.  Random numbers that the method itself draws every step (the
Brownian force) are not made here: the GPU library and the oracle each
generate them from one counter-based Philox4x32-10 stream.

Workloads (lattice units, dx = dt = rho0 = 1), all periodic cubes with the
nineteen-velocity lattice, particle mass 10 and friction constant 1:

* ``relaxation32``  -- 32^3, tau 1.0, FP64, one particle kicked to 0.01 along x
  at a seeded off-lattice position, kT = 0, 1000 steps.
* ``vacf128``       -- 128^3, tau 0.8, FP32, 64 particles, kT = 1e-4, 20000 steps.
* ``suspension256`` -- 256^3, tau 0.6, 4096 particles, kT = 1e-4, 2000 steps,
  FP32 / shifted BF16 / shifted FP16 storage, particle radius 0.5.
* ``suspension512`` -- the same at 512^3.

``radius`` 0 means "from Stokes' law" (gamma = 6 pi rho0 nu R).  At tau 0.6 that
law would give R = 1.59, and the eight-node Stokeslet fit returns negative
friction once R exceeds about 0.87 (the fitted gain for a particle at a cell
centre in a uniform stream is 1 - 2R/sqrt(3)), so the coupled run diverges; the
suspensions therefore keep the friction constant 1 and fix R = 0.5.

* ``fig2thermal100`` -- the thermal suspension of the paper's Fig. 2 (section 3)
  in lattice units: 100^3, tau 0.5534 (nu = 0.89e-6 m^2/s at dx = 5 nm,
  dt = 0.5 ps), 500 particles of R = 1 and M = 16, friction 6 pi rho0 nu R,
  kT = 3.3e-7 (300 K), the fit and the spreading on the (2 dx)^3 cube (the
  unit-cell fit has negative gain at R = 1), 12000 steps, lags to 1000.

* ``ENSEMBLE64``    -- 64 independent cubic boxes with edges drawn from
  {48, 64, 80, 96}, tau 0.8, 8 particles each, kT = 1e-4, FP32.

They stand in for the paper's own runs (a 100^3 box of 500 particles), which
use no external dataset.
"""
from __future__ import annotations

import numpy as np

WORKLOADS = {
    "relaxation32": dict(L=32, tau=1.0, storage="f64", n=1, mass=10.0, gamma=1.0, kT=0.0,
                         radius=0.0, steps=1000, seed=1001, kick=0.01),
    "vacf128": dict(L=128, tau=0.8, storage="f32", n=64, mass=10.0, gamma=1.0, kT=1e-4,
                    radius=0.0, steps=20000, seed=2002, max_lag=2000, stride=10),
    "suspension256": dict(L=256, tau=0.6, storage="f32", n=4096, mass=10.0, gamma=1.0, kT=1e-4,
                          radius=0.5, steps=2000, seed=3003, max_lag=500, stride=10),
    "suspension512": dict(L=512, tau=0.6, storage="f32", n=4096, mass=10.0, gamma=1.0, kT=1e-4,
                          radius=0.5, steps=2000, seed=3004, max_lag=500, stride=10),
    "fig2thermal100": dict(L=100, tau=0.5534, storage="f32", n=500, mass=16.0,
                           gamma=6.0 * np.pi * (0.5534 - 0.5) / 3.0, kT=3.3e-7, radius=1.0,
                           friction="stokeslet_cube", steps=12000, seed=2019, max_lag=1000,
                           stride=10),
}


ENSEMBLE64 = dict(replicas=64, sizes=(48, 64, 80, 96), tau=0.8, n=8, mass=10.0, gamma=1.0,
                  kT=1e-4, seed=4000, steps=5000, max_lag=1000, stride=10, storage="f32")

# Reverse-mode workload: 64^3, tau 0.8, FP32, 16 particles, gradients over
# 2000 steps with a checkpoint every 100.
ADJOINT64 = dict(L=64, tau=0.8, storage="f32", n=16, mass=10.0, gamma=1.0, kT=1e-4, steps=2000,
                 every=100, seed=2024)


def ensemble_replicas(replicas: int = 64, sizes=(48, 64, 80, 96), n: int = 8, tau: float = 0.8,
                      kT: float = 1e-4, mass: float = 10.0, seed: int = 4000):
    """Replica list for an ensemble of cubic boxes with edges drawn uniformly
    from `sizes`; replica k gets Philox key seed + k and counter word k."""
    rng = np.random.default_rng([seed, 0x5EED, 4])
    edges = rng.choice(np.asarray(sizes), size=replicas)
    out = []
    for k, L in enumerate(edges):
        L = int(L)
        out.append(dict(nx=L, ny=L, nz=L, tau=tau, seed=seed + k, replica=k,
                        r=particle_positions(n, L, seed + k),
                        v=particle_velocities(n, kT / mass, seed + k)))
    return out


def particle_positions(n: int, box, seed: int) -> np.ndarray:
    """n positions uniform in [0, box) per axis, FP64 [n, 3] (x, y, z)."""
    box = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    rng = np.random.default_rng([seed, 0x5EED, 1])
    return rng.random((n, 3)) * box


def particle_velocities(n: int, variance: float, seed: int) -> np.ndarray:
    """n velocities with independent normal components of the given variance."""
    rng = np.random.default_rng([seed, 0x5EED, 2])
    if variance <= 0.0:
        return np.zeros((n, 3))
    return rng.standard_normal((n, 3)) * np.sqrt(variance)


def workload_particles(name: str):
    """(r, v) for a named workload.  The kicked-relaxation case starts at rest
    except for the kick along x; the suspensions draw Maxwellian velocities of
    variance kT / M."""
    w = WORKLOADS[name]
    r = particle_positions(w["n"], w["L"], w["seed"])
    if "kick" in w:
        v = np.zeros((w["n"], 3))
        v[:, 0] = w["kick"]
    else:
        v = particle_velocities(w["n"], w["kT"] / w["mass"], w["seed"])
    return r, v


def perturbed_fields(shape, seed: int, amp_rho: float = 1e-3, amp_u: float = 1e-3):
    """Smooth-ish random density and velocity fields for parity tests:
    rho [nz, ny, nx] around 1 and u [3, nz, ny, nx]."""
    rng = np.random.default_rng([seed, 0x5EED, 3])
    rho = 1.0 + amp_rho * rng.standard_normal(shape)
    u = amp_u * rng.standard_normal((3,) + tuple(shape))
    return rho, u
