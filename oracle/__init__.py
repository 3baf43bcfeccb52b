"""FP64 CPU oracle for the coupled lattice-Boltzmann / Brownian-particle step.

TEST INFRASTRUCTURE ONLY.  This package wraps ``oracle.c`` (plain C, FP64) with
ctypes and numpy.  Only the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the GPU product path never
does, and it imports nothing from the GPU package.

Method: Yoshida, Kinjo & Washizu, arXiv:1909.13412 -- section 2.1 (friction
fit, Eq. s2-slet-v; reaction force, first Eq. s2-force; Langevin equation,
Eqs. s2-langevin, s2-langevin2) and section 2.2 (lattice Boltzmann equation,
Eqs. s2-density to s2-trans).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 19
FRICTION = {"stokeslet": 0, "pointwise": 1, "bd": 2, "stokeslet2dx": 3, "stokeslet_cube": 4}

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    i32, u32, u64, i64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    vp = ctypes.c_void_p
    sig = {
        "ora_lattice": (None, [vp, dp]),
        "ora_lattice_q": (None, [i32, vp, dp]),
        "ora_equilibrium": (None, [ctypes.c_double, dp, dp]),
        "ora_equilibrium_q": (None, [i32, ctypes.c_double, dp, dp]),
        "ora_philox4x32_10": (None, [vp, vp, vp]),
        "ora_gauss3": (None, [u64, u32, u32, u32, u32, dp]),
        "ora_friction_force": (None, [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]),
        "ora_create": (vp, [i32, i32, i32, ctypes.c_double]),
        "ora_create_q": (vp, [i32, i32, i32, ctypes.c_double, i32]),
        "ora_destroy": (None, [vp]),
        "ora_set_equilibrium": (None, [vp, dp, dp]),
        "ora_set_populations": (None, [vp, dp]),
        "ora_get_populations": (None, [vp, dp]),
        "ora_get_moments": (None, [vp, dp, dp]),
        "ora_set_body_force": (None, [vp, dp]),
        "ora_set_particles": (ctypes.c_int, [vp, i32, dp, dp, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, u64, u32, i32]),
        "ora_get_particles": (None, [vp, dp, dp]),
        "ora_get_particle_forces": (None, [vp, dp, dp]),
        "ora_set_particle_force": (None, [vp, dp]),
        "ora_set_pair_force": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double]),
        "ora_get_pair_forces": (None, [vp, dp]),
        "ora_radius": (ctypes.c_double, [vp]),
        "ora_vacf_config": (ctypes.c_int, [vp, i32, i32]),
        "ora_vacf_get": (None, [vp, dp, ctypes.POINTER(i64)]),
        "ora_step": (None, [vp, i32]),
        "ora_step_count": (i64, [vp]),
        "ora_observables": (None, [vp, dp]),
        "ora_num_threads": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def lattice(q: int = Q):
    """(e[q,3] int, w[q]) of the oracle's velocity set with q = 19 or 15."""
    lib = _load()
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    lib.ora_lattice_q(int(q), e.ctypes.data_as(ctypes.c_void_p), _dp(w))
    return e, w


def equilibrium(rho: float, u, q: int = Q) -> np.ndarray:
    lib = _load()
    u = _f64(u, (3,))
    out = np.zeros(q)
    lib.ora_equilibrium_q(int(q), float(rho), _dp(u), _dp(out))
    return out


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.zeros(4, dtype=np.uint32)
    lib.ora_philox4x32_10(c.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p),
                          out.ctypes.data_as(ctypes.c_void_p))
    return out


def gauss3(seed: int, step: int, particle: int, replica: int = 0, stream: int = 0) -> np.ndarray:
    lib = _load()
    z = np.zeros(3)
    lib.ora_gauss3(seed, step, particle, replica, stream, _dp(z))
    return z


def friction_force(mode, R, gamma, s, V, u8) -> np.ndarray:
    lib = _load()
    mode = FRICTION[mode] if isinstance(mode, str) else int(mode)
    s = _f64(s, (3,))
    V = _f64(V, (3,))
    u8 = _f64(u8, (8, 3))
    out = np.zeros(3)
    lib.ora_friction_force(mode, float(R), float(gamma), _dp(s), _dp(V), _dp(u8), _dp(out))
    return out


def num_threads() -> int:
    return int(_load().ora_num_threads())


class Sim:
    """One periodic box.  Arrays follow the oracle's layouts:
    populations [q, nz, ny, nx], velocity [3, nz, ny, nx], particles [n, 3];
    q = 19 or 15 velocities."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float, q: int = Q):
        self._lib = _load()
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        self.tau = tau
        self.q = int(q)
        self._h = self._lib.ora_create_q(nx, ny, nz, float(tau), self.q)
        if not self._h:
            raise ValueError("oracle: invalid grid or tau")
        self.np = 0

    def close(self):
        if self._h:
            self._lib.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_equilibrium(self, rho=None, u=None):
        rho = None if rho is None else _f64(rho, (self.ncell,))
        u = None if u is None else _f64(u, (3 * self.ncell,))
        self._lib.ora_set_equilibrium(self._h, _dp(rho), _dp(u))

    def set_populations(self, f):
        f = _f64(f, (self.q * self.ncell,))
        self._lib.ora_set_populations(self._h, _dp(f))

    def populations(self) -> np.ndarray:
        f = np.zeros((self.q,) + self.shape)
        self._lib.ora_get_populations(self._h, _dp(f))
        return f

    def moments(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        self._lib.ora_get_moments(self._h, _dp(rho), _dp(u))
        return rho, u

    def set_body_force(self, F=None):
        F = None if F is None else _f64(F, (3 * self.ncell,))
        self._lib.ora_set_body_force(self._h, _dp(F))

    def set_particles(self, r, v, mass=10.0, gamma=1.0, kT=0.0, radius=0.0, seed=0,
                      replica=0, friction="stokeslet"):
        r = _f64(r).reshape(-1, 3)
        v = _f64(v).reshape(-1, 3)
        if r.shape != v.shape:
            raise ValueError("r and v must have the same shape")
        mode = FRICTION[friction] if isinstance(friction, str) else int(friction)
        rc = self._lib.ora_set_particles(self._h, r.shape[0], _dp(r), _dp(v), float(mass),
                                         float(gamma), float(kT), float(radius), int(seed),
                                         int(replica), mode)
        if rc != 0:
            raise ValueError("oracle: invalid particle parameters")
        self.np = r.shape[0]

    def set_particle_force(self, F=None):
        """Constant force F_C on each particle, [n, 3] (None: none)."""
        self._fc = None if F is None else _f64(F, (self.np, 3))
        self._lib.ora_set_particle_force(self._h, _dp(self._fc))

    def set_pair_force(self, a_f: float, r_c: float = 1.0):
        """Soft pair repulsion a_f (1 - r/r_c) for r < r_c (a_f = 0: off)."""
        if self._lib.ora_set_pair_force(self._h, float(a_f), float(r_c)) != 0:
            raise ValueError("oracle: invalid pair force")

    def pair_forces(self) -> np.ndarray:
        F = np.zeros((self.np, 3))
        self._lib.ora_get_pair_forces(self._h, _dp(F))
        return F

    def particles(self):
        r = np.zeros((self.np, 3))
        v = np.zeros((self.np, 3))
        self._lib.ora_get_particles(self._h, _dp(r), _dp(v))
        return r, v

    def particle_forces(self):
        fh = np.zeros((self.np, 3))
        fr = np.zeros((self.np, 3))
        self._lib.ora_get_particle_forces(self._h, _dp(fh), _dp(fr))
        return fh, fr

    @property
    def radius(self) -> float:
        return float(self._lib.ora_radius(self._h))

    def vacf_config(self, max_lag: int, stride: int):
        if self._lib.ora_vacf_config(self._h, int(max_lag), int(stride)) != 0:
            raise ValueError("oracle: invalid VACF configuration")
        self._vacf_lags = int(max_lag) + 1

    def vacf(self):
        acc = np.zeros((self.np, self._vacf_lags))
        cnt = np.zeros(self._vacf_lags, dtype=np.int64)
        self._lib.ora_vacf_get(self._h, _dp(acc), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return acc, cnt

    def step(self, n: int = 1):
        self._lib.ora_step(self._h, int(n))

    @property
    def step_count(self) -> int:
        return int(self._lib.ora_step_count(self._h))

    def observables(self) -> np.ndarray:
        out = np.zeros(7)
        self._lib.ora_observables(self._h, _dp(out))
        return out
