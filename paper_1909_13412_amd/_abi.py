"""ctypes declarations of the C ABI in include/lbmbp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbmbp.so")

LBM_Q = 19
STATUS = {0: "LBM_OK", 1: "LBM_E_INVAL", 2: "LBM_E_DEVICE", 3: "LBM_E_STATE",
          4: "LBM_E_NONFINITE", 5: "LBM_E_UNSUPPORTED"}
STORAGE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
FRICTION = {"stokeslet": 0, "pointwise": 1, "bd": 2, "stokeslet2dx": 3, "stokeslet_cube": 4}

# every entry point of include/lbmbp.h
EXPORTS = [
    "lbm_lattice_bytes", "lbm_grid_scratch_bytes", "lbm_particle_scratch_bytes",
    "lbm_vacf_origin_bytes", "lbm_init", "lbm_set_equilibrium", "lbm_set_populations",
    "lbm_set_body_force", "lbm_get_populations", "lbm_get_moments", "particles_couple", "lbm_set_particle_force", "lbm_set_pair_force", "lbm_pair_forces", "lbm_particle_radius", "lbm_warnings",
    "lbm_particle_forces", "lbm_vacf_config", "lbm_vacf_counts", "lbm_step", "lbm_series_config",
    "lbm_series_count", "lbm_observables", "lbm_observables_noalloc",
    "lbm_profile_enable", "lbm_profile_read", "lbm_autotune", "lbm_stream_ceiling", "lbm_set_shape", "lbm_get_shape", "lbm_set_sweep_launch", "lbm_get_sweep_launch", "lbm_set_layout", "lbm_get_layout", "lbm_ens_set_layout", "lbm_ens_get_layout", "lbm_ens_set_sweep_launch", "lbm_ens_get_sweep_launch", "lbm_ens_set_shape", "lbm_get_step", "lbm_destroy",
    "lbm_tape_bytes", "lbm_record", "lbm_adjoint_work_bytes", "lbm_adjoint",
    "lbm_ens_bytes", "lbm_ens_init", "lbm_ens_use_graph", "lbm_ens_vacf_config",
    "lbm_ens_vacf_counts", "lbm_ens_step", "lbm_ens_autotune", "lbm_ens_stream_ceiling", "lbm_ens_get_shape", "lbm_ens_observables",
    "lbm_ens_get_populations", "lbm_ens_get_step", "lbm_ens_graph_replays", "lbm_ens_destroy",
    "lbm_status_string",
]
LBM_NUM_SHAPES = 10
LBM_ENS_GRAPH_STEPS = 16
# advisory bits of lbm_warnings
WARNINGS = {
    1: "radius beyond sqrt(3) dx (2 sqrt(3) dx for the (2 dx)^3 fit): the particle covers the fitting nodes",
    2: "radius beyond sqrt(3)/2 dx (sqrt(3) dx for the (2 dx)^3 fit): the fit's gain turns negative at the cell centre",
    4: "volume fraction above 0.1, beyond the range the method was checked for",
}


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("storage", ctypes.c_int32),
                ("f16_scale_log2", ctypes.c_int32), ("velocities", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ParticleDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("friction", ctypes.c_int32), ("mass", ctypes.c_double),
                ("gamma", ctypes.c_double), ("kT", ctypes.c_double), ("radius", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class EnsembleDesc(ctypes.Structure):
    _fields_ = [("nrep", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("f16_scale_log2", ctypes.c_int32), ("friction", ctypes.c_int32),
                ("mass", ctypes.c_double), ("gamma", ctypes.c_double), ("kT", ctypes.c_double),
                ("radius", ctypes.c_double), ("reserved", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ReplicaDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n", ctypes.c_int32), ("tau", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class LbmError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        super().__init__(f"{fn} failed: {STATUS.get(code, code)}")


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbmbp.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dp = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                            ctypes.c_void_p)
    gd, pd = ctypes.POINTER(GridDesc), ctypes.POINTER(ParticleDesc)
    sig = {
        "lbm_lattice_bytes": [gd, ctypes.POINTER(sz)],
        "lbm_grid_scratch_bytes": [gd, ctypes.POINTER(sz)],
        "lbm_particle_scratch_bytes": [gd, i32, ctypes.POINTER(sz)],
        "lbm_vacf_origin_bytes": [i32, i32, i32, ctypes.POINTER(sz)],
        "lbm_init": [gd, vp, vp, vp, vp, ctypes.POINTER(vp)],
        "lbm_set_equilibrium": [vp, dp, dp],
        "lbm_set_populations": [vp, dp],
        "lbm_set_body_force": [vp, ctypes.POINTER(ctypes.c_double)],
        "lbm_get_populations": [vp, dp],
        "lbm_get_moments": [vp, dp, dp],
        "particles_couple": [vp, pd, dp, dp, vp],
        "lbm_particle_forces": [vp, dp, dp],
        "lbm_set_particle_force": [vp, dp],
        "lbm_set_pair_force": [vp, ctypes.c_double, ctypes.c_double],
        "lbm_pair_forces": [vp, dp],
        "lbm_vacf_config": [vp, i32, i32, dp, dp],
        "lbm_vacf_counts": [vp, ctypes.POINTER(i64)],
        "lbm_step": [vp, i32],
        "lbm_series_config": [vp, i32, dp, i64],
        "lbm_series_count": [vp, ctypes.POINTER(i64)],
        "lbm_observables": [vp, ctypes.POINTER(ctypes.c_double)],
        "lbm_observables_noalloc": [vp, ctypes.POINTER(ctypes.c_double)],
        "lbm_profile_enable": [vp, i32],
        "lbm_profile_read": [vp, ctypes.POINTER(ctypes.c_double)],
        "lbm_autotune": [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
        "lbm_stream_ceiling": [vp, i32, i32, ctypes.POINTER(ctypes.c_double)],
        "lbm_set_shape": [vp, i32],
        "lbm_get_shape": [vp, ctypes.POINTER(i32)],
        "lbm_set_sweep_launch": [vp, i32, i32],
        "lbm_get_sweep_launch": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lbm_set_layout": [vp, i32],
        "lbm_get_layout": [vp, ctypes.POINTER(i32)],
        "lbm_ens_set_layout": [vp, i32],
        "lbm_ens_get_layout": [vp, i32, ctypes.POINTER(i32)],
        "lbm_ens_set_sweep_launch": [vp, i32, i32],
        "lbm_ens_set_shape": [vp, i32],
        "lbm_ens_get_sweep_launch": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lbm_warnings": [vp, ctypes.POINTER(ctypes.c_uint32)],
        "lbm_get_step": [vp, ctypes.POINTER(i64)],
        "lbm_destroy": [vp],
        "lbm_tape_bytes": [vp, i32, i32, ctypes.POINTER(sz)],
        "lbm_record": [vp, i32, i32, vp],
        "lbm_adjoint_work_bytes": [vp, ctypes.POINTER(sz)],
        "lbm_adjoint": [vp, vp, vp, dp, dp, dp, dp],
        "lbm_ens_bytes": [ctypes.POINTER(EnsembleDesc), ctypes.POINTER(ReplicaDesc),
                          ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "lbm_ens_init": [ctypes.POINTER(EnsembleDesc), ctypes.POINTER(ReplicaDesc), vp, vp, vp,
                         dp, dp, vp, ctypes.POINTER(vp)],
        "lbm_ens_use_graph": [vp, i32],
        "lbm_ens_vacf_config": [vp, i32, i32, dp, dp],
        "lbm_ens_vacf_counts": [vp, ctypes.POINTER(i64)],
        "lbm_ens_step": [vp, i32],
        "lbm_ens_autotune": [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
        "lbm_ens_stream_ceiling": [vp, i32, i32, ctypes.POINTER(ctypes.c_double)],
        "lbm_ens_observables": [vp, i32, ctypes.POINTER(ctypes.c_double)],
        "lbm_ens_get_populations": [vp, i32, dp],
        "lbm_ens_get_step": [vp, ctypes.POINTER(i64)],
        "lbm_ens_get_shape": [vp, ctypes.POINTER(i32)],
        "lbm_ens_graph_replays": [vp, ctypes.POINTER(i64)],
        "lbm_ens_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lbm_particle_radius.argtypes = [vp]
    lib.lbm_particle_radius.restype = ctypes.c_double
    lib.lbm_status_string.argtypes = [ctypes.c_int]
    lib.lbm_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(fn: str, code: int, allow=()) -> int:
    if code != 0 and code not in allow:
        raise LbmError(fn, code)
    return code
