"""Thin Python handle over the C ABI: torch provides device memory and the stream,
every step of the method runs in the HIP kernels of liblbmbp.so."""
from __future__ import annotations

import contextlib
import ctypes
import warnings as _warnings

import numpy as np
import torch

from . import _abi

Q = _abi.LBM_Q


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _device_f64(a, device, shape=None):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=torch.float64)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    t = t.contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


def _alloc_bytes(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator hands out 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class _StreamOrder:
    """Ordering between the caller's current stream and the context's stream
    (they differ only when a stream is passed in): work a call enqueues on the
    context's stream starts after what the caller had enqueued on its current
    stream, and tensors a call returns (and r, v) are safe to use on the
    caller's stream.  Waiting for an idle stream costs nothing, so contexts on
    their own streams, driven from one host thread, run concurrently."""

    def _same_stream(self) -> bool:
        return torch.cuda.current_stream(self.device).cuda_stream == self.stream.cuda_stream

    def _after_caller(self):
        if not self._same_stream():
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    @contextlib.contextmanager
    def _staging(self):
        # inputs and buffers are made on the context's stream
        if self._same_stream():
            yield
            return
        self._after_caller()
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            yield

    def _handover(self, *ts):
        if not self._same_stream():
            cur = torch.cuda.current_stream(self.device)
            cur.wait_stream(self.stream)
            for t in ts:
                if t is not None:
                    t.record_stream(cur)
        return ts[0] if len(ts) == 1 else ts

    @property
    def r(self):
        """Particle positions [n, 3] (device FP64, unwrapped), updated in place by every step."""
        return self._handover(self._r)

    @property
    def v(self):
        """Particle velocities [n, 3] (device FP64), updated in place by every step."""
        return self._handover(self._v)


class Tape:
    """Checkpoints of a recorded run (device buffer owned here)."""

    def __init__(self, buf: torch.Tensor, nsteps: int, every: int, n: int):
        self.buf, self.nsteps, self.every, self.n = buf, nsteps, every, n


class Lattice(_StreamOrder):
    """One periodic box of nx*ny*nz nodes with two population lattices.

    storage: "f64", "f32", "bf16" (shifted, round-to-nearest-even) or "f16"
    (shifted, scaled by 2^f16_scale_log2).  velocities: 19 (D3Q19) or 15 (D3Q15).
    """

    def __init__(self, nx: int, ny: int, nz: int, tau: float, storage: str = "f32",
                 f16_scale_log2: int = 16, device="cuda:0", stream: torch.cuda.Stream | None = None,
                 velocities: int = 19):
        self.lib = _abi.load()
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        self.tau = float(tau)
        self.storage = storage
        if velocities not in (15, 19):
            raise ValueError("velocities must be 19 or 15")
        self.q = int(velocities)
        self.desc = _abi.GridDesc(nx, ny, nz, float(tau), _abi.STORAGE[storage], int(f16_scale_log2),
                                  self.q, 0)
        sz = ctypes.c_size_t()
        _abi.check("lbm_lattice_bytes", self.lib.lbm_lattice_bytes(ctypes.byref(self.desc), ctypes.byref(sz)))
        self.lattice_bytes = sz.value
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with self._staging():
            self.pop_a = _alloc_bytes(self.lattice_bytes, self.device)
            self.pop_b = _alloc_bytes(self.lattice_bytes, self.device)
            _abi.check("lbm_grid_scratch_bytes",
                       self.lib.lbm_grid_scratch_bytes(ctypes.byref(self.desc), ctypes.byref(sz)))
            self.grid_scratch = _alloc_bytes(sz.value, self.device)
            ctx = ctypes.c_void_p()
            _abi.check("lbm_init", self.lib.lbm_init(ctypes.byref(self.desc), _ptr(self.pop_a),
                                                     _ptr(self.pop_b), _ptr(self.grid_scratch),
                                                     ctypes.c_void_p(self.stream.cuda_stream),
                                                     ctypes.byref(ctx)))
        self.ctx = ctx
        self.n = 0
        self._r = self._v = None
        self._vacf = None

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- fluid ------------------------------------------------------------
    def set_equilibrium(self, rho=None, u=None):
        with self._staging():
            self._rho_in = _device_f64(rho, self.device, (self.ncell,))
            self._u_in = _device_f64(u, self.device, (3 * self.ncell,))
            _abi.check("lbm_set_equilibrium",
                       self.lib.lbm_set_equilibrium(self.ctx, _ptr(self._rho_in), _ptr(self._u_in)))

    def set_populations(self, f):
        with self._staging():
            self._f_in = _device_f64(f, self.device, (self.q * self.ncell,))
            _abi.check("lbm_set_populations", self.lib.lbm_set_populations(self.ctx, _ptr(self._f_in)))

    def set_body_force(self, g=None):
        """Uniform body force (gx, gy, gz) on every node from the next step on."""
        arr = None if g is None else (ctypes.c_double * 3)(*[float(x) for x in g])
        _abi.check("lbm_set_body_force", self.lib.lbm_set_body_force(self.ctx, arr))

    def populations(self) -> torch.Tensor:
        with self._staging():
            out = torch.empty((self.q,) + self.shape, dtype=torch.float64, device=self.device)
            _abi.check("lbm_get_populations", self.lib.lbm_get_populations(self.ctx, _ptr(out)))
        return self._handover(out)

    def moments(self):
        with self._staging():
            rho = torch.empty(self.shape, dtype=torch.float64, device=self.device)
            u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
            _abi.check("lbm_get_moments", self.lib.lbm_get_moments(self.ctx, _ptr(rho), _ptr(u)))
        return self._handover(rho, u)

    # -- particles --------------------------------------------------------
    def particles_couple(self, r, v, mass=10.0, gamma=1.0, kT=0.0, radius=0.0, seed=0,
                         replica=0, friction="stokeslet"):
        with self._staging():
            self._couple(r, v, mass, gamma, kT, radius, seed, replica, friction)
        for bit, text in _abi.WARNINGS.items():
            if self.warnings & bit:
                _warnings.warn(f"particles_couple: {text} (R = {self.radius:.4g})", stacklevel=2)

    def _couple(self, r, v, mass, gamma, kT, radius, seed, replica, friction):
        r = _device_f64(r, self.device).reshape(-1, 3).clone()
        v = _device_f64(v, self.device).reshape(-1, 3).clone()
        n = r.shape[0]
        if v.shape != r.shape:
            raise ValueError("r and v must both be [n, 3]")
        pd = _abi.ParticleDesc(n, _abi.FRICTION[friction], float(mass), float(gamma), float(kT),
                               float(radius), int(seed), int(replica), 0)
        sz = ctypes.c_size_t()
        _abi.check("lbm_particle_scratch_bytes",
                   self.lib.lbm_particle_scratch_bytes(ctypes.byref(self.desc), n, ctypes.byref(sz)))
        scratch = _alloc_bytes(sz.value, self.device)
        _abi.check("particles_couple", self.lib.particles_couple(self.ctx, ctypes.byref(pd), _ptr(r),
                                                                 _ptr(v), _ptr(scratch)))
        self.n, self._r, self._v, self.pdesc, self._pscratch = n, r, v, pd, scratch
        self._vacf = None
        self.fh = torch.zeros((n, 3), dtype=torch.float64, device=self.device)
        self.fr = torch.zeros((n, 3), dtype=torch.float64, device=self.device)

    @property
    def warnings(self) -> int:
        """LBM_WARN_* bits of the attached particle set (advisory, not errors)."""
        f = ctypes.c_uint32()
        _abi.check("lbm_warnings", self.lib.lbm_warnings(self.ctx, ctypes.byref(f)))
        return f.value

    def set_particle_force(self, F=None):
        """Constant force F_C on each particle ([n, 3]; None detaches it)."""
        with self._staging():
            self._fext = None if F is None else _device_f64(F, self.device).reshape(self.n, 3).contiguous()
            _abi.check("lbm_set_particle_force", self.lib.lbm_set_particle_force(self.ctx, _ptr(self._fext)))

    def set_pair_force(self, a_f: float, r_c: float = 1.0):
        """Soft pair repulsion a_f (1 - r/r_c) for r < r_c (a_f = 0: off)."""
        _abi.check("lbm_set_pair_force", self.lib.lbm_set_pair_force(self.ctx, float(a_f), float(r_c)))

    def pair_forces(self) -> torch.Tensor:
        with self._staging():
            out = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
            _abi.check("lbm_pair_forces", self.lib.lbm_pair_forces(self.ctx, _ptr(out)))
        return self._handover(out)

    @property
    def radius(self) -> float:
        return float(self.lib.lbm_particle_radius(self.ctx))

    def particles(self):
        """(r, v) device tensors [n, 3]; updated in place by every step."""
        return self.r, self.v

    def particle_forces(self):
        with self._staging():
            _abi.check("lbm_particle_forces", self.lib.lbm_particle_forces(self.ctx, _ptr(self.fh), _ptr(self.fr)))
        return self._handover(self.fh, self.fr)

    # -- velocity autocorrelation ----------------------------------------
    def vacf_config(self, max_lag: int, stride: int):
        sz = ctypes.c_size_t()
        _abi.check("lbm_vacf_origin_bytes",
                   self.lib.lbm_vacf_origin_bytes(self.n, max_lag, stride, ctypes.byref(sz)))
        with self._staging():
            acc = torch.empty((max_lag + 1, self.n), dtype=torch.float64, device=self.device)  # lag-major
            origins = _alloc_bytes(sz.value, self.device)
            _abi.check("lbm_vacf_config",
                       self.lib.lbm_vacf_config(self.ctx, max_lag, stride, _ptr(acc), _ptr(origins)))
        self._vacf = (acc, origins, max_lag)

    def vacf(self):
        """(acc [n, max_lag+1] device FP64 (a view of the lag-major buffer),
        counts [max_lag+1] numpy int64)."""
        acc, _, max_lag = self._vacf
        cnt = np.zeros(max_lag + 1, dtype=np.int64)
        _abi.check("lbm_vacf_counts", self.lib.lbm_vacf_counts(
            self.ctx, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return self._handover(acc).t(), cnt

    # -- recorded observables --------------------------------------------
    def series_config(self, every: int, capacity: int):
        """Record {step, mass, fluid momentum, particle momentum} every `every`
        steps (fused into the step kernels) into a device buffer."""
        with self._staging():
            self._series = torch.zeros((max(int(capacity), 1), 8), dtype=torch.float64, device=self.device)
            _abi.check("lbm_series_config", self.lib.lbm_series_config(
                self.ctx, int(every), _ptr(self._series), int(capacity) if every > 0 else 0))

    def series(self) -> np.ndarray:
        """[count, 8] numpy array: step, mass, P_fluid (3), P_particle (3)."""
        n = ctypes.c_int64()
        _abi.check("lbm_series_count", self.lib.lbm_series_count(self.ctx, ctypes.byref(n)))
        return self._handover(self._series)[: n.value].cpu().numpy()

    # -- stepping and diagnostics ----------------------------------------
    def step(self, nsteps: int = 1):
        self._after_caller()
        _abi.check("lbm_step", self.lib.lbm_step(self.ctx, int(nsteps)))

    def observables(self, allow_nonfinite: bool = False) -> np.ndarray:
        self._after_caller()
        out = np.zeros(7)
        code = self.lib.lbm_observables(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        _abi.check("lbm_observables", code, allow=(4,) if allow_nonfinite else ())
        return out

    def observables_noalloc(self, allow_nonfinite: bool = False) -> np.ndarray:
        """The same sums through lbm_observables_noalloc (the library's own
        fixed device array instead of the context's scratch)."""
        self._after_caller()
        out = np.zeros(7)
        code = self.lib.lbm_observables_noalloc(self.ctx,
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        _abi.check("lbm_observables_noalloc", code, allow=(4,) if allow_nonfinite else ())
        return out

    def profile_enable(self, enable: bool = True):
        _abi.check("lbm_profile_enable", self.lib.lbm_profile_enable(self.ctx, int(bool(enable))))

    def profile_read(self) -> dict:
        """Accumulated per-kernel event timings since the last read (then reset)."""
        out = np.zeros(4)
        _abi.check("lbm_profile_read",
                   self.lib.lbm_profile_read(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return {"collide_ms": out[0], "collide_launches": int(out[1]),
                "particle_ms": out[2], "particle_launches": int(out[3])}

    def autotune(self, iters: int = 20):
        """Time the stream-collide launch options (configuration, block order,
        residency cap, storage layout) on this lattice (state values unchanged)
        and keep the fastest.  Returns (chosen configuration, best ms per launch
        of each configuration)."""
        self._after_caller()
        ms = np.zeros(_abi.LBM_NUM_SHAPES)
        chosen = ctypes.c_int32()
        _abi.check("lbm_autotune", self.lib.lbm_autotune(
            self.ctx, int(iters), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(chosen)))
        return chosen.value, ms

    def stream_ceiling(self, iters: int = 20, config: int = -1) -> float:
        """Milliseconds per launch of the stream-collide's data movement alone
        (pull and store, no arithmetic) in launch configuration `config`
        (-1: the current one); state unchanged (see lbm_stream_ceiling)."""
        self._after_caller()
        ms = ctypes.c_double()
        _abi.check("lbm_stream_ceiling", self.lib.lbm_stream_ceiling(self.ctx, int(config), int(iters), ctypes.byref(ms)))
        return ms.value

    def set_shape(self, k: int):
        """Use stream-collide launch configuration k (see lbm_set_shape)."""
        _abi.check("lbm_set_shape", self.lib.lbm_set_shape(self.ctx, int(k)))

    @property
    def launch_config(self) -> int:
        """The stream-collide launch configuration later steps use."""
        k = ctypes.c_int32()
        _abi.check("lbm_get_shape", self.lib.lbm_get_shape(self.ctx, ctypes.byref(k)))
        return k.value

    def set_sweep_launch(self, order: int = 0, waves_per_simd: int = 0):
        """Block order (0 node order, 1 per-XCD slabs) and residency cap (0, 6,
        5, 4, 3 or 2 waves per SIMD) of the stream-collide; same results."""
        _abi.check("lbm_set_sweep_launch",
                   self.lib.lbm_set_sweep_launch(self.ctx, int(order), int(waves_per_simd)))

    @property
    def sweep_launch(self):
        """(block order, residency cap in waves per SIMD) of later steps."""
        o, w = ctypes.c_int32(), ctypes.c_int32()
        _abi.check("lbm_get_sweep_launch",
                   self.lib.lbm_get_sweep_launch(self.ctx, ctypes.byref(o), ctypes.byref(w)))
        return o.value, w.value

    def set_layout(self, rows_per_group: int):
        """Storage layout of the lattice buffers: lattice rows grouped
        rows_per_group at a time (1, 2, 4, ..., 64, dividing ny), each
        population's rows of a group one run; the current populations move
        into it unchanged (same results in every layout)."""
        with self._staging():
            _abi.check("lbm_set_layout", self.lib.lbm_set_layout(self.ctx, int(rows_per_group)))

    @property
    def layout(self) -> int:
        """Rows per group of the lattice buffers' layout."""
        y = ctypes.c_int32()
        _abi.check("lbm_get_layout", self.lib.lbm_get_layout(self.ctx, ctypes.byref(y)))
        return y.value

    @property
    def step_count(self) -> int:
        s = ctypes.c_int64()
        _abi.check("lbm_get_step", self.lib.lbm_get_step(self.ctx, ctypes.byref(s)))
        return s.value

    # -- reverse mode -----------------------------------------------------
    def record(self, nsteps: int, every: int = 100) -> "Tape":
        """Take nsteps steps (exactly as step()) keeping a checkpoint every
        `every` steps, for a later adjoint()."""
        sz = ctypes.c_size_t()
        _abi.check("lbm_tape_bytes", self.lib.lbm_tape_bytes(self.ctx, int(nsteps), int(every),
                                                             ctypes.byref(sz)))
        with self._staging():
            tape = Tape(_alloc_bytes(sz.value, self.device), int(nsteps), int(every), self.n)
            _abi.check("lbm_record", self.lib.lbm_record(self.ctx, int(nsteps), int(every),
                                                         _ptr(tape.buf)))
        self._tape = tape
        return tape

    def adjoint(self, tape: "Tape", adj_pop=None, adj_r=None, adj_v=None) -> dict:
        """Gradient of J = <adj_pop, f^N> + <adj_r, r^N> + <adj_v, V^N> of the
        recorded run with respect to its initial populations ("pop", canonical
        [19, nz, ny, nx]), particle positions and velocities ("r", "v", [n, 3])
        and the parameters ("params": gamma, tau, M, kT).  Missing cotangents
        are zero."""
        if tape is not getattr(self, "_tape", None):
            raise ValueError("adjoint() needs the tape of this lattice's last record()")
        with self._staging():
            pop = torch.zeros((self.q,) + self.shape, dtype=torch.float64, device=self.device)
            if adj_pop is not None:
                pop.copy_(_device_f64(adj_pop, self.device).reshape(pop.shape))
            n = tape.n
            r = torch.zeros((n, 3), dtype=torch.float64, device=self.device)
            v = torch.zeros((n, 3), dtype=torch.float64, device=self.device)
            if adj_r is not None:
                r.copy_(_device_f64(adj_r, self.device).reshape(n, 3))
            if adj_v is not None:
                v.copy_(_device_f64(adj_v, self.device).reshape(n, 3))
            params = torch.zeros(4, dtype=torch.float64, device=self.device)
            sz = ctypes.c_size_t()
            _abi.check("lbm_adjoint_work_bytes",
                       self.lib.lbm_adjoint_work_bytes(self.ctx, ctypes.byref(sz)))
            work = _alloc_bytes(sz.value, self.device)
            _abi.check("lbm_adjoint", self.lib.lbm_adjoint(
                self.ctx, _ptr(tape.buf), _ptr(work), _ptr(pop), _ptr(r if n else None),
                _ptr(v if n else None), _ptr(params)))
            self._adj_keep = (pop, r, v, params, work)  # alive until the stream reaches them
        pop, r, v, params = self._handover(pop, r, v, params)
        return {"pop": pop, "r": r, "v": v, "params": params}


class Ensemble(_StreamOrder):
    """Many independent periodic boxes stepped together (one launch per kernel
    per step, replayed from a captured graph of several steps).

    replicas: list of dicts with keys nx, ny, nz, r [n, 3], v [n, 3], tau, seed,
    replica (Philox third counter word).  Shared: storage, mass, gamma, kT,
    radius, friction."""

    def __init__(self, replicas, storage="f32", mass=10.0, gamma=1.0, kT=0.0, radius=0.0,
                 friction="stokeslet", f16_scale_log2=16, device="cuda:0", stream=None):
        self.lib = _abi.load()
        self.device = torch.device(device)
        self.nrep = len(replicas)
        self.desc = _abi.EnsembleDesc(self.nrep, _abi.STORAGE[storage], int(f16_scale_log2),
                                      _abi.FRICTION[friction], float(mass), float(gamma),
                                      float(kT), float(radius), 0, 0)
        reps = (_abi.ReplicaDesc * self.nrep)()
        rs, vs = [], []
        for k, rd in enumerate(replicas):
            r = np.asarray(rd["r"], dtype=np.float64).reshape(-1, 3)
            v = np.asarray(rd["v"], dtype=np.float64).reshape(-1, 3)
            reps[k] = _abi.ReplicaDesc(int(rd["nx"]), int(rd["ny"]), int(rd["nz"]), r.shape[0],
                                       float(rd["tau"]), int(rd["seed"]), int(rd.get("replica", k)), 0)
            rs.append(r)
            vs.append(v)
        self.reps = reps
        self.shapes = [(int(rd["nz"]), int(rd["ny"]), int(rd["nx"])) for rd in replicas]
        self.offsets = np.concatenate([[0], np.cumsum([len(r) for r in rs])])
        self.n = int(self.offsets[-1])
        lat, scr = ctypes.c_size_t(), ctypes.c_size_t()
        _abi.check("lbm_ens_bytes", self.lib.lbm_ens_bytes(ctypes.byref(self.desc), reps,
                                                           ctypes.byref(lat), ctypes.byref(scr)))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with self._staging():
            self.pop_a = _alloc_bytes(lat.value, self.device)
            self.pop_b = _alloc_bytes(lat.value, self.device)
            self.scratch = _alloc_bytes(scr.value, self.device)
            self._r = _device_f64(np.concatenate(rs), self.device).clone()
            self._v = _device_f64(np.concatenate(vs), self.device).clone()
            ctx = ctypes.c_void_p()
            _abi.check("lbm_ens_init", self.lib.lbm_ens_init(
                ctypes.byref(self.desc), reps, _ptr(self.pop_a), _ptr(self.pop_b), _ptr(self.scratch),
                _ptr(self._r), _ptr(self._v), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self.ctx = ctx
        self._vacf = None

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            self.lib.lbm_ens_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_graph(self, use: bool = True):
        _abi.check("lbm_ens_use_graph", self.lib.lbm_ens_use_graph(self.ctx, int(bool(use))))

    def step(self, nsteps: int = 1):
        self._after_caller()
        _abi.check("lbm_ens_step", self.lib.lbm_ens_step(self.ctx, int(nsteps)))

    @property
    def graph_replays(self) -> int:
        n = ctypes.c_int64()
        _abi.check("lbm_ens_graph_replays", self.lib.lbm_ens_graph_replays(self.ctx, ctypes.byref(n)))
        return n.value

    def autotune(self, iters: int = 10):
        self._after_caller()
        ms = np.zeros(_abi.LBM_NUM_SHAPES)
        chosen = ctypes.c_int32()
        _abi.check("lbm_ens_autotune", self.lib.lbm_ens_autotune(
            self.ctx, int(iters), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(chosen)))
        return chosen.value, ms

    def stream_ceiling(self, iters: int = 20, config: int = -1) -> float:
        """Milliseconds per launch of the ensemble stream-collide's data movement
        alone in launch configuration `config` (-1: the current one); state
        unchanged (see lbm_ens_stream_ceiling)."""
        self._after_caller()
        ms = ctypes.c_double()
        _abi.check("lbm_ens_stream_ceiling",
                   self.lib.lbm_ens_stream_ceiling(self.ctx, int(config), int(iters), ctypes.byref(ms)))
        return ms.value

    def set_layout(self, rows_per_group: int):
        """Storage layout of every box (see Lattice.set_layout): each box takes
        the largest power of two not above rows_per_group that divides its ny;
        the populations move into it unchanged."""
        self._after_caller()
        _abi.check("lbm_ens_set_layout", self.lib.lbm_ens_set_layout(self.ctx, int(rows_per_group)))

    def layout(self, k: int) -> int:
        """Rows per group of replica k's lattice layout."""
        y = ctypes.c_int32()
        _abi.check("lbm_ens_get_layout", self.lib.lbm_ens_get_layout(self.ctx, int(k), ctypes.byref(y)))
        return y.value

    @property
    def launch_config(self) -> int:
        """The stream-collide launch configuration later steps use."""
        k = ctypes.c_int32()
        _abi.check("lbm_ens_get_shape", self.lib.lbm_ens_get_shape(self.ctx, ctypes.byref(k)))
        return k.value

    def set_launch_config(self, k: int):
        """Stream-collide launch configuration k (0..7) of later steps; same
        results, drops the captured graph."""
        _abi.check("lbm_ens_set_shape", self.lib.lbm_ens_set_shape(self.ctx, int(k)))

    def set_sweep_launch(self, order: int = 0, waves_per_simd: int = 0):
        """Block order and residency cap of the ensemble stream-collide (see
        Lattice.set_sweep_launch); same results, drops the captured graph."""
        _abi.check("lbm_ens_set_sweep_launch",
                   self.lib.lbm_ens_set_sweep_launch(self.ctx, int(order), int(waves_per_simd)))

    @property
    def sweep_launch(self):
        """(block order, residency cap in waves per SIMD) of later steps."""
        o, w = ctypes.c_int32(), ctypes.c_int32()
        _abi.check("lbm_ens_get_sweep_launch",
                   self.lib.lbm_ens_get_sweep_launch(self.ctx, ctypes.byref(o), ctypes.byref(w)))
        return o.value, w.value

    def vacf_config(self, max_lag: int, stride: int):
        sz = ctypes.c_size_t()
        _abi.check("lbm_vacf_origin_bytes",
                   self.lib.lbm_vacf_origin_bytes(self.n, max_lag, stride, ctypes.byref(sz)))
        with self._staging():
            acc = torch.empty((max_lag + 1, self.n), dtype=torch.float64, device=self.device)  # lag-major
            origins = _alloc_bytes(sz.value, self.device)
            _abi.check("lbm_ens_vacf_config",
                       self.lib.lbm_ens_vacf_config(self.ctx, max_lag, stride, _ptr(acc), _ptr(origins)))
        self._vacf = (acc, origins, max_lag)

    def vacf(self):
        acc, _, max_lag = self._vacf
        cnt = np.zeros(max_lag + 1, dtype=np.int64)
        _abi.check("lbm_ens_vacf_counts", self.lib.lbm_ens_vacf_counts(
            self.ctx, cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return self._handover(acc).t(), cnt  # [all particles, max_lag+1] view of the lag-major buffer

    def particles(self, k: int):
        a, b = int(self.offsets[k]), int(self.offsets[k + 1])
        return self.r[a:b], self.v[a:b]

    def populations(self, k: int) -> torch.Tensor:
        with self._staging():
            out = torch.empty((Q,) + self.shapes[k], dtype=torch.float64, device=self.device)
            _abi.check("lbm_ens_get_populations", self.lib.lbm_ens_get_populations(self.ctx, int(k), _ptr(out)))
        return self._handover(out)

    def observables(self, k: int) -> np.ndarray:
        self._after_caller()
        out = np.zeros(7)
        _abi.check("lbm_ens_observables", self.lib.lbm_ens_observables(
            self.ctx, int(k), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out
