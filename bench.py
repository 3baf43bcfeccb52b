#!/usr/bin/env python3
"""Benchmark of the coupled lattice-Boltzmann / Brownian-particle step on one MI355X.

A step is the whole hot path: VACF sample, particle coupling (gather at the eight
neighbour nodes, Stokeslet fit, Philox Brownian force, reaction-force spreading,
Langevin update) and the fused stream-collide with forcing; every 10th step also
records the FP64 mass and momentum sums (fused into the same kernels).  Workload (default):
256^3 periodic box, tau 0.6, 4096 particles (M 10, gamma 1, R 0.5, kT 1e-4), VACF with
lags up to 500 and origins every 10 steps; synthetic seeded initial state.

Prints ONE JSON line.  `value` is whole-step MLUPS (nodes x steps / s / 1e6) with
FP32 population storage; `variants` repeats the timing for shifted BF16 and FP16
storage; `roofline` prices the stream-collide kernel (the dominant one) against
the 8 TB/s HBM peak from HIP-event timings of every launch in a second timed
region (events add a few microseconds per step, so `value` comes from a region
without them);
`cpu_baseline` times the FP64 oracle on a few steps of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ELEM = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
METRIC = "MLUPS & % HBM roofline, FP32 vs shifted-BF16 storage at stated VACF error"


PMC_PROFILE = os.path.join(ROOT, "profiles", "k_stream_collide_suspension256.md")


def kernel_source_hash() -> str:
    """SHA-256 over the sources the stream-collide kernel is compiled from (its
    header, the codecs, the lattice constants) and the hipcc flags: the PMC
    traffic figure is reported only while this matches the profiled build."""
    import hashlib

    from paper_1909_13412_amd import build as hip_build

    h = hashlib.sha256()
    for name in ("collide.hpp", "codec.hpp", "velocities.hpp"):
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1909_13412_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(hip_build.HIPCC_FLAGS).encode())
    return h.hexdigest()


def pmc_traffic(storage: str):
    """HBM bytes per stream-collide launch from the committed counter profile:
    the L2's read requests to memory counted by size (32 x TCC_EA0_RDREQ_32B +
    64 x TCC_EA0_RDREQ_64B + 128 x TCC_EA0_RDREQ_128B) plus its write requests
    (64 x TCC_EA0_WRREQ_64B + 32 x the rest), the rule that gives a plain
    device copy's bytes exactly; None when the kernel sources changed since
    the counters were taken."""
    try:
        with open(PMC_PROFILE) as fh:
            line = next(ln for ln in fh if ln.strip().startswith("PMC_TRAFFIC "))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.strip()[len("PMC_TRAFFIC "):])
    if rec.get("source_sha256") != kernel_source_hash() or not rec.get(storage):
        return None
    c = rec[storage]
    return float(c["read_bytes"] + c["write_bytes"])


def parse_variant(name: str):
    """'bf16' -> ('bf16', 19); 'f32q15' -> ('f32', 15): storage and velocity set."""
    if name.endswith("q15"):
        return name[:-3], 15
    return name, 19


def collide_bytes_per_node(storage: str, q: int = 19) -> float:
    """Algorithmic bytes of one stream-collide node update: q population loads
    and q stores, plus the one-bit forcing flag."""
    return 2 * q * ELEM[storage] + 1.0 / 8.0


SERIES_EVERY = 10  # FP64 mass/momentum sums recorded inside the step kernels every 10 steps


def make_lattice(w, storage, device="cuda:0", series_capacity=0, q=19):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import workload_particles

    L = w["L"]
    lat = Lattice(L, L, L, w["tau"], storage=storage, device=device, velocities=q)
    r, v = workload_particles(w["name"])
    lat.particles_couple(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                         seed=w["seed"], friction=w.get("friction", "stokeslet"))
    lat.vacf_config(w["max_lag"], w["stride"])
    if series_capacity > 0:
        lat.series_config(SERIES_EVERY, series_capacity)
    return lat


def time_storage(w, variant, steps, warmup, prof_steps, pair=None, repeats=0):
    """Autotune the stream-collide launch shape, time `steps` whole steps with
    nothing but the kernels on the stream (-> MLUPS), then time `prof_steps`
    more with HIP events around every kernel launch (-> per-kernel durations;
    the events themselves add a few microseconds per step, so they stay out
    of the first region)."""
    import torch

    storage, q = parse_variant(variant)
    lat = make_lattice(w, storage, q=q,
                       series_capacity=(2 * warmup + steps + prof_steps) // SERIES_EVERY + 2)
    if pair is not None:
        lat.set_pair_force(*pair)
    lat.step(warmup)
    torch.cuda.synchronize()
    shape, shape_ms = lat.autotune(20)
    order, cap = lat.sweep_launch
    rows = lat.layout
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # further regions of the same `steps` steps, for the spread of the figure
    more = []
    for _ in range(repeats):
        a = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        more.append(w["L"] ** 3 * steps / (time.perf_counter() - a) / 1e6)
    lat.profile_enable(True)
    lat.profile_read()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lat.step(prof_steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = lat.profile_read()
    lat.profile_enable(False)
    # the same data movement without the arithmetic, same launch configuration
    ceil_ms = lat.stream_ceiling(20)
    obs = lat.observables()
    ncell = w["L"] ** 3
    coll_ms = prof["collide_ms"] / max(prof["collide_launches"], 1)
    part_ms = prof["particle_ms"] / max(prof["particle_launches"], 1)
    achieved = ncell * collide_bytes_per_node(storage, q) / (coll_ms * 1e-3) / 1e9
    res = {
        "storage": storage,
        "velocities": q,
        "mlups": ncell * steps / (t1 - t0) / 1e6,
        "mlups_more_regions": more,
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "profiled_ms_per_step": (t3 - t2) * 1e3 / prof_steps,
        "collide_ms": coll_ms,
        "particle_phase_ms": part_ms,
        "collide_GBs": achieved,
        "collide_frac": achieved / HBM_PEAK_GBS,
        "collide_shape": shape,
        "collide_order": order,
        "collide_waves_per_simd_cap": cap,
        "layout_rows_per_group": rows,
        "stream_only_ms": ceil_ms,
        "of_stream_only": ceil_ms / coll_ms,
        "autotune_ms": [round(float(x), 5) for x in shape_ms],
        "mass": obs[0],
    }
    del lat
    torch.cuda.empty_cache()
    return res


def copy_probe(nbytes, reps=20):
    """Plain device copy of `nbytes` (one lattice's worth): the practical
    read+write ceiling next to the stream-collide, and the reference kernel
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": round(ms, 5),
            "GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_fixture(name: str):
    """The FP64 oracle's long run of a workload (written by
    tests/golden/make_oracle_fixtures.py from the oracle alone), or None."""
    path = os.path.join(GOLDEN, f"oracle_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def vacf_errors(c, c_ref, tail, per_particle=None):
    """Errors of a velocity autocorrelation C(l) = <V(t0).V(t0 + l)> (section
    2.1; lags 0..L, not normalised) against the reference curve c_ref:
    c0_rel, the relative error of C(0) (the particles' kinetic temperature);
    vacf_abs_err, max over lags of |C - C_ref| / C_ref(0) (every lag, C(0)
    included, in units of the reference's C(0): the "within 1%" figure);
    vacf_err, the same between the curves each normalised by its own C(0)
    (shape only).  Over the tail window tail = (lo, hi): tail_integral_rel,
    the relative error of sum C(l) (the tail's share of the diffusion
    coefficient); tail_amplitude_rel, the relative error of the least-squares
    amplitude B of C(l) = B l^(-3/2) (the long-time tail of section 3);
    tail_window_err, max |C - C_ref| over the window / max |C_ref| there.
    per_particle ([n, L + 1] per-particle curves of the run under test):
    tail_integral_se_rel, the standard error of the tail sum over particles,
    relative: the estimator's own sampling uncertainty, against which the
    tail errors are to be read."""
    import numpy as np

    c = np.asarray(c, dtype=np.float64)
    c_ref = np.asarray(c_ref, dtype=np.float64)
    lo, hi = tail
    w = slice(lo, hi + 1)
    lag = np.arange(lo, hi + 1, dtype=np.float64)
    basis = lag ** -1.5

    def amp(x):
        return float(np.sum(x[w] * basis) / np.sum(basis * basis))

    out = {
        "c0_rel": float(abs(c[0] - c_ref[0]) / abs(c_ref[0])),
        "vacf_abs_err": float(np.max(np.abs(c - c_ref)) / abs(c_ref[0])),
        "vacf_err": float(np.max(np.abs(c / c[0] - c_ref / c_ref[0]))),
        "tail_window": [lo, hi],
        "tail_integral_rel": float(abs(c[w].sum() - c_ref[w].sum()) / abs(c_ref[w].sum())),
        "tail_amplitude_rel": float(abs(amp(c) - amp(c_ref)) / abs(amp(c_ref))),
        "tail_window_err": float(np.max(np.abs(c[w] - c_ref[w])) / np.max(np.abs(c_ref[w]))),
    }
    if per_particle is not None:
        t = np.asarray(per_particle)[:, w].sum(axis=1)
        out["tail_integral_se_rel"] = float(np.std(t, ddof=1) / np.sqrt(len(t)) / abs(t.mean()))
    return out


# Tail windows of the precision study: past the Brownian relaxation time
# M / gamma = 10 steps, up to a lag where the reference curve is still a few
# per mille of C(0).
TAIL = {"vacf128": (50, 500), "suspension256": (50, 250), "fig2thermal100": (100, 1000)}


def run_precision(w, storage, steps, every):
    """One storage on a workload: VACF curve C(l) and the FP64 sums every
    `every` steps (as the oracle fixture records them)."""
    import numpy as np
    import torch

    lat = make_lattice(w, storage)
    rows = []
    done = 0
    while True:
        o = lat.observables()
        rows.append([float(done)] + [float(x) for x in o])
        if done >= steps:
            break
        k = min(every, steps - done)
        lat.step(k)
        done += k
    acc, cnt = lat.vacf()
    acc = acc.cpu().numpy() / np.maximum(np.asarray(cnt), 1)  # per-particle curves
    c = acc.mean(axis=0)
    del lat
    torch.cuda.empty_cache()
    return c, np.array(rows), np.asarray(cnt), acc


def series_errors(ser, ref):
    """Fluid and particle momentum of the FP64 sums against the oracle's, each
    normalised by the largest reference value over the run, and the fluid
    mass relative error."""
    import numpy as np

    ref = np.asarray(ref)
    return {
        "fluid_mass_rel": float(np.max(np.abs(ser[:, 1] - ref[:, 1]) / ref[:, 1])),
        "fluid_momentum_err": float(np.max(np.abs(ser[:, 2:5] - ref[:, 2:5])) /
                                    np.max(np.abs(ref[:, 2:5]))),
        "particle_momentum_err": float(np.max(np.abs(ser[:, 5:8] - ref[:, 5:8])) /
                                       np.max(np.abs(ref[:, 5:8]))),
    }


def precision_study(w, storages=("f64", "f32", "bf16", "f16")):
    """VACF and momentum error of each storage against the FP64 oracle's own
    run of the same workload and seed (tests/golden/oracle_<workload>.json)."""
    import numpy as np

    ref = oracle_fixture(w["name"])
    if ref is None:
        return {"reference": f"missing oracle fixture for {w['name']}"}
    steps, every = ref["steps"], ref["series_every"]
    c_ref = np.asarray(ref["vacf"])
    out = {"reference": f"FP64 oracle, {steps} steps (tests/golden/oracle_{w['name']}.json)",
           "steps": steps, "max_lag": ref["max_lag"]}
    for s in storages:
        t0 = time.perf_counter()
        c, ser, cnt, per = run_precision(w, s, steps, every)
        rec = vacf_errors(c, c_ref, TAIL[w["name"]], per)
        rec.update(series_errors(ser, ref["series"]))
        rec["counts_match"] = bool(np.array_equal(cnt, ref["vacf_counts"]))
        rec["gpu_seconds"] = round(time.perf_counter() - t0, 2)
        out[s] = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in rec.items()}
    return out


def time_ensemble(steps, warmup):
    """The 64-replica ensemble (edges 48..96, tau 0.8, 8 particles each, FP32,
    VACF on): whole-ensemble MLUPS with graph-replayed steps and with plain
    launches, and the ensemble-averaged VACF.  The graph-replayed run takes
    exactly `steps` steps from the initial state (the autotuner leaves the
    state untouched), so at 5000 steps its smallest and largest boxes are
    compared with the oracle's own run of that box alone
    (tests/golden/oracle_ensemble64_edges.json)."""
    import numpy as np
    import torch

    from paper_1909_13412_amd import Ensemble
    from paper_1909_13412_amd.inputs import ENSEMBLE64, ensemble_replicas

    w = ENSEMBLE64
    reps = ensemble_replicas(w["replicas"], w["sizes"], w["n"], w["tau"], w["kT"], w["mass"], w["seed"])
    nodes = sum(r["nx"] * r["ny"] * r["nz"] for r in reps)
    out = {"workload": "ensemble64", "replicas": len(reps), "nodes": nodes,
           "particles": sum(len(r["r"]) for r in reps), "storage": w["storage"], "steps": steps}
    for use_graph in (True, False):
        ens = Ensemble(reps, storage=w["storage"], mass=w["mass"], gamma=w["gamma"], kT=w["kT"])
        ens.vacf_config(w["max_lag"], w["stride"])
        ens.use_graph(use_graph)
        shape, tune_ms = ens.autotune(10)
        if use_graph:
            # the stream-collide (autotuner timing) against the same data
            # movement without the arithmetic, same configuration
            ceil = ens.stream_ceiling(10)
            out["collide_ms"] = round(float(tune_ms[shape]), 5)
            out["collide_frac"] = round(nodes * collide_bytes_per_node(w["storage"]) / (tune_ms[shape] * 1e-3)
                                        / 1e9 / HBM_PEAK_GBS, 4)
            out["stream_only_ms"] = round(ceil, 5)
            out["of_stream_only"] = round(ceil / float(tune_ms[shape]), 4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "graph" if use_graph else "plain"
        out[f"mlups_{key}"] = round(nodes * steps / dt / 1e6, 1)
        out[f"ms_per_step_{key}"] = round(dt * 1e3 / steps, 5)
        out["launch_shape"] = shape
        out["launch_order"], out["launch_waves_per_simd_cap"] = ens.sweep_launch
        if use_graph:
            out["graph_replays"] = ens.graph_replays
            acc, cnt = ens.vacf()
            acc = acc.cpu().numpy()
            c = acc.sum(0) / (acc.shape[0] * np.maximum(cnt, 1))
            out["vacf_norm_lag"] = {str(l): round(float(c[l] / c[0]), 5) for l in (0, 10, 50, 100, 500)}
            ref = oracle_fixture("ensemble64_edges")
            if ref is not None and ref["steps"] == steps:
                checks = []
                for rec in ref["replicas"]:
                    k = rec["index"]
                    rows = acc[w["n"] * k: w["n"] * (k + 1)] / np.maximum(cnt, 1)
                    e = vacf_errors(rows.mean(axis=0), rec["vacf"], (50, 250), rows)
                    _, vk = ens.particles(k)
                    e["final_v_err"] = float(np.max(np.abs(vk.cpu().numpy() - np.asarray(rec["final_v"]))) /
                                             np.max(np.abs(rec["final_v"])))
                    checks.append({"replica": k, "edge": rec["edge"],
                                   **{kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv)
                                      for kk, vv in e.items()}})
                out["vs_oracle"] = checks
            # every box: the ensemble-averaged VACF over all particles against
            # the average of the oracle's single-box runs, and how many boxes
            # still follow the oracle's trajectories (final velocities 1e-3)
            full = oracle_fixture("ensemble64_all")
            if full is not None and full["steps"] == steps:
                recs = sorted(full["replicas"], key=lambda r: r["index"])
                per = acc / np.maximum(cnt, 1)
                c_ref = np.mean([np.asarray(r["vacf"]) for r in recs], axis=0)
                e = vacf_errors(per.mean(axis=0), c_ref, (50, 250), per)
                follow = 0
                for r in recs:
                    _, vk = ens.particles(r["index"])
                    fv = np.asarray(r["final_v"])
                    follow += int(np.max(np.abs(vk.cpu().numpy() - fv)) / np.max(np.abs(fv)) < 1e-3)
                out["vs_oracle_all_boxes"] = {
                    "boxes": len(recs), "boxes_following_oracle_trajectories": follow,
                    **{kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv) for kk, vv in e.items()}}
        del ens
        torch.cuda.empty_cache()
    return out


def _msd_forward(storage, gamma, tau, v_shift=None, grad=False):
    """The 64^3 reverse-mode workload: loss J = mean over particles of
    |r^N - r^0|^2 (unwrapped positions) after its steps; with grad, also the
    adjoint's dJ/d(gamma, tau) and dJ/dV^0 [n, 3]."""
    import numpy as np

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import ADJOINT64, particle_positions, particle_velocities

    w = ADJOINT64
    L, n = w["L"], w["n"]
    r0 = particle_positions(n, L, w["seed"])
    v0 = particle_velocities(n, w["kT"] / w["mass"], w["seed"])
    if v_shift is not None:
        v0 = v0 + v_shift
    lat = Lattice(L, L, L, tau, storage=storage)
    lat.particles_couple(r0, v0, mass=w["mass"], gamma=gamma, kT=w["kT"], seed=w["seed"])
    tape = lat.record(w["steps"], w["every"]) if grad else None
    if not grad:
        lat.step(w["steps"])
    rN = lat.r.cpu().numpy()
    J = float(np.mean(np.sum((rN - r0) ** 2, axis=1)))
    if not grad:
        return J, None, None
    g = lat.adjoint(tape, None, 2.0 * (rN - r0) / n, None)
    return J, g["params"].cpu().numpy()[:2], g["v"].cpu().numpy()


def time_adjoint(steps, warmup):
    """Reverse mode on the 64^3 / 16-particle workload (tau 0.8, FP32, kT
    1e-4, 2000 steps, a checkpoint every 100): the recorded forward and the
    adjoint sweep (segment recompute plus the reverse step kernels) against
    plain forward steps; then the gradient of the mean-squared displacement
    of the 16 particles with respect to gamma, tau and the 16 x 3 initial
    velocities, from the FP32 and FP64 adjoints, beside central finite
    differences of the FP64 forward with h = 1e-3 and 1e-6 (absolute for
    gamma and tau, times sqrt(kT/M) for the velocities).  The Stokeslet fit
    changes its node set when a particle crosses a cell face, so the loss is
    only piecewise smooth and the wide difference can straddle a crossing."""
    import numpy as np
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import ADJOINT64, particle_positions, particle_velocities

    w = ADJOINT64
    L, n, every = w["L"], w["n"], w["every"]
    lat = Lattice(L, L, L, w["tau"], storage=w["storage"])
    r = particle_positions(n, L, w["seed"])
    v = particle_velocities(n, w["kT"] / w["mass"], w["seed"])
    lat.particles_couple(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], seed=w["seed"])
    cr = torch.ones((n, 3), dtype=torch.float64, device=lat.device)
    tape = lat.record(2 * every, every)
    lat.adjoint(tape, None, cr, None)
    lat.step(warmup)
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    _, t_fwd = timed(lambda: lat.step(steps))
    tape, t_rec = timed(lambda: lat.record(steps, every))
    g, t_adj = timed(lambda: lat.adjoint(tape, None, cr, None))
    work = lat._adj_keep[4].numel()
    out = {"workload": "adjoint64", "box": [L] * 3, "tau": w["tau"], "particles": n,
           "storage": w["storage"], "steps": steps, "checkpoint_every": every,
           "tape_MB": round(tape.buf.numel() / 2**20, 1), "work_MB": round(work / 2**20, 1),
           "forward_ms_per_step": round(t_fwd * 1e3 / steps, 5),
           "record_ms_per_step": round(t_rec * 1e3 / steps, 5),
           "adjoint_ms_per_step": round(t_adj * 1e3 / steps, 5),
           "adjoint_over_forward": round(t_adj / t_fwd, 3)}
    del lat, tape
    torch.cuda.empty_cache()
    if steps != w["steps"]:
        return out
    # gradient of the mean-squared displacement
    t0 = time.perf_counter()
    J32, p32, v32 = _msd_forward("f32", w["gamma"], w["tau"], grad=True)
    J64, p64, v64 = _msd_forward("f64", w["gamma"], w["tau"], grad=True)
    sv = np.sqrt(w["kT"] / w["mass"])
    fd = {}
    for h in (1e-3, 1e-6):
        def J(dg=0.0, dt=0.0, dv=None):
            return _msd_forward("f64", w["gamma"] + dg, w["tau"] + dt, dv)[0]

        gv = np.zeros((n, 3))
        for i in range(n):
            for k in range(3):
                e = np.zeros((n, 3))
                e[i, k] = h * sv
                gv[i, k] = (J(dv=e) - J(dv=-e)) / (2 * h * sv)
        fd[h] = ((J(dg=h) - J(dg=-h)) / (2 * h), (J(dt=h) - J(dt=-h)) / (2 * h), gv)

    def rel(a, b):
        return float(f"{abs(a - b) / abs(b):.3g}")

    def vrel(a, b):
        return float(f"{np.max(np.abs(a - b)) / np.max(np.abs(b)):.3g}")

    out["msd"] = {
        "loss": "mean over the 16 particles of |r(2000) - r(0)|^2 (unwrapped)",
        "J_f32": J32, "J_f64": J64,
        "adjoint_f32": {"gamma": float(p32[0]), "tau": float(p32[1]),
                        "v0": [[float(f"{x:.6g}") for x in row] for row in v32]},
        "adjoint_f64": {"gamma": float(p64[0]), "tau": float(p64[1]),
                        "v0": [[float(f"{x:.6g}") for x in row] for row in v64]},
        "fd_f64": {str(h): {"gamma": fd[h][0], "tau": fd[h][1],
                            "v0": [[float(f"{x:.6g}") for x in row] for row in fd[h][2]]}
                   for h in fd},
        "f32_vs_fd_1e-6": {"gamma": rel(p32[0], fd[1e-6][0]), "tau": rel(p32[1], fd[1e-6][1]),
                           "v0": vrel(v32, fd[1e-6][2])},
        "f64_vs_fd_1e-6": {"gamma": rel(p64[0], fd[1e-6][0]), "tau": rel(p64[1], fd[1e-6][1]),
                           "v0": vrel(v64, fd[1e-6][2])},
        "f64_vs_fd_1e-3": {"gamma": rel(p64[0], fd[1e-3][0]), "tau": rel(p64[1], fd[1e-3][1]),
                           "v0": vrel(v64, fd[1e-3][2])},
        "fd_runs": 4 * (2 + 3 * n), "seconds": round(time.perf_counter() - t0, 1),
    }
    return out


def time_large(steps, warmup):
    """The same workload at 512^3 (134M nodes, 19 x 512^3 > 2^31 population
    elements), FP32 and BF16 storage: whole-step MLUPS and the stream-collide's
    fraction of the HBM peak."""
    import torch

    from paper_1909_13412_amd.inputs import WORKLOADS

    w = dict(WORKLOADS["suspension512"])
    w["name"] = "suspension512"
    out = {"box": [w["L"]] * 3, "nodes": w["L"] ** 3, "particles": w["n"], "steps": steps}
    for storage in ("f32", "bf16"):
        r = time_storage(w, storage, steps, min(warmup, 20), min(steps, 50))
        out[storage] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 5),
                        "collide_ms": round(r["collide_ms"], 5), "collide_GBs": round(r["collide_GBs"], 1),
                        "collide_frac": round(r["collide_frac"], 4), "collide_shape": r["collide_shape"],
                        "collide_order": r["collide_order"],
                        "collide_waves_per_simd_cap": r["collide_waves_per_simd_cap"],
                        "layout_rows_per_group": r["layout_rows_per_group"],
                        "stream_only_ms": round(r["stream_only_ms"], 5),
                        "of_stream_only": round(r["of_stream_only"], 4)}
        torch.cuda.empty_cache()
    return out



def size_sweep(sizes, storages):
    """Stream-collide of cubic boxes of the given edges (tau 0.6, 200
    particles): every launch configuration's milliseconds (autotuner timing,
    best of two rounds), the best flat (0-7) and row-aligned (8, 9) ones, and
    the streaming-only ceiling of the best."""
    import numpy as np
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    out = []
    for st in storages:
        for L in sizes:
            lat = Lattice(L, L, L, 0.6, storage=st)
            lat.particles_couple(particle_positions(200, L, seed=3), particle_velocities(200, 1e-5, seed=3),
                                 radius=0.5, kT=1e-4, seed=3)
            lat.step(10)
            ms = np.min(np.array([lat.autotune(20)[1] for _ in range(2)]), axis=0)
            valid = ms > 0
            k = int(np.argmin(np.where(valid, ms, np.inf)))
            ceil = lat.stream_ceiling(20, config=k)
            alg = collide_bytes_per_node(st) * L ** 3
            flat = ms[:8][valid[:8]]
            row = ms[8:][valid[8:]]
            out.append({"box": L, "storage": st, "config": k, "ms": round(float(ms[k]), 5),
                        "GBs": round(alg / (ms[k] * 1e-3) / 1e9, 1),
                        "frac": round(alg / (ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "flat_best_ms": round(float(flat.min()), 5),
                        "row_best_ms": round(float(row.min()), 5) if row.size else None,
                        "stream_only_ms": round(ceil, 5), "of_stream_only": round(ceil / float(ms[k]), 4),
                        "all_ms": [round(float(x), 5) for x in ms]})
            print(f"[bench] size sweep {L}^3 {st}: config {k} {ms[k]:.4f} ms", file=sys.stderr, flush=True)
            del lat
            torch.cuda.empty_cache()
    return out

def time_pairs(w, steps, warmup, prof_steps, main):
    """The same FP32 workload with the soft pair repulsion switched on (a_f =
    0.05, cutoff 2R = 1): cost of the cell list and the neighbour sums, which
    run in the particle phase."""
    pair = (0.05, 2.0 * w["radius"])
    r = time_storage(w, "f32", steps, warmup, prof_steps, pair=pair)
    return {"a_f": pair[0], "r_c": pair[1], "mlups": round(r["mlups"], 1),
            "ms_per_step": round(r["ms_per_step"], 5),
            "particle_phase_ms": round(r["particle_phase_ms"], 5),
            "particle_phase_ms_without": round(main["particle_phase_ms"], 5),
            "pair_ms": round(r["particle_phase_ms"] - main["particle_phase_ms"], 5)}


def cpu_baseline(w, steps):
    import oracle
    from paper_1909_13412_amd.inputs import workload_particles

    oracle.build(force=False)
    L = w["L"]
    sim = oracle.Sim(L, L, L, w["tau"])
    r, v = workload_particles(w["name"])
    sim.set_particles(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                      seed=w["seed"])
    sim.vacf_config(w["max_lag"], w["stride"])
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    sim.close()
    return {
        "value": L**3 * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} steps of the {L}^3 / {w['n']}-particle workload, FP64, "
                  f"{dt:.1f} s",
    }



def cpu_baseline_one_thread(w, steps):
    """The same oracle run on one host thread (OMP_NUM_THREADS=1), in a child
    process that never touches the GPU; None if it fails."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, {root!r}); import bench; "
            "print(json.dumps(bench.cpu_baseline({w!r}, {steps})))").format(root=ROOT, w=dict(w), steps=int(steps))
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if res.returncode != 0:
        print(f"[bench] one-thread oracle run failed: {res.stderr[-500:]}", file=sys.stderr, flush=True)
        return None
    return json.loads(res.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="suspension256")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--variants", default="bf16,f16,f64,f32q15,bf16q15",
                    help="storages to time besides --storage; a q15 suffix selects D3Q15")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed regions of --steps steps for the main storage: `value` is the first, "
                         "`value_regions` lists all with their median (1 = the first only)")
    ap.add_argument("--size-sweep", default="",
                    help="comma-separated box edges for a stream-collide size sweep (off by default), "
                         "e.g. 48,64,96,100,128,200,250,256")
    ap.add_argument("--size-sweep-storages", default="f32,bf16")
    ap.add_argument("--vacf128-steps", type=int, default=20000,
                    help="0 = skip the precision study on the 128^3 / 64-particle VACF workload "
                         "(its 20,000 steps against the oracle's run; also skipped with "
                         "--precision-steps 0)")
    ap.add_argument("--fig2-steps", type=int, default=12000,
                    help="0 = skip the precision study on the paper's thermal Fig. 2 suspension "
                         "(100^3, 500 particles of R = 1 on the (2 dx)^3 cube; its 12,000 steps "
                         "against the oracle's run; also skipped with --precision-steps 0)")
    ap.add_argument("--cpu-steps", type=int, default=90, help="oracle steps timed (0 = skip; 90 is ~11 s on 16 host threads)")
    ap.add_argument("--cpu-steps-one-thread", type=int, default=6,
                    help="oracle steps timed on one host thread, in a child process (0 = skip; also skipped with --cpu-steps 0; 6 is ~10 s)")
    ap.add_argument("--precision-steps", type=int, default=2000,
                    help="0 = skip the VACF error study (the workload's 2000 steps against the "
                         "oracle's run)")
    ap.add_argument("--prof-steps", type=int, default=300, help="steps timed with per-kernel events")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=5000,
                    help="0 = skip the ensemble timing (5000: the workload's length, checked against "
                         "the oracle's runs of its smallest and largest boxes)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="0 = skip the reverse-mode leg (2000: the workload's length, with the "
                         "mean-squared-displacement gradient and its finite differences)")
    ap.add_argument("--no-pairs", action="store_true", help="skip the pair-repulsion timing")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="steps of the 512^3 leg per storage (0 = skip)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; no multi-GPU path is implemented "
              "(see the sharding design).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_13412_amd.inputs import WORKLOADS

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    w = dict(WORKLOADS[args.workload])
    w["name"] = args.workload

    copy = None
    if not args.no_copy_probe:
        print("[bench] copy probe", file=sys.stderr, flush=True)
        copy = copy_probe(19 * w["L"] ** 3 * ELEM[args.storage])
    print(f"[bench] timing {args.workload} storage={args.storage} steps={args.steps}", file=sys.stderr,
          flush=True)
    main_res = time_storage(w, args.storage, args.steps, args.warmup, args.prof_steps,
                            repeats=max(args.repeats - 1, 0))
    variants = {}
    for s in [v for v in args.variants.split(",") if v and v != args.storage]:
        print(f"[bench] timing storage={s}", file=sys.stderr, flush=True)
        r = time_storage(w, s, args.steps, args.warmup, args.prof_steps)
        r["speedup_vs_main"] = r["mlups"] / main_res["mlups"]
        r["traffic"] = pmc_traffic(s)
        variants[s] = r
    large = None
    if args.large_steps > 0 and args.workload == "suspension256":
        print(f"[bench] suspension512 ({args.large_steps} steps per storage)", file=sys.stderr, flush=True)
        large = time_large(args.large_steps, args.warmup)
    pairs = None
    if not args.no_pairs:
        print("[bench] pair repulsion", file=sys.stderr, flush=True)
        pairs = time_pairs(w, min(args.steps, 300), args.warmup, args.prof_steps, main_res)
    ensemble = None
    if args.ensemble_steps > 0:
        print(f"[bench] ensemble ({args.ensemble_steps} steps)", file=sys.stderr, flush=True)
        ensemble = time_ensemble(args.ensemble_steps, args.warmup)
    adjoint = None
    if args.adjoint_steps > 0:
        print(f"[bench] reverse mode ({args.adjoint_steps} steps)", file=sys.stderr, flush=True)
        adjoint = time_adjoint(args.adjoint_steps, args.warmup)
    precision = None
    if args.precision_steps > 0:
        print(f"[bench] precision study ({args.precision_steps} steps per storage)", file=sys.stderr,
              flush=True)
        precision = precision_study(w)
    sweep = None
    if args.size_sweep:
        sweep = size_sweep([int(x) for x in args.size_sweep.split(",") if x],
                           [x for x in args.size_sweep_storages.split(",") if x])
    precision128 = None
    if args.precision_steps > 0 and args.vacf128_steps > 0:
        print(f"[bench] precision study, vacf128 ({args.vacf128_steps} steps per storage)", file=sys.stderr,
              flush=True)
        from paper_1909_13412_amd.inputs import WORKLOADS

        w128 = dict(WORKLOADS["vacf128"])
        w128["name"] = "vacf128"
        precision128 = precision_study(w128)
    precision_fig2 = None
    if args.precision_steps > 0 and args.fig2_steps > 0:
        print(f"[bench] precision study, fig2thermal100 ({args.fig2_steps} steps per storage)",
              file=sys.stderr, flush=True)
        from paper_1909_13412_amd.inputs import WORKLOADS

        wf2 = dict(WORKLOADS["fig2thermal100"])
        wf2["name"] = "fig2thermal100"
        precision_fig2 = precision_study(wf2)
    cpu = None
    if args.cpu_steps > 0:
        print(f"[bench] oracle baseline ({args.cpu_steps} steps)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_steps)
    cpu1 = None
    if args.cpu_steps > 0 and args.cpu_steps_one_thread > 0:
        print(f"[bench] oracle baseline, one thread ({args.cpu_steps_one_thread} steps)", file=sys.stderr,
              flush=True)
        cpu1 = cpu_baseline_one_thread(w, args.cpu_steps_one_thread)

    ncell = w["L"] ** 3
    regions = [main_res["mlups"]] + main_res["mlups_more_regions"]
    traffic = pmc_traffic(args.storage)
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "value_regions": {"mlups": [round(x, 1) for x in regions],
                          "median": round(statistics.median(regions), 1)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "box": [w["L"]] * 3, "nodes": ncell, "tau": w["tau"],
                   "particles": w["n"], "kT": w["kT"], "gamma": w["gamma"], "radius": w["radius"],
                   "mass": w["mass"], "storage": args.storage,
                   "vacf": {"max_lag": w["max_lag"], "stride": w["stride"]},
                   "fp64_sums_every": SERIES_EVERY,
                   "parallelism": "single GPU"},
        "roofline": {
            "kernel": "k_stream_collide",
            "bound": "hbm",
            "achieved": round(main_res["collide_GBs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_res["collide_frac"], 4),
            "traffic": traffic,
            "traffic_frac": (round(traffic / (main_res["collide_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic else None),
            "traffic_unit": "bytes per launch (rocprofv3: L2 read requests to memory x their size "
                            "(32/64/128 B) + write requests x their size; a plain copy reads "
                            "exactly its bytes this way; null if the kernels changed since)",
            "algorithmic_bytes_per_launch": collide_bytes_per_node(args.storage) * ncell,
            "bytes_per_node": collide_bytes_per_node(args.storage),
            "avg_launch_ms": round(main_res["collide_ms"], 5),
            "launch_shape": main_res["collide_shape"],
            "launch_order": main_res["collide_order"],
            "launch_waves_per_simd_cap": main_res["collide_waves_per_simd_cap"],
            "layout_rows_per_group": main_res["layout_rows_per_group"],
            "autotune_ms": main_res["autotune_ms"],
            "pattern_ceiling": {
                "kernel": "k_stream_only",
                "what": "the stream-collide's pulls and stores alone (no arithmetic), same layout and launch configuration",
                "avg_launch_ms": round(main_res["stream_only_ms"], 5),
                "bytes_per_node": 2 * 19 * ELEM[args.storage],
                "achieved": round(2 * 19 * ELEM[args.storage] * ncell / (main_res["stream_only_ms"] * 1e-3) / 1e9, 1),
                "frac": round(2 * 19 * ELEM[args.storage] * ncell / (main_res["stream_only_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "kernel_vs_ceiling": round(main_res["of_stream_only"], 4),
            },
        },
        "profiled_ms_per_step": round(main_res["profiled_ms_per_step"], 5),
        "particle_phase_ms": round(main_res["particle_phase_ms"], 5),
        "copy_probe": copy,
        "variants": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in variants.items()},
        "suspension512": large,
        "pairs": pairs,
        "ensemble": ensemble,
        "adjoint": adjoint,
        "precision": precision,
        "precision_vacf128": precision128,
        "precision_fig2thermal100": precision_fig2,
        "size_sweep": sweep,
        "cpu_baseline": cpu,
        "cpu_baseline_one_thread": cpu1,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
