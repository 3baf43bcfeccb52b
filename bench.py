#!/usr/bin/env python3
"""Benchmark of the coupled lattice-Boltzmann / Brownian-particle step on one MI355X.

A step is the whole hot path: VACF sample, particle coupling (gather at the eight
neighbour nodes, Stokeslet fit, Philox Brownian force, reaction-force spreading,
Langevin update) and the fused stream-collide with forcing.  Workload (default):
256^3 periodic box, tau 0.6, 4096 particles (M 10, gamma 1, R 0.5, kT 1e-4), VACF with
lags up to 500 and origins every 10 steps; synthetic seeded initial state.

Prints ONE JSON line.  `value` is whole-step MLUPS (nodes x steps / s / 1e6) with
FP32 population storage; `variants` repeats the timing for shifted BF16 and FP16
storage; `roofline` prices the stream-collide kernel (the dominant one) against
the 8 TB/s HBM peak from HIP-event timings taken inside the timed region;
`cpu_baseline` times the FP64 oracle on a few steps of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ELEM = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
METRIC = "MLUPS & % HBM roofline, FP32 vs shifted-BF16 storage at stated VACF error"


def collide_bytes_per_node(storage: str) -> float:
    """Algorithmic bytes of one stream-collide node update: 19 population loads
    and 19 stores, plus the one-bit forcing flag."""
    return 2 * 19 * ELEM[storage] + 1.0 / 8.0


def make_lattice(w, storage, device="cuda:0"):
    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import workload_particles

    L = w["L"]
    lat = Lattice(L, L, L, w["tau"], storage=storage, device=device)
    r, v = workload_particles(w["name"])
    lat.particles_couple(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                         seed=w["seed"])
    lat.vacf_config(w["max_lag"], w["stride"])
    return lat


def time_storage(w, storage, steps, warmup):
    import torch

    lat = make_lattice(w, storage)
    lat.step(warmup)
    torch.cuda.synchronize()
    lat.profile_enable(True)
    lat.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = lat.profile_read()
    lat.profile_enable(False)
    obs = lat.observables()
    ncell = w["L"] ** 3
    ms_step = (t1 - t0) * 1e3 / steps
    mlups = ncell * steps / (t1 - t0) / 1e6
    coll_ms = prof["collide_ms"] / max(prof["collide_launches"], 1)
    part_ms = prof["particle_ms"] / max(prof["particle_launches"], 1)
    achieved = ncell * collide_bytes_per_node(storage) / (coll_ms * 1e-3) / 1e9
    res = {
        "storage": storage,
        "mlups": mlups,
        "ms_per_step": ms_step,
        "collide_ms": coll_ms,
        "particle_phase_ms": part_ms,
        "collide_GBs": achieved,
        "collide_frac": achieved / HBM_PEAK_GBS,
        "mass": obs[0],
    }
    del lat
    torch.cuda.empty_cache()
    return res


def precision_study(w, steps, storages=("f32", "bf16", "f16")):
    """VACF and momentum error of each storage against the FP64 path (itself
    matched to the FP64 oracle to 1e-10) on the same workload and seed."""
    import numpy as np
    import torch

    def run(storage):
        lat = make_lattice(w, storage)
        mom = []
        chunk = 100
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            lat.step(k)
            done += k
            o = lat.observables()
            mom.append(np.concatenate([o[1:4], o[4:7]]))
        acc, cnt = lat.vacf()
        acc = acc.cpu().numpy()
        c = acc.sum(0) / (acc.shape[0] * np.maximum(cnt, 1))
        valid = cnt > 0
        curve = np.where(valid, c / c[0], 0.0)
        del lat
        torch.cuda.empty_cache()
        return curve, np.array(mom), valid

    ref_curve, ref_mom, valid = run("f64")
    out = {"reference": "f64 storage (FP64 path)", "steps": steps}
    for s in storages:
        curve, mom, _ = run(s)
        out[s] = {
            "vacf_err": float(np.max(np.abs(curve[valid] - ref_curve[valid]))),
            "particle_momentum_err": float(np.max(np.abs(mom[:, 3:] - ref_mom[:, 3:])) /
                                           np.max(np.abs(ref_mom[:, 3:]))),
            "fluid_momentum_err": float(np.max(np.abs(mom[:, :3] - ref_mom[:, :3])) /
                                        np.max(np.abs(ref_mom[:, :3]))),
        }
    return out


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="suspension256")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--variants", default="bf16,f16")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps timed (0 = skip)")
    ap.add_argument("--precision-steps", type=int, default=2000, help="0 = skip the VACF error study")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU path is not built "
              "(see the sharding design).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_13412_amd.inputs import WORKLOADS

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    w = dict(WORKLOADS[args.workload])
    w["name"] = args.workload

    print(f"[bench] timing {args.workload} storage={args.storage} steps={args.steps}", file=sys.stderr,
          flush=True)
    main_res = time_storage(w, args.storage, args.steps, args.warmup)
    variants = {}
    for s in [v for v in args.variants.split(",") if v and v != args.storage]:
        print(f"[bench] timing storage={s}", file=sys.stderr, flush=True)
        r = time_storage(w, s, args.steps, args.warmup)
        r["speedup_vs_main"] = r["mlups"] / main_res["mlups"]
        variants[s] = r
    precision = None
    if args.precision_steps > 0:
        print(f"[bench] precision study ({args.precision_steps} steps per storage)", file=sys.stderr,
              flush=True)
        precision = precision_study(w, args.precision_steps)
    cpu = None
    if args.cpu_steps > 0:
        print(f"[bench] oracle baseline ({args.cpu_steps} steps)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, args.cpu_steps)

    ncell = w["L"] ** 3
    out = {
        "metric": METRIC,
        "value": round(main_res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "box": [w["L"]] * 3, "nodes": ncell, "tau": w["tau"],
                   "particles": w["n"], "kT": w["kT"], "gamma": w["gamma"], "radius": w["radius"],
                   "mass": w["mass"], "storage": args.storage,
                   "vacf": {"max_lag": w["max_lag"], "stride": w["stride"]},
                   "parallelism": "single GPU"},
        "roofline": {
            "kernel": "k_stream_collide",
            "bound": "hbm",
            "achieved": round(main_res["collide_GBs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_res["collide_frac"], 4),
            "traffic": None,
            "bytes_per_node": collide_bytes_per_node(args.storage),
            "avg_launch_ms": round(main_res["collide_ms"], 5),
        },
        "particle_phase_ms": round(main_res["particle_phase_ms"], 5),
        "variants": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in variants.items()},
        "precision": precision,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
