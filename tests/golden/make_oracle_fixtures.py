#!/usr/bin/env python3
"""Write the FP64 oracle's long-run reference values for the precision study.

Calls only the oracle (``oracle/``) and the seeded initial conditions of
``paper_1909_13412_amd/inputs.py`` (loaded by file path, so nothing else of
the GPU package is imported).  Each fixture is one JSON file in this folder:

* ``oracle_vacf128.json``: the 128^3 VACF workload (tau 0.8, 64 particles,
  R from Stokes' law, kT 1e-4, seed 2002) over its full 20,000 steps: the
  velocity autocorrelation C(l) = <V(t0).V(t0 + l)> averaged over particles
  and origins (section 2.1; origins every 10 steps, lags 0..2000) and the FP64
  mass / momentum sums every 100 steps.
* ``oracle_suspension256.json``: the 256^3 suspension (tau 0.6, 4096
  particles, R 0.5, kT 1e-4, seed 3003) over 2,000 steps: C(l) for lags
  0..500 and the sums every 10 steps.
* ``oracle_fig2thermal100.json``: the paper's thermal Fig. 2 suspension
  (100^3, tau 0.5534, 500 particles, R = 1, M = 16, kT 3.3e-7, fit and
  spreading on the (2 dx)^3 cube, seed 2019) over 12,000 steps: C(l) for lags
  0..1000 and the sums every 100 steps.
* ``oracle_ensemble64_edges.json``: the smallest and the largest box of the
  64-box ensemble (edges 48 and 96, tau 0.8, 8 particles, kT 1e-4) over
  5,000 steps, each run as the single box the ensemble replica stands for:
  C(l) for lags 0..1000 and the final particle state.
* ``oracle_ensemble64_all.json``: the same for every one of the 64 boxes.

Usage: python tests/golden/make_oracle_fixtures.py [vacf128] [suspension256]
[fig2thermal100] [ensemble] [ensemble_all]   (no argument: all but
ensemble_all).  The 128^3 and 256^3 runs take about 20 minutes each on 8 host
threads, ensemble_all about as long.
"""
from __future__ import annotations

import importlib.util
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def _inputs():
    spec = importlib.util.spec_from_file_location(
        "lbmbp_inputs", os.path.join(ROOT, "paper_1909_13412_amd", "inputs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


INPUTS = _inputs()

CITATION = ("Yoshida, Kinjo & Washizu, arXiv:1909.13412: section 2.1 (friction fit Eq. s2-slet-v, "
            "Langevin update Eqs. s2-langevin, s2-langevin2, random force Eqs. s2-rf1, s2-rf2, "
            "C_v(t) = <V(0).V(t)>), section 2.2 (lattice Boltzmann Eqs. s2-density to s2-trans)")


def _curve(sim, n):
    acc, cnt = sim.vacf()
    c = acc.sum(axis=0) / (n * np.maximum(cnt, 1))
    return c, cnt


def _series_run(sim, steps, every):
    rows = []
    done = 0
    while True:
        o = sim.observables()
        rows.append([float(done)] + [float(x) for x in o])
        if done >= steps:
            break
        k = min(every, steps - done)
        sim.step(k)
        done += k
    return rows


def _write(name, rec):
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
        fh.write("\n")
    os.replace(path + ".tmp", path)
    print(f"wrote {path} ({os.path.getsize(path)} bytes)", flush=True)


def make_workload(name, series_every):
    w = dict(INPUTS.WORKLOADS[name])
    w["name"] = name
    L = w["L"]
    sim = oracle.Sim(L, L, L, w["tau"])
    r, v = INPUTS.workload_particles(name)
    sim.set_particles(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                      seed=w["seed"], friction=w.get("friction", "stokeslet"))
    sim.vacf_config(w["max_lag"], w["stride"])
    t0 = time.time()
    series = _series_run(sim, w["steps"], series_every)
    wall = time.time() - t0
    c, cnt = _curve(sim, w["n"])
    rf, vf = sim.particles()
    rec = {
        "workload": name, "box": [L, L, L], "tau": w["tau"], "particles": w["n"],
        "mass": w["mass"], "gamma": w["gamma"], "kT": w["kT"], "radius": sim.radius,
        "friction": w.get("friction", "stokeslet"),
        "seed": w["seed"], "steps": w["steps"], "max_lag": w["max_lag"], "stride": w["stride"],
        "storage": "oracle FP64", "citation": CITATION,
        "vacf": [float(x) for x in c], "vacf_counts": [int(x) for x in cnt],
        "series_every": series_every,
        "series_columns": ["step", "fluid mass", "fluid Px", "fluid Py", "fluid Pz",
                           "particle Px", "particle Py", "particle Pz"],
        "series": series,
        "final_v": vf.tolist() if w["n"] <= 500 else None,
        "oracle_threads": oracle.num_threads(), "oracle_seconds": round(wall, 1),
        "generator": "tests/golden/make_oracle_fixtures.py",
    }
    _write(f"oracle_{name}.json", rec)


def make_ensemble_edges(every_box=False):
    w = INPUTS.ENSEMBLE64
    reps = INPUTS.ensemble_replicas(w["replicas"], w["sizes"], w["n"], w["tau"], w["kT"],
                                    w["mass"], w["seed"])
    edges = [rp["nx"] for rp in reps]
    picks = list(range(len(reps))) if every_box else [edges.index(min(edges)), edges.index(max(edges))]
    out = {"workload": "ensemble64", "steps": w["steps"], "max_lag": w["max_lag"],
           "stride": w["stride"], "tau": w["tau"], "mass": w["mass"], "gamma": w["gamma"],
           "kT": w["kT"], "storage": "oracle FP64", "citation": CITATION, "replicas": [],
           "generator": "tests/golden/make_oracle_fixtures.py"}
    for k in picks:
        rp = reps[k]
        L = rp["nx"]
        sim = oracle.Sim(L, L, L, rp["tau"])
        sim.set_particles(rp["r"], rp["v"], mass=w["mass"], gamma=w["gamma"], kT=w["kT"],
                          seed=rp["seed"], replica=rp["replica"])
        sim.vacf_config(w["max_lag"], w["stride"])
        t0 = time.time()
        sim.step(w["steps"])
        wall = time.time() - t0
        c, cnt = _curve(sim, len(rp["r"]))
        rf, vf = sim.particles()
        out["replicas"].append({
            "index": k, "edge": L, "seed": rp["seed"], "replica": rp["replica"],
            "particles": len(rp["r"]), "radius": sim.radius,
            "vacf": [float(x) for x in c], "vacf_counts": [int(x) for x in cnt],
            "final_r": rf.tolist(), "final_v": vf.tolist(),
            "observables": [float(x) for x in sim.observables()],
            "oracle_seconds": round(wall, 1)})
        print(f"ensemble replica {k} (edge {L}) done in {wall:.0f} s", flush=True)
    _write("oracle_ensemble64_all.json" if every_box else "oracle_ensemble64_edges.json", out)


def main(argv):
    what = argv or ["vacf128", "suspension256", "fig2thermal100", "ensemble"]
    oracle.build(force=False)
    for item in what:
        t = time.time()
        if item == "vacf128":
            make_workload("vacf128", 100)
        elif item == "suspension256":
            make_workload("suspension256", 10)
        elif item == "fig2thermal100":
            make_workload("fig2thermal100", 100)
        elif item == "ensemble":
            make_ensemble_edges()
        elif item == "ensemble_all":
            make_ensemble_edges(every_box=True)
        else:
            raise SystemExit(f"unknown fixture {item!r}")
        print(f"{item}: {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
