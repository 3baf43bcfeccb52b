"""Split steps (the particle kernel on a second stream overlapping the second
part of the stream-collide, lbm_set_overlap) against plain steps: the same
bits for every output, over storages, friction models, launch configurations,
pair forces, VACF and recorded sums, and the 256^3 benchmark workload."""
import numpy as np
import pytest

from helpers import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _run(L, tau, storage, r, v, steps, overlap, *, friction="stokeslet", kT=1e-4, seed=3, radius=0.0,
         shape=None, pairs=None, vacf=(12, 3), series=None, chunks=(1,)):
    import torch

    from paper_1909_13412_amd import Lattice

    lat = Lattice(*L, tau, storage=storage)
    if shape is not None:
        lat.set_shape(shape)
    lat.particles_couple(r, v, kT=kT, seed=seed, radius=radius, friction=friction)
    if pairs:
        lat.set_pair_force(*pairs)
    if vacf:
        lat.vacf_config(*vacf)
    if series:
        lat.series_config(series, steps + 2)
    lat.set_overlap(overlap)
    done = 0
    k = 0
    while done < steps:  # several lbm_step calls of different lengths
        n = min(chunks[k % len(chunks)], steps - done)
        lat.step(n)
        done += n
        k += 1
    torch.cuda.synchronize()
    out = {"f": lat.populations().cpu().numpy(), "r": lat.r.cpu().numpy(), "v": lat.v.cpu().numpy()}
    if vacf:
        out["acc"] = lat.vacf()[0].cpu().numpy()
    if series:
        out["series"] = lat.series()
    out["fh"] = lat.particle_forces()[0].cpu().numpy()
    return out


def _same(a, b, what):
    for key in a:
        assert np.array_equal(a[key], b[key]), (what, key)


CASES = [
    # box, storage, friction, particles, launch configuration, pairs
    ((48, 40, 36), "f32", "stokeslet", 60, None, None),
    ((48, 40, 36), "bf16", "stokeslet", 60, None, None),
    ((37, 30, 22), "f32", "stokeslet2dx", 40, None, None),
    ((37, 30, 22), "f32", "pointwise", 40, 8, None),
    ((40, 24, 30), "f64", "stokeslet", 30, 3, None),
    ((40, 24, 30), "f32", "bd", 30, None, None),
    ((130, 20, 12), "f32", "stokeslet", 50, 9, (0.05, 1.5)),
    ((32, 32, 32), "f32", "stokeslet", 300, 6, (0.05, 1.2)),
]


@pytest.mark.parametrize("L,storage,friction,n,shape,pairs", CASES)
def test_split_steps_are_bit_identical(L, storage, friction, n, shape, pairs):
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    r = particle_positions(n, L, seed=41)
    v = particle_velocities(n, 1e-4 / 10.0, seed=41)
    announce(f"split steps: {L} {storage} {friction} n={n} shape={shape} pairs={pairs}")
    kw = dict(friction=friction, shape=shape, pairs=pairs, series=5, chunks=(1, 7, 3, 12))
    plain = _run(L, 0.7, storage, r, v, 31, 0, **kw)
    split = _run(L, 0.7, storage, r, v, 31, 1, **kw)
    _same(plain, split, (L, storage, friction))


def test_split_steps_benchmark_workload():
    # 256^3, 4096 particles, FP32, VACF on, in the autotuned configuration.
    from paper_1909_13412_amd.inputs import WORKLOADS, workload_particles

    import torch

    from paper_1909_13412_amd import Lattice

    w = WORKLOADS["suspension256"]
    r, v = workload_particles("suspension256")
    outs = []
    for overlap in (0, 1):
        lat = Lattice(256, 256, 256, w["tau"], storage="f32")
        lat.particles_couple(r, v, mass=w["mass"], gamma=w["gamma"], kT=w["kT"], radius=w["radius"],
                             seed=w["seed"])
        lat.vacf_config(w["max_lag"], w["stride"])
        lat.autotune(5)
        lat.set_overlap(overlap)
        lat.step(12)
        torch.cuda.synchronize()
        outs.append((lat.populations().cpu().numpy(), lat.r.cpu().numpy(), lat.v.cpu().numpy(),
                     lat.vacf()[0].cpu().numpy()))
        del lat
        torch.cuda.empty_cache()
    announce("split steps at 256^3: comparing")
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_split_steps_recorded_tape():
    # lbm_record with split steps reaches the same state, and the adjoint
    # (which recomputes from its checkpoints) gives the same gradients.
    import torch

    from paper_1909_13412_amd import Lattice
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    L = (24, 20, 16)
    r = particle_positions(12, L, seed=5)
    v = particle_velocities(12, 1e-5, seed=5)
    grads = []
    for overlap in (0, 1):
        lat = Lattice(*L, 0.8, storage="f32")
        lat.particles_couple(r, v, kT=1e-4, seed=7)
        lat.set_overlap(overlap)
        tape = lat.record(20, 4)
        f_end = lat.populations().cpu().numpy()
        g = lat.adjoint(tape, adj_r=torch.ones((12, 3), dtype=torch.float64, device=lat.device))
        torch.cuda.synchronize()
        grads.append((f_end, {k: x.cpu().numpy() for k, x in g.items()}))
    assert np.array_equal(grads[0][0], grads[1][0])
    for k in grads[0][1]:
        assert np.array_equal(grads[0][1][k], grads[1][1][k]), k
