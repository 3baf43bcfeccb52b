"""GPU parity of the ensemble path (many boxes in one launch per kernel, steps
replayed from a captured graph): every replica against the FP64 oracle and
against a single-box run with the same inputs."""
import numpy as np
import pytest

from helpers import announce, nmax_err, pulled, raw_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _small_replicas(kT=1e-4):
    from paper_1909_13412_amd.inputs import particle_positions, particle_velocities

    boxes = [((12, 10, 8), 0.7, 4), ((9, 9, 9), 0.8, 3), ((16, 6, 10), 0.9, 5), ((7, 13, 11), 0.75, 2)]
    reps = []
    for k, (L, tau, n) in enumerate(boxes):
        reps.append(dict(nx=L[0], ny=L[1], nz=L[2], tau=tau, seed=900 + k, replica=k,
                         r=particle_positions(n, L, 60 + k), v=particle_velocities(n, kT / 10.0, 60 + k)))
    return reps


def test_ensemble_replicas_match_oracle(oracle_mod):
    from paper_1909_13412_amd import Ensemble, _abi

    reps = _small_replicas()
    ens = Ensemble(reps, storage="f64", kT=1e-4)
    ens.vacf_config(9, 4)
    G = _abi.LBM_ENS_GRAPH_STEPS
    steps = 2 * G + 5  # two graph replays and five plain steps
    ens.step(steps)
    assert ens.graph_replays == 2
    for k, rd in enumerate(reps):
        ref = oracle_mod.Sim(rd["nx"], rd["ny"], rd["nz"], rd["tau"])
        ref.set_particles(rd["r"], rd["v"], kT=1e-4, seed=rd["seed"], replica=rd["replica"])
        ref.vacf_config(9, 4)
        ref.step(steps)
        rr, vr = ref.particles()
        rg, vg = ens.particles(k)
        e_v = nmax_err(vg.cpu().numpy(), vr)
        e_r = np.max(np.abs(rg.cpu().numpy() - rr))
        w = oracle_mod.lattice()[1][:, None, None, None]
        e_g = nmax_err(ens.populations(k).cpu().numpy() - w, ref.populations() - w)
        acc_g, cnt_g = ens.vacf()
        a, b = int(ens.offsets[k]), int(ens.offsets[k + 1])
        acc_r, cnt_r = ref.vacf()
        e_acc = nmax_err(acc_g.cpu().numpy()[a:b], acc_r)
        o_g = ens.observables(k)
        o_r = ref.observables()
        announce(f"  replica {k}: v {e_v:.2e} r {e_r:.2e} g {e_g:.2e} vacf {e_acc:.2e}")
        assert e_v < 1e-10 and e_r < 1e-10 and e_g < 1e-10 and e_acc < 1e-10
        assert np.array_equal(cnt_g, cnt_r)
        assert abs(o_g[0] - o_r[0]) < 1e-10 * o_r[0]
        assert nmax_err(o_g[1:], o_r[1:]) < 1e-10


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16", "f64"])
def test_ensemble_equals_single_box_runs(storage):
    from paper_1909_13412_amd import Ensemble, Lattice

    reps = _small_replicas()
    ens = Ensemble(reps, storage=storage, kT=1e-4)
    ens.step(24)
    # The ensemble kernels run the single-box node and particle updates with
    # the same rounding (multiply-adds fuse only within one expression), so
    # every replica must reproduce its single-box run bit for bit, in every
    # storage.
    for k, rd in enumerate(reps):
        one = Lattice(rd["nx"], rd["ny"], rd["nz"], rd["tau"], storage=storage)
        one.particles_couple(rd["r"], rd["v"], kT=1e-4, seed=rd["seed"], replica=rd["replica"])
        one.step(24)
        fe, fo = ens.populations(k).cpu().numpy(), one.populations().cpu().numpy()
        ve, vo = ens.particles(k)[1].cpu().numpy(), one.v.cpu().numpy()
        assert np.array_equal(fe, fo) and np.array_equal(ve, vo), (k, np.max(np.abs(fe - fo)), nmax_err(ve, vo))


def test_ensemble_on_its_own_stream():
    # An ensemble driven on a stream of its own (graph replays included) gives
    # the bits it gives on the caller's stream, and its results are safe to
    # read on the caller's stream.
    import torch

    from paper_1909_13412_amd import Ensemble

    reps = _small_replicas()
    out = []
    for stream in (None, torch.cuda.Stream()):
        e = Ensemble(reps, storage="f32", kT=1e-4, stream=stream)
        e.vacf_config(9, 4)
        e.step(21)
        acc, cnt = e.vacf()
        out.append(([e.populations(k).cpu().numpy() for k in range(len(reps))],
                    e.v.cpu().numpy(), acc.cpu().numpy(), cnt))
        e.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][1:], out[1][1:]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_ensemble_stream_ceiling_pulls_every_population(storage):
    # The ensemble's streaming-only kernel (lbm_ens_stream_ceiling) moves
    # exactly the ensemble stream-collide's bytes: box after box in the spare
    # lattice, every population pulled from x - e_a unchanged, in every
    # configuration that applies (two-node shapes need an even ny in every box);
    # the state is left as it was.
    import torch

    from paper_1909_13412_amd import Ensemble

    reps = _small_replicas()
    e = Ensemble(reps, storage=storage, kT=1e-4)
    e.step(6)  # even: the current populations are back in the first buffer
    f0 = [e.populations(k).clone() for k in range(len(reps))]
    torch.cuda.synchronize()
    dt, el = {"f32": (torch.float32, 4), "bf16": (torch.int16, 2)}[storage]
    sizes = [19 * rd["nx"] * rd["ny"] * rd["nz"] for rd in reps]
    offs = np.concatenate([[0], np.cumsum(sizes)])

    def raw(buf):
        # box after box as [nz, ny, 19, nx], whatever each box's rows per group
        a = buf[: int(offs[-1]) * el].view(dt).cpu().numpy()
        return np.concatenate([raw_rows(a[offs[k]:offs[k + 1]], rd["nx"], rd["ny"], rd["nz"],
                                        e.layout(k)).ravel() for k, rd in enumerate(reps)])

    a0 = raw(e.pop_a)
    expect = np.concatenate([pulled(a0[offs[k]:offs[k + 1]], rd["nx"], rd["ny"], rd["nz"]).ravel()
                             for k, rd in enumerate(reps)])
    even_ny = all(rd["ny"] % 2 == 0 for rd in reps)
    # in the layouts with one row per group, and with up to two and four
    # (boxes whose ny the request does not divide take fewer)
    for rows in (1, 2, 4):
        e.set_layout(rows)
        assert [e.layout(k) for k in range(len(reps))] == [
            max(y for y in (1, 2, 4) if y <= rows and rd["ny"] % y == 0) for rd in reps]
        assert np.array_equal(raw(e.pop_a), a0), (storage, rows)
        for k in range(8):
            if (k & 3) >= 2 and not even_ny:
                with pytest.raises(Exception):
                    e.stream_ceiling(1, config=k)
                continue
            e.pop_b.zero_()
            torch.cuda.synchronize()
            assert e.stream_ceiling(1, config=k) > 0.0
            assert np.array_equal(raw(e.pop_b), expect), (storage, rows, k)
    with pytest.raises(Exception):
        e.stream_ceiling(1, config=8)  # row-aligned: single boxes only
    assert np.array_equal(raw(e.pop_a), a0)
    for k in range(len(reps)):
        assert torch.equal(e.populations(k), f0[k])


def test_ensemble_layouts_are_bit_identical():
    # The same ensemble run with one row per group, with up to four rows per
    # group (mixed across the boxes), and with the layout switched between
    # graph-replayed steps: the same populations, particles and VACF.
    import torch

    from paper_1909_13412_amd import Ensemble

    reps = _small_replicas()
    out = []
    for rows0, rows1 in ((1, 1), (4, 4), (2, 1), (1, 4)):
        e = Ensemble(reps, storage="f32", kT=1e-4)
        e.set_layout(rows0)
        e.vacf_config(6, 3)
        e.step(8)
        e.set_layout(rows1)
        e.step(9)
        torch.cuda.synchronize()
        out.append(([e.populations(k).cpu().numpy() for k in range(len(reps))],
                    e.v.cpu().numpy(), e.vacf()[0].cpu().numpy()))
        e.close()
    for o in out[1:]:
        for a, b in zip(out[0][0], o[0]):
            assert np.array_equal(a, b)
        assert np.array_equal(out[0][1], o[1]) and np.array_equal(out[0][2], o[2])


def test_ensemble_launch_options_are_bit_identical():
    # Launch configuration, block order and residency cap change only which
    # lanes and blocks update which nodes, and when: the same run with each
    # choice, also switched between graph-replayed steps (the graph is
    # captured again after a change), gives the same populations, particles
    # and VACF.
    import torch

    from paper_1909_13412_amd import Ensemble, _abi

    G = _abi.LBM_ENS_GRAPH_STEPS
    reps = _small_replicas()  # odd ny in two boxes: one node per lane only
    runs = [((k, 0, 0), (k, 0, 0)) for k in (0, 1, 4, 5)]
    # caps that 160 KiB of LDS per compute unit can impose even with only
    # 64 KiB per block: 6 waves per SIMD for 512-lane blocks, 6 and 4 for
    # 256-lane ones
    runs += [((k, o, w), (k, o, w)) for k, ws in ((0, (0, 6)), (5, (0, 6, 4))) for o in (0, 1)
             for w in ws if (o, w) != (0, 0)]
    runs += [((1, 1, 4), (4, 0, 0)), ((4, 1, 6), (1, 0, 4)), ((5, 0, 6), (0, 1, 0))]
    out = []
    for (k0, o0, w0), (k1, o1, w1) in runs:
        e = Ensemble(reps, storage="f32", kT=1e-4)
        e.set_launch_config(k0)
        e.set_sweep_launch(o0, w0)
        assert (e.launch_config, e.sweep_launch) == (k0, (o0, w0))
        e.vacf_config(6, 3)
        e.step(G + 3)
        e.set_launch_config(k1)
        e.set_sweep_launch(o1, w1)
        assert (e.launch_config, e.sweep_launch) == (k1, (o1, w1))
        e.step(G + 1)
        torch.cuda.synchronize()
        assert e.graph_replays == 2
        out.append(([e.populations(k).cpu().numpy() for k in range(len(reps))],
                    e.v.cpu().numpy(), e.vacf()[0].cpu().numpy()))
        e.close()
    for (a0, a1), o in zip(runs[1:], out[1:]):
        for a, b in zip(out[0][0], o[0]):
            assert np.array_equal(a, b), (a0, a1)
        assert np.array_equal(out[0][1], o[1]) and np.array_equal(out[0][2], o[2]), (a0, a1)
    e = Ensemble(reps, storage="f32", kT=1e-4)
    for k in (2, 3, 6, 7, 8, 9):  # two nodes per lane (odd ny), row-aligned (single boxes)
        with pytest.raises(_abi.LbmError):
            e.set_launch_config(k)
    with pytest.raises(_abi.LbmError):
        e.set_sweep_launch(2, 0)
    with pytest.raises(_abi.LbmError):
        e.set_sweep_launch(0, 7)
    e.close()


def test_graph_replays_match_plain_launches():
    # Replays of the captured graph, with eager work and synchronisation
    # between them, against the same ensemble stepped with plain launches:
    # every replay compared; a call of fewer steps than one graph, and an odd
    # start, run plainly.
    import torch

    from paper_1909_13412_amd import Ensemble, _abi

    G = _abi.LBM_ENS_GRAPH_STEPS
    reps = _small_replicas()
    g = Ensemble(reps, storage="f32", kT=1e-4)
    e = Ensemble(reps, storage="f32", kT=1e-4)
    e.use_graph(False)
    g.vacf_config(6, 3)
    e.vacf_config(6, 3)
    step, replays = 0, 0
    for rep, n in enumerate((G, G, 3, G + 1, 2 * G + 1, 5)):
        g.step(n)
        e.step(n)
        # from an odd step one plain step first; then one replay per whole
        # graph; the rest plain
        if step % 2 and n > 0:
            step, n = step + 1, n - 1
        replays += n // G
        step += n
        assert g.graph_replays == replays and e.graph_replays == 0, rep
        torch.cuda.synchronize()
        for k in range(len(reps)):
            assert np.array_equal(g.populations(k).cpu().numpy(), e.populations(k).cpu().numpy()), (rep, k)
            assert np.array_equal(g.particles(k)[1].cpu().numpy(), e.particles(k)[1].cpu().numpy())
        g.observables(rep % len(reps))
        _ = torch.ones(1000, device="cuda").sum().item()
    assert np.array_equal(g.vacf()[0].cpu().numpy(), e.vacf()[0].cpu().numpy())


def test_ensemble64_workload():
    # The 64-replica workload (edges 48..96), checked replica by replica for
    # the smallest and largest boxes against single-box runs.
    from paper_1909_13412_amd import Ensemble, Lattice
    from paper_1909_13412_amd.inputs import ENSEMBLE64, ensemble_replicas

    w = ENSEMBLE64
    reps = ensemble_replicas(w["replicas"], w["sizes"], w["n"], w["tau"], w["kT"], w["mass"], w["seed"])
    announce(f"ensemble64: edges {sorted(set(r['nx'] for r in reps))}, "
             f"{sum(r['nx'] ** 3 for r in reps)} nodes")
    ens = Ensemble(reps, storage="f32", kT=w["kT"], mass=w["mass"], gamma=w["gamma"])
    ens.vacf_config(50, 10)
    chosen, ms = ens.autotune(5)
    announce(f"  autotune shape {chosen} ms {np.round(ms, 4)}")
    ens.step(20)
    edges = [r["nx"] for r in reps]
    for k in (int(np.argmin(edges)), int(np.argmax(edges))):
        rd = reps[k]
        one = Lattice(rd["nx"], rd["ny"], rd["nz"], rd["tau"], storage="f32")
        one.particles_couple(rd["r"], rd["v"], mass=w["mass"], gamma=w["gamma"], kT=w["kT"],
                             seed=rd["seed"], replica=rd["replica"])
        one.step(20)
        assert np.allclose(ens.populations(k).cpu().numpy(), one.populations().cpu().numpy(),
                           rtol=0, atol=1e-12)
        assert nmax_err(ens.particles(k)[1].cpu().numpy(), one.v.cpu().numpy()) < 1e-12
    for k in range(len(reps)):
        o = ens.observables(k)
        assert abs(o[0] - reps[k]["nx"] ** 3) < 1e-6 * reps[k]["nx"] ** 3


def test_ensemble64_full_run_against_oracle():
    # The 64-replica workload over its full 5000 steps, graph-replayed, FP32:
    # every box against the FP64 oracle's own run of that box alone
    # (tests/golden/oracle_ensemble64_all.json): velocity autocorrelation
    # (lags 0..1000, origins every 10 steps) and the final particle velocities.
    # A box whose FP32 trajectories still follow the oracle's (final velocities
    # within 1e-3) must match its VACF to 1e-4 of C(0).  In a box where the
    # rounding differences have grown (the fit is nonlinear in the nodal
    # velocities, and eight particles give a noisy estimator), C(0) must agree
    # within four standard errors of the box's own estimate.  The
    # ensemble-averaged VACF over all 512 particles (the workload's observable)
    # must match the oracle's average to 1% of C(0), and its tail sum (lags
    # 50-250) within twice its sampling error.
    import bench
    from paper_1909_13412_amd import Ensemble
    from paper_1909_13412_amd.inputs import ENSEMBLE64, ensemble_replicas

    w = ENSEMBLE64
    ref = bench.oracle_fixture("ensemble64_all")
    assert ref is not None and ref["steps"] == w["steps"]
    reps = ensemble_replicas(w["replicas"], w["sizes"], w["n"], w["tau"], w["kT"], w["mass"], w["seed"])
    ens = Ensemble(reps, storage="f32", kT=w["kT"], mass=w["mass"], gamma=w["gamma"])
    ens.vacf_config(w["max_lag"], w["stride"])
    ens.step(w["steps"])
    acc, cnt = ens.vacf()
    acc = acc.cpu().numpy() / np.maximum(cnt, 1)
    assert sorted(rec["index"] for rec in ref["replicas"]) == list(range(len(reps)))
    following = 0
    for rec in ref["replicas"]:
        k = rec["index"]
        assert reps[k]["nx"] == rec["edge"] and reps[k]["seed"] == rec["seed"]
        assert np.array_equal(cnt, rec["vacf_counts"])
        rows = acc[w["n"] * k: w["n"] * (k + 1)]
        e = bench.vacf_errors(rows.mean(axis=0), rec["vacf"], (50, 250), rows)
        ev = nmax_err(ens.particles(k)[1].cpu().numpy(), rec["final_v"])
        c0 = rows[:, 0]
        se_c0 = np.std(c0, ddof=1) / np.sqrt(len(c0)) / abs(c0.mean())
        announce(f"  replica {k} (edge {rec['edge']}): C(0) {e['c0_rel']:.2e} (se {se_c0:.1e}), VACF "
                 f"{e['vacf_abs_err']:.2e}, tail sum {e['tail_integral_rel']:.2e}, final V {ev:.2e}")
        if ev < 1e-3:
            following += 1
            assert e["c0_rel"] < 1e-4 and e["vacf_abs_err"] < 1e-4, k
        else:
            assert e["c0_rel"] < 4.0 * se_c0, k
    # the ensemble average over every particle of every box
    c_ref = np.mean([np.asarray(rec["vacf"]) for rec in sorted(ref["replicas"], key=lambda r: r["index"])],
                    axis=0)
    e = bench.vacf_errors(acc.mean(axis=0), c_ref, (50, 250), acc)
    announce(f"  {following} of {len(reps)} boxes follow the oracle's trajectories; ensemble: C(0) "
             f"{e['c0_rel']:.2e}, VACF {e['vacf_abs_err']:.2e}, tail sum {e['tail_integral_rel']:.2e} "
             f"(se {e['tail_integral_se_rel']:.2e})")
    assert following >= len(reps) // 2
    assert e["c0_rel"] < 1e-2 and e["vacf_abs_err"] < 1e-2
    assert e["tail_integral_rel"] < 2.0 * e["tail_integral_se_rel"]


def test_autotune_choice_is_remembered():
    # lbm_ens_autotune's choice is kept for the process: a later ensemble of
    # the same boxes (same order, storage, device) starts from it; other box
    # lists start from the size-based default.
    from paper_1909_13412_amd import Ensemble

    reps = _small_replicas()
    a = Ensemble(reps, storage="f32", kT=1e-4)
    k, ms = a.autotune(3)
    assert a.launch_config == k and ms[k] > 0.0
    b = Ensemble(reps, storage="f32", kT=1e-4)
    assert b.launch_config == k
    c = Ensemble(reps[::-1], storage="f32", kT=1e-4)
    assert c.launch_config == 0  # small boxes: one node per lane, 512 lanes, plain stores
