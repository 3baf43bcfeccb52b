"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte counts, the gate on the committed PMC traffic figure, and the
one-thread oracle leg."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr or "one GPU" in res.stdout


def test_algorithmic_bytes_per_node():
    import bench

    # Q loads + Q stores of a population and the one-bit forcing flag
    assert bench.collide_bytes_per_node("f64") == 304.125
    assert bench.collide_bytes_per_node("f32") == 152.125
    assert bench.collide_bytes_per_node("bf16") == 76.125
    assert bench.collide_bytes_per_node("f16") == 76.125
    assert bench.collide_bytes_per_node("f32", 15) == 120.125
    assert bench.parse_variant("bf16q15") == ("bf16", 15)
    assert bench.parse_variant("f64") == ("f64", 19)


def test_traffic_figure_is_gated_on_the_kernel_sources(monkeypatch):
    import bench
    from paper_1909_13412_amd import build as hip_build

    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 64
    with open(bench.PMC_PROFILE) as fh:
        line = next(ln for ln in fh if ln.strip().startswith("PMC_TRAFFIC "))
    rec = json.loads(line.strip()[len("PMC_TRAFFIC "):])
    t = bench.pmc_traffic("f32")
    if rec["source_sha256"] == h:
        # profiled build: the counters give the stream-collide's HBM bytes,
        # within a few per cent of the algorithmic 152.125 B per node
        alg = bench.collide_bytes_per_node("f32") * 256 ** 3
        assert t is not None and 0.99 < t / alg < 1.03
    else:
        assert t is None
    # any change to the compile flags (or the kernel sources) withdraws it
    monkeypatch.setattr(hip_build, "HIPCC_FLAGS", hip_build.HIPCC_FLAGS + ["-DPROBE"])
    assert bench.kernel_source_hash() != h
    assert bench.pmc_traffic("f32") is None


def test_one_thread_oracle_leg():
    import bench
    from paper_1909_13412_amd.inputs import WORKLOADS

    w = dict(WORKLOADS["relaxation32"])
    w["name"] = "relaxation32"
    w.setdefault("max_lag", 10)
    w.setdefault("stride", 2)
    out = bench.cpu_baseline_one_thread(w, 2)
    assert out is not None
    assert out["cores"] == 1 and out["kind"] == "oracle" and out["value"] > 0


def test_row_group_layout_formula():
    # helpers.raw_rows decodes a raw lattice of the documented layout, element
    # (a, x, y, z) at ((z ny + R (y / R)) Q + y mod R) nx + a R nx + x: a buffer
    # filled with each element's own (a, x, y, z) code decodes to the
    # canonical [z][y][a][x] array of codes, for every R dividing ny.
    import numpy as np

    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import raw_rows

    nx, ny, nz, q = 5, 12, 3, 19
    a_, x_, y_, z_ = np.meshgrid(np.arange(q), np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    code = ((z_ * ny + y_) * q + a_) * nx + x_
    want = np.empty((nz, ny, q, nx), dtype=np.int64)
    want[z_, y_, a_, x_] = code
    for R in (1, 2, 3, 4, 6, 12):
        raw = np.empty(q * nx * ny * nz, dtype=np.int64)
        idx = ((z_ * ny + R * (y_ // R)) * q + y_ % R) * nx + a_ * R * nx + x_
        raw[idx] = code
        assert np.array_equal(raw_rows(raw, nx, ny, nz, R), want), R
