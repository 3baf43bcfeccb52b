"""Host-side checks of the C ABI: the library loads, exports every entry point the
header declares, sizes its buffers, and rejects bad arguments before touching a
device.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_13412_amd import _abi

    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("liblbmbp.so is not built (run __graft_entry__.build())")
    return _abi.load()


def _header_functions():
    text = open(os.path.join(ROOT, "include", "lbmbp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_and_binding_agree():
    from paper_1909_13412_amd import _abi

    assert sorted(_abi.EXPORTS) == _header_functions()
    for name in ("lbm_init", "lbm_step", "particles_couple", "lbm_observables", "lbm_vacf_config"):
        assert name in _abi.EXPORTS


def test_library_exports_every_declared_symbol(lib):
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(lib):
    from paper_1909_13412_amd import _abi

    assert ctypes.sizeof(_abi.GridDesc) == 40
    assert ctypes.sizeof(_abi.ParticleDesc) == 56
    assert ctypes.sizeof(_abi.EnsembleDesc) == 56
    assert ctypes.sizeof(_abi.ReplicaDesc) == 40


def _grid(nx=16, ny=16, nz=16, tau=0.8, storage=1, s=16, q=0, reserved=0):
    from paper_1909_13412_amd import _abi

    return _abi.GridDesc(nx, ny, nz, tau, storage, s, q, reserved)


def test_lattice_and_scratch_sizes(lib):
    sz = ctypes.c_size_t()
    for storage, elem in ((0, 8), (1, 4), (2, 2), (3, 2)):
        g = _grid(nx=37, ny=23, nz=19, storage=storage)
        assert lib.lbm_lattice_bytes(ctypes.byref(g), ctypes.byref(sz)) == 0
        ncell = 37 * 23 * 19
        assert sz.value >= 19 * ncell * elem
        assert sz.value % 256 == 0
        # unpadded rows, the total rounded up to 256 bytes
        assert sz.value == -(-(19 * 37 * 23 * 19 * elem) // 256) * 256
    g = _grid(nx=256, ny=256, nz=256)
    assert lib.lbm_lattice_bytes(ctypes.byref(g), ctypes.byref(sz)) == 0
    assert sz.value == 19 * 256**3 * 4
    for q in (19, 15):
        gq = _grid(nx=256, ny=256, nz=256, q=q)
        assert lib.lbm_lattice_bytes(ctypes.byref(gq), ctypes.byref(sz)) == 0
        assert sz.value == q * 256**3 * 4
    assert lib.lbm_grid_scratch_bytes(ctypes.byref(g), ctypes.byref(sz)) == 0
    assert sz.value >= 2 * 256**3 // 8
    assert lib.lbm_particle_scratch_bytes(ctypes.byref(g), 4096, ctypes.byref(sz)) == 0
    assert sz.value > 0
    assert lib.lbm_particle_scratch_bytes(ctypes.byref(g), 0, ctypes.byref(sz)) == 0
    assert sz.value == 0
    # the particle count's documented range is 0..2^24
    assert lib.lbm_particle_scratch_bytes(ctypes.byref(g), 1 << 24, ctypes.byref(sz)) == 0
    assert sz.value >= (1 << 24) * 8 * 4  # at least each lane's last node
    assert lib.lbm_particle_scratch_bytes(ctypes.byref(g), (1 << 24) + 1, ctypes.byref(sz)) == 1
    assert lib.lbm_particle_scratch_bytes(ctypes.byref(g), -1, ctypes.byref(sz)) == 1
    assert lib.lbm_vacf_origin_bytes(64, 2000, 10, ctypes.byref(sz)) == 0
    assert sz.value == 201 * 64 * 3 * 8


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(ny=0), dict(nz=-4), dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")),
    dict(storage=7), dict(storage=3, s=40), dict(nx=2048, ny=2048, nz=1024), dict(q=27),
    dict(q=16), dict(reserved=1),
])
def test_invalid_grids_rejected(lib, bad):
    kw = dict(nx=8, ny=8, nz=8, tau=0.8, storage=1, s=16)
    kw.update(bad)
    g = _grid(**kw)
    sz = ctypes.c_size_t()
    assert lib.lbm_lattice_bytes(ctypes.byref(g), ctypes.byref(sz)) == 1
    assert lib.lbm_grid_scratch_bytes(ctypes.byref(g), ctypes.byref(sz)) == 1
    ctx = ctypes.c_void_p()
    buf = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    assert lib.lbm_init(ctypes.byref(g), buf, ctypes.c_void_p(512), buf, None, ctypes.byref(ctx)) == 1


def test_init_rejects_null_and_misaligned_buffers(lib):
    g = _grid()
    ctx = ctypes.c_void_p()
    assert lib.lbm_init(ctypes.byref(g), None, ctypes.c_void_p(512), ctypes.c_void_p(1024), None,
                        ctypes.byref(ctx)) == 1
    assert lib.lbm_init(ctypes.byref(g), ctypes.c_void_p(260), ctypes.c_void_p(512),
                        ctypes.c_void_p(1024), None, ctypes.byref(ctx)) == 1
    assert lib.lbm_init(ctypes.byref(g), ctypes.c_void_p(512), ctypes.c_void_p(512),
                        ctypes.c_void_p(1024), None, ctypes.byref(ctx)) == 1
    assert lib.lbm_init(ctypes.byref(g), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                        ctypes.c_void_p(2048), None, None) == 1


def test_null_context_rejected(lib):
    out = (ctypes.c_double * 7)()
    assert lib.lbm_step(None, 1) == 1
    assert lib.lbm_observables(None, out) == 1
    assert lib.lbm_destroy(None) == 1
    assert lib.lbm_particle_radius(None) < 0
    k = ctypes.c_int32()
    assert lib.lbm_get_shape(None, ctypes.byref(k)) == 1
    assert lib.lbm_ens_get_shape(None, ctypes.byref(k)) == 1
    assert lib.lbm_set_shape(None, 0) == 1
    o = ctypes.c_int32()
    assert lib.lbm_set_sweep_launch(None, 0, 0) == 1
    assert lib.lbm_get_sweep_launch(None, ctypes.byref(o), ctypes.byref(k)) == 1
    assert lib.lbm_set_layout(None, 1) == 1
    assert lib.lbm_get_layout(None, ctypes.byref(k)) == 1
    assert lib.lbm_ens_set_layout(None, 1) == 1
    assert lib.lbm_ens_get_layout(None, 0, ctypes.byref(k)) == 1
    assert lib.lbm_ens_set_sweep_launch(None, 0, 0) == 1
    assert lib.lbm_ens_get_sweep_launch(None, ctypes.byref(o), ctypes.byref(k)) == 1
    assert lib.lbm_observables_noalloc(None, out) == 1
    assert lib.lbm_set_pair_force(None, ctypes.c_double(0.1), ctypes.c_double(1.0)) == 1
    assert lib.lbm_pair_forces(None, None) == 1
    assert lib.lbm_autotune(None, 5, None, None) == 1
    ms = ctypes.c_double()
    assert lib.lbm_stream_ceiling(None, -1, 5, ctypes.byref(ms)) == 1
    f = ctypes.c_uint32()
    assert lib.lbm_warnings(None, ctypes.byref(f)) == 1


def test_every_entry_point_validates_null_arguments(lib):
    # Every status-returning entry point, called with each pointer NULL and
    # each number zero, rejects the call (LBM_E_INVAL) before it touches
    # memory or the device.
    from paper_1909_13412_amd import _abi

    numbers = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t,
               ctypes.c_int)
    checked = 0
    for name in _abi.EXPORTS:
        fn = getattr(lib, name)
        if fn.restype is not ctypes.c_int:
            continue  # lbm_particle_radius, lbm_status_string
        args = [0.0 if t is ctypes.c_double else 0 if t in numbers else None for t in fn.argtypes]
        assert fn(*args) == 1, name
        checked += 1
    assert checked >= 40


def test_status_strings(lib):
    for code in range(6):
        s = lib.lbm_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert lib.lbm_status_string(0) == b"ok"
    assert lib.lbm_status_string(99) == b"unknown status"


def test_ensemble_sizes_and_validation(lib):
    from paper_1909_13412_amd import _abi

    d = _abi.EnsembleDesc(3, 1, 16, 0, 10.0, 1.0, 1e-4, 0.0, 0, 0)
    reps = (_abi.ReplicaDesc * 3)(_abi.ReplicaDesc(48, 48, 48, 8, 0.8, 1, 0, 0),
                                  _abi.ReplicaDesc(37, 20, 11, 3, 0.7, 2, 1, 0),
                                  _abi.ReplicaDesc(96, 96, 96, 8, 0.8, 3, 2, 0))
    lat, scr = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lbm_ens_bytes(ctypes.byref(d), reps, ctypes.byref(lat), ctypes.byref(scr)) == 0
    want = 19 * 4 * (48 * 48 * 48 + 37 * 20 * 11 + 96 * 96 * 96)
    assert lat.value == -(-want // 256) * 256
    cells = 48**3 + 37 * 20 * 11 + 96**3
    assert scr.value > 2 * 24 * cells
    bad = (_abi.ReplicaDesc * 3)(*reps)
    bad[1].tau = 0.5
    assert lib.lbm_ens_bytes(ctypes.byref(d), bad, ctypes.byref(lat), ctypes.byref(scr)) == 1
    bad[1].tau = 0.7
    bad[2].n = 0
    assert lib.lbm_ens_bytes(ctypes.byref(d), bad, ctypes.byref(lat), ctypes.byref(scr)) == 1
    # one box of 19 x 620^3 >= 2^32 population elements: beyond a box's 32-bit index
    big = (_abi.ReplicaDesc * 1)(_abi.ReplicaDesc(620, 620, 620, 8, 0.8, 1, 0, 0))
    d1 = _abi.EnsembleDesc(1, 1, 16, 0, 10.0, 1.0, 1e-4, 0.0, 0, 0)
    assert lib.lbm_ens_bytes(ctypes.byref(d1), big, ctypes.byref(lat), ctypes.byref(scr)) == 1
    big[0].nx = 580  # 19 x 580 x 620 x 620 < 2^32
    assert lib.lbm_ens_bytes(ctypes.byref(d1), big, ctypes.byref(lat), ctypes.byref(scr)) == 0
    d.nrep = 0
    assert lib.lbm_ens_bytes(ctypes.byref(d), reps, ctypes.byref(lat), ctypes.byref(scr)) == 1
    out = ctypes.c_void_p()
    assert lib.lbm_ens_init(None, reps, None, None, None, None, None, None, ctypes.byref(out)) == 1
    assert lib.lbm_ens_step(None, 1) == 1


def test_launch_configuration_count_matches_header():
    from paper_1909_13412_amd import _abi

    text = open(os.path.join(ROOT, "include", "lbmbp.h")).read()
    m = re.search(r"#define LBM_NUM_SHAPES (\d+)", text)
    assert m and int(m.group(1)) == _abi.LBM_NUM_SHAPES == 10
    m = re.search(r"#define LBM_ENS_GRAPH_STEPS (\d+)", text)
    assert m and int(m.group(1)) == _abi.LBM_ENS_GRAPH_STEPS


def test_binding_attributes_not_shadowed_by_properties():
    # An attribute the binding assigns on its instances must not also be a
    # read-only property of the class (the assignment would fail at run time,
    # and only on a GPU).
    import ast

    src = open(os.path.join(ROOT, "paper_1909_13412_amd", "sim.py")).read()
    classes = {n.name: n for n in ast.parse(src).body if isinstance(n, ast.ClassDef)}

    def props_of(cls):
        own = {fn.name for fn in cls.body if isinstance(fn, ast.FunctionDef)
               and any(isinstance(d, ast.Name) and d.id == "property" for d in fn.decorator_list)}
        for b in cls.bases:  # properties inherited from classes of the same module
            if isinstance(b, ast.Name) and b.id in classes:
                own |= props_of(classes[b.id])
        return own

    checked = 0
    for cls in classes.values():
        assigned = set()
        for fn in (n for n in cls.body if isinstance(n, ast.FunctionDef)):
            for node in ast.walk(fn):
                targets = node.targets if isinstance(node, ast.Assign) else (
                    [node.target] if isinstance(node, (ast.AugAssign, ast.AnnAssign)) else [])
                for t in targets:
                    for e in (t.elts if isinstance(t, ast.Tuple) else [t]):
                        if isinstance(e, ast.Attribute) and isinstance(e.value, ast.Name) and e.value.id == "self":
                            assigned.add(e.attr)
        assert not (props_of(cls) & assigned), (cls.name, props_of(cls) & assigned)
        checked += "r" in props_of(cls)
    assert checked >= 2  # Lattice and Ensemble inherit r and v


def test_row_aligned_mapping_covers_every_node_once():
    # The lane -> node map of the row-aligned stream-collide configurations,
    # restated: each row takes nx rounded up to whole 64-lane wavefronts; a
    # 256-lane block holds 256 // lanes whole rows (lanes past them idle) or a
    # row spans several blocks.  Every node must be visited exactly once for
    # widths that divide the block, that do not, and rows longer than a block.
    BS = 256
    for nx in (2, 40, 48, 64, 65, 100, 129, 130, 192, 193, 250, 256, 257, 300, 513, 700):
        ny, nz = 3, 2
        lpr = (nx + 63) // 64 * 64
        nrows = ny * nz
        grid = -(-nrows // (BS // lpr)) if lpr <= BS else nrows * -(-lpr // BS)
        count = {}
        for b in range(grid):
            for t in range(BS):
                if lpr <= BS:
                    slot = t // lpr
                    ok, row, x = slot < BS // lpr, b * (BS // lpr) + slot, t % lpr
                else:
                    bpr = -(-lpr // BS)
                    ok, row, x = True, b // bpr, (b % bpr) * BS + t
                if ok and x < nx and row < nrows:
                    count[row * nx + x] = count.get(row * nx + x, 0) + 1
        assert sorted(count) == list(range(nx * nrows)) and set(count.values()) == {1}, nx
