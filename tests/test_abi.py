"""The C-ABI library loads, exports every entry point include/*.h declares,
and its host-side validation works (no GPU needed: nothing here launches a
kernel or touches device memory)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1601_00918_amd import _lib, binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(lbm(?:3d)?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_list():
    assert _declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert "gfx950" in binding.lbm_version()


def _geom(**kw):
    d = dict(kind="channel", nx=256, ny=26, lam=64.0, h0=8.0, a=4.0)
    d.update(kw)
    return binding.geom_struct(**d)


def test_required_bytes_scales_with_storage_of_populations():
    one = binding.lbm_required_bytes([_geom()])
    two = binding.lbm_required_bytes([_geom(), _geom()])
    pops = 2 * 18 * 4 * 256 * 26   # two population buffers, FP32
    assert one >= pops
    assert pops <= two - one <= pops + 64 * 1024


def test_required_bytes_rejects_bad_geometry():
    with pytest.raises(_lib.LbmError) as e:
        binding.lbm_required_bytes([_geom(nx=0)])
    assert e.value.status == 1 and "out of range" in str(e.value)
    with pytest.raises(_lib.LbmError):
        binding.lbm_required_bytes([_geom(h0=-1.0)])
    g = [_geom()]
    n = ctypes.c_size_t()
    assert _lib.load().lbm_required_bytes(binding._arr(g, _lib.LbmGeom), 1, 7,
                                          ctypes.byref(n)) == 6   # unknown storage format
    half = binding.lbm_required_bytes(g, storage="f16")
    assert half < binding.lbm_required_bytes(g) and binding.lbm_required_bytes(g, "bf16") == half


def _try_init(geoms, fluids, inits, ws_bytes=1 << 30):
    # A fake, aligned, never-dereferenced workspace pointer: every case below
    # must be rejected on the host before any device work is enqueued.
    return binding.lbm_init(geoms, fluids, inits, "f32", 1 << 20, ws_bytes, 0)


def test_init_rejects_bad_fluid_and_init_on_host():
    g = [_geom()]
    ok_init = [binding.init_struct("uniform")]
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, [binding.fluid_struct((0.5, 1.0), -2.7)], ok_init)
    assert e.value.status == 1 and "tau" in str(e.value)
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, [binding.fluid_struct((1.0, 1.0), -2.7, g=(0.5, 0))], ok_init)
    assert "g[0]" in str(e.value)
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, [binding.fluid_struct((1.0, 1.0), -2.7)], [binding.init_struct(4)])
    assert e.value.status == 1 and "unknown init kind" in str(e.value)
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, [binding.fluid_struct((1.0, 1.0), -2.7)], ok_init, ws_bytes=1024)
    assert e.value.status == 3
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, [binding.fluid_struct((1.0, 1.0), -2.7, reg_order=4)], ok_init)
    assert e.value.status == 1 and "reg_order" in str(e.value)


def test_mask_with_three_fluid_runs_in_a_column_is_unsupported():
    """Two runs per column (a bypass) are supported; a third is rejected on
    the host."""
    mask = np.ones((10, 8), dtype=np.uint8)
    mask[4, 3] = 0
    mask[7, 3] = 0
    keep = []
    g = binding.geom_struct("mask", 8, 10, mask=mask, _keep=keep)
    with pytest.raises(_lib.LbmError) as e:
        _try_init([g], [binding.fluid_struct((1.0, 1.0), -2.7)], [binding.init_struct("uniform")])
    assert e.value.status == 6 and "column 3" in str(e.value)


def test_island_parameters_validate_on_the_host():
    fl = [binding.fluid_struct((1.0, 1.0), -2.7)]
    ini = [binding.init_struct("uniform")]
    g = binding.geom_struct("channel", 256, 26, 64.0, 8.0, 4.0, island=(-1.0, 32.0))
    with pytest.raises(_lib.LbmError) as e:
        _try_init([g], fl, ini)
    assert e.value.status == 1 and "island" in str(e.value)
    g = binding.geom_struct("channel", 256, 26, 64.0, 8.0, 4.0, wall_interp=1, island=(2.0, 32.0))
    with pytest.raises(_lib.LbmError) as e:
        _try_init([g], fl, ini)
    assert e.value.status == 6 and "island" in str(e.value)


def test_mlp_entry_points_validate_on_the_host():
    lib = _lib.load()
    assert lib.lbm_mlp_workspace_bytes(0) == 0
    # nine [B_padded x 128] planes plus one loss partial per 16 samples
    assert lib.lbm_mlp_workspace_bytes(20) == 4 * (9 * 32 * 128 + 2)
    null = ctypes.c_void_p(0)
    assert lib.lbm_mlp_forward(null, null, 4, null, null, 0, null) == 1
    assert lib.lbm_mlp_adam(null, null, null, null, 0, 1e-3, 0.9, 0.999, 1e-8, null) == 1
    # the allocation-free variant: null pointers, B < 1 and B beyond its fixed
    # scratch are rejected before any device call (never dereferenced)
    fake = ctypes.c_void_p(1 << 20)
    assert lib.lbm_mlp_gradient_noalloc(null, fake, fake, 4, fake, fake, null, null) == 1
    assert lib.lbm_mlp_gradient_noalloc(fake, fake, fake, 0, fake, fake, null, null) == 1
    assert lib.lbm_mlp_gradient_noalloc(fake, fake, fake, 2049, fake, fake, null, null) == 1
    assert b"2048" in lib.lbm_last_error()


def test_bench_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reports measured traffic only while the step kernel's source is
    the one the counters were taken with."""
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rec = json.load(open(os.path.join(ROOT, "profiles", "step_kernel_batch256_traffic.txt")))
    t = bench.measured_traffic("f32")
    expect = 1024.0 * (rec["f32"]["fetch_kib"] * rec["fetch_scale"] +
                       rec["f32"]["write_kib"] * rec["write_scale"])
    if t is not None:           # the record matches the current kernel source
        assert t == expect
    assert bench.measured_traffic("bf16") is None   # never profiled
    # the D3Q19 tube record, keyed by the D3Q19 kernel sources
    rec3 = json.load(open(os.path.join(ROOT, "profiles", "step3_kernel_tube_traffic.txt")))
    t3 = bench.measured_traffic("f16", "step3_kernel_tube_traffic.txt", bench.KERNEL3_SOURCES)
    if t3 is not None:
        assert t3 == 1024.0 * (rec3["f16"]["fetch_kib"] * rec3["fetch_scale"] +
                               rec3["f16"]["write_kib"] * rec3["write_scale"])
    # a changed kernel source voids the record
    fake_root = tmp_path
    (fake_root / "profiles").mkdir()
    (fake_root / "paper_1601_00918_amd" / "csrc").mkdir(parents=True)
    (fake_root / "profiles" / "step_kernel_batch256_traffic.txt").write_text(json.dumps(rec))
    (fake_root / "paper_1601_00918_amd" / "csrc" / "lbm_kernels.hip").write_text("// other\n")
    for f in ("lbm_store.h", "lbm_internal.h"):
        (fake_root / "paper_1601_00918_amd" / "csrc" / f).write_text("// other\n")
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    assert bench.measured_traffic("f32") is None


def test_degenerate_and_oversized_inputs_are_rejected():
    with pytest.raises(_lib.LbmError):
        binding.lbm_required_bytes([])                      # no instance
    # an instance whose population block would exceed 32-bit offsets
    with pytest.raises(_lib.LbmError) as e:
        binding.lbm_required_bytes([_geom(nx=1 << 16, ny=1 << 12, lam=16384.0, h0=1000.0,
                                          a=10.0)])
    assert e.value.status == 1


def test_lbm3d_required_bytes_and_validation():
    from paper_1601_00918_amd import binding3d as b3
    g = b3.geom3_struct("tube", 96, 18, 18, lam=32.0, r0=6.0, a=2.0)
    f32 = b3.lbm3d_required_bytes(g, "f32")
    f16 = b3.lbm3d_required_bytes(g, "f16")
    snap = b3.lbm3d_required_bytes(g, "f32", snapshot=True)
    pops32 = 2 * 18 * 18 * 19 * 128 * 8    # two buffers, 19 planes of 128 FP32 pairs per row
    pops16 = 2 * 18 * 18 * 20 * 128 * 4    # 20 planes (references included) of 4-byte pairs
    assert f32 - f16 == pops32 - pops16
    assert snap - f32 == pops32 // 2
    with pytest.raises(_lib.LbmError) as e:
        b3.lbm3d_required_bytes(b3.geom3_struct("tube", 2, 18, 18, lam=32.0, r0=6.0, a=2.0))
    assert e.value.status == 1
    with pytest.raises(_lib.LbmError) as e:   # one buffer would exceed 32-bit offsets
        b3.lbm3d_required_bytes(b3.geom3_struct("box", 4096, 1024, 64))
    assert e.value.status == 6
    with pytest.raises(_lib.LbmError):
        b3.lbm3d_required_bytes(b3.geom3_struct("tube", 96, 18, 18, lam=32.0, r0=-1.0, a=2.0))
    n = ctypes.c_size_t()
    assert _lib.load().lbm3d_required_bytes(ctypes.byref(g), 9, ctypes.byref(n)) == 6


def test_lbm3d_interpolated_wall_table_size_and_validation():
    """The workspace grows by the column table (8 bytes per (x, y) column) and
    one row of 18 FP32 link fractions per fluid node with a solid neighbour,
    counted here from the mask with numpy; interpolated walls exist only for
    the analytic tube."""
    import synth
    from paper_1601_00918_amd import binding3d as b3
    cx, cy, cz = (np.array(v) for v in zip(*b3.C3))
    for lam, r0, a in ((32.0, 6.0, 2.0), (64.0, 9.3, 3.7)):
        nx, side = int(3 * lam), int(2 * (r0 + a) + 2)
        plain = b3.lbm3d_required_bytes(b3.geom3_struct("tube", nx, side, side, lam=lam,
                                                        r0=r0, a=a), "f16")
        interp = b3.lbm3d_required_bytes(b3.geom3_struct("tube", nx, side, side, lam=lam,
                                                         r0=r0, a=a, wall_interp=True), "f16")
        m = synth.tube_mask(nx, side, side, lam, r0, a).astype(bool)
        padded = np.zeros((side + 2, side + 2, nx), dtype=bool)
        padded[1:-1, 1:-1] = m
        walled = np.zeros_like(m)
        for i in range(1, 19):   # source x - c_i solid
            src = np.roll(padded, int(cx[i]), axis=2)[1 - cz[i]:side + 1 - cz[i],
                                                       1 - cy[i]:side + 1 - cy[i]]
            walled |= m & ~src
        rows = int(walled.sum())
        up = lambda v: (v + 255) // 256 * 256
        assert interp - plain == up(8 * nx * side) + up(72 * rows), (rows, interp - plain)
    for kind in ("box", "mask"):
        g = b3.geom3_struct(kind, 8, 8, 8, mask=np.ones((8, 8, 8), np.uint8),
                            wall_interp=True)
        with pytest.raises(_lib.LbmError) as e:
            b3.lbm3d_required_bytes(g)
        assert e.value.status == 6 and "tube" in str(e.value)
    g = b3.geom3_struct("tube", 96, 18, 18, lam=32.0, r0=6.0, a=2.0)
    g.wall_interp = 2
    with pytest.raises(_lib.LbmError) as e:
        b3.lbm3d_required_bytes(g)
    assert e.value.status == 1


def test_lbm3d_critical_pressure_validates_on_the_host():
    """Rejected before any device work (the workspace pointer is never used)."""
    import synth
    from paper_1601_00918_amd import binding3d as b3
    box = b3.cp3_problem(synth.config_box3d(n=16, r=4.0), 1e-5, 1e-4, 0.195, 1.03, 10, 100)
    tube = b3.cp3_problem(synth.config_tube(lam=32, r0=6.0, a=2.0), 1e-4, 1e-5, 0.195, 1.03,
                          10, 100)
    res = (_lib.LbmCpResult * 1)()
    opts = binding.cp_options()
    lib = _lib.load()
    for prob, what in ((box, "tube geometry"), (tube, "bracket")):
        arr = (_lib.Lbm3dCpProblem * 1)(prob)
        st = lib.lbm3d_critical_pressure(arr, 1, ctypes.byref(opts), ctypes.c_void_p(1 << 20),
                                         1 << 30, None, res)
        assert st == 1 and what in lib.lbm_last_error().decode()
    # options are checked first: verbose is 0 or 1
    bad = binding.cp_options(verbose=2)
    arr = (_lib.Lbm3dCpProblem * 1)(box)
    st = lib.lbm3d_critical_pressure(arr, 1, ctypes.byref(bad), ctypes.c_void_p(1 << 20),
                                     1 << 30, None, res)
    assert st == 1 and "options" in lib.lbm_last_error().decode()


def test_interpolated_walls_validate_on_the_host():
    fl = [binding.fluid_struct((1.0, 1.0), -2.7)]
    ini = [binding.init_struct("uniform")]
    flat = dict(lam=64.0, h0=8.0, a=0.0)
    plain = binding.lbm_required_bytes([binding.geom_struct("channel", 64, 18, **flat)])
    interp = binding.lbm_required_bytes(
        [binding.geom_struct("channel", 64, 18, wall_interp=1, **flat)])
    assert interp - plain >= 64 * 32 * 4      # the wall table: 32 floats per column
    cases = [
        (binding.geom_struct("box", 32, 32, wall_interp=1), "f32", 6, "analytic channel"),
        (binding.geom_struct("channel", 64, 18, wall_interp=2, **flat), "f32", 1, "0 or 1"),
        (binding.geom_struct("channel", 64, 18, y_offset=1.5, **flat), "f32", 1, "y_offset"),
        # slope a 2 pi / lambda = 1.57: fluid runs of neighbouring columns
        # differ by two rows
        (binding.geom_struct("channel", 32, 20, wall_interp=1, lam=16.0, h0=6.0, a=4.0),
         "f32", 6, "steeper"),
    ]
    for g, storage, status, text in cases:
        with pytest.raises(_lib.LbmError) as e:
            binding.lbm_init([g], fl, ini, storage, 1 << 20, 1 << 30, 0)
        assert e.value.status == status and text in str(e.value), (text, str(e.value))


def test_multiple_slugs_validate_on_the_host():
    """Rejected before any device work (the workspace pointer is never used)."""
    from paper_1601_00918_amd import binding3d as b3
    g = [_geom()]
    fl = [binding.fluid_struct((1.0, 1.0), -2.7)]
    bad = [binding.init_struct("slug", slugs=[(0.0, 10.0)] * 9),            # > LBM_MAX_SLUGS
           binding.init_struct("slug", slugs=[(0.0, 10.0), (40.0, -1.0)]),  # negative length
           binding.init_struct("slug", slugs=[(0.0, 10.0), (float("nan"), 5.0)])]
    for ini in bad:
        with pytest.raises(_lib.LbmError) as e:
            _try_init(g, fl, [ini])
        assert e.value.status == 1 and "slug" in str(e.value)
    nul = binding.init_struct("slug")
    nul.n_slugs = 1                                   # count without the array
    with pytest.raises(_lib.LbmError) as e:
        _try_init(g, fl, [nul])
    assert "slugs array" in str(e.value)
    g3 = b3.geom3_struct("tube", 96, 18, 18, lam=32.0, r0=6.0, a=2.0)
    f3 = b3.fluid3_struct((1.0, 1.0), -2.7)
    i3 = b3.init3_struct("slug", slugs=[(0.0, 10.0)] * 9)
    with pytest.raises(_lib.LbmError) as e:
        b3.lbm3d_init(g3, f3, i3, "f32", 1 << 20, 1 << 30, 0)
    assert e.value.status == 1 and "n_slugs" in str(e.value)


def test_stream_copy_validates_on_the_host():
    """Null or misaligned pointers, sizes not a multiple of 4 and chunk sizes
    that are not multiples of 16 KiB are rejected before anything is
    launched."""
    import ctypes
    lib = _lib.load()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)  # never dereferenced
    assert lib.lbm_stream_copy(None, b, 64, 1 << 18, None) == 1
    assert lib.lbm_stream_copy(a, b, 62, 1 << 18, None) == 1
    assert lib.lbm_stream_copy(ctypes.c_void_p((1 << 20) + 4), b, 64, 1 << 18, None) == 1
    assert lib.lbm_stream_copy(a, b, 64, 1000, None) == 1
    assert lib.lbm_stream_copy(a, b, 64, 0, None) == 1


def test_slug_interface_width_validates_on_the_host():
    g = [_geom()]
    fl = [binding.fluid_struct((1.0, 1.0), -2.7)]
    for w in (-1.0, float("nan"), float("inf")):
        with pytest.raises(_lib.LbmError) as e:
            _try_init(g, fl, [binding.init_struct("slug", x0=4.0, length=20.0, width=w)])
        assert e.value.status == 1 and "width" in str(e.value)
