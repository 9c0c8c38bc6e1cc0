"""The C-ABI library on the CPU: it loads, exports every function that
include/fof.h declares, and rejects bad arguments on the host before touching
a device (no compute call is made here)."""
import ctypes
import re

import numpy as np
import pytest

import paper_2003_11468_amd as fof


def declared_functions():
    text = open(fof.HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fof_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    lib = fof.load_library()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(fof.EXPORTS)


def test_status_strings():
    for s in range(7):
        assert fof.fof_status_string(s)
    assert fof.fof_status_string(0) == "ok"


def test_default_options():
    o = fof.fof_default_options()
    assert o.predicate == fof.FOF_PRED_FP32_FILTER and o.strict_less == 0 and o.cell_factor == 0.0


def _ctx(**kw):
    return fof.fof_create(fof.make_options(**kw))


def test_create_rejects_bad_options():
    for kw in (dict(cell_factor=0.5), dict(cell_factor=float("inf")), dict(segment_log2=5), dict(segment_log2=17),
               dict(segment_log2=-1), dict(domains=-1), dict(domains=4097)):
        with pytest.raises(fof.FoFError) as e:
            _ctx(**kw)
        assert e.value.status == fof.FOF_ERR_INVALID_ARG
    o = fof.fof_default_options()
    o.predicate = 7
    with pytest.raises(fof.FoFError):
        fof.fof_create(o)
    o = fof.fof_default_options()
    o.reserved[1] = 1
    with pytest.raises(fof.FoFError):
        fof.fof_create(o)
    for bad in (-1, 2):
        o = fof.fof_default_options()
        o.link_order = bad
        with pytest.raises(fof.FoFError) as e:
            fof.fof_create(o)
        assert e.value.status == fof.FOF_ERR_INVALID_ARG
    o = fof.fof_default_options()
    o.link_order = 1
    fof.fof_destroy(fof.fof_create(o))
    o = fof.make_options(schedule=fof.schedule_bits(giant_skip=True), domains=4)   # no domain mode with it
    with pytest.raises(fof.FoFError) as e:
        fof.fof_create(o)
    assert e.value.status == fof.FOF_ERR_INVALID_ARG
    fof.fof_destroy(fof.fof_create(fof.make_options(schedule=fof.schedule_bits(giant_skip=True))))
    fof.fof_destroy(fof.fof_create(fof.make_options(schedule=fof.schedule_bits(tile_join=False))))
    assert fof.schedule_bits(tile_join=False) == 64
    for field, bad in (("schedule", 128), ("schedule", -1), ("compression", 2), ("compression", -1)):
        o = fof.fof_default_options()
        setattr(o, field, bad)
        with pytest.raises(fof.FoFError) as e:
            fof.fof_create(o)
        assert e.value.status == fof.FOF_ERR_INVALID_ARG, field
    o = fof.make_options(schedule=fof.schedule_bits(4096, 8192, False), compression="depth2")
    assert o.schedule == 3 | (3 << 2) | 16 and o.compression == 1
    fof.fof_destroy(fof.fof_create(o))


def test_workspace_bytes_scales_with_particles_and_cells():
    ctx = _ctx()
    try:
        small = fof.fof_workspace_bytes(ctx, [0, 1000], 1.0, 0.02)
        big = fof.fof_workspace_bytes(ctx, [0, 100000], 1.0, 0.002)
        assert big > small > 1000 * 36
        two = fof.fof_workspace_bytes(ctx, [0, 1000, 3000], [1.0, 2.0], [0.02, 0.03])
        assert two > small
        assert fof.fof_workspace_bytes(ctx, [0, 0], 1.0, 0.1) > 0          # empty box
    finally:
        fof.fof_destroy(ctx)


@pytest.mark.parametrize("offsets,box,lx", [
    ([0, 10], 1.0, 0.0),                 # l_x <= 0
    ([0, 10], 1.0, -0.1),
    ([0, 10], 1.0, float("nan")),
    ([0, 10], 0.0, 0.1),                 # L <= 0
    ([0, 10], float("inf"), 0.1),
    ([0, 10], 1.0, 0.34),                # fewer than 3 cells of side >= l_x
    ([1, 10], 1.0, 0.1),                 # offsets must start at 0
    ([0, 10, 5], [1.0, 1.0], [0.1, 0.1]),  # decreasing offsets
    ([0, 2 ** 31], 1.0, 0.1),            # too many particles
])
def test_host_validation(offsets, box, lx):
    ctx = _ctx()
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_workspace_bytes(ctx, offsets, box, lx)
        assert e.value.status == fof.FOF_ERR_INVALID_ARG
        with pytest.raises(fof.FoFError) as e:
            fof.fof_build_cells(ctx, None, offsets, box, lx)
        assert e.value.status == fof.FOF_ERR_INVALID_ARG
    finally:
        fof.fof_destroy(ctx)


def test_cells_per_axis_up_to_2048():
    # up to 2048 cells per axis (2^33 cells in a box), and at most 2^34 cells in all
    opt = fof.make_options(cell_factor=1.0)
    assert fof.fof_describe_box(1000, 1.0, 1.0 / 2048.5, opt)["cells_per_axis"] == 2048
    with pytest.raises(fof.FoFError) as e:
        fof.fof_describe_box(1000, 1.0, 1.0 / 2049.5, opt)
    assert e.value.status == fof.FOF_ERR_UNSUPPORTED
    ctx = _ctx(cell_factor=1.0)
    try:
        assert fof.fof_workspace_bytes(ctx, [0, 1000], 1.0, 1.0 / 1800.5) > (1800 ** 3) // 4   # occupancy words
        assert fof.fof_workspace_bytes(ctx, [0, 10, 20], 1.0, 1.0 / 2048.5) > 0                  # 2^34 cells
        with pytest.raises(fof.FoFError) as e:
            fof.fof_workspace_bytes(ctx, [0, 10, 20, 30], 1.0, 1.0 / 2048.5)
        assert e.value.status == fof.FOF_ERR_UNSUPPORTED
    finally:
        fof.fof_destroy(ctx)


def test_too_many_cells_is_unsupported():
    ctx = _ctx(cell_factor=1.0)
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_workspace_bytes(ctx, [0, 10 ** 9], 1.0, 1e-4)
        assert e.value.status == fof.FOF_ERR_UNSUPPORTED
    finally:
        fof.fof_destroy(ctx)


def test_call_order_and_missing_workspace():
    ctx = _ctx()
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_link(ctx)
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        with pytest.raises(fof.FoFError) as e:
            fof.fof_finalize(ctx, None, None)
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        with pytest.raises(fof.FoFError) as e:       # valid boxes, no workspace set
            fof.fof_build_cells(ctx, None, [0, 0], 1.0, 0.1)
        assert e.value.status == fof.FOF_ERR_WORKSPACE
        with pytest.raises(fof.FoFError) as e:       # misaligned workspace pointer
            fof.load_library()
            st = fof.load_library().fof_set_workspace(ctx, ctypes.c_void_p(0x1001), 4096)
            fof._check(st, "fof_set_workspace")
        assert e.value.status == fof.FOF_ERR_WORKSPACE
        with pytest.raises(fof.FoFError) as e:
            fof.fof_graph_launch(ctx)
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        with pytest.raises(fof.FoFError):
            fof.fof_read_n_groups(ctx, 1)
    finally:
        fof.fof_destroy(ctx)


def test_null_arguments():
    lib = fof.load_library()
    assert lib.fof_create(None, None, None) == fof.FOF_ERR_INVALID_ARG
    assert lib.fof_link(None) == fof.FOF_ERR_INVALID_ARG
    assert lib.fof_destroy(None) == fof.FOF_OK
    ctx = _ctx()
    try:
        assert lib.fof_workspace_bytes(ctx, None, None, None, 1, None) == fof.FOF_ERR_INVALID_ARG
        off = np.array([0, 4], dtype=np.int64)
        L = np.ones(1)
        assert lib.fof_build_cells(ctx, None, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   L.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   (L * 0.1).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1) \
            == fof.FOF_ERR_INVALID_ARG          # 4 particles but no position pointer
    finally:
        fof.fof_destroy(ctx)


def test_catalogue_validation():
    ctx = _ctx()
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_catalogue(ctx, None, None, 1)
        assert e.value.status == fof.FOF_ERR_BAD_STATE       # nothing built yet
        for bad in (0, -3):
            with pytest.raises(fof.FoFError) as e:
                fof.fof_catalogue(ctx, None, None, bad)
            assert e.value.status == fof.FOF_ERR_INVALID_ARG
    finally:
        fof.fof_destroy(ctx)


def test_relink_needs_a_build():
    ctx = _ctx()
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_relink(ctx, 0.01, 1)
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        assert fof.load_library().fof_relink(ctx, None, 1) == fof.FOF_ERR_INVALID_ARG
    finally:
        fof.fof_destroy(ctx)


def test_kernel_times_need_the_option():
    ctx = _ctx()
    try:
        with pytest.raises(fof.FoFError) as e:
            fof.fof_get_kernel_times(ctx)
        assert e.value.status == fof.FOF_ERR_BAD_STATE
    finally:
        fof.fof_destroy(ctx)
    names = [fof.fof_kernel_name(k) for k in range(15)]
    assert names[0] == "k_clear" and "k_link_dense" in names and "k_dense_premerge" in names and "?" not in names
    assert fof.fof_kernel_name(15) == "?"
    assert fof.fof_kernel_name(99) == "?"


def test_tune_workload_key_and_cache(tmp_path):
    from paper_2003_11468_amd import tune

    k1 = tune.workload_key([0, 256 ** 3], 1.0, 0.2 / 256, "fp32_filter")
    k2 = tune.workload_key([0, 255 ** 3], 1.0, 0.2 / 255, "fp32_filter")
    k3 = tune.workload_key([0, 256 ** 3], 1.0, 0.5 / 256, "fp32_filter")
    assert k1 == k2 and k1 != k3 and "b0.2" in k1
    assert tune.workload_key([0, 1000, 3000], [1.0, 1.0], [0.02, 0.02], "fp64").startswith("fp64|le|")
    path = str(tmp_path / "t.json")
    tune._save(path, {"a": {"cell_factor": 2.0, "dense_min": 16}})
    assert tune._load(path)["a"]["dense_min"] == 16
    assert tune._load(str(tmp_path / "missing.json")) == {}


def test_noalloc_host_validation():
    """fof_label_noalloc rejects bad arguments and oversize runs on the host,
    before it looks for a device (none here)."""
    lib = fof.load_library()
    ng = ctypes.c_int64(0)
    st = lib.fof_label_noalloc(None, None, None, 10, 1.0, 0.1, None, None, ctypes.byref(ng))
    assert st == fof.FOF_ERR_INVALID_ARG                  # positions and outputs missing
    fake = ctypes.c_void_p(0x10000)
    for n, box, lx in ((-1, 1.0, 0.1), (10, 1.0, 0.0), (10, 0.0, 0.1), (10, 1.0, 0.4)):
        assert lib.fof_label_noalloc(None, None, fake, n, box, lx, fake, fake, None) == fof.FOF_ERR_INVALID_ARG
    n = 4_000_000
    assert lib.fof_label_noalloc(None, None, fake, n, 1.0, 0.2 / n ** (1 / 3), fake, fake, None) \
        == fof.FOF_ERR_UNSUPPORTED
    o = fof.make_options(timings=True)
    assert lib.fof_label_noalloc(ctypes.byref(o), None, fake, 10, 1.0, 0.1, fake, fake, None) \
        == fof.FOF_ERR_INVALID_ARG
    o = fof.fof_default_options()
    o.predicate = 9
    assert lib.fof_label_noalloc(ctypes.byref(o), None, fake, 10, 1.0, 0.1, fake, fake, None) \
        == fof.FOF_ERR_INVALID_ARG
