"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Labels (group minimum index), sizes and group counts are integers, so every
comparison is exact, element by element. Both link predicates must give the
oracle's result; the FP32 filter is exact by construction of its guard band.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from cases import chain_across_boundary, lattice, load_fixture

torch = pytest.importorskip("torch")
fof = pytest.importorskip("paper_2003_11468_amd")

pytestmark = pytest.mark.gpu
PREDICATES = ["fp32_filter", "fp64"]


def gpu_run(pos, offsets, box, lx, predicate="fp32_filter", strict=False, cell_factor=0.0, stats=False,
            dense_min=0, segment_log2=0, domains=0, link_order="index"):
    f = fof.FoF(predicate, strict, cell_factor, stats, dense_min=dense_min, segment_log2=segment_log2,
                domains=domains, link_order=link_order)
    try:
        p = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float32)).cuda()
        label, size, ng = f.run(p, offsets, box, lx)
        st = f.stats() if stats else None
        return label.cpu().numpy(), size.cpu().numpy(), ng, st
    finally:
        f.close()


def assert_single(pos, lx, box=1.0, strict=False, predicate="fp32_filter", cell_factor=0.0, dense_min=0,
                  segment_log2=0):
    ref = oracle.fof(pos, lx, box, strict=strict)
    lab, size, ng, _ = gpu_run(pos, [0, len(pos)], box, lx, predicate, strict, cell_factor, dense_min=dense_min,
                               segment_log2=segment_log2)
    assert np.array_equal(lab, ref[0])
    assert np.array_equal(size, ref[1])
    assert int(ng[0]) == ref[2]
    return ref


# ----------------------------------------------------------- hand cases --

@pytest.mark.parametrize("predicate", PREDICATES)
@pytest.mark.parametrize("strict", [False, True])
def test_golden_fixture(predicate, strict):
    fx = load_fixture("fig2_indirect_u.txt")
    tag = "lt" if strict else "le"
    lab, size, ng, _ = gpu_run(fx["pos"], [0, len(fx["pos"])], fx["box"], fx["lx"], predicate, strict)
    assert np.array_equal(lab, fx["labels_" + tag])
    assert np.array_equal(size, fx["sizes_" + tag])
    assert int(ng[0]) == int(fx["groups_" + tag][0])


@pytest.mark.parametrize("predicate", PREDICATES)
def test_lattice_below_and_above_spacing(predicate):
    pos = lattice(16, seed=3)
    lab, _, ng, _ = gpu_run(pos, [0, len(pos)], 1.0, (1 - 1e-3) / 16, predicate)
    assert int(ng[0]) == 16 ** 3 and np.array_equal(lab, np.arange(16 ** 3))
    lab, size, ng, _ = gpu_run(pos, [0, len(pos)], 1.0, (1 + 1e-3) / 16, predicate)
    assert int(ng[0]) == 1 and np.all(lab == 0) and size[0] == 16 ** 3


@pytest.mark.parametrize("predicate", PREDICATES)
@pytest.mark.parametrize("strict,groups", [(False, 1), (True, 64 ** 3)])
def test_dyadic_tie_lattice(predicate, strict, groups):
    pos = lattice(64, seed=1)
    lab, size, ng, _ = gpu_run(pos, [0, len(pos)], 1.0, 2.0 ** -6, predicate, strict)
    assert int(ng[0]) == groups
    if groups == 1:
        assert np.all(lab == 0) and size[0] == 64 ** 3


@pytest.mark.parametrize("predicate", PREDICATES)
def test_chains_across_each_face(predicate):
    for axis in range(3):
        pos = chain_across_boundary(40, 0.0234375, axis)
        assert_single(pos, 0.03125, predicate=predicate)
        assert_single(pos, 0.0234375 * (1 - 1e-3), predicate=predicate)


@pytest.mark.parametrize("predicate", PREDICATES)
def test_edge_cases(predicate):
    lab, size, ng, _ = gpu_run(np.zeros((0, 3), np.float32), [0, 0], 1.0, 0.1, predicate)
    assert len(lab) == 0 and int(ng[0]) == 0
    lab, size, ng, _ = gpu_run(np.float32([[0.3, 0.3, 0.3]]), [0, 1], 1.0, 0.1, predicate)
    assert list(lab) == [0] and list(size) == [1] and int(ng[0]) == 1
    pos = np.float32([[0.3, 0.3, 0.3], [0.9, 0.9, 0.9], [0.3, 0.3, 0.3]])
    lab, size, ng, _ = gpu_run(pos, [0, 3], 1.0, 1e-6, predicate)
    assert list(lab) == [0, 1, 0] and list(size) == [2, 1, 0] and int(ng[0]) == 2


def test_out_of_box_coordinate_is_reported():
    pos = synth.uniform(1000, 5)
    pos[17, 2] = 1.0
    p = torch.from_numpy(pos).cuda()
    f = fof.FoF()
    try:
        with pytest.raises(fof.FoFError) as e:
            f.run(p, [0, 1000], 1.0, 0.02)
        assert e.value.status == fof.FOF_ERR_OUT_OF_BOX
        pos[17, 2] = np.nan
        p = torch.from_numpy(pos).cuda()
        with pytest.raises(fof.FoFError) as e:
            f.run(p, [0, 1000], 1.0, 0.02)
        assert e.value.status == fof.FOF_ERR_OUT_OF_BOX
        pos[17, 2] = 0.5                         # a clean run afterwards clears the latch
        p = torch.from_numpy(pos).cuda()
        f.run(p, [0, 1000], 1.0, 0.02)
    finally:
        f.close()


# ------------------------------------------------------- seeded random --

@pytest.mark.parametrize("predicate", PREDICATES)
@pytest.mark.parametrize("n", [2, 63, 64, 65, 257, 1000, 4097, 65537])
def test_uniform_sizes(predicate, n):
    pos = synth.uniform(n, 40 + n)
    assert_single(pos, synth.linking_length(0.6, n) if n > 27 else 0.2, predicate=predicate)


@pytest.mark.parametrize("predicate", PREDICATES)
@pytest.mark.parametrize("b", [0.2, 0.5, 0.9, 1.5])
def test_clustered_linking_lengths(predicate, b):
    n = 200003
    pos = synth.clustered(n, 77, 0, 0.6)
    lx = synth.linking_length(b, n)
    if lx * (1 + 2 ** -20) * 3 > 1.0:
        pytest.skip("fewer than 3 cells")
    assert_single(pos, lx, predicate=predicate)


@pytest.mark.parametrize("cell_factor", [1.0, 1.375, 1.5, 2.0, 3.0, 7.0])
def test_cell_sizes(cell_factor):
    n = 150000
    pos = synth.clustered(n, 5, 0, 0.6)
    lx = synth.linking_length(0.2, n)
    for predicate in PREDICATES:
        assert_single(pos, lx, predicate=predicate, cell_factor=cell_factor)


# Above 1290 cells per axis a box has more than 2^31 cells: the cell index is
# 64-bit in the sort keys, the occupancy words, the neighbour rows and the
# dense work items. Clustered points so that dense cells and the pre-merge
# take part too.
@pytest.mark.parametrize("nc", [1300, 1800])
def test_more_than_2_to_the_31_cells(nc):
    n = 150000
    pos = synth.clustered(n, 23, 0, 0.9, m_max=2e4)
    lx = 1.0 / (nc + 0.5)
    assert fof.fof_describe_box(n, 1.0, lx, fof.make_options(cell_factor=1.0))["cells_per_axis"] == nc
    for predicate in PREDICATES:
        for dense_min in (8, 1 << 30):
            ref = assert_single(pos, lx, predicate=predicate, cell_factor=1.0, dense_min=dense_min)
    assert int(ref[1].max()) >= 8   # groups with many members


# dense_min = 1: every non-empty cell is searched by whole wavefronts;
# dense_min = 1 << 30: every cell per lane; between: both kernels meet.
@pytest.mark.parametrize("dense_min", [1, 2, 8, 64, 100, 1 << 30])
@pytest.mark.parametrize("predicate", PREDICATES)
def test_dense_and_sparse_kernels(dense_min, predicate):
    n = 120000
    pos = synth.clustered(n, 17, 0, 0.7)
    for b, cf in ((0.2, 0.0), (0.5, 1.0), (0.3, 2.5)):
        assert_single(pos, synth.linking_length(b, n), predicate=predicate, cell_factor=cf, dense_min=dense_min)


# More links between tiles than the edge list holds (2^20 queued pairs at
# this size): the per-particle search merges the surplus at once while other
# tiles hook their own links, so some tile hooks find their slot hooked
# already and fall back to an ordinary union. Both tile-join settings.
@pytest.mark.parametrize("tile_join", [True, False])
def test_edge_list_overflow_with_tile_join(tile_join):
    n = 120000
    pos = synth.clustered(n, 17, 0, 0.7)
    lx = synth.linking_length(0.5, n)
    ref = oracle.fof(pos, lx, 1.0)
    f = fof.FoF("fp32_filter", cell_factor=1.0, stats=True, dense_min=1 << 30,
                schedule=fof.schedule_bits(tile_join=tile_join))
    try:
        label, size, ng = f.run(torch.from_numpy(pos).cuda(), [0, n], 1.0, lx)
        st = f.stats()
        assert st["queued_links"] > (1 << 20)   # the list overflowed
        assert np.array_equal(label.cpu().numpy(), ref[0]) and np.array_equal(size.cpu().numpy(), ref[1])
        assert int(ng[0]) == ref[2]
    finally:
        f.close()


@pytest.mark.parametrize("dense_min", [1, 1 << 30])
def test_kernel_paths_on_hand_cases(dense_min):
    fx = load_fixture("fig2_indirect_u.txt")
    for strict, tag in ((False, "le"), (True, "lt")):
        for predicate in PREDICATES:
            lab, size, ng, _ = gpu_run(fx["pos"], [0, len(fx["pos"])], fx["box"], fx["lx"], predicate, strict,
                                       dense_min=dense_min)
            assert np.array_equal(lab, fx["labels_" + tag]) and np.array_equal(size, fx["sizes_" + tag])
    pos = lattice(16, seed=5)
    for predicate in PREDICATES:
        lab, size, ng, _ = gpu_run(pos, [0, len(pos)], 1.0, (1 + 1e-3) / 16, predicate, dense_min=dense_min)
        assert int(ng[0]) == 1
    for axis in range(3):
        assert_single(chain_across_boundary(40, 0.0234375, axis), 0.03125, dense_min=dense_min)
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    for predicate in PREDICATES:
        lab, size, ng, _ = gpu_run(w.pos, w.offsets, w.box, w.lx, predicate, dense_min=dense_min)
        assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and np.array_equal(ng, ref[2])


# The cell sort counts 2^k cells per work-group: small k gives many segments
# per bucket, k >= 14 one segment per bucket and above 2^14 cells several
# occupancy words per thread; 16^3 and 32^3 cells fill their last segment
# exactly (the end marker comes from the last work-group).
@pytest.mark.parametrize("segment_log2", [6, 7, 9, 11, 12, 13, 14, 15, 16])
def test_cell_sort_segments(segment_log2):
    n = 120000
    pos = synth.clustered(n, 23, 0, 0.7)
    for b, cf in ((0.2, 0.0), (0.4, 1.0), (0.2, 3.0)):
        assert_single(pos, synth.linking_length(b, n), cell_factor=cf, segment_log2=segment_log2)
    # about one particle per cell: segments of 2^13 and 2^14 cells hold more
    # occupied cells than one counting window, so they are sorted in windows
    for nside in (16, 32, 48):
        u = synth.uniform(nside ** 3, 29)
        lx = synth.linking_length(0.9, nside ** 3)
        assert oracle.cells_per_axis(nside ** 3, lx) == nside
        assert_single(u, lx, segment_log2=segment_log2)
    w = synth.make("batched256", n_boxes=20, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    lab, size, ng, _ = gpu_run(w.pos, w.offsets, w.box, w.lx, segment_log2=segment_log2)
    assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and np.array_equal(ng, ref[2])


# Tight clumps fill sub-cells of dense cells with many particles, so the
# sub-cell pre-merge does most of the merging before the pair search.
def test_dense_cells_premerged_by_sub_cells():
    rng = np.random.default_rng(41)
    centres = rng.random((300, 3))
    pts = (centres[:, None, :] + rng.normal(0.0, 0.002, (300, 60, 3))) % 1.0
    pos = pts.reshape(-1, 3).astype(np.float32)
    pos[pos >= np.float32(1.0)] = 0
    for cf in (1.0, 2.0, 4.0):
        assert fof.fof_describe_box(len(pos), 1.0, 0.004, fof.make_options(cell_factor=cf))["sub_cells_per_axis"] > 0
        for strict in (False, True):
            for predicate in PREDICATES:
                assert_single(pos, 0.004, strict=strict, predicate=predicate, cell_factor=cf, dense_min=8)


def _catalogue_reference(label, size, offsets, min_size):
    idx = np.flatnonzero(size >= min_size)
    box = np.searchsorted(np.asarray(offsets), idx, side="right") - 1
    return label[idx], size[idx], box


def test_group_catalogue():
    n = 120000
    pos = synth.clustered(n, 37, 0, 0.7)
    lx = synth.linking_length(0.2, n)
    ref = oracle.fof(pos, lx)
    w = synth.make("batched256", n_boxes=20, size_scale=0.05)
    sizes = np.diff(w.offsets)
    sizes[4] = 0                                   # an empty box
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bpos = np.concatenate([w.pos[w.offsets[k]:w.offsets[k] + sizes[k]] for k in range(20)])
    bref = oracle.fof_boxes(bpos, offsets, w.box, w.lx)
    for p_np, off, L, l, r in ((pos, [0, n], 1.0, lx, ref), (bpos, offsets, w.box, w.lx, bref)):
        f = fof.FoF()
        try:
            p = torch.from_numpy(np.ascontiguousarray(p_np)).cuda()
            label, size, ng = f.run(p, off, L, l)
            assert np.array_equal(label.cpu().numpy(), r[0])
            for min_size in (1, 2, 20, 10 ** 9):
                first, gsize, gbox = (t.cpu().numpy() for t in f.catalogue(label, size, min_size))
                e_first, e_size, e_box = _catalogue_reference(r[0], r[1], off, min_size)
                assert np.array_equal(first, e_first) and np.array_equal(gsize, e_size)
                assert np.array_equal(gbox, e_box)
                if min_size == 1:   # every group once: the sizes add up to N, one entry per group
                    assert int(gsize.sum()) == len(p_np) and len(first) == int(np.sum(ng))
            # a capacity below the count: the count is still exact, the first entries are written
            full = fof.fof_catalogue(f.ctx, label, size, 2)
            cap = max(1, full // 3)
            a, b_, c = (torch.full((cap,), -7, dtype=torch.int32, device="cuda") for _ in range(3))
            assert fof.fof_catalogue(f.ctx, label, size, 2, a, b_, c, cap) == full
            e_first, e_size, e_box = _catalogue_reference(r[0], r[1], off, 2)
            assert np.array_equal(a.cpu().numpy(), e_first[:cap]) and np.array_equal(b_.cpu().numpy(), e_size[:cap])
        finally:
            f.close()


# Domain-decomposed merge on one GPU (Section 3.3): union-find inside slabs
# along x, the links across slabs collected, their groups numbered densely and
# merged. The labels must not change; the boundary list must be in use.
@pytest.mark.parametrize("domains", [2, 3, 7, 16])
def test_domain_decomposed_merge(domains):
    n = 150000
    pos = synth.clustered(n, 43, 0, 0.7)
    for b, cf, dm in ((0.2, 2.0, 32), (0.5, 1.0, 8), (0.9, 0.0, 4)):
        lx = synth.linking_length(b, n)
        ref = oracle.fof(pos, lx)
        for predicate in PREDICATES:
            lab, size, ng, st = gpu_run(pos, [0, n], 1.0, lx, predicate, cell_factor=cf, dense_min=dm, stats=True,
                                        domains=domains)
            assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and int(ng[0]) == ref[2]
            assert st["boundary_links"] > 0 and 0 < st["boundary_groups"] <= 2 * st["boundary_links"]
    for axis in range(3):   # chains across each periodic face, the x face being a slab face too
        pc = chain_across_boundary(40, 0.0234375, axis)
        ref = oracle.fof(pc, 0.03125)
        lab, size, ng, _ = gpu_run(pc, [0, len(pc)], 1.0, 0.03125, domains=domains)
        assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1])
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    for predicate in PREDICATES:
        lab, size, ng, _ = gpu_run(w.pos, w.offsets, w.box, w.lx, predicate, dense_min=16, domains=domains)
        assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and np.array_equal(ng, ref[2])


# Randomised linking (Section 3.2): roots hook by a fixed pseudo-random
# priority of the index instead of the index. Which node ends up a root
# changes; the labels (smallest original index of each group), the sizes and
# the group counts must not. Every kernel path, both predicates, domain mode,
# one lattice-wide group (the most contended case) and batches.
def test_randomised_linking_same_labels():
    n = 150000
    pos = synth.clustered(n, 53, 0, 0.7)
    for b, cf, dm in ((0.2, 2.0, 32), (0.5, 1.0, 8), (0.9, 0.0, 4)):
        lx = synth.linking_length(b, n)
        ref = oracle.fof(pos, lx)
        for predicate in PREDICATES:
            for domains in (0, 3):
                lab, size, ng, st = gpu_run(pos, [0, n], 1.0, lx, predicate, cell_factor=cf, dense_min=dm,
                                            stats=True, domains=domains, link_order="random")
                assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and int(ng[0]) == ref[2]
                assert st["links"] >= n - ref[2]
    fx = load_fixture("fig2_indirect_u.txt")
    lab, size, _, _ = gpu_run(fx["pos"], [0, len(fx["pos"])], fx["box"], fx["lx"], link_order="random")
    assert np.array_equal(lab, fx["labels_le"]) and np.array_equal(size, fx["sizes_le"])
    pos = lattice(40, seed=5)
    for dm in (1, 1 << 30):
        lab, size, ng, _ = gpu_run(pos, [0, len(pos)], 1.0, (1 + 1e-3) / 40, dense_min=dm, link_order="random")
        assert int(ng[0]) == 1 and np.all(lab == 0) and size[0] == 40 ** 3
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    lab, size, ng, _ = gpu_run(w.pos, w.offsets, w.box, w.lx, dense_min=16, link_order="random")
    assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and np.array_equal(ng, ref[2])


# The contention input at a size the oracle handles: a jittered lattice that
# is one group. Both link orders, both predicates, sparse and dense paths.
def test_jittered_lattice_one_group_both_link_orders():
    w = synth.make("lattice1024", n=64 ** 3)
    ref = oracle.fof(w.pos, float(w.lx[0]))
    assert ref[2] == 1
    for order in ("index", "random"):
        for predicate in PREDICATES:
            for cf, dm in ((0.0, 0), (2.0, 4)):
                lab, size, ng, st = gpu_run(w.pos, w.offsets, w.box, w.lx, predicate, cell_factor=cf, dense_min=dm,
                                            stats=True, link_order=order)
                assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1]) and int(ng[0]) == 1
                assert st["links"] >= w.n - 1


# Find depth statistics: every non-root is at least one step from its root,
# a forest of singletons has depth 0, and the sum is bounded by max x n.
def test_find_depth_statistics():
    n = 100000
    pos = synth.clustered(n, 57, 0, 0.6)
    lx = synth.linking_length(0.5, n)
    ref = oracle.fof(pos, lx)
    for order in ("index", "random"):
        _, _, ng, st = gpu_run(pos, [0, n], 1.0, lx, stats=True, link_order=order)
        assert int(ng[0]) == ref[2]
        assert st["find_depth_max"] >= 1
        assert n - ref[2] <= st["find_depth_sum"] <= st["find_depth_max"] * n
    pos = lattice(16, seed=3)
    _, _, ng, st = gpu_run(pos, [0, len(pos)], 1.0, (1 - 1e-3) / 16, stats=True)
    assert int(ng[0]) == 16 ** 3 and st["find_depth_max"] == 0 and st["find_depth_sum"] == 0


# Relink: new linking lengths over the cells of the last build (each at most
# the build's), several in a row, single box and batches, both predicates.
def test_relink_reuses_the_cells():
    n = 120000
    pos = synth.clustered(n, 47, 0, 0.6)
    lx0 = synth.linking_length(0.5, n)
    p = torch.from_numpy(pos).cuda()
    for predicate in PREDICATES:
        f = fof.FoF(predicate, dense_min=16)
        try:
            label, size, ng = f.run(p, [0, n], 1.0, lx0)
            ref = oracle.fof(pos, lx0)
            assert np.array_equal(label.cpu().numpy(), ref[0])
            for scale in (0.4, 1.0, 0.15, 0.8):
                lab, sz, ng = f.relink(lx0 * scale, 1)
                ref = oracle.fof(pos, lx0 * scale)
                assert np.array_equal(lab.cpu().numpy(), ref[0]) and np.array_equal(sz.cpu().numpy(), ref[1])
                assert int(ng[0]) == ref[2]
            with pytest.raises(fof.FoFError) as e:      # cells too small for a longer linking length
                fof.fof_relink(f.ctx, lx0 * 1.01, 1)
            assert e.value.status == fof.FOF_ERR_INVALID_ARG
        finally:
            f.close()
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    f = fof.FoF(dense_min=16)
    try:
        f.run(torch.from_numpy(w.pos).cuda(), w.offsets, w.box, w.lx)
        lx1 = np.asarray(w.lx) * 0.6
        lab, sz, ng = f.relink(lx1, w.n_boxes)
        ref = oracle.fof_boxes(w.pos, w.offsets, w.box, lx1)
        assert np.array_equal(lab.cpu().numpy(), ref[0]) and np.array_equal(sz.cpu().numpy(), ref[1])
        assert np.array_equal(ng, ref[2])
    finally:
        f.close()


def test_uniform32k_and_strict():
    w = synth.make("uniform32k")
    for predicate in PREDICATES:
        for strict in (False, True):
            assert_single(w.pos, float(w.lx[0]), strict=strict, predicate=predicate)


def test_box_side_other_than_one():
    pos = (synth.clustered(50000, 8, 0, 0.6).astype(np.float64) * 8.0).astype(np.float32)  # exact scaling
    lx = synth.linking_length(0.3, 50000, box=8.0)
    for predicate in PREDICATES:
        assert_single(pos, lx, box=8.0, predicate=predicate)


def test_box_side_not_exact_in_fp32_falls_back_to_fp64():
    L = 0.1
    pos = np.minimum(synth.uniform(20000, 3).astype(np.float64) * L, np.nextafter(L, 0)).astype(np.float32)
    pos = np.where(pos.astype(np.float64) >= L, np.float32(0), pos).astype(np.float32)
    lx = synth.linking_length(0.7, 20000, box=L)
    ref = oracle.fof(pos, lx, L)
    lab, size, ng, st = gpu_run(pos, [0, len(pos)], L, lx, "fp32_filter", stats=True)
    assert np.array_equal(lab, ref[0]) and np.array_equal(size, ref[1])
    assert st["fp64_boxes"] == 1


# -------------------------------------------------------------- batched --

@pytest.mark.parametrize("predicate", PREDICATES)
def test_batched_boxes(predicate):
    w = synth.make("batched256", n_boxes=24, size_scale=0.05)
    sizes = np.diff(w.offsets)
    sizes[3] = 0                      # an empty box
    sizes[7] = 1                      # a single particle
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([w.pos[w.offsets[k]:w.offsets[k] + sizes[k]] for k in range(24)])
    ref = oracle.fof_boxes(pos, offsets, w.box, w.lx)
    lab, size, ng, _ = gpu_run(pos, offsets, w.box, w.lx, predicate)
    assert np.array_equal(lab, ref[0])
    assert np.array_equal(size, ref[1])
    assert np.array_equal(ng, ref[2])


def test_graph_replays_match_eager():
    w = synth.make("batched256", n_boxes=16, size_scale=0.03)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    f = fof.FoF()
    try:
        p = torch.from_numpy(w.pos).cuda()
        label, size = f.outputs(w.n)
        f.capture(p, w.offsets, w.box, w.lx, label, size)
        for rep in range(4):
            label.fill_(-7)
            size.fill_(-7)
            f.replay()
            ng = f.n_groups(w.n_boxes)
            assert np.array_equal(label.cpu().numpy(), ref[0]), rep
            assert np.array_equal(size.cpu().numpy(), ref[1]), rep
            assert np.array_equal(ng, ref[2]), rep
            # eager work on the same stream between replays
            lab2, size2, ng2 = f.run(p[: w.offsets[3]].contiguous(), w.offsets[:4], w.box[:3], w.lx[:3])
            assert np.array_equal(lab2.cpu().numpy(), ref[0][: w.offsets[3]])
            f.capture(p, w.offsets, w.box, w.lx, label, size)
    finally:
        f.close()


@pytest.mark.parametrize("predicate", PREDICATES)
@pytest.mark.parametrize("premerge,stats", [(True, False), (False, False), (True, True)])
def test_graph_with_dense_cells_matches_oracle(predicate, premerge, stats):
    """A graph over boxes with many dense cells: the captured link phase runs
    the sub-cell pre-merge on a second captured stream beside the union pass;
    every replay (with eager work between) equals the oracle."""
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    f = fof.FoF(predicate, cell_factor=1.5, dense_min=8, stats=stats,
                schedule=fof.schedule_bits(premerge=premerge))
    try:
        p = torch.from_numpy(w.pos).cuda()
        label, size = f.outputs(w.n)
        f.run(p, w.offsets, w.box, w.lx, label, size)
        if stats:
            assert f.stats()["dense_items"] > 0
        f.capture(p, w.offsets, w.box, w.lx, label, size)
        for rep in range(3):
            label.fill_(-7)
            size.fill_(-7)
            f.replay()
            ng = f.n_groups(w.n_boxes)
            assert np.array_equal(label.cpu().numpy(), ref[0]), rep
            assert np.array_equal(size.cpu().numpy(), ref[1]), rep
            assert np.array_equal(ng, ref[2]), rep
            lab2, _, _ = f.run(p[: w.offsets[2]].contiguous(), w.offsets[:3], w.box[:2], w.lx[:2])
            assert np.array_equal(lab2.cpu().numpy(), ref[0][: w.offsets[2]])
            f.run(p, w.offsets, w.box, w.lx, label, size)   # the captured geometry back in the workspace
    finally:
        f.close()


def test_graph_refused_after_its_box_table_is_replaced():
    """A multi-box graph reads the box table in the workspace: after an eager
    build of another geometry (or of one box, or a relink) the host refuses to
    replay it, so nothing runs with a replaced table; an eager build of the
    captured geometry puts the table back and replays work again."""
    w = synth.make("batched256", n_boxes=12, size_scale=0.03)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    f = fof.FoF()
    try:
        p = torch.from_numpy(w.pos).cuda()
        label, size = f.outputs(w.n)
        f.capture(p, w.offsets, w.box, w.lx, label, size)
        f.replay()
        assert np.array_equal(label.cpu().numpy(), ref[0])
        k = 5   # another geometry: the first five boxes
        f.run(p[: w.offsets[k]].contiguous(), w.offsets[: k + 1], w.box[:k], w.lx[:k])
        with pytest.raises(fof.FoFError) as e:
            f.replay()
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        f.run(p[: w.offsets[1]].contiguous(), w.offsets[:2], w.box[:1], w.lx[:1])   # one box
        with pytest.raises(fof.FoFError) as e:
            f.replay()
        assert e.value.status == fof.FOF_ERR_BAD_STATE
        f.run(p, w.offsets, w.box, w.lx)    # the captured geometry again: its table is back
        label.fill_(-7)
        f.replay()
        assert np.array_equal(label.cpu().numpy(), ref[0])
        f.relink([float(v) * 0.9 for v in w.lx], w.n_boxes)   # new thresholds in the table
        with pytest.raises(fof.FoFError) as e:
            f.replay()
        assert e.value.status == fof.FOF_ERR_BAD_STATE
    finally:
        f.close()


def test_single_box_graph_survives_other_runs():
    w = synth.make("batched256", n_boxes=4, size_scale=0.03)
    p = torch.from_numpy(w.pos).cuda()
    n0 = int(w.offsets[1])
    ref = oracle.fof(w.pos[:n0], float(w.lx[0]))
    f = fof.FoF()
    try:
        p0 = p[:n0].contiguous()
        label, size = f.outputs(n0)
        f.run(p, w.offsets, w.box, w.lx)          # sizes the workspace for the larger run
        f.capture(p0, [0, n0], w.box[0], w.lx[0], label, size)
        f.run(p, w.offsets, w.box, w.lx)          # a multi-box run on the same workspace
        label.fill_(-7)
        f.replay()
        assert np.array_equal(label.cpu().numpy(), ref[0])
        assert np.array_equal(size.cpu().numpy(), ref[1])
    finally:
        f.close()


# ---------------------------------------------------------- properties --

def test_repeated_runs_identical():
    n = 300000
    pos = synth.clustered(n, 99, 0, 0.6)
    lx = synth.linking_length(0.5, n)
    first = gpu_run(pos, [0, n], 1.0, lx)
    for _ in range(5):
        again = gpu_run(pos, [0, n], 1.0, lx)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])


def test_stats_count_band_and_links():
    n = 100000
    pos = synth.clustered(n, 12, 0, 0.6)
    lx = synth.linking_length(0.2, n)
    ref = oracle.fof(pos, lx)
    lab, size, ng, st = gpu_run(pos, [0, n], 1.0, lx, "fp32_filter", stats=True)
    assert np.array_equal(lab, ref[0])
    assert st["pair_tests"] > st["links"] >= n - ref[2]
    assert 0 <= st["band_hits"] < max(10, st["links"] // 1000)
    assert st["n_groups"] == ref[2]


def test_near_threshold_pairs_fp32_filter_is_exact():
    """Pairs at distances within a few FP32 ulps of l_x, several orientations
    and periodic wraps: the filter must reproduce the double decision."""
    rng = np.random.default_rng(2024)
    m = 20000
    lx = 0.01
    a = rng.uniform(0, 1, size=(m, 3))
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rel = rng.choice([-4e-7, -2e-7, -6e-8, 0.0, 6e-8, 2e-7, 4e-7], size=m) + rng.normal(0, 1e-7, size=m)
    b = np.mod(a + d * lx * (1 + rel)[:, None], 1.0)
    pos = np.empty((2 * m, 3), dtype=np.float32)
    pos[0::2] = a.astype(np.float32)
    pos[1::2] = b.astype(np.float32)
    pos[pos >= 1.0] = 0.0
    ref = oracle.fof(pos, lx)
    for predicate in PREDICATES:
        lab, size, ng, st = gpu_run(pos, [0, 2 * m], 1.0, lx, predicate, stats=(predicate == "fp32_filter"))
        assert np.array_equal(lab, ref[0]), predicate
        assert np.array_equal(size, ref[1]), predicate
        if st is not None:
            assert st["band_hits"] > 0


def test_autotuner_choice_is_exact(tmp_path):
    from paper_2003_11468_amd import tune

    n = 200000
    pos_np = synth.clustered(n, 21, 0, 0.6)
    lx = synth.linking_length(0.2, n)
    pos = torch.from_numpy(pos_np).cuda()
    cache = str(tmp_path / "tune.json")
    r = tune.autotune(pos, [0, n], 1.0, lx, cache_path=cache, repeats=1, cell_factors=(0.0, 2.0, 3.0),
                      dense_mins=(8, 32))
    assert not r["cached"] and len(r["tried"]) == 6 + sum(len(v) - 1 for v in tune.AXES.values())
    assert "gfx950" in r["key"] and "|clu" in r["key"]
    again = tune.autotune(pos, [0, n], 1.0, lx, cache_path=cache)
    assert again["cached"] and again["cell_factor"] == r["cell_factor"]
    ref = oracle.fof(pos_np, lx)
    f = fof.FoF(cell_factor=r["cell_factor"], dense_min=r["dense_min"], schedule=r["schedule"],
                link_order=r["link_order"], compression=r["compression"], segment_log2=r["segment_log2"])
    try:
        label, size, ng = f.run(pos, [0, n], 1.0, lx)
        assert np.array_equal(label.cpu().numpy(), ref[0]) and np.array_equal(size.cpu().numpy(), ref[1])
    finally:
        f.close()


TUNER_OPTIONS = ([dict(schedule=fof.schedule_bits(sg, dg, pm)) for sg, dg, pm in
                  ((512, 1024, True), (2048, 4096, True), (4096, 8192, True), (1024, 2048, False))] +
                 [dict(schedule=fof.schedule_bits(tile_join=False)),
                  dict(schedule=fof.schedule_bits(giant_skip=True)),
                  dict(schedule=fof.schedule_bits(giant_skip=True), link_order="random", compression="depth2"),
                  dict(link_order="random"), dict(compression="depth2"),
                  dict(compression="depth2", link_order="random"), dict(segment_log2=12)])


@pytest.mark.parametrize("opt", TUNER_OPTIONS, ids=lambda o: "-".join(f"{k}{v}" for k, v in o.items()))
@pytest.mark.parametrize("predicate", PREDICATES)
def test_every_tuner_option_is_exact(opt, predicate):
    """Every work-schedule and contention option the autotuner may pick gives
    the oracle's labels: on a batch with dense halo cells (both kernels and
    the pre-merge run) and on a jittered lattice that is one group."""
    w = synth.make("batched256", n_boxes=12, size_scale=0.05)
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx)
    f = fof.FoF(predicate, cell_factor=1.5, dense_min=16, **opt)
    try:
        label, size, ng = f.run(torch.from_numpy(w.pos).cuda(), w.offsets, w.box, w.lx)
        assert np.array_equal(label.cpu().numpy(), ref[0]) and np.array_equal(size.cpu().numpy(), ref[1])
        assert np.array_equal(ng, ref[2])
    finally:
        f.close()
    lat = synth.make("lattice1024", n=64 ** 3)   # 64^3 sites, spacing 0.9 l_x: one group
    f = fof.FoF(predicate, cell_factor=0.0, dense_min=32, **opt)
    try:
        label, size, ng = f.run(torch.from_numpy(lat.pos).cuda(), lat.offsets, lat.box, lat.lx)
        assert int(ng[0]) == 1 and int(label.count_nonzero()) == 0 and int(size[0]) == lat.n
    finally:
        f.close()


def test_kernel_times_cover_every_kernel():
    n = 100000
    pos = torch.from_numpy(synth.clustered(n, 3, 0, 0.6)).cuda()
    f = fof.FoF(timings=True)
    try:
        for _ in range(3):
            f.run(pos, [0, n], 1.0, synth.linking_length(0.2, n))
        kt = f.kernel_times()
        assert set(kt) == {fof.fof_kernel_name(k) for k in range(15)}
        for name, (ms, launches) in kt.items():
            assert launches == 3 and ms > 0.0, name
        assert all(c == 0 for _, c in f.kernel_times().values())   # the record was cleared
    finally:
        f.close()
