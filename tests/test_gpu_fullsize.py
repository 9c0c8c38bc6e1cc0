"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (the autotuner's choice).

clustered256 (16.8M) and batched256 (34.3M in 256 boxes) are compared with the
full oracle element by element. clustered512 (134M) and percolate1024 (1.07B)
are checked by invariants that hold at any size (labels are group minima,
sizes count members, the group count is the number of roots) and by
breadth-first search of the groups of sampled particles -- including the
largest group -- which must have the GPU's label (its minimum), size and
exact member set. lattice1024 (1.07B on a jittered lattice) is one group by
construction, which fixes every label and size.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
fof = pytest.importorskip("paper_2003_11468_amd")
from paper_2003_11468_amd import tune  # noqa: E402

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def tuned(pos, w, predicate="fp32_filter", **kw):
    return tune.autotune(pos, w.offsets, w.box, w.lx, predicate, cache_path=None, repeats=1, **kw)


def run(pos, w, cfg, predicate="fp32_filter"):
    f = fof.FoF(predicate, cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"])
    try:
        label, size, ng = f.run(pos, w.offsets, w.box, w.lx)
        return label.cpu().numpy(), size.cpu().numpy(), ng
    finally:
        f.close()


def check_invariants(label, size, n_groups, offsets):
    for k in range(len(offsets) - 1):
        o0, o1 = int(offsets[k]), int(offsets[k + 1])
        lab = label[o0:o1].astype(np.int64)
        sz = size[o0:o1]
        idx = np.arange(o1 - o0)
        assert np.all(lab <= idx) and np.all(lab >= 0)
        assert np.all(lab[lab] == lab)
        roots = lab == idx
        assert int(roots.sum()) == int(n_groups[k])
        counts = np.bincount(lab, minlength=o1 - o0)
        assert np.array_equal(sz, np.where(roots, counts, 0))


def check_sampled_groups(pos, lx, label, size, starts):
    sizes, mins, mark = oracle.components_of(pos, lx, starts)
    for k, s in enumerate(starts):
        assert mins[k] == label[s], (k, s)
        assert sizes[k] == size[label[s]], (k, s)
        if mark[s] == k:   # first start of its group: compare the member sets
            assert np.array_equal(np.flatnonzero(mark == k), np.flatnonzero(label == label[s])), (k, s)


def test_clustered256_full_size_matches_oracle():
    w = synth.make("clustered256")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w)
    label, size, ng = run(pos, w, cfg)
    ref = oracle.fof(w.pos, float(w.lx[0]))
    assert np.array_equal(label, ref[0])
    assert np.array_equal(size, ref[1])
    assert int(ng[0]) == ref[2]


def test_batched256_full_size_matches_oracle_in_a_graph():
    w = synth.make("batched256")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w)
    f = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"])
    try:
        label, size = f.outputs(w.n)
        f.capture(pos, w.offsets, w.box, w.lx, label, size)
        f.replay()
        f.replay()
        ng = f.n_groups(w.n_boxes)
        lab, sz = label.cpu().numpy(), size.cpu().numpy()
    finally:
        f.close()
    ref = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx, threads=THREADS)
    assert np.array_equal(lab, ref[0])
    assert np.array_equal(sz, ref[1])
    assert np.array_equal(ng, ref[2])


def _sampled_case(name, seed):
    w = synth.make(name)
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w, cell_factors=(0.0, 2.0, 3.0), dense_mins=(16, 32))
    label, size, ng = run(pos, w, cfg)
    del pos
    torch.cuda.empty_cache()
    check_invariants(label, size, ng, w.offsets)
    rng = np.random.default_rng(seed)
    starts = list(rng.integers(0, w.n, size=6))
    starts.append(int(np.argmax(size)))                        # the largest group
    members = np.flatnonzero(size > 1)
    if len(members):
        starts += list(rng.choice(members, size=min(3, len(members)), replace=False))
    check_sampled_groups(w.pos, float(w.lx[0]), label, size, [int(s) for s in starts])
    return label, size, ng


def test_clustered512_full_size_invariants_and_sampled_groups():
    _sampled_case("clustered512", 512)


def test_percolate1024_full_size_invariants_and_sampled_groups():
    label, size, ng = _sampled_case("percolate1024", 1024)
    assert int(ng[0]) < 1024 ** 3


# The most contended input: 1024^3 particles that form one group. Both link
# orders, in the benchmark's kind of configuration (tuned over a few cell sizes).
def test_lattice1024_is_one_group_under_both_link_orders():
    w = synth.make("lattice1024")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w, cell_factors=(0.0, 2.0), dense_mins=(32,))
    for order in ("index", "random"):
        f = fof.FoF("fp32_filter", cell_factor=cfg["cell_factor"], dense_min=cfg["dense_min"], link_order=order)
        try:
            label, size, ng = f.run(pos, w.offsets, w.box, w.lx)
            assert int(ng[0]) == 1, order
            assert int(label.count_nonzero()) == 0, order
            assert int(size[0]) == w.n and int(size.count_nonzero()) == 1, order
        finally:
            f.close()
        torch.cuda.empty_cache()
