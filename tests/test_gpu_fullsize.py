"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses (the autotuner's choice).

Every full-size workload is compared with the oracle element by element:
clustered256 (16.8M), batched256 (34.3M in 256 boxes, in a graph),
clustered512 (134M, the precision form: the FP32 filter and the all-FP64
path, which must also equal each other) and percolate1024 (1.07B, both
predicates). The large ones use the oracle's threaded variant (the same
components, the link search over host threads), pinned against the
sequential oracle, brute force and scipy on the CPU. lattice1024 (1.07B on a
jittered lattice) is one group by construction, which fixes every label and
size.
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
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def note(msg):
    print(msg, flush=True)


OPTION_KEYS = ("cell_factor", "dense_min", "schedule", "link_order", "compression", "segment_log2")


def tuned(pos, w, predicate="fp32_filter", **kw):
    return tune.autotune(pos, w.offsets, w.box, w.lx, predicate, cache_path=None, repeats=1, **kw)


def run(pos, w, cfg, predicate="fp32_filter"):
    f = fof.FoF(predicate, **{k: cfg[k] for k in OPTION_KEYS if k in cfg})
    try:
        label, size, ng = f.run(pos, w.offsets, w.box, w.lx)
        return label.cpu().numpy(), size.cpu().numpy(), ng
    finally:
        f.close()


def assert_equal_to(ref, label, size, ng, what):
    assert np.array_equal(label, ref[0]), what + ": labels"
    assert np.array_equal(size, ref[1]), what + ": sizes"
    assert int(np.sum(ng)) == int(np.sum(ref[2])), what + ": group count"


def test_clustered256_full_size_matches_oracle():
    w = synth.make("clustered256")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w)
    label, size, ng = run(pos, w, cfg)
    ref = oracle.fof_parallel(w.pos, float(w.lx[0]), threads=THREADS)
    assert_equal_to(ref, label, size, ng, "clustered256")


def test_batched256_full_size_matches_oracle_in_a_graph():
    w = synth.make("batched256")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w)
    f = fof.FoF("fp32_filter", **{k: cfg[k] for k in OPTION_KEYS if k in cfg})
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


def _both_predicates_against_oracle(name, cell_factors, dense_mins):
    """The FP32 filter and the all-FP64 path, each in its tuned configuration,
    element by element against one oracle run and against each other."""
    note(f"{name}: generating")
    w = synth.make(name)
    pos = torch.from_numpy(w.pos).cuda()
    out = {}
    for predicate in ("fp32_filter", "fp64"):
        cfg = tuned(pos, w, predicate, cell_factors=cell_factors, dense_mins=dense_mins, axes={})
        note(f"{name}: {predicate} at cell factor {cfg['cell_factor']}, dense threshold {cfg['dense_min']}")
        out[predicate] = run(pos, w, cfg, predicate)
        torch.cuda.empty_cache()
    del pos
    torch.cuda.empty_cache()
    a, b = out["fp32_filter"], out["fp64"]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), f"{name}: FP32 filter != FP64"
    note(f"{name}: oracle on {THREADS} host threads")
    ref = oracle.fof_parallel(w.pos, float(w.lx[0]), threads=THREADS)
    for predicate, (label, size, ng) in out.items():
        assert_equal_to(ref, label, size, ng, f"{name} {predicate}")
    return ref


def test_clustered512_both_predicates_match_oracle():
    ref = _both_predicates_against_oracle("clustered512", (0.0, 1.5, 2.0, 3.0), (16, 32))
    assert int(ref[1].max()) >= 2


def test_percolate1024_both_predicates_match_oracle():
    ref = _both_predicates_against_oracle("percolate1024", (0.0, 1.5, 2.0), (32,))
    assert ref[2] < 1024 ** 3


# The most contended input: 1024^3 particles that form one group. Both link
# orders, in the benchmark's kind of configuration (tuned over a few cell sizes).
def test_lattice1024_is_one_group_under_both_link_orders():
    w = synth.make("lattice1024")
    pos = torch.from_numpy(w.pos).cuda()
    cfg = tuned(pos, w, cell_factors=(0.0, 2.0), dense_mins=(32,), axes={})
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
