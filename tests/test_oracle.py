"""Pins for the CPU oracle: it is checked against things other than itself.

- hand-derived fixture (golden/fig2_indirect_u.txt): U-shaped indirect chain
  (Fig. 2 of the paper), wrap and corner pairs, an exact tie;
- closed forms: dyadic distances with each axis wrapping separately;
- lattices just below / above the spacing (N singletons / one group), and the
  exact dyadic tie that fixes "<=" against "<";
- brute force O(N^2) (Listing 1) on small inputs;
- a library routine: scipy's periodic k-d tree pair search plus
  scipy.sparse.csgraph connected components;
- invariants: periodic translation and axis permutation leave the partition
  unchanged; labels are the group minima; sizes count the members;
- statistics: Poisson expectations for i.i.d. uniform points;
- planted mistakes: mutated copies of the oracle must fail at least one pin.

The threaded variant (oracle_fof_parallel, for the full-size parity checks)
has pins of its own: the hand fixture, lattices, the tie lattice, brute force,
scipy's periodic k-d tree, and planted mistakes in its own code (slot
grouping, shell enumeration, the label and size at the group minimum).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

import oracle
import synth
from cases import chain_across_boundary, labels_from_partition, lattice, load_fixture

pytestmark = pytest.mark.filterwarnings("ignore")


def canonical_from_components(comp: np.ndarray) -> np.ndarray:
    """Map component ids to the minimum member index."""
    n = len(comp)
    mins = np.full(comp.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp]


def scipy_labels(pos: np.ndarray, lx: float, box: float = 1.0) -> np.ndarray:
    tree = cKDTree(pos.astype(np.float64), boxsize=box)
    pairs = tree.query_pairs(lx, output_type="ndarray")
    n = len(pos)
    g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    return canonical_from_components(comp)


def check_invariants(label, size, n_groups):
    n = len(label)
    idx = np.arange(n)
    assert np.all(label <= idx)
    assert np.all(label[label] == label)
    roots = label == idx
    assert n_groups == int(roots.sum())
    counts = np.bincount(label, minlength=n)
    assert np.array_equal(size, np.where(roots, counts, 0))
    assert int(size.sum()) == n


# ----------------------------------------------------------------- fixture --

@pytest.mark.parametrize("brute", [False, True])
def test_golden_fixture(brute):
    fx = load_fixture("fig2_indirect_u.txt")
    for strict, tag in ((False, "le"), (True, "lt")):
        label, size, ng = oracle.fof(fx["pos"], fx["lx"], fx["box"], strict=strict, brute=brute)
        assert np.array_equal(label, fx["labels_" + tag])
        assert np.array_equal(size, fx["sizes_" + tag])
        assert ng == int(fx["groups_" + tag][0])


# ------------------------------------------------------------ closed forms --

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_r2_closed_forms(axis):
    def pt(v):
        p = np.full(3, 0.5, dtype=np.float32)
        p[axis] = v
        return p

    assert oracle.r2(pt(0.875), pt(0.125)) == 0.0625        # wraps: |0.75| -> 0.25
    assert oracle.r2(pt(0.125), pt(0.875)) == 0.0625        # other sign
    assert oracle.r2(pt(0.75), pt(0.25)) == 0.25            # exactly L/2: no wrap
    assert oracle.r2(pt(0.625), pt(0.25)) == 0.140625       # 0.375, no wrap
    a = np.array([0.25, 0.5, 0.75], dtype=np.float32)
    b = np.array([0.75, 0.5, 0.25], dtype=np.float32)
    assert oracle.r2(a, b) == 0.5
    # distinct per-axis offsets pin that each axis uses its own coordinates
    a = np.array([0.0625, 0.125, 0.9375], dtype=np.float32)
    b = np.array([0.9375, 0.375, 0.875], dtype=np.float32)
    assert oracle.r2(a, b) == 0.125 ** 2 + 0.25 ** 2 + 0.0625 ** 2
    # box side other than 1
    assert oracle.r2(np.float32([7.0, 0, 0]), np.float32([1.0, 0, 0]), box=8.0) == 4.0


# ---------------------------------------------------------------- lattices --

@pytest.mark.parametrize("n", [4, 16])
def test_lattice_below_and_above_spacing(n):
    pos = lattice(n, seed=n)
    s = 1.0 / n
    label, size, ng = oracle.fof(pos, s * (1 - 1e-3))
    assert ng == n ** 3 and np.array_equal(label, np.arange(n ** 3))
    label, size, ng = oracle.fof(pos, s * (1 + 1e-3))
    assert ng == 1 and np.all(label == 0) and size[0] == n ** 3


@pytest.mark.parametrize("strict,expect_groups", [(False, 1), (True, 64 ** 3)])
def test_dyadic_tie_lattice(strict, expect_groups):
    pos = lattice(64, seed=1)
    label, size, ng = oracle.fof(pos, 2.0 ** -6, strict=strict)
    assert ng == expect_groups
    check_invariants(label, size, ng)


def test_chains_across_each_face():
    for axis in range(3):
        pos = chain_across_boundary(40, 0.0234375, axis)          # step < l_x, 40 steps wrap the face
        label, size, ng = oracle.fof(pos, 0.03125)
        assert ng == 1 and size[0] == 40
        label, size, ng = oracle.fof(pos, 0.0234375 * (1 - 1e-3))
        assert ng == 40


def clump_and_pair():
    """1998 coincident particles at the centre plus two particles 0.095 apart
    on the x axis (l_x = 0.1). Many particles with a long linking length make
    the cell grid fine, so this pins that cells never get narrower than l_x."""
    pos = np.full((2000, 3), 0.5, dtype=np.float32)
    pos[3] = [0.16, 0.1, 0.1]
    pos[1500] = [0.255, 0.1, 0.1]
    return pos


def test_sparse_pair_beside_dense_clump():
    label, size, ng = oracle.fof(clump_and_pair(), 0.1)
    assert ng == 2 and label[1500] == 3 and size[3] == 2 and size[0] == 1998


def test_edge_cases():
    label, size, ng = oracle.fof(np.zeros((0, 3), np.float32), 0.1)
    assert ng == 0 and len(label) == 0
    label, size, ng = oracle.fof(np.float32([[0.3, 0.3, 0.3]]), 0.1)
    assert ng == 1 and label[0] == 0 and size[0] == 1
    pos = np.float32([[0.3, 0.3, 0.3], [0.9, 0.9, 0.9], [0.3, 0.3, 0.3]])  # coincident 0 and 2
    label, size, ng = oracle.fof(pos, 1e-6)
    assert list(label) == [0, 1, 0] and list(size) == [2, 1, 0] and ng == 2


@pytest.mark.parametrize("bad", [np.nan, -0.0625, 1.0, np.inf])
def test_rejects_bad_coordinates(bad):
    pos = np.float32([[0.5, 0.5, 0.5], [0.25, 0.25, 0.25]])
    pos[1, 1] = bad
    if bad == -0.0625 or bad == 1.0 or not np.isfinite(bad):
        with pytest.raises(oracle.OracleError):
            oracle.fof(pos, 0.1)


def test_rejects_bad_parameters():
    pos = np.float32([[0.5, 0.5, 0.5]])
    for lx, box in ((0.0, 1.0), (-1.0, 1.0), (np.nan, 1.0), (0.1, 0.0), (0.1, np.inf)):
        with pytest.raises(oracle.OracleError):
            oracle.fof(pos, lx, box)


# ------------------------------------------------------------- brute force --

@pytest.mark.parametrize("b", [0.2, 0.5, 0.9, 1.5])
@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_cells_equal_brute_force(b, kind):
    for seed in range(6):
        n = 2048
        pos = synth.uniform(n, 100 + seed) if kind == "uniform" else synth.clustered(n, 200 + seed, 0, 0.6)
        lx = synth.linking_length(b, n)
        got = oracle.fof(pos, lx)
        ref = oracle.fof(pos, lx, brute=True)
        for g, r in zip(got[:2], ref[:2]):
            assert np.array_equal(g, r)
        assert got[2] == ref[2]
        check_invariants(*got)


def test_brute_force_with_few_cells():
    # fewer than 3 cells per axis fit: the oracle falls back to brute force
    pos = synth.uniform(500, 7)
    assert oracle.cells_per_axis(500, 0.4) == 0
    a = oracle.fof(pos, 0.4)
    b = oracle.fof(pos, 0.4, brute=True)
    assert np.array_equal(a[0], b[0])


# ------------------------------------------------------------------- scipy --

@pytest.mark.parametrize("b", [0.2, 0.5, 1.0])
def test_matches_scipy_periodic_kdtree(b):
    n = 30000
    pos = synth.clustered(n, 11, 0, 0.6)
    lx = synth.linking_length(b, n)
    label, size, ng = oracle.fof(pos, lx)
    assert np.array_equal(label, scipy_labels(pos, lx))
    check_invariants(label, size, ng)


# -------------------------------------------------------------- invariants --

def partition_key(label: np.ndarray) -> np.ndarray:
    return label  # canonical labels already identify the partition


def test_translation_and_axis_permutation_invariance():
    n = 20000
    pos = synth.uniform(n, 21)          # coordinates are multiples of 2^-24: shifts by 1/2 are exact
    lx = synth.linking_length(0.9, n)
    base, _, _ = oracle.fof(pos, lx)
    shifted = np.mod(pos.astype(np.float64) + np.array([0.5, 0.25, 0.75]), 1.0).astype(np.float32)
    assert np.array_equal(oracle.fof(shifted, lx)[0], base)
    perm = np.ascontiguousarray(pos[:, [2, 0, 1]])
    assert np.array_equal(oracle.fof(perm, lx)[0], base)


def test_component_bfs_matches_union_find():
    n = 20000
    pos = synth.clustered(n, 31, 0, 0.6)
    lx = synth.linking_length(0.2, n)
    label, size, _ = oracle.fof(pos, lx)
    big = np.argsort(-size)[:3]
    for start in list(big) + [int(np.argmax(label != np.arange(n))), 5]:
        members = oracle.component(pos, lx, start)
        assert np.array_equal(members, np.flatnonzero(label == label[start]))


def test_components_of_match_union_find():
    n = 30000
    pos = synth.clustered(n, 41, 0, 0.6)
    lx = synth.linking_length(0.3, n)
    label, size, _ = oracle.fof(pos, lx)
    starts = [int(np.argmax(size)), 7, 123, int(np.argmax(size)) + 0, 29999]
    sizes, mins, mark = oracle.components_of(pos, lx, starts)
    for k, s in enumerate(starts):
        assert mins[k] == label[s] and sizes[k] == size[label[s]]
        first = next(q for q in range(k + 1) if mark[starts[q]] == mark[s])
        assert np.array_equal(np.flatnonzero(mark == first), np.flatnonzero(label == label[s]))


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_oracle_equals_sequential(threads):
    cases = []
    for b in (0.2, 0.5, 0.9):
        n = 40000
        cases.append((synth.clustered(n, 300 + int(10 * b), 0, 0.6), synth.linking_length(b, n), 1.0))
    n = 20000
    cases.append((synth.uniform(n, 77), synth.linking_length(0.8, n), 1.0))
    p = synth.clustered(n, 78, 0, 0.6).astype(np.float64) * 2.5
    cases.append((np.ascontiguousarray(np.mod(p, 2.5).astype(np.float32)), 2.5 * synth.linking_length(0.6, n), 2.5))
    for pos, lx, box in cases:
        for strict in (False, True):
            ref = oracle.fof(pos, lx, box, strict=strict)
            got = oracle.fof_parallel(pos, lx, box, strict=strict, threads=threads)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2]


def test_threaded_oracle_tie_lattice_chains_and_edges():
    pos = lattice(64, seed=1)
    assert oracle.fof_parallel(pos, 2.0 ** -6, threads=4)[2] == 1
    assert oracle.fof_parallel(pos, 2.0 ** -6, strict=True, threads=4)[2] == 64 ** 3
    for axis in range(3):
        pos = chain_across_boundary(50, 0.01, axis)
        label, size, ng = oracle.fof_parallel(pos, 0.0101, threads=2)
        assert ng == 1 and size[0] == 50
    assert oracle.fof_parallel(np.zeros((0, 3), np.float32), 0.1, threads=2)[2] == 0
    label, size, ng = oracle.fof_parallel(np.array([[0.3, 0.3, 0.3]], np.float32), 0.1, threads=2)
    assert ng == 1 and label[0] == 0 and size[0] == 1
    with pytest.raises(oracle.OracleError):
        oracle.fof_parallel(np.array([[1.0, 0.3, 0.3]], np.float32), 0.1, threads=2)


def test_threaded_oracle_equals_brute_force():
    for seed in range(4):
        n = 2048
        pos = synth.clustered(n, 400 + seed, 0, 0.6)
        for b in (0.5, 1.5):
            lx = synth.linking_length(b, n)
            got = oracle.fof_parallel(pos, lx, threads=4)
            ref = oracle.fof(pos, lx, brute=True)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2]


def test_boxes_equal_single_box_runs():
    w = synth.make("batched256", n_boxes=6, size_scale=0.02)
    lab1, size1, ng1 = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx, threads=1)
    lab4, size4, ng4 = oracle.fof_boxes(w.pos, w.offsets, w.box, w.lx, threads=4)
    assert np.array_equal(lab1, lab4) and np.array_equal(size1, size4) and np.array_equal(ng1, ng4)
    for k in range(w.n_boxes):
        o0, o1 = w.offsets[k], w.offsets[k + 1]
        lab, size, ng = oracle.fof(w.pos[o0:o1], w.lx[k])
        assert np.array_equal(lab1[o0:o1], lab) and ng1[k] == ng


def test_explicit_partition_helper_roundtrip():
    label, size = labels_from_partition([[3, 1], [4, 2, 0]], 6)
    assert list(label) == [0, 1, 0, 1, 0, 5] and list(size) == [3, 2, 0, 0, 0, 1]


# -------------------------------------------------------------- statistics --

def test_poisson_expectations_uniform32k():
    """i.i.d. uniform, N = 32^3, l_x = 0.2/32: expected links N(N-1)/2 * 4/3 pi l_x^3
    = 549.0 and singleton fraction exp(-N 4/3 pi l_x^3) = 0.96705; groups ~ N - links."""
    n, lx = 32 ** 3, 0.2 / 32
    vol = 4.0 / 3.0 * np.pi * lx ** 3
    e_links = n * (n - 1) / 2 * vol
    p_single = np.exp(-(n - 1) * vol)
    groups, singles = [], []
    for seed in range(8):
        label, size, ng = oracle.fof(synth.uniform(n, 1000 + seed), lx)
        groups.append(ng)
        singles.append(np.mean(size == 1))
    assert abs(e_links - 549.0) < 0.1 and abs(p_single - 0.96705) < 1e-5
    sigma = np.sqrt(e_links / 8)
    assert abs(np.mean(groups) - (n - e_links)) < 4 * sigma + 2
    assert abs(np.mean(singles) - p_single) < 4 * np.sqrt(2 * e_links / 8) / n + 1e-4


# --------------------------------------------------------- planted mistakes --

MUTANTS = {
    "drop_z_term": ("return sxy + tz * tz;", "return sxy;"),
    "wrap_sign": ("if (t > half) return t - L;", "if (t > half) return t + L;"),
    "no_wrap": ("if (t < -half) return t + L;", "if (t < -half) return t;"),
    "strict_swapped": ("return strict ? (r2 < l2) : (r2 <= l2);", "return strict ? (r2 <= l2) : (r2 < l2);"),
    "transposed_axis": ("(double)a[1] - (double)b[1]", "(double)a[0] - (double)b[1]"),
    "union_by_max": ("if (ra < rb) parent[rb] = ra;", "if (ra > rb) parent[rb] = ra;"),
    "missing_cell_offset": ("for (int dx = -1; dx <= 1; ++dx) {\n                                int64_t ox",
                            "for (int dx = -1; dx <= 0; ++dx) {\n                                int64_t ox"),
    "cell_side_too_small": ("floor(L / (lx * (1.0 + 1.0 / 1048576.0)))", "floor(L / (lx * 0.5))"),
    "size_not_at_root": ("size[r] += 1;", "size[i] += 1;"),
}


def _mutant_lib(name, tmp, table=None):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "fof_oracle.c")).read()
    old, new = (table or MUTANTS)[name]
    assert src.count(old) >= 1, name
    src = src.replace(old, new)
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"],
                   check=True)
    return ctypes.CDLL(so)


# Mistakes in the threaded variant's own code (its slots, shell, outputs).
PARALLEL_MUTANTS = {
    "par_own_cell_only": ("for (k = 0; k < 27; ++k)\n", "for (k = 13; k < 14; ++k)\n"),
    "par_label_root_slot": ("label[orig[s]] = low[r];", "label[orig[s]] = orig[r];"),
    "par_size_at_root_slot": ("size[orig[s]] = orig[s] == low[r] ? count[r] : 0;",
                              "size[orig[s]] = r == s ? count[r] : 0;"),
    "par_no_x_wrap": ("ox += ox < 0 ? nc : (ox >= nc ? -nc : 0);", "ox += ox < 0 ? 1 : (ox >= nc ? -1 : 0);"),
    "par_cell_ends_as_starts": ("    memmove(first + 1, first, sizeof(uint32_t) * (size_t)ncell);\n", "\n"),
    "par_skip_last_cell_slot": ("for (uint32_t t = lo[k]; t < hi[k]; ++t)", "for (uint32_t t = lo[k]; t + 1 < hi[k]; ++t)"),
}


def _run(lib, pos, lx, box=1.0, strict=False, brute=False, parallel=False):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    n = len(pos)
    label = np.empty(n, np.int32)
    size = np.empty(n, np.int32)
    ng = ctypes.c_int64()
    args = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    if parallel:
        fn = lib.oracle_fof_parallel
        fn.argtypes = args + [ctypes.c_int]
        st = fn(n, pos.ctypes.data, box, lx, int(strict), label.ctypes.data, size.ctypes.data, ctypes.byref(ng), 3)
    else:
        fn = lib.oracle_fof_brute if brute else lib.oracle_fof
        fn.argtypes = args
        st = fn(n, pos.ctypes.data, box, lx, int(strict), label.ctypes.data, size.ctypes.data, ctypes.byref(ng))
    assert st == 0
    return label, size, ng.value


def _pins_pass(lib, parallel=False) -> bool:
    """The pin battery above, run against an arbitrary oracle library (its
    sequential or its threaded function)."""
    try:
        fx = load_fixture("fig2_indirect_u.txt")
        for strict, tag in ((False, "le"), (True, "lt")):
            for brute in (False, True):
                l, s, g = _run(lib, fx["pos"], fx["lx"], fx["box"], strict, brute and not parallel, parallel)
                if not (np.array_equal(l, fx["labels_" + tag]) and np.array_equal(s, fx["sizes_" + tag])):
                    return False
        l, s, g = _run(lib, clump_and_pair(), 0.1, parallel=parallel)
        if g != 2 or l[1500] != 3:
            return False
        pos = lattice(16, seed=3)
        if _run(lib, pos, (1 - 1e-3) / 16, parallel=parallel)[2] != 16 ** 3 or \
                _run(lib, pos, (1 + 1e-3) / 16, parallel=parallel)[2] != 1:
            return False
        n = 20000
        pos = synth.clustered(n, 11, 0, 0.6)
        lx = synth.linking_length(0.5, n)
        l, s, g = _run(lib, pos, lx, parallel=parallel)
        if not np.array_equal(l, scipy_labels(pos, lx)):
            return False
        check_invariants(l, s, g)
        pos = synth.uniform(2048, 5)
        for b in (0.9, 1.5):
            lx = synth.linking_length(b, 2048)
            if not np.array_equal(_run(lib, pos, lx, parallel=parallel)[0], _run(lib, pos, lx, brute=True)[0]):
                return False
        return True
    except AssertionError:
        return False


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass(oracle._load())
    assert _pins_pass(oracle._load(), parallel=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        assert not _pins_pass(_mutant_lib(name, tmp)), f"mutant {name} passed every pin"


@pytest.mark.parametrize("name", sorted(PARALLEL_MUTANTS))
def test_planted_mistake_in_the_threaded_oracle_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _mutant_lib(name, tmp, PARALLEL_MUTANTS)
        assert _pins_pass(lib), "the sequential functions are untouched"
        assert not _pins_pass(lib, parallel=True), f"mutant {name} passed every pin"
