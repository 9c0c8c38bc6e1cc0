"""Certification of the FP32 filter's guard band on the CPU (no GPU needed).

For pairs placed within a few FP32 ulps of the linking length -- random
orientations, coordinates near the periodic faces, several box sides and
linking lengths -- the FP32 squared distance is computed with the kernels'
operation order (each axis: one rounded subtraction of exact values, the
periodic image applied as home - L or neighbour - L; then x*x, y*y, z*z
summed with and without fused multiply-adds), and the thresholds the library
derives (fof_describe_box) are checked against the double predicate:
R32 < lo32 must mean linked and R32 > hi32 must mean not linked.
"""
import numpy as np
import pytest

import paper_2003_11468_amd as fof

CASES = [
    (1.0, 0.2 / 32), (1.0, 0.2 / 256), (1.0, 0.2 / 512), (1.0, 0.5 / 1024), (1.0, 1e-4), (1.0, 0.3),
    (8.0, 0.05), (1024.0, 3.0), (0.125, 0.001), (1.0, 2.0 ** -6),
]
PAIRS_PER_CASE = 10_000_000
CHUNK = 2_000_000


def f32_fma(a, b, c):
    """FP32 fused multiply-add: the product of two FP32 values is exact in
    double; the sum is rounded once in double, then to FP32 (the double
    rounding this adds is covered by the band's slack)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def kernel_r32(a, b, L):
    L32 = np.float32(L)
    d = []
    for k in range(3):
        h, q = a[:, k], b[:, k]
        t = h.astype(np.float64) - q.astype(np.float64)
        home_top = t > L / 2          # neighbour across the high face: (h - L) - q
        nb_top = t < -L / 2           # neighbour is the top cell across the low face: h - (q - L)
        hh = np.where(home_top, h - L32, h).astype(np.float32)
        qq = np.where(nb_top, q - L32, q).astype(np.float32)
        d.append((hh - qq).astype(np.float32))
    dx, dy, dz = d
    plain = ((dx * dx + dy * dy).astype(np.float32) + (dz * dz).astype(np.float32)).astype(np.float32)
    fused = f32_fma(dz, dz, f32_fma(dy, dy, (dx * dx).astype(np.float32)))
    return plain, fused


def canonical_r2(a, b, L):
    t = a.astype(np.float64) - b.astype(np.float64)
    t = np.where(t > L / 2, t - L, np.where(t < -L / 2, t + L, t))
    return (t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2]


def near_pairs(rng, n, L, lx):
    a = rng.uniform(0, L, size=(n, 3))
    face = rng.random(n) < 0.3            # a third start right at a face
    a[face, 0] = rng.choice([0.0, L], size=face.sum()) + rng.uniform(-lx, lx, size=face.sum())
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rel = rng.normal(0, 2e-6, size=n) * rng.choice([1.0, 0.05, 20.0], size=n)
    b = a + d * (lx * (1 + rel))[:, None]
    a = np.mod(a, L).astype(np.float32)
    b = np.mod(b, L).astype(np.float32)
    a[a >= np.float32(L)] = 0
    b[b >= np.float32(L)] = 0
    return a, b


@pytest.mark.parametrize("L,lx", CASES)
def test_thresholds_never_contradict_the_double_predicate(L, lx):
    info = fof.fof_describe_box(10 ** 6, L, lx)
    assert info["fp64_only"] == 0
    lo, hi, l2 = np.float32(info["lo32"]), np.float32(info["hi32"]), info["l2"]
    assert lo < l2 < hi and (hi - lo) / l2 < 2e-6
    rng = np.random.default_rng(int(lx * 1e9) % 2 ** 32)
    band = 0
    for _ in range(PAIRS_PER_CASE // CHUNK):
        a, b = near_pairs(rng, CHUNK, L, lx)
        r64 = canonical_r2(a, b, L)
        for r32 in kernel_r32(a, b, L):
            assert np.all(r64[r32 < lo] < l2)         # linked under both <= and <
            assert np.all(r64[r32 > hi] > l2)         # not linked
            band += int(np.count_nonzero((r32 >= lo) & (r32 <= hi)))
    assert band > 0            # the pairs really straddle the threshold


def test_boxes_the_filter_cannot_serve_fall_back_to_double():
    assert fof.fof_describe_box(1000, 0.1, 0.002)["fp64_only"] == 1      # 0.1 is not an FP32 value
    assert fof.fof_describe_box(1000, 2.0 ** 70, 2.0 ** 60)["fp64_only"] == 1
    info = fof.fof_describe_box(1000, 0.1, 0.002)
    assert info["lo32"] == -np.inf and info["hi32"] == np.inf


def test_cells_per_axis():
    assert fof.fof_describe_box(256 ** 3, 1.0, 0.2 / 256)["cells_per_axis"] == 256
    opt = fof.make_options(cell_factor=2.0)
    assert fof.fof_describe_box(256 ** 3, 1.0, 0.2 / 256, opt)["cells_per_axis"] == 640
    opt = fof.make_options(cell_factor=1.0)
    assert fof.fof_describe_box(10, 1.0, 0.25, opt)["cells_per_axis"] == 3
    with pytest.raises(fof.FoFError):
        fof.fof_describe_box(10, 1.0, 0.34)


def test_without_the_band_fp32_alone_would_be_wrong():
    """Deciding in FP32 against l2 itself (no band) contradicts the double
    predicate for some near-threshold pairs: the band is doing real work."""
    L, lx = 1.0, 0.2 / 512
    l2 = lx * lx
    rng = np.random.default_rng(7)
    wrong = 0
    for _ in range(3):
        a, b = near_pairs(rng, CHUNK, L, lx)
        r64 = canonical_r2(a, b, L)
        plain, fused = kernel_r32(a, b, L)
        l2_32 = np.float32(l2)
        wrong += int(np.count_nonzero((plain <= l2_32) != (r64 <= l2)))
        wrong += int(np.count_nonzero((fused <= l2_32) != (r64 <= l2)))
    assert wrong > 0


def test_premerge_sub_cells_are_inside_the_linking_length():
    """Dense cells are pre-merged by k^3 sub-cells: every two points of one
    must be linked, and with sub_cells_adjacent every two points of two
    touching sub-cells too, so the sub-cell diagonal (twice it for touching
    sub-cells) must stay below l_x with room for the double predicate's
    rounding; k must be the smallest such count, the touching criterion
    first."""
    rng = np.random.default_rng(11)
    seen = set()
    for _ in range(400):
        n = int(rng.integers(27, 10 ** 7))
        L = float(rng.choice([1.0, 8.0, 0.125, 1024.0, 0.1]))
        lx = L * float(rng.uniform(0.001, 0.3)) / max(1.0, n ** (1 / 3) / 4)
        cf = float(rng.choice([0.0, 1.0, 1.5, 2.0, 3.0, 4.0, 7.0]))
        try:
            info = fof.fof_describe_box(n, L, lx, fof.make_options(cell_factor=cf))
        except fof.FoFError:
            continue
        nc, k, adj = info["cells_per_axis"], info["sub_cells_per_axis"], info["sub_cells_adjacent"]
        side = L / nc
        need_one = side * np.sqrt(3.0) / (lx * (1 - 1e-6))
        need_adj = 2.0 * need_one
        if k:
            assert 1 <= k <= 8
            s = side / k
            if adj:
                assert k == int(np.ceil(need_adj))
                assert 2.0 * s * np.sqrt(3.0) <= lx * (1 - 1e-6) * (1 + 1e-12)
                reach = 2.0 * s        # far corners of two sub-cells touching at a corner
            else:
                assert need_adj > 8 and k == int(np.ceil(need_one))
                assert s * np.sqrt(3.0) <= lx * (1 - 1e-6) * (1 + 1e-12)
                reach = s              # far corners of one sub-cell
            # the FP64 predicate of two such points links
            a = np.zeros(3, dtype=np.float32)
            b = np.full(3, reach * (1 - 1e-7), dtype=np.float64).astype(np.float32)
            t = b.astype(np.float64) - a.astype(np.float64)
            assert float((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]) < info["l2"]
        else:
            assert need_one > 8 and adj == 0
        seen.add((k, adj))
    assert (0, 0) in seen and any(a for _, a in seen) and any(k and not a for k, a in seen)
