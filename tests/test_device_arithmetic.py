"""Host checks of the integer arithmetic that the kernels do in floating point.

The cell sort recovers a dense cell's coordinates from its box-local index by
truncated double quotients, the pre-merge a sub-cell's coordinates by
truncated float quotients of t + 1/2, and the cell sort picks the t-th
occupied cell of a word by halving it with population counts. Each kernel
comment states why the result equals the integer one; these tests restate the
same formulas with IEEE arithmetic on the host (numpy's float64 and float32
operations round to nearest like the device's) and compare them with integer
division, over the full ranges the library admits and their edges.
"""
import numpy as np

MAX_NC = 2048          # cells per box axis the library accepts
MAX_SUB_K = 16         # sub-cells per cell axis, beyond the largest in use (k^3 <= 512)


def cell_coords_by_double(local, nc):
    nc2 = nc * nc
    cz = np.trunc(local.astype(np.float64) / nc2.astype(np.float64)).astype(np.int64)
    rem = local - cz * nc2
    cy = np.trunc(rem.astype(np.float64) / nc.astype(np.float64)).astype(np.int64)
    return rem - cy * nc, cy, cz


def test_dense_cell_coordinates_by_double_quotients():
    rng = np.random.default_rng(7)
    nc = rng.integers(3, MAX_NC + 1, 400000)
    cells = nc * nc * nc
    local = (rng.random(nc.size) * cells).astype(np.int64)
    # the edges: first and last cell, the ends of every plane and row
    nc2 = nc * nc
    q = local // nc2
    edges = np.concatenate([np.zeros_like(nc), cells - 1, q * nc2, q * nc2 + nc2 - 1,
                            (local // nc) * nc, (local // nc) * nc + nc - 1])
    ncs = np.concatenate([nc] * 6)
    for loc, n in ((local, nc), (edges, ncs)):
        loc = np.minimum(loc, n * n * n - 1)
        cx, cy, cz = cell_coords_by_double(loc, n)
        assert np.array_equal(cx, loc % n)
        assert np.array_equal(cy, (loc // n) % n)
        assert np.array_equal(cz, loc // (n * n))


def test_sub_cell_coordinates_by_float_quotients():
    for k in range(1, MAX_SUB_K + 1):
        inv_k = np.float32(1.0) / np.float32(k)
        inv_k2 = np.float32(1.0) / np.float32(k * k)
        t = np.arange(k ** 3, dtype=np.int64)
        sz = ((t.astype(np.float32) + np.float32(0.5)) * inv_k2).astype(np.int64)
        r = t - sz * k * k
        sy = ((r.astype(np.float32) + np.float32(0.5)) * inv_k).astype(np.int64)
        sx = r - sy * k
        assert np.array_equal(sx, t % k), k
        assert np.array_equal(sy, (t // k) % k), k
        assert np.array_equal(sz, t // (k * k)), k


def nth_bit(m, t):
    """Position of the t-th lowest set bit of the 32-bit word m, by halving."""
    pos = 0
    w = 16
    while w > 0:
        low = m & ((1 << w) - 1)
        c = bin(low).count("1")
        if t >= c:
            t -= c
            m >>= w
            pos += w
        else:
            m = low
        w >>= 1
    return pos


def test_nth_set_bit_by_population_counts():
    rng = np.random.default_rng(11)
    words = [0xFFFFFFFF, 0x80000000, 0x00000001, 0x55555555, 0xAAAAAAAA, 0x0000FFFF, 0xFFFF0000]
    words += [int(x) for x in rng.integers(0, 1 << 32, 3000, dtype=np.uint64)]
    words += [int(x) & int(y) for x, y in zip(rng.integers(0, 1 << 32, 1000, dtype=np.uint64),
                                               rng.integers(0, 1 << 32, 1000, dtype=np.uint64))]
    for m in words:
        bits = [i for i in range(32) if (m >> i) & 1]
        for t, want in enumerate(bits):
            assert nth_bit(m, t) == want, (hex(m), t)
