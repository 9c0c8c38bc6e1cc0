"""The seeded input generator: published Philox known answers, the shuffle is a
bijection, coordinates stay in [0, L), and the halo mass law has its mean."""
import numpy as np

import synth


def test_philox_known_answers():
    # Random123 known-answer vectors for Philox4x32-10
    assert list(synth.philox4x32_10([0, 0, 0, 0], [0, 0])) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert list(synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert list(synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                                    [0xA4093822, 0x299F31D0])) == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_shuffle_is_a_bijection():
    for n in (1, 2, 7, 1000, 4097):
        img = [synth.permute(n, 3, 1, k) for k in range(n)]
        assert sorted(img) == list(range(n))


def test_coordinates_in_box_and_reproducible():
    a = synth.clustered(50000, 9, 0, 0.7)
    b = synth.clustered(50000, 9, 0, 0.7)
    assert np.array_equal(a, b)
    assert a.dtype == np.float32 and np.all(a >= 0) and np.all(a < 1)
    c = synth.clustered(50000, 9, 1, 0.7)
    assert not np.array_equal(a, c)
    u = synth.uniform(10000, 4)
    assert np.all(u >= 0) and np.all(u < 1)
    assert np.all(np.mod(u * 2.0 ** 24, 1.0) == 0)      # 24-bit grid


def test_halo_mass_law_mean():
    c = synth.halo_counts(int(0.6 * 256 ** 3), 20.0, 1e5, 1.9, 1)
    assert c.sum() == int(0.6 * 256 ** 3)
    # mean of M^-1.9 on [20, 1e5] is 242; the sample mean of the heavy tail is noisy
    assert 200 < c[:-1].mean() < 300 and c[:-1].min() >= 20 and c.max() <= 100000


def test_workload_shapes():
    w = synth.make("uniform32k")
    assert w.n == 32768 and abs(w.lx[0] - 0.00625) < 1e-18
    w = synth.make("batched256", n_boxes=4, size_scale=0.01)
    assert w.n_boxes == 4 and w.offsets[-1] == len(w.pos)
    assert synth.linking_length(0.2, 256 ** 3) == 0.2 / 256


def test_jittered_lattice_links_exactly_six_axis_neighbours():
    """The contention input: one particle per lattice site within 2 % of a
    spacing of its centre; by brute-force periodic distances every particle
    has exactly six neighbours within l_x, so the box is one group (the
    oracle agrees)."""
    import oracle

    side = 12
    w = synth.make("lattice1024", n=side ** 3)
    assert w.n == side ** 3 and abs(w.lx[0] - (1.0 / side) / 0.9) < 1e-15
    p = w.pos.astype(np.float64)
    s = 1.0 / side
    site = np.floor(p / s).astype(np.int64)
    key = (site[:, 2] * side + site[:, 1]) * side + site[:, 0]
    assert np.array_equal(np.sort(key), np.arange(side ** 3))
    assert np.abs(p / s - (site + 0.5)).max() <= 0.02 + 1e-5
    d = p[:, None, :] - p[None, :, :]
    d -= np.round(d)                                   # minimum image in the unit box
    r2 = (d * d).sum(-1)
    np.fill_diagonal(r2, np.inf)
    near = r2 <= w.lx[0] ** 2
    assert np.all(near.sum(1) == 6)
    steps = np.abs(site[:, None, :] - site[None, :, :]) % side
    steps = np.minimum(steps, side - steps).sum(-1)   # lattice (Manhattan) distance of the sites
    assert np.all(steps[near] == 1)
    w = synth.make("lattice1024", n=24 ** 3)
    label, size, ng = oracle.fof(w.pos, float(w.lx[0]))
    assert ng == 1 and not label.any() and size[0] == 24 ** 3
