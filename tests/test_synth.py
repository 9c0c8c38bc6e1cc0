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
