"""Seeded input generators (no GPU)."""
import numpy as np

import synth


def test_splitmix64_known_answers():
    """The first outputs of SplitMix64 seeded with 1234567, as produced by the
    generator's reference C implementation (state += golden gamma, then the
    30/27/31 finaliser)."""
    got = [int(x) for x in synth.splitmix64(1234567, 0, 5)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_splitmix64_is_counter_based():
    a = synth.splitmix64(99, 0, 1000)
    assert np.array_equal(a[400:700], synth.splitmix64(99, 400, 300))
    imgs = synth.block_images(5, 3, 4, 16, 4)
    assert np.array_equal(imgs[2], synth.sample_images(5, [5], 16, 4)[0])


def test_erasure_masks_fixed_count_uniform():
    n = 6
    m = synth.erasure_masks(synth.SEED_ERASE, 60000, n, 2)
    pc = np.array([bin(int(x)).count("1") for x in m])
    assert (pc == 2).all()
    assert int(m.max()) < (1 << n)
    vals, counts = np.unique(m, return_counts=True)
    assert len(vals) == 15
    assert counts.min() > 60000 / 15 * 0.9 and counts.max() < 60000 / 15 * 1.1


def test_erasure_masks_range_count():
    m = synth.erasure_masks(11, 30000, 6, (0, 2))
    pc = np.array([bin(int(x)).count("1") for x in m])
    for c in (0, 1, 2):
        assert abs((pc == c).mean() - 1 / 3) < 0.02
    # counter-based: a slice of blocks is reproducible on its own
    part = synth.erasure_masks(11, 100, 6, (0, 2), first_block=500)
    assert np.array_equal(part, m[500:600])


def test_centered_dirs():
    assert synth.centered_dirs(6) == [-3, -2, -1, 0, 1, 2]
    assert synth.centered_dirs(12) == list(range(-6, 6))
    assert synth.centered_dirs(16) == list(range(-8, 8))
