"""Pins for the oracle's 128-bit pixel code (Section 3.1; no GPU).

The oracle runs the 64-bit transform on each word plane.  These checks fix it
against Eq. 1 evaluated directly on 128-bit Python integers, the group-sum
invariant in 128 bits, and round trips under every erasure pattern the code
tolerates, with the erased bins overwritten so that a decode reading them
would fail.
"""
import itertools

import numpy as np
import pytest

import synth

MASK64 = (1 << 64) - 1


def wide_image(rng, nblocks, P, Q):
    return rng.integers(0, 2**64, size=(nblocks, Q, P, 2), dtype=np.uint64)


def as_int(words):
    """A 16-byte pixel or bin as one integer, word 0 in the low half."""
    return int(words[0]) | (int(words[1]) << 64)


def brute_forward(img, P, Q, p):
    """Eq. 1 with q = 1 on 128-bit integers: bin b is the XOR of the pixels
    (k, l) with b = -k + l*p, bins in ascending b."""
    bins = {}
    for l in range(Q):
        for k in range(P):
            b = -k + l * p
            bins[b] = bins.get(b, 0) ^ as_int(img[l, k])
    lo = min(bins)
    assert sorted(bins) == list(range(lo, lo + len(bins)))
    return [bins[b] for b in range(lo, lo + len(bins))]


@pytest.mark.parametrize("P,Q,n", [(7, 3, 5), (5, 4, 6), (1, 2, 3), (9, 1, 2)])
def test_wide_forward_matches_eq1_on_128bit_integers(orc, P, Q, n):
    rng = np.random.default_rng(11 + P * Q + n)
    ps = synth.centered_dirs(n)
    imgs = wide_image(rng, 3, P, Q)
    out = orc.encode_blocks_wide(imgs, P, Q, ps)
    assert out.shape == (3, orc.block_stride(P, Q, ps), 2)
    for b in range(3):
        off = 0
        for p in ps:
            want = brute_forward(imgs[b], P, Q, p)
            got = [as_int(out[b, off + j]) for j in range(len(want))]
            assert got == want
            off += len(want)


def test_wide_projection_xor_equals_image_xor(orc):
    """Every bin sums one line and the lines of a direction partition the
    image, so each projection's bins XOR to the XOR of all pixels."""
    P, Q, n = 64, 4, 6
    ps = synth.centered_dirs(n)
    img = wide_image(np.random.default_rng(3), 1, P, Q)
    total = 0
    for w in img.reshape(-1, 2):
        total ^= as_int(w)
    out = orc.encode_blocks_wide(img, P, Q, ps)[0]
    off = 0
    for p in ps:
        B = orc.proj_size(p, 1, P, Q)
        acc = 0
        for w in out[off:off + B]:
            acc ^= as_int(w)
        assert acc == total
        off += B


def test_wide_paper_geometry_4k_block():
    """A 4 KB block of the (6,4) code with 16-byte pixels is 64 x 4 pixels
    (Section 3.1); Eq. 2 gives 6*64 + 3*(3+2+1+0+1+2) = 411 bins of 16 bytes."""
    import oracle

    ps = synth.centered_dirs(6)
    assert oracle.block_stride(64, 4, ps) == 411


def test_wide_roundtrip_every_erasure_pattern(orc):
    """(6,4) code, P = 64 pixels of 16 bytes: any 4 of 6 projections give the
    block back; erased projections are overwritten with noise first."""
    P, Q, n = 64, 4, 6
    ps = synth.centered_dirs(n)
    rng = np.random.default_rng(5)
    imgs = wide_image(rng, 1, P, Q)
    pool = orc.encode_blocks_wide(imgs, P, Q, ps)
    sizes = [orc.proj_size(p, 1, P, Q) for p in ps]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for r in range(0, 3):
        for lost in itertools.combinations(range(n), r):
            bad = pool.copy()
            mask = 0
            for i in lost:
                bad[0, offs[i]:offs[i + 1]] = rng.integers(0, 2**64, size=(sizes[i], 2),
                                                          dtype=np.uint64)
                mask |= 1 << i
            out = orc.decode_blocks_wide(bad, np.array([mask], dtype=np.uint16), P, Q, ps)
            assert np.array_equal(out, imgs)


def test_wide_word_planes_are_not_mixed(orc):
    """An image whose second words are all zero has projections whose second
    words are all zero (no carry or mixing between the two 64-bit halves)."""
    P, Q, n = 16, 4, 6
    ps = synth.centered_dirs(n)
    imgs = wide_image(np.random.default_rng(9), 2, P, Q)
    imgs[..., 1] = 0
    out = orc.encode_blocks_wide(imgs, P, Q, ps)
    assert not out[..., 1].any()
    assert out[..., 0].any()
