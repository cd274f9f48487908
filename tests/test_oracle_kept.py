"""Pins for the oracle's never-used-bin code (Section 2.3; no GPU).

The kept bins are found by enumerating every erasure pattern, so they are
checked against totals computed independently when the scope was surveyed,
against the closed form of the interval the fixed path reads, and by round
trips in which only the kept bins exist.
"""
import itertools

import numpy as np
import pytest

import synth


def test_kept_totals_match_the_independent_count(orc):
    """773 of 795 bins for the 4 KB (6,4) code and 1,590 of 1,788 for the
    8 KB (12,8) code (P = 128), as counted independently of this code."""
    ps6 = synth.centered_dirs(6)
    assert sum(c for _, c in orc.kept_bins(ps6, 128, 4)) == 773
    assert orc.block_stride(128, 4, ps6) == 795
    ps12 = synth.centered_dirs(12)
    assert sum(c for _, c in orc.kept_bins(ps12, 128, 8)) == 1590
    assert orc.block_stride(128, 8, ps12) == 1788


@pytest.mark.parametrize("n,Q,P", [(6, 4, 128), (12, 8, 64), (6, 3, 40), (8, 4, 9), (4, 2, 5),
                                   (3, 3, 7)])
def test_kept_interval_closed_form(orc, n, Q, P):
    """The r-th used survivor reads bins r*p - P + 1 .. r*p; projection i of
    the sorted directions can be the r-th for r = max(0, i-m) .. min(i, Q-1)
    (m = n - Q), so it keeps P + (r_hi - r_lo)*|p| bins."""
    ps = synth.centered_dirs(n)
    keep = orc.kept_bins(ps, P, Q)
    m = n - Q
    for i, p in enumerate(sorted(ps)):
        r_lo, r_hi = max(0, i - m), min(i, Q - 1)
        first = min(r_lo * p, r_hi * p) - P + 1
        idx = ps.index(p)
        assert keep[idx] == (first - orc.bin_min(p, 1, P, Q), P + (r_hi - r_lo) * abs(p))


@pytest.mark.parametrize("n,Q,P", [(6, 4, 16), (6, 4, 128), (8, 4, 12), (6, 3, 10)])
def test_kept_roundtrip_every_erasure_pattern(orc, n, Q, P):
    ps = synth.centered_dirs(n)
    imgs = synth.block_images(21 + n, 0, 1, P, Q)
    kept = orc.encode_blocks_kept(imgs, P, Q, ps)
    keep = orc.kept_bins(ps, P, Q)
    offs = np.concatenate([[0], np.cumsum([c for _, c in keep])])
    for r in range(0, n - Q + 1):
        for lost in itertools.combinations(range(n), r):
            bad = kept.copy()
            mask = 0
            for i in lost:
                bad[0, offs[i]:offs[i + 1]] = np.uint64(0xDEADBEEFCAFEF00D)
                mask |= 1 << i
            out = orc.decode_blocks_kept(bad, np.array([mask], dtype=np.uint16), P, Q, ps)
            assert np.array_equal(out, imgs)


def test_kept_encode_is_a_restriction_of_eq1(orc):
    P, Q, n = 32, 4, 6
    ps = synth.centered_dirs(n)
    imgs = synth.block_images(5, 0, 3, P, Q)
    kept = orc.encode_blocks_kept(imgs, P, Q, ps)
    for b in range(3):
        full = orc.forward(imgs[b], [(p, 1) for p in ps])
        parts = [full[i][lo:lo + c] for i, (lo, c) in enumerate(orc.kept_bins(ps, P, Q))]
        assert np.array_equal(kept[b], np.concatenate(parts))


def test_missing_bins_are_never_read(orc):
    """With the full window the kept peeling is the plain one; with an empty
    window a projection counts as lost (its zero-filled bins are not used)."""
    import ctypes

    P, Q = 12, 3
    ps = [-1, 0, 1]
    img = synth.block_images(8, 0, 1, P, Q)[0]
    projs = orc.forward(img, [(p, 1) for p in ps])
    flat = np.concatenate(projs)
    off = np.concatenate([[0], np.cumsum([len(x) for x in projs])[:-1]]).astype(np.int64)
    p = np.array(ps, dtype=np.int32)
    q = np.ones(3, dtype=np.int32)
    lib = orc._load()

    def run(lo, cnt, src):
        out = np.zeros((Q, P), dtype=np.uint64)
        lo_a = np.array(lo, dtype=np.int64)     # kept alive across the call
        cnt_a = np.array(cnt, dtype=np.int64)
        rc = lib.orc_inverse_kept(orc.XOR, 0, orc._ptr(src), orc._ptr(off), orc._ptr(p),
                                  orc._ptr(q), 3, P, Q, orc._ptr(lo_a), orc._ptr(cnt_a),
                                  orc._ptr(out), 1, ctypes.c_void_p(0))
        return rc, out

    rc, out = run([0, 0, 0], [len(x) for x in projs], flat)
    assert rc == orc.OK and np.array_equal(out, img)
    # projection 1 stores nothing: two projections cannot rebuild 3 rows
    src = np.concatenate([projs[0], projs[2]])
    off2 = np.array([0, len(projs[0]), len(projs[0])], dtype=np.int64)
    off[:] = off2
    rc, _ = run([0, 0, 0], [len(projs[0]), 0, len(projs[2])], src)
    assert rc == orc.ENOTRECON
