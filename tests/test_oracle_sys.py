"""Pins for the oracle's systematic code (Section 2.3; no GPU): data lines
stored as they are, m parity projections beside them."""
import ctypes
import itertools

import numpy as np
import pytest

import synth

POISON = np.uint64(0xDEADBEEFCAFEF00D)


def lose(imgs, parity, mask, P, Q, pdirs, orc):
    """Copies with every lost packet overwritten."""
    im, pa = imgs.copy(), parity.copy()
    offs = np.concatenate([[0], np.cumsum([orc.proj_size(p, 1, P, Q) for p in pdirs])])
    for i in range(Q + len(pdirs)):
        if (mask >> i) & 1:
            if i < Q:
                im[:, i] = POISON
            else:
                pa[:, offs[i - Q]:offs[i - Q + 1]] = POISON
    return im, pa


@pytest.mark.parametrize("P,Q,pdirs", [(128, 4, [-1, 1]), (16, 4, [0, 1]), (32, 8, [-2, -1, 1, 2]),
                                       (10, 3, [-1, 0, 1]), (7, 2, [3])])
def test_sys_roundtrip_every_erasure_pattern(orc, P, Q, pdirs):
    imgs = synth.block_images(40 + P, 0, 1, P, Q)
    parity = orc.encode_blocks_sys(imgs, P, Q, pdirs)
    m = len(pdirs)
    for r in range(m + 1):
        for lost in itertools.combinations(range(Q + m), r):
            mask = sum(1 << i for i in lost)
            im, pa = lose(imgs, parity, mask, P, Q, pdirs, orc)
            out, rc = orc.decode_blocks_sys(im, pa, np.array([mask], dtype=np.uint16), P, Q,
                                            pdirs, return_rc=True)
            assert rc[0] == orc.OK and np.array_equal(out, imgs)


def test_sys_parity_is_the_forward_transform(orc):
    P, Q, pdirs = 24, 4, [-1, 1]
    imgs = synth.block_images(3, 0, 2, P, Q)
    parity = orc.encode_blocks_sys(imgs, P, Q, pdirs)
    for b in range(2):
        assert np.array_equal(parity[b], np.concatenate(orc.forward(imgs[b], [(-1, 1), (1, 1)])))
    # the p = 0 parity of a (k, 1) code is the XOR of the data lines (RAID-4/5),
    # bin j holding column P-1-j (bins ascend in b = -k)
    par0 = orc.encode_blocks_sys(imgs, P, Q, [0])
    assert np.array_equal(par0, np.bitwise_xor.reduce(imgs, axis=1)[:, ::-1])


def test_sys_too_many_lost_lines(orc):
    P, Q, pdirs = 16, 4, [-1, 1]
    imgs = synth.block_images(9, 0, 1, P, Q)
    parity = orc.encode_blocks_sys(imgs, P, Q, pdirs)
    for mask in (0b0111, 0b010011, 0b100001 | 0b1000):   # 3 lines; 2 lines + 1 parity
        im, pa = lose(imgs, parity, mask, P, Q, pdirs, orc)
        _, rc = orc.decode_blocks_sys(im, pa, np.array([mask], dtype=np.uint16), P, Q, pdirs,
                                      return_rc=True)
        assert rc[0] == orc.ENOTRECON


def test_sys_intact_lines_need_no_peeling(orc):
    """All lines present: the decode is a copy; the peeling subtracts nothing."""
    P, Q, pdirs = 20, 4, [-1, 1]
    img = synth.block_images(5, 0, 1, P, Q)[0]
    parity = orc.encode_blocks_sys(img[None], P, Q, pdirs)[0]
    known = np.ones((Q, P), dtype=np.uint8)
    cur = img.copy()
    p = np.array(pdirs, dtype=np.int32)
    q = np.ones(2, dtype=np.int32)
    off = np.array([0, orc.proj_size(-1, 1, P, Q)], dtype=np.int64)
    ops = ctypes.c_int64(-1)
    rc = orc._load().orc_inverse_known(orc.XOR, 0, orc._ptr(parity), orc._ptr(off),
                                       orc._ptr(p), orc._ptr(q), 2, P, Q, orc._ptr(known),
                                       orc._ptr(cur), 1, ctypes.addressof(ops))
    assert rc == orc.OK and ops.value == 0 and np.array_equal(cur, img)


def test_sys_all_lines_lost_equals_the_plain_inverse(orc):
    """With m >= Q and every line lost, the systematic decode is the
    non-systematic one from the parity projections alone."""
    P, Q, pdirs = 12, 2, [-1, 0, 2]
    imgs = synth.block_images(6, 0, 1, P, Q)
    parity = orc.encode_blocks_sys(imgs, P, Q, pdirs)
    mask = 0b011 | (1 << (Q + 1))          # both lines and the p = 0 parity lost
    im, pa = lose(imgs, parity, mask, P, Q, pdirs, orc)
    out = orc.decode_blocks_sys(im, pa, np.array([mask], dtype=np.uint16), P, Q, pdirs)
    full = np.zeros((1, orc.block_stride(P, Q, pdirs)), dtype=np.uint64)
    full[:] = parity
    plain = orc.decode_blocks(full, np.array([0b010], dtype=np.uint16), P, Q, pdirs)
    assert np.array_equal(out, imgs) and np.array_equal(plain, imgs)
