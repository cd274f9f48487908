"""Two-corner decode (mojette_decode_batch_two_corner): every block swept
from both ends, each sweep stopping past the middle; bit-identical to the
oracle's peeling and to the one-sided sweep, from pools whose erased
projections are overwritten, on codes of 1 to 16 rows, odd and even row
lengths, every erasure pattern of the (6,4) code, and undecodable blocks."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import masks_to_dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

POISON = np.uint64(0xDEADBEEFCAFEF00D)


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def poisoned(enc, masks, P, Q, dirs):
    out = enc.copy()
    off = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
    for i in range(len(dirs)):
        out[np.flatnonzero((masks >> i) & 1), off[i]:off[i + 1]] = POISON
    return out


def both_decodes(mj, imgs, masks, P, Q, dirs, nbw=0):
    nb = imgs.shape[0]
    enc = oracle.encode_blocks(imgs, P, Q, dirs)
    d_src = to_dev(poisoned(enc, masks, P, Q, dirs))
    d_mask = masks_to_dev(masks)
    two = torch.full((nb * Q * P,), -1, dtype=torch.int64, device="cuda")
    one = torch.full_like(two, -1)
    st2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    st1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_two_corner(d_src, d_mask, nb, P, Q, dirs, two, st2, nbw)
    mj.mojette_decode_batch(d_src, d_mask, nb, P, Q, dirs, one, st1)
    torch.cuda.synchronize()
    return enc, to_np(two).reshape(nb, Q, P), to_np(one).reshape(nb, Q, P), int(st2.item()), \
        int(st1.item())


GEOMS = [
    # (P, Q, dirs, erasures, nblocks)
    (128, 4, synth.centered_dirs(6), 2, 300),
    (129, 4, synth.centered_dirs(6), (0, 2), 200),
    (128, 8, synth.centered_dirs(12), 4, 200),
    (1024, 8, synth.centered_dirs(12), (0, 4), 40),
    (1366, 6, synth.centered_dirs(9), (0, 3), 30),
    (683, 12, synth.centered_dirs(16), (0, 4), 20),
    (64, 16, synth.centered_dirs(16), 0, 12),
    (17, 3, [2, -1, 0, 5], 1, 100),
    (3, 2, [-1, 0, 1], 1, 100),
    (1, 1, [0], 0, 50),
    (1, 4, [-2, -1, 0, 1, 2], 1, 50),
    (40, 5, [7, -6, 0, 2, -3, 1], 1, 60),
    (2048, 4, synth.centered_dirs(6), (0, 2), 30),
]


@pytest.mark.parametrize("P,Q,dirs,ner,nb", GEOMS)
def test_two_corner_matches_oracle_and_one_sided(mj, P, Q, dirs, ner, nb):
    say(f"two-corner: P={P} Q={Q} dirs={dirs} erasures={ner} blocks={nb}")
    imgs = synth.block_images(P * 7 + Q, 0, nb, P, Q)
    masks = synth.erasure_masks(P + 3 * Q, nb, len(dirs), ner)
    enc, two, one, st2, st1 = both_decodes(mj, imgs, masks, P, Q, dirs)
    assert st2 == 0 and st1 == 0
    assert np.array_equal(one, imgs)
    assert np.array_equal(two, imgs)
    src = poisoned(enc, masks, P, Q, dirs)
    sample = np.unique([0, nb // 2, nb - 1])
    assert np.array_equal(two[sample], oracle.decode_blocks(src[sample], masks[sample], P, Q, dirs))


def test_two_corner_every_erasure_pattern_and_blocks_per_wave(mj):
    P, Q, dirs = 200, 4, synth.centered_dirs(6)
    pats = [0]
    for r in (1, 2):
        for lost in itertools.combinations(range(6), r):
            pats.append(sum(1 << i for i in lost))
    masks = np.array(pats * 10, dtype=np.uint16)
    imgs = synth.block_images(8, 0, len(masks), P, Q)
    for nbw in (0, 1, 3, 16):
        _, two, _, st, _ = both_decodes(mj, imgs, masks, P, Q, dirs, nbw)
        assert st == 0 and np.array_equal(two, imgs), nbw


def test_two_corner_undecodable_blocks(mj):
    P, Q, n, nb = 96, 4, 6, 60
    dirs = synth.centered_dirs(n)
    imgs = synth.block_images(4, 0, nb, P, Q)
    masks = synth.erasure_masks(5, nb, n, 2)
    bad = np.arange(0, nb, 7)
    masks[bad] |= np.uint16(0b111000)
    _, two, _, st, _ = both_decodes(mj, imgs, masks, P, Q, dirs)
    assert st == mj.MOJETTE_ENOTRECON
    good = np.setdiff1d(np.arange(nb), bad)
    assert np.array_equal(two[good], imgs[good])
    assert (two[bad] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()


def test_two_corner_full_size_12_8(mj):
    """2^19 blocks of 8 KB, the (12,8) code, exactly 4 erasures per block,
    poisoned on the device: the round trip over every block."""
    from tests.gpuutil import poison_erased_dev

    P, Q, n, nb = 128, 8, 12, 1 << 19
    dirs = synth.centered_dirs(n)
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), 33)
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    masks = synth.erasure_masks(34, nb, n, 4)
    poison_erased_dev(d_proj, masks, [mj.mojette_proj_size(p, P, Q) for p in dirs])
    out = torch.empty_like(d_img)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_two_corner(d_proj, masks_to_dev(masks), nb, P, Q, dirs, out, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(out, d_img)
