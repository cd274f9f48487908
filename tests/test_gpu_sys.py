"""GPU parity for the systematic code (Section 2.3's systematic version, as
built here): the HIP library's systematic entry points against the oracle."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import masks_to_dev, say, to_dev, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


POISON = np.uint64(0xDEADBEEFCAFEF00D)


def run_sys(mj, imgs, masks, P, Q, pdirs):
    """Encode, poison every lost packet, decode in place; returns (parity,
    decoded images, status)."""
    nb = imgs.shape[0]
    words = mj.mojette_block_words(pdirs, P, Q)
    d_img = to_dev(imgs)
    d_par = torch.full((nb * words,), -1, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch_sys(d_img, nb, P, Q, pdirs, d_par)
    torch.cuda.synchronize()
    par = to_np(d_par).reshape(nb, words)
    lossy = imgs.copy()
    bad = par.copy()
    offs = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in pdirs])
    for l in range(Q):
        lossy[np.flatnonzero((masks >> l) & 1), l] = POISON
    for j in range(len(pdirs)):
        bad[np.flatnonzero((masks >> (Q + j)) & 1), offs[j]:offs[j + 1]] = POISON
    d_img2 = to_dev(lossy)
    ws = torch.full((max(1, mj.mojette_sys_workspace(pdirs, P, Q, nb)),), -1, dtype=torch.int64,
                    device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_sys(d_img2, to_dev(bad), masks_to_dev(masks), nb, P, Q, pdirs, ws,
                                d_status)
    torch.cuda.synchronize()
    return par, to_np(d_img2).reshape(nb, Q, P), int(d_status.item()), lossy


@pytest.mark.parametrize("P,Q,pdirs", [(128, 4, [-1, 0]), (37, 3, [-1, 0, 1]), (16, 2, [3]),
                                       (64, 8, [-2, -1, 0, 1])])
def test_sys_every_erasure_pattern(mj, P, Q, pdirs):
    """Every pattern of at most m lost packets, several blocks each."""
    m = len(pdirs)
    pats = [sum(1 << i for i in c) for r in range(m + 1)
            for c in itertools.combinations(range(Q + m), r)]
    masks = np.array([x for x in pats for _ in range(3)], dtype=np.uint16)
    nb = len(masks)
    say(f"sys patterns P={P} Q={Q} m={m} blocks={nb}")
    imgs = synth.block_images(500 + P + Q, 0, nb, P, Q)
    par, dec, st, _ = run_sys(mj, imgs, masks, P, Q, pdirs)
    assert np.array_equal(par, oracle.encode_blocks_sys(imgs, P, Q, pdirs))
    assert st == 0
    assert np.array_equal(dec, imgs)


@pytest.mark.parametrize("P,Q,pdirs,ner,nb", [(256, 4, [-1, 0], (0, 2), 200),
                                              (300, 2, [-1, 1], 2, 30),
                                              (48, 12, [-2, -1, 0, 1], 4, 57),
                                              (128, 8, [-2, -1, 0, 1], (0, 4), 101),
                                              (9, 5, [-3, -2, -1, 0, 1, 2, 3, 4], (0, 8), 40)])
def test_sys_random_erasures_match_the_oracle(mj, P, Q, pdirs, ner, nb):
    m = len(pdirs)
    say(f"sys random P={P} Q={Q} m={m} blocks={nb}")
    imgs = synth.block_images(600 + P, 0, nb, P, Q)
    masks = synth.erasure_masks(31 + Q, nb, Q + m, ner)
    par, dec, st, lossy = run_sys(mj, imgs, masks, P, Q, pdirs)
    assert st == 0
    assert np.array_equal(dec, imgs)
    bad = par.copy()   # the oracle ignores lost packets' contents
    want = oracle.decode_blocks_sys(lossy[:8], bad[:8], masks[:8], P, Q, pdirs)
    assert np.array_equal(dec[:8], want)


def test_sys_too_many_lost_lines_are_reported_and_left_alone(mj):
    P, Q, pdirs = 64, 4, [-1, 0]
    masks = np.array([0b000111, 0b010011, 0b000001, 0b110000, 0b101001], dtype=np.uint16)
    imgs = synth.block_images(77, 0, len(masks), P, Q)
    _, dec, st, lossy = run_sys(mj, imgs, masks, P, Q, pdirs)
    assert st == -2                             # MOJETTE_ENOTRECON
    for b in (0, 1, 4):                         # 3 lines; 2 lines + 1 parity; 2 lines + 1 parity
        assert np.array_equal(dec[b], lossy[b])   # untouched
    for b in (2, 3):
        assert np.array_equal(dec[b], imgs[b])


def test_sys_full_size_4k(mj):
    """2^21 blocks of 4 KB, 4 lines + 2 parity projections, 2 of the 6 packets
    lost per block; round trip over every block, oracle on a sample."""
    P, Q, pdirs, nb = 128, 4, [-1, 0], 1 << 21
    words = mj.mojette_block_words(pdirs, P, Q)
    say(f"sys full size: {nb} blocks")
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), synth.SEED_DATA + 11)
    ref = d_img.clone()
    masks = synth.erasure_masks(synth.SEED_ERASE, nb, Q + 2, 2)
    d_par = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    ws = torch.empty(mj.mojette_sys_workspace(pdirs, P, Q, nb), dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batch_sys(d_img, nb, P, Q, pdirs, d_par)
    # lose the lines: overwrite them on the device
    lost = torch.from_numpy(((masks[:, None] >> np.arange(Q)) & 1).astype(bool)).cuda()
    d_img.view(nb, Q, P).masked_fill_(lost[:, :, None], -1)
    mj.mojette_decode_batch_sys(d_img, d_par, masks_to_dev(masks), nb, P, Q, pdirs, ws, d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    assert torch.equal(d_img, ref)
    rng = np.random.default_rng(12)
    sample = np.unique(np.concatenate([[0, nb - 1], rng.integers(0, nb, 40)]))
    idx = torch.from_numpy(sample).cuda()
    imgs = to_np(ref.view(nb, -1)[idx]).reshape(len(sample), Q, P)
    got = to_np(d_par.view(nb, words)[idx])
    assert np.array_equal(got, oracle.encode_blocks_sys(imgs, P, Q, pdirs))
    del d_img, ref, d_par, ws
    torch.cuda.empty_cache()


def test_sys_argument_checks(mj):
    d = torch.zeros(16, dtype=torch.int64, device="cuda")
    m16 = torch.zeros(4, dtype=torch.int16, device="cuda")
    assert mj.mojette_sys_workspace([0, 1], 8, 15, 4) == -1          # 15 + 2 > 16 packets
    assert mj.mojette_sys_workspace(list(range(-4, 5)), 8, 4, 4) == -1   # m > 8
    assert mj.mojette_decode_batch_sys(d, d, m16, 1, 8, 15, [0, 1], d,
                                       check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_decode_batch_sys(d, d, None, 4, 8, 2, [0, 1], d) == 0   # nothing lost
