"""GPU parity for the 128-bit pixel code (Section 3.1): the HIP library's wide
entry points against the oracle, bit for bit."""
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


def wide_images(seed, nblocks, P, Q):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**64, size=(nblocks, Q, P, 2), dtype=np.uint64)


def run_wide(mj, imgs, masks, P, Q, dirs):
    nb = imgs.shape[0]
    words = 2 * mj.mojette_block_words(dirs, P, Q)
    d_img = to_dev(imgs)
    d_proj = torch.full((nb * words,), -1, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch_wide(d_img, nb, P, Q, dirs, d_proj)
    torch.cuda.synchronize()
    enc = to_np(d_proj).reshape(nb, words // 2, 2)
    # overwrite every erased projection so that a decode reading it fails
    src = enc.copy()
    off = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
    for i in range(len(dirs)):
        rows = np.flatnonzero((masks >> i) & 1)
        src[rows, off[i]:off[i + 1]] = POISON
    d_out = torch.full((nb * Q * P * 2,), -1, dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_wide(to_dev(src), masks_to_dev(masks), nb, P, Q, dirs, d_out,
                                 d_status)
    torch.cuda.synchronize()
    return enc, to_np(d_out).reshape(nb, Q, P, 2), int(d_status.item())


@pytest.mark.parametrize("P,Q,n,ner,nblocks", [
    (64, 4, 6, 2, 67),        # 4 KB block of the (6,4) code in the paper's pixels
    (128, 4, 6, (0, 2), 40),  # 8 KB (4,2)
    (64, 8, 12, 4, 21),       # 8 KB (8,4)
    (37, 3, 5, 2, 33),        # odd row length, ragged batch
    (1, 1, 2, 1, 5),
    (300, 2, 4, 2, 9),        # rows wider than one encode tile of 64 columns
])
def test_wide_parity(mj, P, Q, n, ner, nblocks):
    dirs = synth.centered_dirs(n)
    say(f"wide parity P={P} Q={Q} n={n} blocks={nblocks}")
    imgs = wide_images(100 + P + Q + n, nblocks, P, Q)
    masks = synth.erasure_masks(7 + n, nblocks, n, ner)
    enc, dec, st = run_wide(mj, imgs, masks, P, Q, dirs)
    assert np.array_equal(enc, oracle.encode_blocks_wide(imgs, P, Q, dirs))
    assert st == 0
    assert np.array_equal(dec, imgs)


def test_wide_full_size_4k_6_4(mj):
    """2^21 blocks of 4 KB with 16-byte pixels (P = 64 x Q = 4), two erasures
    per block: round trip over every block, oracle on a sample."""
    P, Q, n, nblocks = 64, 4, 6, 1 << 21
    dirs = synth.centered_dirs(n)
    words = 2 * mj.mojette_block_words(dirs, P, Q)
    say(f"wide full size: {nblocks} blocks P={P} Q={Q} n={n}")
    d_img = torch.empty(nblocks * Q * P * 2, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), synth.SEED_DATA + 5)
    masks = synth.erasure_masks(synth.SEED_ERASE, nblocks, n, 2)
    d_proj = torch.empty(nblocks * words, dtype=torch.int64, device="cuda")
    d_out = torch.empty_like(d_img)
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batch_wide(d_img, nblocks, P, Q, dirs, d_proj)
    mj.mojette_decode_batch_wide(d_proj, masks_to_dev(masks), nblocks, P, Q, dirs, d_out,
                                 d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    assert torch.equal(d_out, d_img)
    rng = np.random.default_rng(4)
    sample = np.unique(np.concatenate([[0, nblocks - 1], rng.integers(0, nblocks, 48)]))
    idx = torch.from_numpy(sample).cuda()
    imgs = to_np(d_img.view(nblocks, -1)[idx]).reshape(len(sample), Q, P, 2)
    got = to_np(d_proj.view(nblocks, words)[idx]).reshape(len(sample), words // 2, 2)
    assert np.array_equal(got, oracle.encode_blocks_wide(imgs, P, Q, dirs))
    del d_img, d_proj, d_out
    torch.cuda.empty_cache()


def test_wide_argument_checks(mj):
    dirs = synth.centered_dirs(6)
    d = torch.zeros(16, dtype=torch.int64, device="cuda")
    assert mj.mojette_encode_batch_wide(d, 0, 64, 4, dirs, d) == 0
    assert mj.mojette_encode_batch_wide(d, 1, (1 << 23) + 1, 1, [0, 1], d,
                                        check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_decode_batch_wide(d, None, 1, 8, 2, [0, 1 << 15 | 1], d,
                                        check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_encode_batch_wide(d, -1, 8, 2, [0, 1], d,
                                        check=False) == mj.MOJETTE_EINVAL


@pytest.mark.parametrize("P,Q,n,m", [
    (64, 4, 6, 4),      # 4 KB block of the (6,4) code in the paper's pixels
    (37, 3, 5, 5),      # odd row length, every projection given (Q of them used)
    (1, 1, 2, 1),
    (700, 2, 4, 3),     # rows over several tiles, a ragged last one
])
def test_wide_one_block(mj, P, Q, n, m):
    """mojette_encode_wide / mojette_decode_wide: one block, projections at
    separate pointers, against the oracle's wide transform; the decode reads
    m of them (erased ones overwritten) and restores the image."""
    dirs = synth.centered_dirs(n)
    say(f"wide one block P={P} Q={Q} n={n} m={m}")
    img = wide_images(500 + P + n, 1, P, Q)
    want = oracle.encode_blocks_wide(img, P, Q, dirs)[0]
    sizes = [oracle.proj_size(p, 1, P, Q) for p in dirs]
    off = np.cumsum([0] + sizes)
    outs = [torch.full((2 * s,), -1, dtype=torch.int64, device="cuda") for s in sizes]
    assert mj.mojette_encode_wide(to_dev(img), P, Q, dirs, outs) == 0
    torch.cuda.synchronize()
    for i in range(n):
        assert np.array_equal(to_np(outs[i]).reshape(-1, 2), want[off[i]:off[i + 1]]), i
    ids = sorted(np.random.default_rng(P + m).choice(n, m, replace=False).tolist())
    for i in set(range(n)) - set(ids):
        outs[i].fill_(int(POISON.astype(np.int64)))
    d_out = torch.full((Q * P * 2,), -1, dtype=torch.int64, device="cuda")
    assert mj.mojette_decode_wide([outs[i] for i in ids], ids, dirs, P, Q, d_out,
                                  verify=True) == 0
    torch.cuda.synchronize()
    assert np.array_equal(to_np(d_out).reshape(Q, P, 2), img[0])


def test_wide_one_block_verify_finds_a_flipped_word(mj):
    """One flipped word of one 16-byte bin (either half): with every
    projection given the verified decode reports MOJETTE_EINCONSISTENT."""
    P, Q, n = 64, 4, 6
    dirs = synth.centered_dirs(n)
    img = wide_images(31, 1, P, Q)
    want = oracle.encode_blocks_wide(img, P, Q, dirs)[0]
    off = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
    rng = np.random.default_rng(8)
    for trial in range(4):
        i = int(rng.integers(0, n))
        bins = want[off[i]:off[i + 1]].copy()
        bins[int(rng.integers(0, len(bins))), trial % 2] ^= np.uint64(1 << int(rng.integers(64)))
        proj = [to_dev(want[off[t]:off[t + 1]]) for t in range(n)]
        proj[i] = to_dev(bins)
        d_out = torch.empty(Q * P * 2, dtype=torch.int64, device="cuda")
        rc = mj.mojette_decode_wide(proj, list(range(n)), dirs, P, Q, d_out, verify=True,
                                    check=False)
        assert rc == mj.MOJETTE_EINCONSISTENT, (trial, i)


def test_wide_one_block_argument_checks(mj):
    d = torch.zeros(16, dtype=torch.int64, device="cuda")
    assert mj.mojette_encode_wide(d, (1 << 23) + 1, 1, [0, 1], [d, d],
                                  check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_decode_wide([d, d], [0, 1], [0, 1 << 15 | 1], 8, 2, d,
                                  check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_decode_wide([d], [0], [0, 1], 8, 2, d,
                                  check=False) == mj.MOJETTE_ENOTRECON
