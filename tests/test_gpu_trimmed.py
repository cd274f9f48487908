"""GPU parity for the code without never-used bins (Section 2.3): the HIP
library's trimmed entry points against the oracle, bit for bit."""
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


@pytest.mark.parametrize("P,Q,n,ner,nblocks", [
    (128, 4, 6, 2, 70),        # 4 KB (6,4)
    (128, 8, 12, 4, 19),       # 8 KB (8,4)
    (256, 4, 6, (0, 2), 33),   # 8 KB (4,2)
    (64, 4, 12, (0, 8), 25),   # (12,4)
    (37, 3, 6, 3, 41),         # odd row length, ragged batch
    (300, 2, 4, 2, 9),         # rows wider than one encode tile
    (5, 1, 3, 2, 7),
])
def test_trimmed_parity(mj, P, Q, n, ner, nblocks):
    dirs = synth.centered_dirs(n)
    say(f"trimmed parity P={P} Q={Q} n={n} blocks={nblocks}")
    words, keep = mj.mojette_trimmed_layout(dirs, P, Q)
    imgs = synth.block_images(300 + P + n, 0, nblocks, P, Q)
    masks = synth.erasure_masks(17 + n, nblocks, n, ner)
    d_img = to_dev(imgs)
    d_proj = torch.full((nblocks * words,), -1, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch_trimmed(d_img, nblocks, P, Q, dirs, d_proj)
    torch.cuda.synchronize()
    enc = to_np(d_proj).reshape(nblocks, words)
    assert np.array_equal(enc, oracle.encode_blocks_kept(imgs, P, Q, dirs))
    src = enc.copy()
    offs = np.concatenate([[0], np.cumsum([c for _, c in keep])])
    for i in range(n):
        src[np.flatnonzero((masks >> i) & 1), offs[i]:offs[i + 1]] = POISON
    d_out = torch.full((nblocks * Q * P,), -1, dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_trimmed(to_dev(src), masks_to_dev(masks), nblocks, P, Q, dirs,
                                    d_out, d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    out = to_np(d_out).reshape(nblocks, Q, P)
    assert np.array_equal(out, imgs)
    assert np.array_equal(out[:4], oracle.decode_blocks_kept(src[:4], masks[:4], P, Q, dirs))


@pytest.mark.parametrize("P,Q,n,nblocks,ner", [(128, 4, 6, 1 << 21, 2), (128, 8, 12, 1 << 19, 4)])
def test_trimmed_full_size(mj, P, Q, n, nblocks, ner):
    dirs = synth.centered_dirs(n)
    words, _ = mj.mojette_trimmed_layout(dirs, P, Q)
    say(f"trimmed full size: {nblocks} blocks P={P} Q={Q} n={n}")
    d_img = torch.empty(nblocks * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), synth.SEED_DATA + 9)
    masks = synth.erasure_masks(synth.SEED_ERASE, nblocks, n, ner)
    d_proj = torch.empty(nblocks * words, dtype=torch.int64, device="cuda")
    d_out = torch.empty_like(d_img)
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batch_trimmed(d_img, nblocks, P, Q, dirs, d_proj)
    mj.mojette_decode_batch_trimmed(d_proj, masks_to_dev(masks), nblocks, P, Q, dirs, d_out,
                                    d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    assert torch.equal(d_out, d_img)
    rng = np.random.default_rng(6)
    sample = np.unique(np.concatenate([[0, nblocks - 1], rng.integers(0, nblocks, 40)]))
    idx = torch.from_numpy(sample).cuda()
    imgs = to_np(d_img.view(nblocks, -1)[idx]).reshape(len(sample), Q, P)
    got = to_np(d_proj.view(nblocks, words)[idx])
    assert np.array_equal(got, oracle.encode_blocks_kept(imgs, P, Q, dirs))
    del d_img, d_proj, d_out
    torch.cuda.empty_cache()


def test_trimmed_argument_checks(mj):
    d = torch.zeros(16, dtype=torch.int64, device="cuda")
    assert mj.mojette_encode_batch_trimmed(d, 1, 8, 3, [0, 1], d,
                                           check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_decode_batch_trimmed(d, None, -1, 8, 2, [0, 1], d,
                                           check=False) == mj.MOJETTE_EINVAL
    assert mj.mojette_encode_batch_trimmed(d, 0, 8, 2, [0, 1], d) == 0


@pytest.mark.parametrize("P,Q,n,m", [
    (128, 4, 6, 4),     # 4 KB (6,4)
    (128, 8, 12, 9),    # 8 KB (8,4), more survivors than Q
    (37, 3, 6, 3),      # odd row length
    (300, 2, 4, 4),     # rows over several encode tiles, every projection given
])
def test_trimmed_one_block(mj, P, Q, n, m):
    """mojette_encode_trimmed / mojette_decode_trimmed: one block, each
    projection's kept bins at its own pointer, against the oracle's kept-bin
    transform; the verified decode from m of them restores the image."""
    dirs = synth.centered_dirs(n)
    say(f"trimmed one block P={P} Q={Q} n={n} m={m}")
    words, keep = mj.mojette_trimmed_layout(dirs, P, Q)
    img = synth.block_images(700 + P + n, 0, 1, P, Q)
    want = oracle.encode_blocks_kept(img, P, Q, dirs)[0]
    offs = np.concatenate([[0], np.cumsum([c for _, c in keep])]).astype(int)
    outs = [torch.full((c,), -1, dtype=torch.int64, device="cuda") for _, c in keep]
    assert mj.mojette_encode_trimmed(to_dev(img), P, Q, dirs, outs) == 0
    torch.cuda.synchronize()
    for i in range(n):
        assert np.array_equal(to_np(outs[i]), want[offs[i]:offs[i + 1]]), i
    ids = sorted(np.random.default_rng(P + m).choice(n, m, replace=False).tolist())
    for i in set(range(n)) - set(ids):
        outs[i].fill_(int(POISON.astype(np.int64)))
    d_out = torch.full((Q * P,), -1, dtype=torch.int64, device="cuda")
    assert mj.mojette_decode_trimmed([outs[i] for i in ids], ids, dirs, P, Q, d_out,
                                     verify=True) == 0
    torch.cuda.synchronize()
    assert np.array_equal(to_np(d_out).reshape(Q, P), img[0])


def test_trimmed_one_block_verify_finds_a_flipped_bin(mj):
    """A flipped kept bin of a projection the decode does not use (every
    projection given; the Q of smallest p rebuild): the verified decode
    reports MOJETTE_EINCONSISTENT."""
    P, Q, n = 128, 4, 6
    dirs = synth.centered_dirs(n)
    _, keep = mj.mojette_trimmed_layout(dirs, P, Q)
    img = synth.block_images(41, 0, 1, P, Q)
    want = oracle.encode_blocks_kept(img, P, Q, dirs)[0]
    offs = np.concatenate([[0], np.cumsum([c for _, c in keep])]).astype(int)
    unused = np.argsort(dirs)[Q:]
    rng = np.random.default_rng(9)
    for trial in range(4):
        i = int(unused[trial % len(unused)])
        bins = want[offs[i]:offs[i + 1]].copy()
        bins[int(rng.integers(0, len(bins)))] ^= np.uint64(1 << int(rng.integers(64)))
        proj = [to_dev(want[offs[t]:offs[t + 1]]) for t in range(n)]
        proj[i] = to_dev(bins)
        d_out = torch.empty(Q * P, dtype=torch.int64, device="cuda")
        rc = mj.mojette_decode_trimmed(proj, list(range(n)), dirs, P, Q, d_out, verify=True,
                                       check=False)
        assert rc == mj.MOJETTE_EINCONSISTENT, (trial, i)
        assert np.array_equal(to_np(d_out).reshape(Q, P), img[0])
