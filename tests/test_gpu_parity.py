"""Bit-exact parity of the HIP path with the CPU oracle (needs an MI355X).

Every comparison is exact: the arithmetic is XOR on 64-bit words, and with
Katz's criterion satisfied the decoded image is unique (Section 2.2, Eq. 3),
so there is no tolerance anywhere.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import mask_depth, masks_to_dev, poison_erased_dev, say, to_dev, to_np

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


def poison_erased(pool: np.ndarray, masks: np.ndarray, P: int, Q: int, dirs) -> np.ndarray:
    """Overwrite the bins of every erased projection, so a decoder that reads
    them would produce wrong pixels."""
    out = pool.copy()
    off = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
    for i in range(len(dirs)):
        rows = np.flatnonzero((masks >> i) & 1)
        out[rows, off[i]:off[i + 1]] = POISON
    return out


def run_batch(mj, imgs, masks, P, Q, dirs, poison=True):
    nb = imgs.shape[0]
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = to_dev(imgs)
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    torch.cuda.synchronize()
    enc = to_np(d_proj).reshape(nb, words)
    src = poison_erased(enc, masks, P, Q, dirs) if poison else enc
    d_src = to_dev(src)
    d_out = torch.full((nb * Q * P,), -1, dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch(d_src, masks_to_dev(masks), nb, P, Q, dirs, d_out, d_status)
    torch.cuda.synchronize()
    return enc, to_np(d_out).reshape(nb, Q, P), int(d_status.item())


def test_fill_splitmix64_matches_numpy(mj):
    n = 1 << 20
    d = torch.empty(n, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d, n, synth.SEED_DATA, 12345)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(d), synth.splitmix64(synth.SEED_DATA, 12345, n))


def test_config_4k_6_4_as_stated(mj):
    """1,024 blocks of 4 KB, P=128, Q=4, n=6, p in -3..2, two erasures per
    block drawn by the seed; encode and decode bit-exact against the oracle,
    and the round trip gives the blocks back."""
    P, Q, n, nb = 128, 4, 6, 1024
    dirs = synth.centered_dirs(n)
    say(f"config 4K (6,4): {nb} blocks")
    imgs = synth.block_images(synth.SEED_DATA, 0, nb, P, Q)
    masks = synth.erasure_masks(synth.SEED_ERASE, nb, n, 2)
    enc, dec, st = run_batch(mj, imgs, masks, P, Q, dirs)
    assert np.array_equal(enc, oracle.encode_blocks(imgs, P, Q, dirs))
    assert st == 0
    assert np.array_equal(dec, oracle.decode_blocks(enc, masks, P, Q, dirs))
    assert np.array_equal(dec, imgs)


def test_every_erasure_pattern_4k(mj):
    """All 22 patterns of at most two erasures of the (6,4) code."""
    P, Q, n = 128, 4, 6
    dirs = synth.centered_dirs(n)
    pats = [0]
    for r in (1, 2):
        for lost in itertools.combinations(range(n), r):
            pats.append(sum(1 << i for i in lost))
    masks = np.array(pats * 12, dtype=np.uint16)
    imgs = synth.block_images(77, 0, len(masks), P, Q)
    enc, dec, st = run_batch(mj, imgs, masks, P, Q, dirs)
    assert st == 0
    assert np.array_equal(dec, imgs)


GEOMS = [
    # (P, Q, dirs, erasures as int or (lo, hi), nblocks)
    (1, 1, [0], 0, 70),
    (1, 4, [-2, -1, 0, 1, 2], 1, 70),
    (3, 2, [-1, 0, 1], 1, 130),
    (17, 4, [-3, -2, -1, 0, 1, 2], 2, 100),
    (33, 3, [2, -1, 0, 5], 1, 90),
    (100, 8, list(range(-6, 6)), 4, 60),
    (128, 8, list(range(-6, 6)), (0, 4), 60),
    (171, 6, list(range(-4, 5)), (0, 3), 40),
    (129, 12, list(range(-8, 8)), (0, 4), 30),
    (64, 16, list(range(-8, 8)), 0, 12),
    (256, 4, [-3, -2, -1, 0, 1, 2], (0, 2), 80),
    (40, 5, [7, -6, 0, 2, -3, 1], 1, 50),
    (16, 7, [3, -2, 9, -8, 0, 1, 5, -1], 1, 50),
]


@pytest.mark.parametrize("P,Q,dirs,ner,nb", GEOMS)
def test_geometry_parity(mj, P, Q, dirs, ner, nb):
    n = len(dirs)
    say(f"geometry P={P} Q={Q} dirs={dirs} erasures={ner} blocks={nb}")
    imgs = synth.block_images(P * 1000 + Q, 0, nb, P, Q)
    masks = synth.erasure_masks(P + Q, nb, n, ner)
    enc, dec, st = run_batch(mj, imgs, masks, P, Q, dirs)
    assert np.array_equal(enc, oracle.encode_blocks(imgs, P, Q, dirs))
    assert st == 0
    assert np.array_equal(dec, oracle.decode_blocks(enc, masks, P, Q, dirs))


@pytest.mark.parametrize("P,Q,dirs,nb", [
    (32768, 4, [-3, -2, -1, 0, 1, 2], 3),            # 1 MB block, k = 4
    (10923, 12, list(range(-8, 8)), 2),              # 1 MB block, k = 12 (last row padded)
    (1366, 6, list(range(-4, 5)), 4),                # 64 KB block, k = 6
])
def test_large_blocks(mj, P, Q, dirs, nb):
    """Blocks wider than one encode tile and far longer than the decode ring."""
    n = len(dirs)
    say(f"large block P={P} Q={Q} n={n}")
    imgs = synth.block_images(5 + P, 0, nb, P, Q)
    masks = synth.erasure_masks(9, nb, n, (0, n - Q))
    enc, dec, st = run_batch(mj, imgs, masks, P, Q, dirs)
    assert np.array_equal(enc, oracle.encode_blocks(imgs, P, Q, dirs))
    assert st == 0
    assert np.array_equal(dec, imgs)


def test_undecodable_blocks_report_status(mj):
    P, Q, n, nb = 64, 4, 6, 200
    dirs = synth.centered_dirs(n)
    imgs = synth.block_images(3, 0, nb, P, Q)
    masks = synth.erasure_masks(4, nb, n, 2)
    bad = np.arange(0, nb, 7)
    masks[bad] |= np.uint16(0b111)       # at least 3 lost: fewer than Q survive
    enc, dec, st = run_batch(mj, imgs, masks, P, Q, dirs)
    assert st == -2
    good = np.setdiff1d(np.arange(nb), bad)
    assert np.array_equal(dec[good], imgs[good])
    assert (dec[bad] == np.uint64(0xFFFFFFFFFFFFFFFF)).all()  # left unwritten


def test_single_block_calls_match_batch_and_oracle(mj):
    P, Q, n = 128, 4, 6
    dirs = synth.centered_dirs(n)
    imgs = synth.block_images(21, 0, 6, P, Q)
    sizes = [oracle.proj_size(p, 1, P, Q) for p in dirs]
    for b in range(imgs.shape[0]):
        d_img = to_dev(imgs[b])
        outs = [torch.empty(s, dtype=torch.int64, device="cuda") for s in sizes]
        mj.mojette_encode(d_img, P, Q, dirs, outs)
        torch.cuda.synchronize()
        want = oracle.forward(imgs[b], [(p, 1) for p in dirs])
        for o, w in zip(outs, want):
            assert np.array_equal(to_np(o), w)
        # decode from m = 4, 5, 6 survivors given in scrambled order
        for m in (4, 5, 6):
            ids = list(np.random.default_rng(b * 10 + m).permutation(n)[:m])
            d_out = torch.zeros(Q * P, dtype=torch.int64, device="cuda")
            mj.mojette_decode([outs[i] for i in ids], ids, dirs, P, Q, d_out)
            torch.cuda.synchronize()
            assert np.array_equal(to_np(d_out).reshape(Q, P), imgs[b]), (b, ids)
    # errors on the single-block path
    d_out = torch.zeros(Q * P, dtype=torch.int64, device="cuda")
    assert mj.mojette_decode([outs[0], outs[1], outs[2]], [0, 1, 2], dirs, P, Q, d_out,
                             check=False) == mj.MOJETTE_ENOTRECON
    assert mj.mojette_decode([outs[0], outs[0], outs[2], outs[3]], [0, 0, 2, 3], dirs, P, Q,
                             d_out, check=False) == mj.MOJETTE_EINVAL


def test_hip_graph_replay(mj):
    """Encode + decode recorded into a HIP graph: every replay, on inputs
    changed eagerly between replays, matches the eager result."""
    P, Q, n, nb = 128, 4, 6, 4096
    dirs = synth.centered_dirs(n)
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    d_out = torch.empty_like(d_img)
    d_mask = masks_to_dev(synth.erasure_masks(5, nb, n, 2))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mj.mojette_fill_splitmix64(d_img, d_img.numel(), 1)
        mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
        mj.mojette_decode_batch(d_proj, d_mask, nb, P, Q, dirs, d_out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
        mj.mojette_decode_batch(d_proj, d_mask, nb, P, Q, dirs, d_out)
    for rep in range(4):
        mj.mojette_fill_splitmix64(d_img, d_img.numel(), 100 + rep)
        d_out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_proj = d_proj.clone()
        got_out = d_out.clone()
        mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
        mj.mojette_decode_batch(d_proj, d_mask, nb, P, Q, dirs, d_out)
        torch.cuda.synchronize()
        assert torch.equal(got_proj, d_proj)
        assert torch.equal(got_out, d_out)
        assert torch.equal(got_out, d_img)


def full_size_case(mj, P, Q, n, nblocks, ner, seed):
    """Encode and decode at the full batch size, in the launches the library
    picks for it (ring classes and the gathered long-ring launch included),
    from a pool whose erased projections are overwritten on the device: the
    round trip over every block, encode and decode against the oracle on a
    sample that holds the first and last blocks, random ones and blocks of
    the deepest survivor set present."""
    dirs = synth.centered_dirs(n)
    sizes = [oracle.proj_size(p, 1, P, Q) for p in dirs]
    words = mj.mojette_block_words(dirs, P, Q)
    say(f"full size: {nblocks} blocks P={P} Q={Q} n={n}")
    d_img = torch.empty(nblocks * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), seed)
    masks = synth.erasure_masks(synth.SEED_ERASE, nblocks, n, ner)
    d_mask = masks_to_dev(masks)
    d_proj = torch.empty(nblocks * words, dtype=torch.int64, device="cuda")
    d_out = torch.empty_like(d_img)
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batch(d_img, nblocks, P, Q, dirs, d_proj)
    rng = np.random.default_rng(seed)
    depths = {int(m): mask_depth(int(m), dirs, Q) for m in np.unique(masks)}
    dmax = max(depths.values())
    deep_masks = np.array([m for m, d in depths.items() if d == dmax], dtype=np.uint16)
    deepest = np.flatnonzero(np.isin(masks, deep_masks))
    sample = np.unique(np.concatenate([[0, nblocks - 1], rng.integers(0, nblocks, 48),
                                       deepest[:8], deepest[-8:]]))
    idx = torch.from_numpy(sample).cuda()
    proj2 = d_proj.view(nblocks, words)
    torch.cuda.synchronize()
    got = to_np(proj2[idx])                              # encode, before any bin is overwritten
    imgs = synth.sample_images(seed, sample, P, Q)
    want = oracle.encode_blocks(imgs, P, Q, dirs)
    assert np.array_equal(got.reshape(len(sample), words), want)
    poison_erased_dev(d_proj, masks, sizes)
    mj.mojette_decode_batch(d_proj, d_mask, nblocks, P, Q, dirs, d_out, d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    assert torch.equal(d_out, d_img)          # round trip over every block
    src = to_np(proj2[idx]).reshape(len(sample), words)
    assert np.array_equal(src, poison_erased(want, masks[sample], P, Q, dirs))
    dec = oracle.decode_blocks(src, masks[sample], P, Q, dirs)
    assert np.array_equal(dec, imgs)
    assert np.array_equal(to_np(d_out.view(nblocks, -1)[idx]).reshape(len(sample), Q, P), dec)
    del d_img, d_proj, d_out
    torch.cuda.empty_cache()


def test_full_size_4k_6_4(mj):
    """4 KB blocks of the (6,4) code at the benchmark's batch of 2^21 blocks."""
    full_size_case(mj, 128, 4, 6, 1 << 21, 2, synth.SEED_DATA)


def test_full_size_8k_6_4(mj):
    """2^20 blocks of 8 KB, (k=4, m=2), 0-2 erasures per block."""
    full_size_case(mj, 256, 4, 6, 1 << 20, (0, 2), synth.SEED_DATA + 1)


def test_full_size_8k_12_8(mj):
    """2^19 blocks of 8 KB, (k=8, m=4), exactly 4 erasures per block."""
    full_size_case(mj, 128, 8, 12, 1 << 19, 4, synth.SEED_DATA + 2)
