"""Descriptor-driven batched calls (mojette_plan_create, mojette_encode_batched,
mojette_decode_batched): blocks of many codes and row lengths interleaved in
one call, images and projections at scattered places of one pool, against
the oracle bit for bit; erased projections overwritten; short- and
full-ring classes; more classes than the 16 of the class calls; per-block
errors; graph replays."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import POISON_WORD, mask_depth, say, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


CODES = [
    (4, synth.centered_dirs(6)),
    (8, synth.centered_dirs(12)),
    (6, synth.centered_dirs(9)),
    (12, synth.centered_dirs(16)),
    (2, [5, -1, 3]),
    (1, [0]),
    (3, [2, -1, 0, 5]),
]


class Layout:
    """Blocks of given (geom, P) at shuffled places of one word pool."""

    def __init__(self, codes, geom, Ps, masks, seed, gap=3):
        rng = np.random.default_rng(seed)
        self.codes, self.geom, self.P, self.masks = codes, geom, Ps, masks
        nb = len(Ps)
        sizes = []
        for g, P in zip(geom, Ps):
            Q, dirs = codes[g]
            sizes.append((Q * P, sum(oracle.proj_size(p, 1, P, Q) for p in dirs)))
        # pieces (block, kind) in a random order, a few words apart
        pieces = [(b, k) for b in range(nb) for k in (0, 1)]
        order = rng.permutation(len(pieces))
        self.img_off = np.zeros(nb, dtype=np.uint64)
        self.proj_off = np.zeros(nb, dtype=np.uint64)
        at = 5
        for o in order:
            b, k = pieces[o]
            if k == 0:
                self.img_off[b] = at
            else:
                self.proj_off[b] = at
            at += sizes[b][k] + int(rng.integers(0, gap + 1))
        self.words = at + 7
        self.sizes = sizes

    def descriptors(self, mj):
        return mj.make_blocks(self.img_off, self.proj_off, self.P, self.geom, self.masks)


def fill_images(lay, seed):
    """A pool with every block's image (seeded words), projections poisoned."""
    pool = np.full(lay.words, np.uint64(POISON_WORD), dtype=np.uint64)
    imgs = []
    for b in range(len(lay.P)):
        Q, _ = lay.codes[lay.geom[b]]
        img = synth.block_images(seed + b, 0, 1, int(lay.P[b]), Q)[0]
        pool[int(lay.img_off[b]):int(lay.img_off[b]) + img.size] = img.ravel()
        imgs.append(img)
    return pool, imgs


def run_round_trip(mj, codes, geom, Ps, masks, seed, tune=None, poison=True):
    plan = mj.GeomPlan(codes, tune)
    lay = Layout(codes, geom, Ps, masks, seed)
    pool, imgs = fill_images(lay, seed)
    nb = len(Ps)
    d_pool = to_dev(pool)
    d_blocks = lay.descriptors(mj)
    ws = plan.workspace(nb)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batched(plan, d_blocks, nb, d_pool, ws, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    enc = to_np(d_pool)
    # encode: every block's projections equal the oracle's
    for b in range(nb):
        Q, dirs = codes[geom[b]]
        want = oracle.encode_blocks(imgs[b][None], int(Ps[b]), Q, dirs)[0]
        o = int(lay.proj_off[b])
        assert np.array_equal(enc[o:o + want.size], want), f"encode block {b}"
    # decode from pools with the images cleared and erased projections poisoned
    src = enc.copy()
    for b in range(nb):
        Q, dirs = codes[geom[b]]
        o = int(lay.img_off[b])
        src[o:o + imgs[b].size] = np.uint64(POISON_WORD)
        if poison:
            off = int(lay.proj_off[b])
            for i, p in enumerate(dirs):
                s = oracle.proj_size(p, 1, int(Ps[b]), Q)
                if (int(masks[b]) >> i) & 1:
                    src[off:off + s] = np.uint64(POISON_WORD)
                off += s
    d_src = to_dev(src)
    st.zero_()
    mj.mojette_decode_batched(plan, d_blocks, nb, d_src, ws, st)
    torch.cuda.synchronize()
    dec = to_np(d_src)
    plan.close()
    return lay, imgs, src, dec, int(st.item())


def test_interleaved_codes_and_row_lengths(mj):
    rng = np.random.default_rng(3)
    nb = 900
    geom = rng.integers(0, len(CODES), nb)
    Ps = rng.choice([1, 3, 16, 17, 64, 100, 128, 129, 171, 256, 300, 1366], nb)
    masks = np.zeros(nb, dtype=np.uint16)
    for b in range(nb):
        Q, dirs = CODES[geom[b]]
        masks[b] = synth.erasure_masks(10 + b, 1, len(dirs), (0, len(dirs) - Q))[0]
    say(f"descriptor calls: {nb} blocks, {len(CODES)} codes, "
        f"{len(set(zip(geom.tolist(), Ps.tolist())))} (code, P) classes")
    lay, imgs, src, dec, st = run_round_trip(mj, CODES, geom, Ps, masks, 100)
    assert st == 0
    for b in range(nb):
        o = int(lay.img_off[b])
        assert np.array_equal(dec[o:o + imgs[b].size], imgs[b].ravel()), f"decode block {b}"
    # nothing outside the images was written by the decode
    inside = np.zeros(lay.words, dtype=bool)
    for b in range(nb):
        o = int(lay.img_off[b])
        inside[o:o + imgs[b].size] = True
    assert np.array_equal(dec[~inside], src[~inside])
    # the oracle decodes the same poisoned projections to the same images
    for b in rng.choice(nb, 40, replace=False):
        Q, dirs = CODES[geom[b]]
        o = int(lay.proj_off[b])
        words = sum(oracle.proj_size(p, 1, int(Ps[b]), Q) for p in dirs)
        want = oracle.decode_blocks(src[o:o + words][None], masks[b:b + 1], int(Ps[b]), Q, dirs)
        oi = int(lay.img_off[b])
        assert np.array_equal(dec[oi:oi + imgs[b].size].reshape(want[0].shape), want[0])


def test_more_classes_than_the_class_calls_take(mj):
    """300 distinct row lengths of two codes: 600 classes in one call."""
    nb = 1200
    rng = np.random.default_rng(5)
    codes = CODES[:2]
    geom = rng.integers(0, 2, nb)
    Ps = 20 + rng.permutation(np.repeat(np.arange(300), 4))
    masks = np.array([synth.erasure_masks(b, 1, len(codes[g][1]), len(codes[g][1]) - codes[g][0])[0]
                      for b, g in enumerate(geom)], dtype=np.uint16)
    lay, imgs, src, dec, st = run_round_trip(mj, codes, geom, Ps, masks, 200)
    assert st == 0
    for b in range(nb):
        o = int(lay.img_off[b])
        assert np.array_equal(dec[o:o + imgs[b].size], imgs[b].ravel()), b


@pytest.mark.parametrize("split", [0, -1, 1])
def test_ring_classes_of_the_tall_code(mj, split):
    """(12,8) blocks with deep and shallow survivor sets: with the split they
    decode in a short- and a full-ring class, without it in one; the same
    images either way."""
    Q, dirs = CODES[1]
    nb = 700
    rng = np.random.default_rng(7)
    masks = synth.erasure_masks(70, nb, len(dirs), 4)
    depths = np.array([mask_depth(int(m), dirs, Q) for m in masks])
    assert depths.max() > depths.min()
    geom = np.zeros(nb, dtype=np.int64)
    Ps = rng.choice([128, 200], nb)
    lay, imgs, src, dec, st = run_round_trip(mj, [CODES[1]], geom, Ps, masks, 300,
                                             tune=[{"decode_ring_split": split}])
    assert st == 0
    for b in range(nb):
        o = int(lay.img_off[b])
        assert np.array_equal(dec[o:o + imgs[b].size], imgs[b].ravel()), (b, depths[b])


def test_per_block_errors(mj):
    """Blocks with fewer than Q survivors and descriptors with a bad code or
    row length are reported through status and left alone; the others are
    decoded."""
    nb = 60
    geom = np.array([b % 2 for b in range(nb)])
    Ps = np.full(nb, 64)
    masks = np.zeros(nb, dtype=np.uint16)
    lost = [3, 10, 33]
    for b in lost:
        masks[b] = 0b111 if geom[b] == 0 else 0b11111   # more than m lost
    lay, imgs, src, dec, st = run_round_trip(mj, CODES[:2], geom, Ps, masks, 400)
    assert st == mj.MOJETTE_ENOTRECON
    for b in range(nb):
        o = int(lay.img_off[b])
        got = dec[o:o + imgs[b].size]
        if b in lost:
            assert (got == np.uint64(POISON_WORD)).all()
        else:
            assert np.array_equal(got, imgs[b].ravel()), b
    # a bad code id and a zero row length: EINVAL, skipped
    plan = mj.GeomPlan(CODES[:2])
    lay2 = Layout(CODES[:2], [0, 1, 0], [64, 64, 64], np.zeros(3, dtype=np.uint16), 9)
    d = np.frombuffer(lay2.descriptors(mj).cpu().numpy().tobytes(), dtype=mj.block_dtype()).copy()
    d["geom_id"][1] = 7
    d["P"][2] = 0
    d_blocks = torch.from_numpy(d.view(np.uint8).copy()).cuda()
    pool, imgs2 = fill_images(lay2, 9)
    d_pool = to_dev(pool)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batched(plan, d_blocks, 3, d_pool, plan.workspace(3), st)
    torch.cuda.synchronize()
    assert int(st.item()) == mj.MOJETTE_EINVAL
    got = to_np(d_pool)
    want = oracle.encode_blocks(imgs2[0][None], 64, *CODES[0])[0]
    o = int(lay2.proj_off[0])
    assert np.array_equal(got[o:o + want.size], want)
    o = int(lay2.proj_off[1])
    assert (got[o:o + lay2.sizes[1][1]] == np.uint64(POISON_WORD)).all()
    plan.close()


def test_empty_call_and_argument_errors(mj):
    plan = mj.GeomPlan(CODES[:1])
    ws = plan.workspace(0)
    dummy = torch.zeros(3, dtype=torch.uint8, device="cuda")
    pool = torch.zeros(8, dtype=torch.int64, device="cuda")
    assert mj.mojette_encode_batched(plan, dummy, 0, pool, ws) == 0
    assert mj.mojette_decode_batched(plan, dummy, 0, pool, ws) == 0
    L = mj.lib()
    assert L.mojette_decode_batched(plan.handle, dummy.data_ptr(), -1, pool.data_ptr(),
                                    ws.data_ptr(), None, None) == mj.MOJETTE_EINVAL
    assert L.mojette_decode_batched(plan.handle, dummy.data_ptr(), 1, pool.data_ptr(),
                                    ws.data_ptr() + 8, None, None) == mj.MOJETTE_EINVAL
    plan.close()


def test_same_words_as_the_single_geometry_batch(mj):
    """4 KB (6,4) blocks through the descriptor calls and through
    mojette_encode_batch / mojette_decode_batch: identical words."""
    P, Q, dirs, nb = 128, 4, synth.centered_dirs(6), 5000
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), 77)
    masks = synth.erasure_masks(78, nb, 6, 2)
    from tests.gpuutil import masks_to_dev
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    out = torch.empty_like(d_img)
    mj.mojette_decode_batch(d_proj, masks_to_dev(masks), nb, P, Q, dirs, out)
    # the same blocks in one pool: images first, projections after
    plan = mj.GeomPlan([(Q, dirs)])
    pool = torch.empty(nb * Q * P + nb * words, dtype=torch.int64, device="cuda")
    pool[:nb * Q * P] = d_img
    img_off = np.arange(nb, dtype=np.uint64) * (Q * P)
    proj_off = nb * Q * P + np.arange(nb, dtype=np.uint64) * words
    blocks = mj.make_blocks(img_off, proj_off, np.full(nb, P), np.zeros(nb), masks)
    ws = plan.workspace(nb)
    mj.mojette_encode_batched(plan, blocks, nb, pool, ws)
    torch.cuda.synchronize()
    assert torch.equal(pool[nb * Q * P:], d_proj)
    pool[:nb * Q * P] = -1
    mj.mojette_decode_batched(plan, blocks, nb, pool, ws)
    torch.cuda.synchronize()
    assert torch.equal(pool[:nb * Q * P], out)
    assert torch.equal(out, d_img)
    plan.close()


def test_graph_replay(mj):
    """Encode + decode of interleaved codes recorded into a HIP graph: every
    replay, on images changed eagerly in between, matches the eager result."""
    rng = np.random.default_rng(11)
    nb = 400
    codes = CODES[:4]
    geom = rng.integers(0, 4, nb)
    Ps = rng.choice([64, 128, 300], nb)
    masks = np.array([synth.erasure_masks(b, 1, len(codes[g][1]), (0, len(codes[g][1]) - codes[g][0]))[0]
                      for b, g in enumerate(geom)], dtype=np.uint16)
    plan = mj.GeomPlan(codes)
    lay = Layout(codes, geom, Ps, masks, 12)
    pool_np, _ = fill_images(lay, 12)
    d_pool = to_dev(pool_np)
    img_mask = np.zeros(lay.words, dtype=bool)
    for b in range(nb):
        o = int(lay.img_off[b])
        img_mask[o:o + lay.sizes[b][0]] = True
    d_imgmask = torch.from_numpy(img_mask).cuda()
    blocks = lay.descriptors(mj)
    ws = plan.workspace(nb)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        mj.mojette_encode_batched(plan, blocks, nb, d_pool, ws, stream=s.cuda_stream)
        mj.mojette_decode_batched(plan, blocks, nb, d_pool, ws, stream=s.cuda_stream)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        mj.mojette_encode_batched(plan, blocks, nb, d_pool, ws, stream=s.cuda_stream)
        mj.mojette_decode_batched(plan, blocks, nb, d_pool, ws, stream=s.cuda_stream)
    for rep in range(4):
        fresh = torch.empty(lay.words, dtype=torch.int64, device="cuda")
        mj.mojette_fill_splitmix64(fresh, lay.words, 500 + rep)
        d_pool[d_imgmask] = fresh[d_imgmask]
        want_img = d_pool.clone()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = d_pool.clone()
        assert torch.equal(got[d_imgmask], want_img[d_imgmask])   # decode gave the images back
        d_pool.copy_(want_img)
        mj.mojette_encode_batched(plan, blocks, nb, d_pool, ws)
        mj.mojette_decode_batched(plan, blocks, nb, d_pool, ws)
        torch.cuda.synchronize()
        assert torch.equal(got, d_pool)
    plan.close()


def test_mixed_workload_recipe_sample(mj):
    """The mixed workload's recipe (sizes 4K/8K/64K/1M, codes (4,2), (6,3),
    (8,4), (12,4), erasures 0..m per block), a few thousand blocks in block
    order through the descriptor calls with erased projections poisoned,
    padded last rows included: round trip of every block, and encode and
    decode against the oracle on a sample that holds every class present."""
    N = 3000
    size_idx, code_idx, masks = synth.mixed_block_list(N, synth.SEED_DATA)
    codes = [(k, synth.centered_dirs(k + m)) for k, m in synth.MIXED_CODES]
    sizes = np.array(synth.MIXED_SIZES)[size_idx]
    # keep the 1 MB blocks few: every fourth of them
    keep = np.flatnonzero((sizes < (1 << 20)) | (np.arange(N) % 4 == 0))
    size_idx, code_idx, masks, sizes = size_idx[keep], code_idx[keep], masks[keep], sizes[keep]
    Ps = np.array([-(-int(s) // (8 * codes[g][0])) for s, g in zip(sizes, code_idx)])
    say(f"mixed recipe sample: {len(keep)} blocks, {int(sizes.sum()) >> 20} MiB")
    lay, imgs, src, dec, st = run_round_trip(mj, codes, code_idx, Ps, masks, 600)
    assert st == 0
    for b in range(len(keep)):
        o = int(lay.img_off[b])
        assert np.array_equal(dec[o:o + imgs[b].size], imgs[b].ravel()), b
    # oracle on one block of every (size, code) class present
    for key in sorted(set(zip(size_idx.tolist(), code_idx.tolist()))):
        b = int(np.flatnonzero((size_idx == key[0]) & (code_idx == key[1]))[0])
        Q, dirs = codes[code_idx[b]]
        P = int(Ps[b])
        words = sum(oracle.proj_size(p, 1, P, Q) for p in dirs)
        o = int(lay.proj_off[b])
        want_enc = oracle.encode_blocks(imgs[b][None], P, Q, dirs)[0]
        got_src = src[o:o + words]
        keep_bins = np.ones(words, dtype=bool)
        off = 0
        for i, p in enumerate(dirs):
            s = oracle.proj_size(p, 1, P, Q)
            if (int(masks[b]) >> i) & 1:
                keep_bins[off:off + s] = False
            off += s
        assert np.array_equal(got_src[keep_bins], want_enc[keep_bins]), key
        want = oracle.decode_blocks(got_src[None], masks[b:b + 1], P, Q, dirs)[0]
        oi = int(lay.img_off[b])
        assert np.array_equal(dec[oi:oi + imgs[b].size].reshape(Q, P), want), key


@pytest.mark.parametrize("min_p", [1, 100, 1000])
def test_two_corner_classes(mj, min_p):
    """Codes whose rows of at least min_p columns decode from both ends
    (mojette_tune.decode_two_corner_min_P): interleaved codes and row lengths,
    poisoned erasures, against the oracle."""
    rng = np.random.default_rng(min_p)
    nb = 700
    geom = rng.integers(0, len(CODES), nb)
    Ps = rng.choice([1, 3, 17, 99, 100, 128, 300, 999, 1000, 1366, 2048], nb)
    masks = np.zeros(nb, dtype=np.uint16)
    for b in range(nb):
        Q, dirs = CODES[geom[b]]
        masks[b] = synth.erasure_masks(20 + b, 1, len(dirs), (0, len(dirs) - Q))[0]
    tune = [{"decode_two_corner_min_P": min_p} for _ in CODES]
    lay, imgs, src, dec, st = run_round_trip(mj, CODES, geom, Ps, masks, 700 + min_p, tune=tune)
    assert st == 0
    for b in range(nb):
        o = int(lay.img_off[b])
        assert np.array_equal(dec[o:o + imgs[b].size], imgs[b].ravel()), (b, int(Ps[b]))
    for b in rng.choice(nb, 30, replace=False):
        Q, dirs = CODES[geom[b]]
        o = int(lay.proj_off[b])
        words = sum(oracle.proj_size(p, 1, int(Ps[b]), Q) for p in dirs)
        want = oracle.decode_blocks(src[o:o + words][None], masks[b:b + 1], int(Ps[b]), Q, dirs)
        oi = int(lay.img_off[b])
        assert np.array_equal(dec[oi:oi + imgs[b].size].reshape(want[0].shape), want[0])
