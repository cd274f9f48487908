"""Descriptor-driven batched calls over codes with layout options: 128-bit
pixels (MOJETTE_GEOM_WIDE, Section 3.1) and never-used bins left out
(MOJETTE_GEOM_TRIMMED, Section 2.3), interleaved with plain codes in one
plan and one call, blocks at scattered places of one pool.  Encode against
the oracle's wide and kept-bin transforms bit for bit; decode from pools
with the images cleared and the erased projections overwritten, against the
original images (XOR arithmetic is exact: tolerance zero)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import POISON_WORD, say, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def code_table(mj):
    return [
        (4, synth.centered_dirs(6), 0),
        (4, synth.centered_dirs(6), mj.GEOM_WIDE),
        (4, synth.centered_dirs(6), mj.GEOM_TRIMMED),
        (8, synth.centered_dirs(12), mj.GEOM_WIDE),
        (8, synth.centered_dirs(12), mj.GEOM_TRIMMED),
        (2, [5, -1, 3], mj.GEOM_WIDE),
        (3, [2, -1, 0, 5], mj.GEOM_TRIMMED),
        (6, synth.centered_dirs(9), 0),
    ]


def stored(mj, code, P):
    """Words of a block's image and projections, and the oracle's encode of
    an image (image words in memory order -> projection words)."""
    Q, dirs, flags = code
    if flags == mj.GEOM_WIDE:
        img_words = 2 * Q * P
        proj_words = 2 * sum(oracle.proj_size(p, 1, P, Q) for p in dirs)

        def enc(img):
            return oracle.encode_blocks_wide(img.reshape(1, Q, P, 2), P, Q, dirs).ravel()
    elif flags == mj.GEOM_TRIMMED:
        img_words = Q * P
        proj_words = sum(c for _, c in oracle.kept_bins(dirs, P, Q))

        def enc(img):
            return oracle.encode_blocks_kept(img.reshape(1, Q, P), P, Q, dirs).ravel()
    else:
        img_words = Q * P
        proj_words = sum(oracle.proj_size(p, 1, P, Q) for p in dirs)

        def enc(img):
            return oracle.encode_blocks(img.reshape(1, Q, P), P, Q, dirs).ravel()
    return img_words, proj_words, enc


def proj_spans(mj, code, P):
    """(first word, words) of each projection within a block's slice."""
    Q, dirs, flags = code
    if flags == mj.GEOM_TRIMMED:
        sizes = [c for _, c in oracle.kept_bins(dirs, P, Q)]
    else:
        w = 2 if flags == mj.GEOM_WIDE else 1
        sizes = [w * oracle.proj_size(p, 1, P, Q) for p in dirs]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    return [(int(offs[i]), int(sizes[i])) for i in range(len(dirs))]


def round_trip(mj, codes, geom, Ps, masks, seed, tune=None):
    rng = np.random.default_rng(seed)
    nb = len(Ps)
    info = [stored(mj, codes[g], int(P)) for g, P in zip(geom, Ps)]
    pieces = rng.permutation(2 * nb)
    img_off = np.zeros(nb, dtype=np.uint64)
    proj_off = np.zeros(nb, dtype=np.uint64)
    at = 3
    for o in pieces:
        b, k = divmod(int(o), 2)
        if k == 0:
            img_off[b] = at
            at += info[b][0]
        else:
            proj_off[b] = at
            at += info[b][1]
        at += int(rng.integers(0, 4))
    words = at + 5
    pool = np.full(words, np.uint64(POISON_WORD), dtype=np.uint64)
    imgs = []
    for b in range(nb):
        img = synth.splitmix64(seed * 7919 + b, 0, info[b][0])
        pool[int(img_off[b]):int(img_off[b]) + img.size] = img
        imgs.append(img)
    plan = mj.GeomPlan(codes, tune)
    d_pool = to_dev(pool)
    d_blocks = mj.make_blocks(img_off, proj_off, Ps, geom, masks)
    ws = plan.workspace(nb)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_encode_batched(plan, d_blocks, nb, d_pool, ws, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    enc = to_np(d_pool)
    for b in range(nb):
        want = info[b][2](imgs[b])
        o = int(proj_off[b])
        assert np.array_equal(enc[o:o + want.size], want), f"encode block {b} (code {geom[b]})"
    src = enc.copy()
    for b in range(nb):
        src[int(img_off[b]):int(img_off[b]) + info[b][0]] = np.uint64(POISON_WORD)
        for i, (o, n) in enumerate(proj_spans(mj, codes[geom[b]], int(Ps[b]))):
            if (int(masks[b]) >> i) & 1:
                src[int(proj_off[b]) + o:int(proj_off[b]) + o + n] = np.uint64(POISON_WORD)
    d_src = to_dev(src)
    st.zero_()
    mj.mojette_decode_batched(plan, d_blocks, nb, d_src, ws, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    dec = to_np(d_src)
    for b in range(nb):
        o = int(img_off[b])
        assert np.array_equal(dec[o:o + info[b][0]], imgs[b]), f"decode block {b} (code {geom[b]})"
    # outside the images the decode wrote nothing
    inside = np.zeros(words, dtype=bool)
    for b in range(nb):
        inside[int(img_off[b]):int(img_off[b]) + info[b][0]] = True
    assert np.array_equal(dec[~inside], src[~inside])
    plan.close()


def row_lengths(mj, codes, geom, choices, rng):
    """Row lengths drawn from `choices`; a trimmed code's rows are at least
    its largest |p|, where the bins its rows read form one contiguous run
    per projection (the oracle's kept-bin layout is defined there)."""
    Ps = rng.choice(choices, len(geom))
    for b, g in enumerate(geom):
        Q, dirs, flags = codes[g]
        if flags == mj.GEOM_TRIMMED:
            Ps[b] = max(int(Ps[b]), max(abs(p) for p in dirs))
    return Ps


def masks_for(codes, geom, seed):
    out = np.zeros(len(geom), dtype=np.uint16)
    for b, g in enumerate(geom):
        Q, dirs, _ = codes[g]
        out[b] = synth.erasure_masks(seed + b, 1, len(dirs), (0, len(dirs) - Q))[0]
    return out


@pytest.mark.parametrize("seed", [1, 2])
def test_wide_and_trimmed_codes_beside_plain_ones(mj, seed):
    codes = code_table(mj)
    rng = np.random.default_rng(seed)
    nb = 600
    geom = rng.integers(0, len(codes), nb)
    Ps = row_lengths(mj, codes, geom, [1, 2, 15, 16, 17, 64, 100, 128, 171, 300], rng)
    masks = masks_for(codes, geom, 1000 * seed)
    say(f"layout codes: {nb} blocks, {len(codes)} codes (wide, trimmed, plain), seed {seed}")
    round_trip(mj, codes, geom, Ps, masks, seed)


def test_wide_code_decoded_from_both_ends(mj):
    """128-bit pixels with the two-corner decode: the mirrored sweep reads the
    stored bins backwards, each 16-byte bin still in its half order."""
    codes = code_table(mj)
    tune = [{} for _ in codes]
    tune[1] = {"decode_two_corner_min_P": 64}
    tune[3] = {"decode_two_corner_min_P": 64}
    rng = np.random.default_rng(5)
    nb = 300
    geom = rng.choice([0, 1, 3, 5], nb)
    Ps = rng.choice([16, 63, 64, 65, 200, 513], nb)
    masks = masks_for(codes, geom, 77)
    say(f"layout codes, wide from both ends: {nb} blocks")
    round_trip(mj, codes, geom, Ps, masks, 9, tune)


def test_wide_matches_the_batch_call(mj):
    """The wide code through the descriptor call stores the same words as
    mojette_encode_batch_wide."""
    Q, dirs = 4, synth.centered_dirs(6)
    P, nb = 64, 200
    imgs = np.random.default_rng(4).integers(0, 2**64, size=(nb, Q, P, 2), dtype=np.uint64)
    d_img = to_dev(imgs.ravel())
    words = 2 * sum(oracle.proj_size(p, 1, P, Q) for p in dirs)
    d_batch = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch_wide(d_img, nb, P, Q, dirs, d_batch)
    # descriptor call: images and projections in one pool, blocks back to back
    pool = np.zeros(nb * (2 * Q * P + words), dtype=np.uint64)
    pool[:nb * 2 * Q * P] = imgs.ravel()
    img_off = np.arange(nb, dtype=np.uint64) * (2 * Q * P)
    proj_off = nb * 2 * Q * P + np.arange(nb, dtype=np.uint64) * words
    plan = mj.GeomPlan([(Q, dirs, mj.GEOM_WIDE)])
    d_pool = to_dev(pool)
    d_blocks = mj.make_blocks(img_off, proj_off, np.full(nb, P), np.zeros(nb, dtype=int),
                              np.zeros(nb, dtype=np.uint16))
    ws = plan.workspace(nb)
    mj.mojette_encode_batched(plan, d_blocks, nb, d_pool, ws)
    torch.cuda.synchronize()
    got = to_np(d_pool)[nb * 2 * Q * P:]
    assert np.array_equal(got, to_np(d_batch))
    plan.close()


def test_encode_row_windows_of_tall_codes(mj):
    """Codes of 9 to 12 rows encode from LDS row windows (each row holds the
    columns its bins cross): one-signed directions (the window's left or
    right end at the tile's own column), a trimmed 12-row code, tiles at
    the row's ends and in its middle; then codes whose windows exceed the
    register prefetch (the 128-bit 12-row code, an 11-row code with |p| up
    to 20), which keep the tile-and-halo layout.  Against the oracle."""
    rw = [
        (12, synth.centered_dirs(16), 0),
        (12, synth.centered_dirs(16), mj.GEOM_TRIMMED),
        (9, list(range(1, 11)), 0),
        (10, list(range(-12, 0)), 0),
        (4, synth.centered_dirs(6), 0),
    ]
    wide = [
        (12, synth.centered_dirs(16), mj.GEOM_WIDE),
        (11, [-3, 0, 1, 2, 4, 7, 9, 13, 20, -8, 5, 6], 0),
    ]
    for k, codes in enumerate((rw, wide)):
        rng = np.random.default_rng(20 + k)
        nb = 400
        geom = rng.integers(0, len(codes), nb)
        Ps = row_lengths(mj, codes, geom, [1, 2, 15, 16, 17, 64, 100, 128, 171, 300, 700], rng)
        masks = masks_for(codes, geom, 3000 + 100 * k)
        say(f"row windows: {nb} blocks, codes set {k}")
        round_trip(mj, codes, geom, Ps, masks, 40 + k)
