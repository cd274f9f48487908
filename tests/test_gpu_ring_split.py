"""Whole-block decode with two ring classes: in a batch large enough to keep
the chip busy, blocks whose survivor set reads deep (far behind the newest
pixel) and shallow blocks go to different launches.  Batches made only of
deep sets, only of shallow sets, and both mixed at random, against the
oracle."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests.gpuutil import (POISON_WORD, mask_depth, masks_to_dev, poison_erased_dev, say,
                           survivor_depth, to_np)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def masks_by_depth(dirs, Q):
    n = len(dirs)
    out = []
    for keep in itertools.combinations(range(n), Q):
        used = sorted(dirs[i] for i in keep)
        mask = sum(1 << i for i in range(n) if i not in keep)
        out.append((survivor_depth(used), mask))
    return sorted(out)


def run(mj, P, Q, dirs, masks):
    """Round trip of every block on the device from pools whose erased
    projections are overwritten, the oracle on a sample that holds the first,
    middle and last blocks and the deepest blocks of the batch (those of the
    gathered long-ring launch when the library splits it).  The batches are
    large enough for the library to split them."""
    nb = len(masks)
    sizes = [oracle.proj_size(p, 1, P, Q) for p in dirs]
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), 900 + nb)
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    depths = {int(m): mask_depth(int(m), dirs, Q) for m in np.unique(masks)}
    dmax = max(depths.values())
    deepest = np.flatnonzero([depths[int(m)] == dmax for m in masks])
    pick = np.unique(np.concatenate([[0, 1, nb // 2, nb - 1], deepest[:3], deepest[-3:]]))
    idx = torch.from_numpy(pick).cuda()
    torch.cuda.synchronize()
    enc = to_np(d_proj.view(nb, words)[idx])          # before the erased bins are overwritten
    poison_erased_dev(d_proj, masks, sizes)
    d_out = torch.full((nb * Q * P,), -1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch(d_proj, masks_to_dev(masks), nb, P, Q, dirs, d_out, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(d_out, d_img)
    src = to_np(d_proj.view(nb, words)[idx])
    off = np.cumsum([0] + sizes)
    for k, b in enumerate(pick):                     # the device pool really is poisoned
        for i in range(len(dirs)):
            if (int(masks[b]) >> i) & 1:
                assert (src[k, off[i]:off[i + 1]] == np.uint64(POISON_WORD)).all()
    want = oracle.decode_blocks(src, masks[pick], P, Q, dirs)
    assert np.array_equal(want, oracle.decode_blocks(enc, masks[pick], P, Q, dirs))
    assert np.array_equal(to_np(d_out.view(nb, -1)[idx]).reshape(len(pick), Q, P), want)


@pytest.mark.parametrize("n,Q,P,nb", [(12, 8, 128, 12000), (8, 4, 96, 40000),
                                      (16, 12, 40, 12000)])   # the last: one ring for every set
def test_deep_shallow_and_mixed_batches(mj, n, Q, P, nb):
    dirs = synth.centered_dirs(n)
    by_depth = masks_by_depth(dirs, Q)
    deep = np.resize(np.array([m for _, m in by_depth[-5:]], dtype=np.uint16), nb)
    shallow = np.resize(np.array([m for _, m in by_depth[:5]], dtype=np.uint16), nb)
    say(f"ring split n={n} Q={Q} P={P}: depths {by_depth[0][0]}..{by_depth[-1][0]}")
    run(mj, P, Q, dirs, deep)
    run(mj, P, Q, dirs, shallow)
    rng = np.random.default_rng(n)
    mixed = np.array([by_depth[i][1] for i in rng.integers(0, len(by_depth), nb)],
                     dtype=np.uint16)
    run(mj, P, Q, dirs, mixed)


def test_scattered_deep_blocks_at_range_edges(mj):
    """The deep class is gathered from ranges of consecutive blocks: deep
    blocks at the first and last positions of ranges, a dense cluster inside
    one range, and the ragged last range, in a shallow batch."""
    n, Q, P, nb = 12, 8, 128, 20000
    dirs = synth.centered_dirs(n)
    by_depth = masks_by_depth(dirs, Q)
    shallow = [m for _, m in by_depth[:20]]
    deep = [m for _, m in by_depth[-13:]]
    masks = np.array([shallow[i % len(shallow)] for i in range(nb)], dtype=np.uint16)
    at = [0, 1, 63, 64, 65, 127, 255, 256, 257, 511, 512, 767] + list(range(5000, 5030)) + \
         [nb - 257, nb - 256, nb - 2, nb - 1]
    for k, i in enumerate(at):
        masks[i] = deep[k % len(deep)]
    say(f"deep blocks at {len(at)} positions of {nb}")
    run(mj, P, Q, dirs, masks)
