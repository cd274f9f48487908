"""GPU consistency check of decoded blocks (Section 2.2: projections that no
image has leave a bin with a nonzero residue), against the oracle's own
check."""
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


def decode_and_verify(mj, pool, masks, P, Q, dirs):
    nb = masks.shape[0]
    d_pool = to_dev(pool)
    d_out = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch(d_pool, masks_to_dev(masks), nb, P, Q, dirs, d_out, st)
    vst = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_verify_batch(d_pool, masks_to_dev(masks), nb, P, Q, dirs, d_out, vst)
    torch.cuda.synchronize()
    return int(st.item()), int(vst.item()), to_np(d_out).reshape(nb, Q, P)


@pytest.mark.parametrize("P,Q,n,ner", [(128, 4, 6, 2), (128, 8, 12, 4), (37, 3, 5, (0, 2))])
def test_clean_projections_verify(mj, P, Q, n, ner):
    dirs = synth.centered_dirs(n)
    nb = 40
    imgs = synth.block_images(700 + n, 0, nb, P, Q)
    pool = oracle.encode_blocks(imgs, P, Q, dirs)
    masks = synth.erasure_masks(12, nb, n, ner)
    st, vst, out = decode_and_verify(mj, pool, masks, P, Q, dirs)
    assert st == 0 and vst == 0 and np.array_equal(out, imgs)


def test_one_corrupted_bin_is_caught_and_erased_ones_are_not_checked(mj):
    P, Q, n = 64, 4, 6
    dirs = synth.centered_dirs(n)
    imgs = synth.block_images(31, 0, 3, P, Q)
    pool = oracle.encode_blocks(imgs, P, Q, dirs)
    masks = np.array([0b000011, 0b000011, 0b000011], dtype=np.uint16)
    off = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
    bad = pool.copy()
    bad[1, off[4] + 7] ^= np.uint64(1 << 40)     # a surviving projection of block 1
    bad[2, off[0] + 3] ^= np.uint64(5)           # an erased projection of block 2
    for b, want in ((0, 0), (1, -5), (2, 0)):
        st, vst, _ = decode_and_verify(mj, bad[b:b + 1], masks[b:b + 1], P, Q, dirs)
        assert st == 0 and vst == want, (b, vst)
    # the oracle's peeling with its consistency check agrees on block 1
    keep = [i for i in range(n) if not (masks[1] >> i) & 1]
    projs = [bad[1, off[i]:off[i + 1]] for i in keep]
    rc, _ = oracle.inverse(projs, [(dirs[i], 1) for i in keep], P, Q, verify=True)
    assert rc == oracle.EINCONSISTENT


def test_verify_full_size_4k(mj):
    """2^21 4 KB blocks decoded and verified clean; one corrupted bin in one
    block somewhere in the pool is caught."""
    P, Q, n, nb = 128, 4, 6, 1 << 21
    dirs = synth.centered_dirs(n)
    words = mj.mojette_block_words(dirs, P, Q)
    say("verify full size")
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), 3)
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    masks = synth.erasure_masks(synth.SEED_ERASE, nb, n, 2)
    d_mask = masks_to_dev(masks)
    d_out = torch.empty_like(d_img)
    mj.mojette_decode_batch(d_proj, d_mask, nb, P, Q, dirs, d_out)
    vst = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_verify_batch(d_proj, d_mask, nb, P, Q, dirs, d_out, vst)
    torch.cuda.synchronize()
    assert int(vst.item()) == 0
    blk = 1_234_567
    surv = [i for i in range(n) if not (int(masks[blk]) >> i) & 1]
    off = int(sum(mj.mojette_proj_size(p, P, Q) for p in dirs[:surv[-1]]))
    d_proj[blk * words + off + 5] ^= 1
    mj.mojette_verify_batch(d_proj, d_mask, nb, P, Q, dirs, d_out, vst)
    torch.cuda.synchronize()
    assert int(vst.item()) == -5
    del d_img, d_proj, d_out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("P,Q,n", [(128, 4, 6), (60, 8, 12), (9, 2, 3)])
def test_single_block_decode_with_verify_flag(mj, P, Q, n):
    """mojette_decode with MOJETTE_VERIFY: clean projections give OK and the
    image; one corrupted bit in any bin of any given projection gives
    MOJETTE_EINCONSISTENT exactly when the oracle's peeling check (verify)
    flags the same inputs."""
    dirs = synth.centered_dirs(n)
    img = synth.block_images(P + Q, 0, 1, P, Q)[0]
    projs = oracle.forward(img, [(p, 1) for p in dirs])
    rng = np.random.default_rng(P)
    for m in (Q, n):
        ids = sorted(int(i) for i in rng.permutation(n)[:m])
        d_projs = [to_dev(projs[i]) for i in ids]
        out = torch.zeros(Q * P, dtype=torch.int64, device="cuda")
        assert mj.mojette_decode(d_projs, ids, dirs, P, Q, out, verify=True) == 0
        assert np.array_equal(to_np(out).reshape(Q, P), img)
        for trial in range(6):
            t = int(rng.integers(0, m))
            j = int(rng.integers(0, projs[ids[t]].size))
            bad = [p.copy() for p in projs]
            bad[ids[t]][j] ^= np.uint64(1) << np.uint64(int(rng.integers(0, 64)))
            # the oracle's check on the same survivors (erased ones left out)
            st_orc, _ = oracle.inverse([bad[i] for i in ids], [(dirs[i], 1) for i in ids], P, Q,
                                       verify=True)
            d_bad = [to_dev(bad[i]) for i in ids]
            rc = mj.mojette_decode(d_bad, ids, dirs, P, Q, out, verify=True, check=False)
            say(f"verify m={m} proj {ids[t]} bin {j}: library {rc}, oracle {st_orc}")
            assert rc == (mj.MOJETTE_EINCONSISTENT if st_orc == oracle.EINCONSISTENT else 0)
