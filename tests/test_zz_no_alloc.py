"""Allocation-free chunked decode (mojette_decode_batch_chunked_noalloc):
the same words as mojette_decode_batch_chunked with a caller workspace, on
calls in a row through the library's fixed scratch memory (a larger call,
then smaller ones, so the second starts on the scratch contents the first
left), and its limit."""
import numpy as np
import pytest

import synth
from tests.gpuutil import masks_to_dev, poison_erased_dev, say, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def decode_both(mj, plan, P, nb, seed):
    """Encode nb blocks of the plan's code, overwrite the erased projections,
    decode with a caller workspace and without; returns both outputs and
    the images."""
    Q, dirs = plan.Q, plan.dirs
    n = len(dirs)
    words = mj.mojette_block_words(dirs, P, Q)
    d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
    mj.mojette_fill_splitmix64(d_img, d_img.numel(), seed)
    d_proj = torch.empty(nb * words, dtype=torch.int64, device="cuda")
    mj.mojette_encode_batch(d_img, nb, P, Q, dirs, d_proj)
    masks = synth.erasure_masks(seed + 1, nb, n, (0, n - Q))
    poison_erased_dev(d_proj, masks, [mj.mojette_proj_size(p, P, Q) for p in dirs])
    d_mask = masks_to_dev(masks)
    need = plan.workspace_words(P, nb)
    d_ws = torch.full((max(1, need),), -1, dtype=torch.int64, device="cuda")
    out_ws = torch.full_like(d_img, -1)
    out_na = torch.full_like(d_img, -1)
    st_ws = torch.zeros(1, dtype=torch.int32, device="cuda")
    st_na = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_batch_chunked(plan, d_proj, d_mask, nb, P, out_ws, d_ws, status=st_ws)
    mj.mojette_decode_batch_chunked_noalloc(plan, d_proj, d_mask, nb, P, out_na, status=st_na)
    torch.cuda.synchronize()
    assert int(st_ws.item()) == 0 and int(st_na.item()) == 0
    return out_ws, out_na, d_img, need


def test_noalloc_equals_workspace_call_on_calls_in_a_row(mj):
    dirs, Q = synth.centered_dirs(6), 4
    plan = mj.ChunkPlan(dirs, Q, 256)
    # 1 MB blocks, then fewer and shorter blocks on the scratch the first left
    for P, nb, seed in [(32768, 24, 11), (9000, 5, 12), (4000, 2, 13)]:
        out_ws, out_na, img, need = decode_both(mj, plan, P, nb, seed)
        say(f"no-alloc chunked decode: P={P} blocks={nb} scratch words={need}")
        assert 0 < need <= mj.MOJETTE_SCRATCH_WORDS
        assert torch.equal(out_na, out_ws)
        assert torch.equal(out_na, img)
    plan.close()


def test_noalloc_tall_code_and_short_rows(mj):
    dirs, Q = synth.centered_dirs(12), 8
    plan = mj.ChunkPlan(dirs, Q, 512)
    for P, nb, seed in [(16384, 6, 21), (6000, 3, 22), (300, 4, 23)]:
        out_ws, out_na, img, need = decode_both(mj, plan, P, nb, seed)
        say(f"no-alloc chunked decode (8,4): P={P} blocks={nb} scratch words={need}")
        assert (need == 0) == (P == 300)          # rows too short to cut: whole blocks
        assert torch.equal(out_na, out_ws)
        assert torch.equal(out_na, img)
    plan.close()


def test_noalloc_refuses_beyond_its_scratch(mj):
    dirs, Q = synth.centered_dirs(6), 4
    plan = mj.ChunkPlan(dirs, Q, 64)
    P = 32768
    per_block = plan.workspace_words(P, 1)
    nb = mj.MOJETTE_SCRATCH_WORDS // per_block + 1
    assert plan.workspace_words(P, nb) > mj.MOJETTE_SCRATCH_WORDS
    dummy = torch.zeros(8, dtype=torch.int64, device="cuda")
    rc = mj.mojette_decode_batch_chunked_noalloc(plan, dummy, None, nb, P, dummy, check=False)
    assert rc == mj.MOJETTE_ESCRATCH
    assert "scratch" in mj.strerror(rc)
    plan.close()
