"""Mixed batches (several geometry classes in one launch) against the oracle."""
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


def run_classes(mj, classes, seed, ner_max=None, graph_reps=0):
    """classes: [(P, Q, dirs, nblocks)]; returns per-class (imgs, enc, dec)."""
    spec = [(P, Q, d, nb) for P, Q, d, nb in classes]
    iw, pw = mj.mojette_classes_layout(spec)
    imgs, masks, pools = [], [], []
    for c, (P, Q, dirs, nb) in enumerate(spec):
        imgs.append(synth.block_images(seed + c, 0, nb, P, Q))
        m = len(dirs) - Q if ner_max is None else min(ner_max, len(dirs) - Q)
        masks.append(synth.erasure_masks(seed + 100 + c, nb, len(dirs), (0, m)))
    d_img = to_dev(np.concatenate([x.ravel() for x in imgs]))
    assert d_img.numel() == iw
    d_proj = torch.empty(pw, dtype=torch.int64, device="cuda")
    mj.mojette_encode_classes(spec, d_img, d_proj)
    torch.cuda.synchronize()
    enc_all = to_np(d_proj)
    # poison erased projections, then decode
    src = enc_all.copy()
    off = 0
    encs = []
    for c, (P, Q, dirs, nb) in enumerate(spec):
        words = mj.mojette_block_words(dirs, P, Q)
        enc = enc_all[off:off + nb * words].reshape(nb, words)
        encs.append(enc)
        sizes = np.cumsum([0] + [oracle.proj_size(p, 1, P, Q) for p in dirs])
        blk = src[off:off + nb * words].reshape(nb, words)
        for i in range(len(dirs)):
            rows = np.flatnonzero((masks[c] >> i) & 1)
            blk[rows, sizes[i]:sizes[i + 1]] = POISON
        off += nb * words
    d_src = to_dev(src)
    d_mask = masks_to_dev(np.concatenate(masks))
    d_out = torch.full((iw,), -1, dtype=torch.int64, device="cuda")
    d_status = torch.zeros(1, dtype=torch.int32, device="cuda")
    mj.mojette_decode_classes(spec, d_src, d_mask, d_out, d_status)
    torch.cuda.synchronize()
    assert int(d_status.item()) == 0
    if graph_reps:
        g = torch.cuda.CUDAGraph()
        d_out2 = torch.zeros_like(d_out)
        d_proj2 = torch.zeros_like(d_proj)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            mj.mojette_encode_classes(spec, d_img, d_proj2)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            mj.mojette_encode_classes(spec, d_img, d_proj2)
            mj.mojette_decode_classes(spec, d_src, d_mask, d_out2, d_status)
        for _ in range(graph_reps):
            d_out2.zero_()
            d_proj2.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(d_proj2, d_proj)
            assert torch.equal(d_out2, d_out)
    dec_all = to_np(d_out)
    out, off = [], 0
    for c, (P, Q, dirs, nb) in enumerate(spec):
        dec = dec_all[off:off + nb * P * Q].reshape(nb, Q, P)
        out.append((imgs[c], encs[c], dec, masks[c]))
        off += nb * P * Q
    return out


def check(classes, results, sample=None):
    for (P, Q, dirs, nb), (img, enc, dec, mask) in zip(classes, results):
        if nb == 0:
            continue
        idx = np.arange(nb) if sample is None else np.unique(
            np.concatenate([[0, nb - 1], np.random.default_rng(P).integers(0, nb, sample)]))
        want = oracle.encode_blocks(img[idx], P, Q, dirs)
        assert np.array_equal(enc[idx], want), (P, Q)
        assert np.array_equal(oracle.decode_blocks(want, mask[idx], P, Q, dirs), img[idx])
        assert np.array_equal(dec, img), (P, Q)


def test_mixed_codes_4_6_8_12_with_large_blocks(mj):
    classes = [
        (128, 4, synth.centered_dirs(6), 300),
        (256, 4, synth.centered_dirs(6), 150),
        (171, 6, synth.centered_dirs(9), 80),
        (128, 8, synth.centered_dirs(12), 60),
        (1366, 6, synth.centered_dirs(9), 5),
        (10923, 12, synth.centered_dirs(16), 2),
        (32768, 4, synth.centered_dirs(6), 2),
    ]
    say("mixed {4,6,8,12}")
    check(classes, run_classes(mj, classes, 11))


def test_mixed_codes_4_8_graph_replay(mj):
    classes = [
        (128, 4, synth.centered_dirs(6), 500),
        (2048, 4, synth.centered_dirs(6), 40),
        (64, 8, synth.centered_dirs(12), 200),
        (1024, 8, synth.centered_dirs(12), 30),
    ]
    say("mixed {4,8} with graph replay")
    check(classes, run_classes(mj, classes, 21, graph_reps=3))


def test_mixed_row_counts_without_a_compiled_kernel(mj):
    classes = [
        (77, 3, [2, -1, 0, 5], 90),
        (40, 5, [7, -6, 0, 2, -3, 1], 70),
        (33, 3, [-2, -1, 0, 1, 2], 50),
        (5, 2, [1, 0, -1], 0),
    ]
    say("mixed {3,5}: one launch per row count")
    check(classes, run_classes(mj, classes, 31))


def test_mixed_config_sample(mj):
    """The 16 size x code classes of the mixed workload, scaled to 640 blocks."""
    spec = [(P, Q, d, nb) for P, Q, d, nb, _ in synth.mixed_classes(640, 4)]
    say(f"mixed workload classes: {[(P, Q, nb) for P, Q, _, nb in spec]}")
    check(spec, run_classes(mj, spec, 41), sample=6)


def test_jobs_scatter_and_gather_slots(mj):
    """Encode scatters blocks to arbitrary projection slots of an arena,
    decode gathers them back, codes (4,2) and (8,4) in one launch each."""
    rng = np.random.default_rng(5)
    specs = [(128, 4, synth.centered_dirs(6), 300, 1000), (96, 8, synth.centered_dirs(12), 120, 500),
             (2048, 4, synth.centered_dirs(6), 20, 64)]
    arenas, jobs_e, jobs_d, host = [], [], [], []
    for c, (P, Q, dirs, nb, cap) in enumerate(specs):
        words = mj.mojette_block_words(dirs, P, Q)
        imgs = synth.block_images(70 + c, 0, nb, P, Q)
        slots = rng.permutation(cap)[:nb].astype(np.int64)
        masks = synth.erasure_masks(80 + c, nb, len(dirs), (0, len(dirs) - Q))
        arena = torch.full((cap * words,), 7, dtype=torch.int64, device="cuda")
        d_slots = torch.from_numpy(slots).cuda()
        d_img = to_dev(imgs)
        d_out = torch.full_like(d_img, -1)
        jobs_e.append(dict(P=P, Q=Q, dirs=dirs, nblocks=nb, images=d_img, projs=arena,
                           slots=d_slots))
        jobs_d.append(dict(P=P, Q=Q, dirs=dirs, nblocks=nb, images=d_out, projs=arena,
                           slots=d_slots, erased=masks_to_dev(masks)))
        arenas.append(arena)
        host.append((imgs, slots, masks, words, d_out))
    say("jobs: scatter encode")
    mj.mojette_encode_jobs(jobs_e)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    say("jobs: gather decode")
    mj.mojette_decode_jobs(jobs_d, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    for (P, Q, dirs, nb, cap), arena, (imgs, slots, masks, words, d_out) in zip(specs, arenas, host):
        ar = to_np(arena).reshape(cap, words)
        want = oracle.encode_blocks(imgs, P, Q, dirs)
        assert np.array_equal(ar[slots], want)
        untouched = np.setdiff1d(np.arange(cap), slots)
        assert (ar[untouched] == 7).all()
        assert np.array_equal(to_np(d_out).reshape(nb, Q, P), imgs)


def test_jobs_big_job_gets_its_own_launch_with_slots(mj):
    """A job large enough for a launch of its own (here 9,000 4 KB blocks at
    scattered slots) beside a small job sharing the mixed launch: both must
    land exactly where the mixed launch alone would put them."""
    rng = np.random.default_rng(9)
    specs = [(128, 4, synth.centered_dirs(6), 9000, 9500), (64, 8, synth.centered_dirs(12), 50, 80),
             (1024, 4, synth.centered_dirs(6), 40, 40)]
    jobs_e, ref_e, host = [], [], []
    for c, (P, Q, dirs, nb, cap) in enumerate(specs):
        words = mj.mojette_block_words(dirs, P, Q)
        d_img = torch.empty(nb * Q * P, dtype=torch.int64, device="cuda")
        mj.mojette_fill_splitmix64(d_img, d_img.numel(), 40 + c)
        slots = rng.permutation(cap)[:nb].astype(np.int64)
        d_slots = torch.from_numpy(slots).cuda()
        arena = torch.full((cap * words,), 7, dtype=torch.int64, device="cuda")
        jobs_e.append(dict(P=P, Q=Q, dirs=dirs, nblocks=nb, images=d_img, projs=arena,
                           slots=d_slots))
        host.append((d_img, slots, arena, words, cap))
    say("jobs: big job + small jobs")
    mj.mojette_encode_jobs(jobs_e)
    torch.cuda.synchronize()
    for (P, Q, dirs, nb, cap), (d_img, slots, arena, words, _) in zip(specs, host):
        ref = torch.empty(nb * words, dtype=torch.int64, device="cuda")
        mj.mojette_encode_batch(d_img, nb, P, Q, dirs, ref)
        torch.cuda.synchronize()
        ar = to_np(arena).reshape(cap, words)
        assert np.array_equal(ar[slots], to_np(ref).reshape(nb, words))
        untouched = np.setdiff1d(np.arange(cap), slots)
        assert (ar[untouched] == 7).all()
        pick = rng.integers(0, nb, 6)
        imgs = to_np(d_img).reshape(nb, Q, P)[pick]
        assert np.array_equal(ar[slots[pick]], oracle.encode_blocks(imgs, P, Q, dirs))
