"""Serving loop on the GPU: every tracked request's result, taken inside the
concurrent mix, is bit-identical to the same request run alone through the
single-block entry points, and to the oracle.  XOR arithmetic is exact, so the
tolerance is zero."""
import numpy as np
import pytest

import synth
from tests.gpuutil import say, to_dev, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def alone_encode(mj, img_t, g):
    outs = [torch.empty(mj.mojette_proj_size(p, g.P, g.Q), dtype=torch.int64, device="cuda")
            for p in g.dirs]
    mj.mojette_encode(img_t, g.P, g.Q, g.dirs, outs)
    return outs


def alone_decode(mj, projs, mask, g):
    ids = [i for i in range(len(g.dirs)) if not (mask >> i) & 1]
    out = torch.empty(g.img_words, dtype=torch.int64, device="cuda")
    mj.mojette_decode([projs[i] for i in ids], ids, g.dirs, g.P, g.Q, out)
    return out


@pytest.mark.parametrize("budget_mib,prefill,qps,chunk_max,long_reads",
                         [(3072, 0.5, 100000, 512, "chunked"), (640, 1.0, 200000, 512, "chunked"),
                          (3072, 0.5, 100000, 0, "chunked"),     # long rows never chunked
                          (3072, 0.5, 200000, 512, "both_ends"),
                          # both paths by arrival rate and backlog (low
                          # thresholds so that the decode from both ends is taken)
                          (3072, 0.5, 400000, 512, "auto")])
def test_serving_mix_matches_alone_and_oracle(mj, orc, budget_mib, prefill, qps, chunk_max,
                                              long_reads):
    from paper_1504_07038_amd import serving

    seed = 11
    geos = serving.geometries(per_octave=1)
    say(f"serving: budget {budget_mib} MiB, prefill {prefill}, qps {qps}, {len(geos)} classes, "
        f"chunked reads up to {chunk_max} per iteration, long reads {long_reads}")
    srv = serving.Server(budget_bytes=budget_mib << 20, depth=3, seed=seed, geos=geos,
                         prefill=prefill, per_iter_bytes=2 << 20, chunk_max_reads=chunk_max,
                         long_reads=long_reads, auto_backlog=200, auto_rate=3e5)
    assert srv.budget_used <= budget_mib << 20
    tr = serving.make_trace(qps, 0.05, geos, seed=3)
    N = len(tr.arrival)
    rng = np.random.default_rng(1)
    track = set(int(x) for x in rng.choice(N, 48, replace=False))
    # make sure both kinds and both codes are tracked
    for r in (0, 1):
        for k in (4, 8):
            cand = np.flatnonzero((tr.read == r) & (np.array([g.k for g in geos])[tr.cls] == k))
            track |= set(int(x) for x in cand[:3])
    done, res, stats = srv.run(tr, track=track, max_wall=90)
    say(f"serving: {N} requests, {stats}")
    assert np.isfinite(done).all()
    assert int(srv.status.item()) == 0
    assert stats["iterations"] > 1
    if long_reads == "auto":
        assert stats["both_ends_iterations"] > 0
    assert set(res) == track
    lat = done - tr.arrival
    assert (lat > 0).all()
    n_oracle = 0
    for rid in sorted(res):
        kind, c, slot, row, data = res[rid]
        st = srv.cs[c]
        g = st.geo
        assert row >= 0
        # the payload row is the seeded generator's output (inputs tie to the oracle side)
        img = synth.splitmix64(seed * 1000 + c, row * g.img_words, g.img_words)
        payload_t = st.payload[row * g.img_words:(row + 1) * g.img_words]
        assert np.array_equal(to_np(payload_t), img), rid
        projs = alone_encode(mj, payload_t, g)
        if kind == "w":
            mix = to_np(data)
            assert np.array_equal(mix, np.concatenate([to_np(p) for p in projs])), rid
            if n_oracle < 6:
                exp = orc.encode_blocks(img.reshape(1, g.Q, g.P), g.P, g.Q, g.dirs)[0]
                assert np.array_equal(mix, exp), rid
                n_oracle += 1
        else:
            mix = to_np(data)
            assert np.array_equal(mix, img), rid
            alone = alone_decode(mj, projs, int(tr.mask[rid]), g)
            torch.cuda.synchronize()
            assert np.array_equal(to_np(alone), mix), rid
    summ = serving.summarize(tr, done, stats)
    say(f"serving: {summ}")
    assert summ["completed"] == N and summ["p99_us"] >= summ["p50_us"] > 0
