"""Host side of the chunked decode, no GPU: the library's transfer matrices
against a symbolic run of the sweep written here, and the whole chunked
scheme (zero-start sweeps, carry with the library's matrices, exact
re-sweeps) replayed on the CPU against the oracle's decode.

The sweep model: survivors sorted by p, row r uses the r-th (p_r), pixel
(k, r) = bin XOR the pixels (k + (l-r) p_r, l), l != r (Section 2.2), taken
in half-steps: with A_r = 2(p_0 + ... + p_{r-1}) + r, rows of the parity of
max A ("X") take column t*16 + d_r + i at half-step 2i of tile t, the others
at 2i + 1, d_r = -floor((max A - A_r) / 2) (X) or -floor((max A - A_r - 1) / 2)."""
import functools
import itertools
import operator
import os

import numpy as np
import pytest

import synth

TW = 16


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not os.path.exists(mj.LIB_PATH):
        from paper_1504_07038_amd import build

        build.build()
    return mj


def schedule(ps):
    A, s = [], 0
    for r, p in enumerate(ps):
        A.append(2 * s + r)
        s += p
    amax, amin = max(A), min(A)
    isx = [(r & 1) == (amax & 1) for r in range(len(ps))]
    d = [-((amax - A[r]) >> 1) if isx[r] else -((amax - A[r] - 1) >> 1) for r in range(len(ps))]
    return d, isx, -((amax - amin) >> 1)


def sweep(ps, t0, t1, start, bins=None, P=None):
    """Pixels of tiles [t0, t1); `start` maps (row, column) -> value (int or
    bit set) for columns before the run; missing ones count as zero."""
    d, isx, _ = schedule(ps)
    val = dict(start)
    Q = len(ps)
    for t in range(t0, t1):
        for i in range(TW):
            for phase in (True, False):
                for r in range(Q):
                    if isx[r] != phase:
                        continue
                    k = t * TW + d[r] + i
                    v = bins(r, k) if bins else 0
                    for l in range(Q):
                        if l != r:
                            c = k + (l - r) * ps[r]
                            assert (l, c) in val or c < t0 * TW + d[l], "read ahead of the sweep"
                            v ^= val.get((l, c), 0)
                    if P is not None and not 0 <= k < P:
                        v = 0
                    val[(r, k)] = v
    return val


def symbolic_matrix(ps, tiles, E):
    d, _, _ = schedule(ps)
    Q = len(ps)
    B = 100   # an interior chunk: far from column 0
    start = {(r, B * TW + d[r] - E + e): 1 << (r * E + e) for r in range(Q) for e in range(E)}
    out = sweep(ps, B, B + tiles, start)
    return [out[(r, (B + tiles) * TW + d[r] - E + e)] for r in range(Q) for e in range(E)]


def rows_to_ints(rows):
    return [sum(int(w) << (64 * i) for i, w in enumerate(row)) for row in rows]


CODES = [(synth.centered_dirs(6), 4), (synth.centered_dirs(12), 8), (synth.centered_dirs(9), 6),
         ([5, -1, 3], 2), ([0, 1], 1)]


@pytest.mark.parametrize("dirs,Q", CODES)
def test_transfer_matrix_matches_symbolic_sweep(mj, dirs, Q):
    rng = np.random.default_rng(len(dirs) * 10 + Q)
    subsets = list(itertools.combinations(sorted(dirs), Q))
    for ps in [subsets[i] for i in rng.choice(len(subsets), min(4, len(subsets)), replace=False)]:
        for cols in (64, 160):
            try:
                E, rows = mj.mojette_chunk_matrix(list(ps), Q, cols)
            except mj.MojetteError:
                _, _, dmin = schedule(ps)
                assert (cols + TW - 1) // TW * TW < -dmin   # refused only when too short
                continue
            tiles = (cols + TW - 1) // TW
            assert rows_to_ints(rows) == symbolic_matrix(list(ps), tiles, E), (ps, cols)


def test_chunk_matrix_argument_errors(mj):
    with pytest.raises(mj.MojetteError):
        mj.mojette_chunk_matrix([2, 1], 2, 64)        # not ascending
    with pytest.raises(mj.MojetteError):
        # this set's sweep leads in over 32 columns: a 16-column chunk is too short
        mj.mojette_chunk_matrix(list(range(-8, 4)), 12, 16)


def chunked_decode_model(mj, P, Q, dirs, mask, chunk_cols, image, orc):
    """The chunked scheme on the CPU, with the library's matrices."""
    projs = orc.forward(image, [(p, 1) for p in dirs])
    order = sorted(range(len(dirs)), key=lambda i: dirs[i])
    surv = [i for i in order if not (mask >> i) & 1][:Q]
    ps = [dirs[i] for i in surv]
    d, _, dmin = schedule(ps)
    tiles = (chunk_cols + TW - 1) // TW
    E, rows = mj.mojette_chunk_matrix(ps, Q, chunk_cols)
    T = rows_to_ints(rows)

    def bins(r, k):
        if not 0 <= k < P:
            return 0
        return int(projs[surv[r]][r * ps[r] - k - orc.bin_min(ps[r], 1, P, Q)])

    ntiles = (P - 1) // TW + (-dmin + TW - 1) // TW + 1
    nchunks = max(1, (P // TW) // tiles)
    assert nchunks >= 3
    end = lambda v, c: [v.get((r, c * tiles * TW + d[r] - E + e), 0)
                        for r in range(Q) for e in range(E)]
    ys = [end(sweep(ps, c * tiles, (c + 1) * tiles, {}, bins, P), c + 1) for c in range(nchunks - 1)]
    zs = {1: ys[0]}
    for c in range(1, nchunks - 1):
        z = zs[c]
        zs[c + 1] = [functools.reduce(operator.xor,
                                      [z[j] for j in range(len(z)) if (T[i] >> j) & 1], y)
                     for i, y in enumerate(ys[c])]
    out = np.zeros((Q, P), dtype=np.uint64)
    for c in range(nchunks):
        t0, t1 = c * tiles, ((c + 1) * tiles if c < nchunks - 1 else ntiles)
        start = {} if c == 0 else {(r, t0 * TW + d[r] - E + e): zs[c][r * E + e]
                                   for r in range(Q) for e in range(E)}
        v = sweep(ps, t0, t1, start, bins, P)
        for r in range(Q):
            for k in range(max(0, t0 * TW + d[r]), min(P, t1 * TW + d[r])):
                out[r, k] = v[(r, k)]
    return out


@pytest.mark.parametrize("P,Q,dirs,cols", [(300, 4, synth.centered_dirs(6), 48),
                                           (520, 8, synth.centered_dirs(12), 64),
                                           (333, 2, [5, -1, 3], 32)])
def test_chunked_scheme_reproduces_the_image(mj, orc, P, Q, dirs, cols):
    n = len(dirs)
    masks = synth.erasure_masks(17, 4, n, (0, n - Q))
    imgs = synth.block_images(23, 0, 4, P, Q)
    for mask, img in zip(masks, imgs):
        out = chunked_decode_model(mj, P, Q, dirs, int(mask), cols, img, orc)
        assert np.array_equal(out, img), hex(int(mask))
