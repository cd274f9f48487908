"""Pins for the CPU oracle (no GPU).

Each check below fixes the oracle against something other than itself: the
closed form of Eq. 2, invariants that follow from Eq. 1 (group sums, edge bins,
impulse responses, linearity, XOR parity for p = 0), the Katz criterion of
Eq. 3 against brute-force GF(2) rank, the structure of the worked example of
Section 2.1, and brute-force GF(2) elimination for the inverse of Section 2.2.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import synth
from tests import gf2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_image(rng, P, Q, kind=0, mod=0):
    if kind == 0:
        return rng.integers(0, 2**64, size=(Q, P), dtype=np.uint64)
    return rng.integers(0, mod, size=(Q, P)).astype(np.uint64)


COPRIME = [(p, q) for p in range(-3, 4) for q in range(0, 4)
           if math.gcd(p, q) == 1 and not (q == 0 and p != 1)]


# ---------------------------------------------------------------- Eq. 2 ----

@pytest.mark.parametrize("P,Q", [(1, 1), (3, 3), (5, 2), (2, 7), (16, 4), (128, 4)])
def test_proj_size_closed_form_matches_line_span(orc, P, Q):
    """Eq. 2 equals the number of distinct line positions over the image."""
    for p, q in COPRIME + [(5, 1), (-7, 2), (1, 0)]:
        pos = gf2.line_positions(p, q, P, Q)
        span = max(pos.values()) - min(pos.values()) + 1
        assert orc.proj_size(p, q, P, Q) == abs(p) * (Q - 1) + abs(q) * (P - 1) + 1
        assert orc.proj_size(p, q, P, Q) == span
        assert orc.bin_min(p, q, P, Q) == min(pos.values())


def test_q1_every_bin_crosses_between_one_and_Q_pixels(orc):
    """With q = 1 no bin is empty, no bin holds more than Q pixels (at most
    k-1 additions per bin, Section 3.1), and for p != 0 the two edge bins
    hold one pixel each (for p = 0 every bin is a whole column)."""
    P, Q = 9, 4
    ones = np.ones((Q, P), dtype=np.uint64)
    for p in range(-4, 5):
        (proj,) = orc.forward(ones, [(p, 1)], kind=orc.MODN, mod=1 << 40)
        assert proj.min() >= 1 and proj.max() <= Q
        if p != 0:
            assert proj[0] == 1 and proj[-1] == 1
        else:
            assert (proj == Q).all()
        assert int(proj.sum()) == P * Q


# ---------------------------------------------------------------- Eq. 1 ----

def test_impulse_response(orc):
    """A single non-zero pixel lands in exactly one bin per projection, at
    j = -k*q + l*p - b_min (Eq. 1 with the Iverson bracket)."""
    P, Q = 6, 3
    dirs = [(-2, 1), (0, 1), (1, 1), (3, 2), (1, 0)]
    for l in range(Q):
        for k in range(P):
            img = np.zeros((Q, P), dtype=np.uint64)
            img[l, k] = 0xA5A5
            projs = orc.forward(img, dirs)
            for (p, q), pr in zip(dirs, projs):
                nz = np.flatnonzero(pr)
                pos = gf2.line_positions(p, q, P, Q)
                assert list(nz) == [pos[(k, l)] - min(pos.values())]
                assert pr[nz[0]] == 0xA5A5


@pytest.mark.parametrize("kind,mod", [(0, 0), (1, 6), (1, 2**61 - 1)])
def test_projection_sums_equal_image_sum(orc, kind, mod):
    """Every pixel lies on exactly one line per direction, so the group sum of
    any projection's bins equals the group sum of the image."""
    rng = np.random.default_rng(1)
    P, Q = 11, 5
    img = rand_image(rng, P, Q, kind, mod)
    dirs = COPRIME
    projs = orc.forward(img, dirs, kind=kind, mod=mod)
    if kind == 0:
        total = np.bitwise_xor.reduce(img.ravel())
        for pr in projs:
            assert np.bitwise_xor.reduce(pr) == total
    else:
        total = int(sum(int(x) for x in img.ravel()) % mod)
        for pr in projs:
            assert int(sum(int(x) for x in pr) % mod) == total


def test_edge_bins_are_corner_pixels(orc):
    """Section 2.1: some border bins are exact copies of pixels.  For q = 1 and
    p > 0 the first bin is pixel (P-1, 0) and the last is (0, Q-1); for p < 0
    the first is (P-1, Q-1) and the last is (0, 0)."""
    rng = np.random.default_rng(2)
    P, Q = 16, 4
    img = rand_image(rng, P, Q)
    for p in [-3, -2, -1, 1, 2, 3]:
        (pr,) = orc.forward(img, [(p, 1)])
        if p > 0:
            assert pr[0] == img[0, P - 1] and pr[-1] == img[Q - 1, 0]
        else:
            assert pr[0] == img[Q - 1, P - 1] and pr[-1] == img[0, 0]


def test_p0_projection_is_xor_parity_of_the_data_packets(orc):
    """Direction (0,1): bin b = -k collects column k of every row, i.e. the
    RAID-4/5 XOR parity of the Q data packets, in reverse column order."""
    rng = np.random.default_rng(3)
    P, Q = 128, 4
    img = rand_image(rng, P, Q)
    (pr,) = orc.forward(img, [(0, 1)])
    parity = img[0] ^ img[1] ^ img[2] ^ img[3]
    assert np.array_equal(pr, parity[::-1])


def test_single_row_projections_are_the_row(orc):
    """Q = 1: every direction (p,1) has bins b = -k, the row read backwards."""
    rng = np.random.default_rng(4)
    img = rand_image(rng, 37, 1)
    for p in [-3, 0, 2, 5]:
        (pr,) = orc.forward(img, [(p, 1)])
        assert np.array_equal(pr, img[0, ::-1])


@pytest.mark.parametrize("kind,mod", [(0, 0), (1, 1000003)])
def test_linearity(orc, kind, mod):
    rng = np.random.default_rng(5)
    P, Q = 13, 4
    f = rand_image(rng, P, Q, kind, mod)
    g = rand_image(rng, P, Q, kind, mod)
    dirs = [(-3, 1), (-1, 1), (0, 1), (2, 1), (1, 2)]
    pf = orc.forward(f, dirs, kind=kind, mod=mod)
    pg = orc.forward(g, dirs, kind=kind, mod=mod)
    if kind == 0:
        ps = orc.forward(f ^ g, dirs)
        for a, b, c in zip(pf, pg, ps):
            assert np.array_equal(a ^ b, c)
    else:
        s = ((f.astype(object) + g.astype(object)) % mod).astype(np.uint64)
        ps = orc.forward(s, dirs, kind=kind, mod=mod)
        for a, b, c in zip(pf, pg, ps):
            assert np.array_equal(((a.astype(object) + b.astype(object)) % mod).astype(np.uint64), c)


def test_forward_equals_mojette_matrix_product(orc):
    """Bins = (0/1 Mojette matrix) x pixels over GF(2); the matrix is built by
    enumerating pixels, independently of the oracle's indexing."""
    rng = np.random.default_rng(6)
    P, Q = 7, 3
    dirs = [(-2, 1), (1, 1), (1, 2), (1, 0)]
    img = rand_image(rng, P, Q)
    A = gf2.mojette_matrix(dirs, P, Q)
    x = img.ravel()
    want = np.array([np.bitwise_xor.reduce(x[row.astype(bool)]) if row.any() else 0
                     for row in A], dtype=np.uint64)
    got = np.concatenate(orc.forward(img, dirs))
    assert np.array_equal(got, want)


# ---------------------------------------------------------------- Eq. 3 ----

def test_katz_equals_gf2_full_rank():
    """Katz's criterion (Eq. 3) holds exactly when the Mojette matrix has full
    column rank over GF(2), on every small case enumerated here."""
    import oracle

    pool = [(p, q) for p in range(-3, 4) for q in range(0, 3)
            if math.gcd(p, q) == 1 and not (q == 0 and p != 1)]
    checked = 0
    for P in range(1, 5):
        for Q in range(1, 5):
            for r in range(1, 4):
                for dirs in itertools.combinations(pool, r):
                    full = gf2.gf2_rank(gf2.mojette_matrix(dirs, P, Q)) == P * Q
                    assert oracle.katz(P, Q, dirs) == full, (P, Q, dirs)
                    checked += 1
    assert checked > 4000


def test_peeling_succeeds_iff_katz(orc):
    """The inverse (Section 2.2) reconstructs exactly when Katz holds; when it
    does, it returns the original image."""
    rng = np.random.default_rng(7)
    pool = [(p, q) for p in range(-2, 3) for q in range(0, 3)
            if math.gcd(p, q) == 1 and not (q == 0 and p != 1)]
    for P in range(1, 5):
        for Q in range(1, 5):
            img = rand_image(rng, P, Q)
            for r in range(1, 4):
                for dirs in itertools.combinations(pool, r):
                    projs = orc.forward(img, dirs)
                    rc, out = orc.inverse(projs, dirs, P, Q)
                    if orc.katz(P, Q, dirs):
                        assert rc == orc.OK, (P, Q, dirs)
                        assert np.array_equal(out, img)
                    else:
                        assert rc == orc.ENOTRECON, (P, Q, dirs)


# ------------------------------------------------------ worked example ----

def test_worked_example_structure(orc):
    with open(os.path.join(GOLDEN, "worked_example.json")) as fh:
        ex = json.load(fh)
    P, Q, mod = ex["P"], ex["Q"], ex["modulus"]
    dirs = [tuple(d) for d in ex["directions"]]
    rng = np.random.default_rng(1504)
    img = rng.integers(0, mod, size=(Q, P)).astype(np.uint64)
    projs = orc.forward(img, dirs, kind=orc.MODN, mod=mod)
    assert [len(x) for x in projs] == ex["bins_per_projection"]
    for pr in projs:
        assert int(pr.max()) < mod
    k = ex["any_k_of_n"]
    for sub in itertools.combinations(range(len(dirs)), k):
        rc, out = orc.inverse([projs[i] for i in sub], [dirs[i] for i in sub], P, Q,
                              kind=orc.MODN, mod=mod)
        assert rc == orc.OK and np.array_equal(out, img)
    # Two projections: Katz holds through the P branch only for sum|p| >= 3.
    for sub in itertools.combinations(range(len(dirs)), 2):
        d = [dirs[i] for i in sub]
        rc, out = orc.inverse([projs[i] for i in sub], d, P, Q, kind=orc.MODN, mod=mod)
        if sum(abs(p) for p, _ in d) >= P:
            assert rc == orc.OK and np.array_equal(out, img)
        else:
            assert rc == orc.ENOTRECON


# ------------------------------------------------ inverse vs brute force ----

def test_inverse_matches_gf2_elimination(orc):
    """On tiny images with random survivor sets, peeling and Gaussian
    elimination over GF(2) agree on the image and on solvability."""
    rng = np.random.default_rng(8)
    for trial in range(120):
        P = int(rng.integers(1, 7))
        Q = int(rng.integers(1, 5))
        n = int(rng.integers(1, 5))
        ps = rng.choice(np.arange(-3, 4), size=n, replace=False)
        dirs = [(int(p), 1) for p in ps]
        img = rand_image(rng, P, Q)
        projs = orc.forward(img, dirs)
        status, x = gf2.gf2_solve(gf2.mojette_matrix(dirs, P, Q), np.concatenate(projs))
        rc, out = orc.inverse(projs, dirs, P, Q)
        if status == "unique":
            assert rc == orc.OK
            assert np.array_equal(out.ravel(), x)
            assert np.array_equal(out, img)
        else:
            assert status == "singular"
            assert rc == orc.ENOTRECON


def test_inverse_verify_flags_corrupted_bins(orc):
    """With more projections than needed, a flipped bit in a redundant bin
    leaves the system inconsistent; elimination and verify both say so."""
    rng = np.random.default_rng(9)
    P, Q = 6, 3
    dirs = [(-1, 1), (0, 1), (1, 1), (2, 1)]
    img = rand_image(rng, P, Q)
    projs = orc.forward(img, dirs)
    rc, out = orc.inverse(projs, dirs, P, Q, verify=True)
    assert rc == orc.OK and np.array_equal(out, img)
    flat_sizes = np.cumsum([0] + [len(x) for x in projs])
    hits = 0
    for t in range(flat_sizes[-1]):
        bad = [x.copy() for x in projs]
        i = int(np.searchsorted(flat_sizes, t, side="right") - 1)
        bad[i][t - flat_sizes[i]] ^= np.uint64(1 << 17)
        status, _ = gf2.gf2_solve(gf2.mojette_matrix(dirs, P, Q), np.concatenate(bad))
        rc, _ = orc.inverse(bad, dirs, P, Q, verify=True)
        assert status == "inconsistent"
        assert rc == orc.EINCONSISTENT
        hits += 1
    assert hits == flat_sizes[-1]


# ------------------------------------------- the code geometry (Section 2.3) ----

def test_code_roundtrip_every_erasure_pattern(orc):
    """(6,4) code of Section 3, P = 128, uint64 pixels: any 4 of the 6
    projections give back the block (Katz with q_i = 1, Section 2.3)."""
    P, Q, n = 128, 4, 6
    ps = synth.centered_dirs(n)
    img = synth.block_images(synth.SEED_DATA, 0, 1, P, Q)[0]
    projs = orc.forward(img, [(p, 1) for p in ps])
    for r in range(0, 3):
        for lost in itertools.combinations(range(n), r):
            keep = [i for i in range(n) if i not in lost]
            rc, out = orc.inverse([projs[i] for i in keep], [(ps[i], 1) for i in keep], P, Q)
            assert rc == orc.OK and np.array_equal(out, img)
    keep = [0, 2, 5]
    rc, _ = orc.inverse([projs[i] for i in keep], [(ps[i], 1) for i in keep], P, Q)
    assert rc == orc.ENOTRECON


def test_block_helpers_match_single_calls(orc):
    P, Q, n = 32, 8, 12
    ps = synth.centered_dirs(n)
    imgs = synth.block_images(7, 0, 5, P, Q)
    pool = orc.encode_blocks(imgs, P, Q, ps)
    masks = synth.erasure_masks(3, 5, n, 4)
    dec = orc.decode_blocks(pool, masks, P, Q, ps)
    assert np.array_equal(dec, imgs)
    for b in range(5):
        single = np.concatenate(orc.forward(imgs[b], [(p, 1) for p in ps]))
        assert np.array_equal(pool[b], single)


def test_ops_count(orc):
    """Peeling removes every reconstructed pixel from each projection used
    (back-projection, Section 2.2): exactly m*P*Q subtractions."""
    P, Q = 20, 4
    dirs = [(-1, 1), (0, 1), (1, 1), (2, 1)]
    img = synth.block_images(1, 0, 1, P, Q)[0]
    projs = orc.forward(img, dirs)
    rc, out, ops = orc.inverse(projs, dirs, P, Q, return_ops=True)
    assert rc == orc.OK and ops == len(dirs) * P * Q


@pytest.mark.parametrize("P,Q,n,want", [(128, 4, 6, 2277), (256, 4, 6, 4581), (128, 8, 12, 10500),
                                        (1, 1, 1, 0), (7, 3, 5, None), (40, 5, 9, None)])
def test_encode_xor_count(orc, P, Q, n, want):
    """Encoding costs n*P*Q - sum(B_i) XORs: every pixel lands in one bin of
    every projection, and a bin's first pixel is a copy (Section 3.1: at
    most k - 1 XORs per bin, none at the edge bins, which hold one pixel).
    The counts for the 4 KB and 8 KB codes were worked out by hand from
    Eq. 2 when the scope was surveyed: 6*512 - 795, 6*1024 - 1563,
    12*1024 - 1788."""
    dirs = [(i - n // 2, 1) for i in range(n)]
    img = synth.block_images(P * Q + n, 0, 1, P, Q)[0]
    projs, ops = orc.forward(img, dirs, return_ops=True)
    sizes = [orc.proj_size(p, q, P, Q) for p, q in dirs]
    assert ops == n * P * Q - sum(sizes)
    if want is not None:
        assert ops == want
    # the count does not depend on the values; the projections are unchanged
    assert all(np.array_equal(a, b) for a, b in zip(projs, orc.forward(img, dirs)))
    _, ops0 = orc.forward(np.zeros_like(img), dirs, return_ops=True)
    assert ops0 == ops
