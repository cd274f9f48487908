"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds input generation only: no part of the Mojette arithmetic.

Pixels.  The paper's workload is a block "filled with random data" (Section
3.1).  Word ``i`` of a pool is the i-th output of SplitMix64 started from
``seed`` (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each output is the state passed through the
murmur3-style finaliser with shifts 30, 27, 31 and multipliers
0xBF58476D1CE4E5B9, 0x94D049BB133111EB.  Being counter-based, word i is
``mix(seed + (i + 1) * gamma)``, so any block can be generated on its own; the
HIP library carries its own implementation of the same definition for filling
device pools.

Erasures.  Per block, a uniform random subset of the n projections is erased,
drawn from a second SplitMix64 stream (``seed_erase``) by a partial
Fisher-Yates shuffle; the subset size is fixed or itself drawn uniformly.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

SEED_DATA = 1504
SEED_ERASE = 7038


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of SplitMix64 seeded with ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        return _mix(z)


def block_images(seed: int, first_block: int, nblocks: int, P: int, Q: int) -> np.ndarray:
    """Blocks ``first_block ..`` of a pool of (Q, P) images filled word by word."""
    wpb = P * Q
    return splitmix64(seed, first_block * wpb, nblocks * wpb).reshape(nblocks, Q, P)


def sample_images(seed: int, block_ids, P: int, Q: int) -> np.ndarray:
    wpb = P * Q
    return np.stack([splitmix64(seed, int(b) * wpb, wpb).reshape(Q, P) for b in block_ids])


def _uniform_below(r: np.ndarray, bound) -> np.ndarray:
    """Map 64-bit words to [0, bound) by the top 53 bits (bias below 2^-50)."""
    u = (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.minimum((u * bound).astype(np.int64), np.asarray(bound, dtype=np.int64) - 1)


def erasure_masks(seed: int, nblocks: int, n: int, n_erase, first_block: int = 0) -> np.ndarray:
    """uint16 masks, bit i set = projection i of that block erased.

    ``n_erase`` is an int (every block loses exactly that many) or a tuple
    ``(lo, hi)``: the count is drawn uniformly from lo..hi, then the subset.
    Stream layout: block b uses words b*(n+1) .. b*(n+1)+n of the stream, word
    0 for the count and words 1..n for the shuffle.
    """
    if n > 16:
        raise ValueError("at most 16 projections")
    per = n + 1
    r = splitmix64(seed, first_block * per, nblocks * per).reshape(nblocks, per)
    if isinstance(n_erase, tuple):
        lo, hi = n_erase
        cnt = lo + _uniform_below(r[:, 0], hi - lo + 1)
    else:
        cnt = np.full(nblocks, int(n_erase), dtype=np.int64)
    perm = np.tile(np.arange(n, dtype=np.int64), (nblocks, 1))
    rows = np.arange(nblocks)
    mask = np.zeros(nblocks, dtype=np.uint16)
    for t in range(n):
        pick = t + _uniform_below(r[:, 1 + t], n - t)
        a = perm[rows, t].copy()
        b = perm[rows, pick].copy()
        perm[rows, t] = b
        perm[rows, pick] = a
        take = t < cnt
        mask[take] |= (np.uint16(1) << b[take].astype(np.uint16))
    return mask


def centered_dirs(n: int) -> list[int]:
    """p_i = i - floor(n/2): {-3..2} for n=6, {-6..5} for n=12, {-8..7} for n=16."""
    return [i - n // 2 for i in range(n)]


# Mixed batches: four block sizes and four (k, m) codes, each combination a
# geometry class.  Sizes are drawn so that every size is equally likely (the
# set read as log-spaced), codes uniformly; P = ceil(size / (8k)), the last
# row zero-padded when 8k does not divide the size.
MIXED_SIZES = (4096, 8192, 65536, 1 << 20)
MIXED_CODES = ((4, 2), (6, 3), (8, 4), (12, 4))


def mixed_classes(total_blocks: int, seed: int, sizes=MIXED_SIZES, codes=MIXED_CODES):
    """[(P, Q, dirs, nblocks, size_bytes)] for a mixed batch of total_blocks,
    one entry per (size, code) pair, counts drawn from SplitMix64(seed)."""
    r = splitmix64(seed, 0, total_blocks)
    cell = _uniform_below(r, len(sizes) * len(codes))
    counts = np.bincount(cell, minlength=len(sizes) * len(codes))
    out = []
    for si, size in enumerate(sizes):
        for ci, (k, m) in enumerate(codes):
            cnt = int(counts[si * len(codes) + ci])
            P = -(-size // (8 * k))
            out.append((P, k, centered_dirs(k + m), cnt, size))
    return out


def mixed_images(seed: int, P: int, Q: int, nblocks: int, size: int, first_block: int = 0):
    """Images of one class: seeded words, zero past `size` bytes of each block."""
    imgs = block_images(seed, first_block, nblocks, P, Q).reshape(nblocks, Q * P)
    imgs[:, size // 8:] = 0
    return imgs.reshape(nblocks, Q, P)


def mixed_block_list(nblocks: int, seed: int, sizes=MIXED_SIZES, codes=MIXED_CODES):
    """Per-block recipe of a mixed batch: block b's size index and code index
    (each uniform, from SplitMix64(seed) words 2b and 2b+1) and its erasure
    mask (a uniform count 0..m, then a uniform subset of the n projections;
    erasure_masks over the blocks of each code, stream seed + 1 + code).
    Returns (size_idx, code_idx, masks) as numpy arrays."""
    r = splitmix64(seed, 0, 2 * nblocks).reshape(nblocks, 2)
    size_idx = _uniform_below(r[:, 0], len(sizes))
    code_idx = _uniform_below(r[:, 1], len(codes))
    masks = np.zeros(nblocks, dtype=np.uint16)
    for ci, (k, m) in enumerate(codes):
        sel = np.flatnonzero(code_idx == ci)
        masks[sel] = erasure_masks(seed + 1 + ci, len(sel), k + m, (0, m))
    return size_idx, code_idx, masks
