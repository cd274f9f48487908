"""Brute-force references used to pin the oracle (tests only).

Nothing here shares code with the oracle: the Mojette matrix is built by
enumerating pixels and the system is solved by Gaussian elimination over GF(2),
with 64-bit right-hand sides so that every row operation acts on the 64 bit
planes of a word at once.
"""
from __future__ import annotations

import numpy as np


def line_positions(p: int, q: int, P: int, Q: int):
    """Every pixel's line position b = -k*q + l*p (k column, l row), by enumeration."""
    return {(k, l): -k * q + l * p for l in range(Q) for k in range(P)}


def mojette_matrix(dirs, P: int, Q: int):
    """0/1 matrix with one row per bin (all directions stacked) and one column per pixel.

    Bins of a direction are the distinct line positions in ascending order; the
    column of pixel (k, l) is l*P + k.
    """
    rows = []
    for p, q in dirs:
        pos = line_positions(p, q, P, Q)
        lo, hi = min(pos.values()), max(pos.values())
        block = np.zeros((hi - lo + 1, P * Q), dtype=np.uint8)
        for (k, l), b in pos.items():
            block[b - lo, l * P + k] = 1
        rows.append(block)
    return np.concatenate(rows, axis=0) if rows else np.zeros((0, P * Q), dtype=np.uint8)


def gf2_rank(A: np.ndarray) -> int:
    A = (A.copy() & 1).astype(np.uint8)
    rank = 0
    nrows, ncols = A.shape
    for c in range(ncols):
        piv = None
        for r in range(rank, nrows):
            if A[r, c]:
                piv = r
                break
        if piv is None:
            continue
        if piv != rank:
            A[[rank, piv]] = A[[piv, rank]]
        for r in range(nrows):
            if r != rank and A[r, c]:
                A[r] ^= A[rank]
        rank += 1
    return rank


def gf2_solve(A: np.ndarray, rhs: np.ndarray):
    """Solve A x = rhs over GF(2) with uint64 word right-hand sides.

    Returns (status, x): status is "unique", "singular" (rank < columns) or
    "inconsistent" (a zero row with a non-zero right-hand side).
    """
    A = (A.copy() & 1).astype(np.uint8)
    y = rhs.astype(np.uint64).copy()
    nrows, ncols = A.shape
    rank = 0
    pivcol = []
    for c in range(ncols):
        piv = None
        for r in range(rank, nrows):
            if A[r, c]:
                piv = r
                break
        if piv is None:
            continue
        if piv != rank:
            A[[rank, piv]] = A[[piv, rank]]
            y[[rank, piv]] = y[[piv, rank]]
        for r in range(nrows):
            if r != rank and A[r, c]:
                A[r] ^= A[rank]
                y[r] ^= y[rank]
        pivcol.append(c)
        rank += 1
    for r in range(rank, nrows):
        if y[r] != 0:
            return "inconsistent", None
    if rank < ncols:
        return "singular", None
    x = np.zeros(ncols, dtype=np.uint64)
    for r, c in enumerate(pivcol):
        x[c] = y[r]
    return "unique", x
