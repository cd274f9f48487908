"""Helpers for the GPU tests: moving uint64 words between numpy and torch."""
from __future__ import annotations

import numpy as np


def dev():
    import torch

    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).to(dev())


def masks_to_dev(m: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(m, dtype=np.uint16).view(np.int16).copy()).to(dev())


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def say(msg: str) -> None:
    print(msg, flush=True)


POISON_WORD = 0xDEADBEEFCAFEF00D


def poison_erased_dev(d_proj, masks: np.ndarray, sizes) -> None:
    """Overwrite, on the device and in place, every erased projection of a
    pool of blocks laid out back to back (projection i of a block at word
    sum(sizes[:i]) of its slice): a decoder that reads an erased projection
    instead of a survivor then produces wrong pixels."""
    import torch

    nb = len(masks)
    words = int(sum(sizes))
    view = d_proj.view(nb, words)
    poison = torch.tensor(POISON_WORD - (1 << 64), dtype=torch.int64, device=d_proj.device)
    m = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint16).astype(np.int64)).to(d_proj.device)
    off = 0
    for i, s in enumerate(sizes):
        rows = torch.nonzero((m >> i) & 1).flatten()
        if rows.numel():
            view[rows, off:off + s] = poison
        off += s


def survivor_depth(ps_used) -> int:
    """Deepest read behind a row's newest pixel for the used survivors
    (ascending p; the r-th rebuilds row r): the maximum over row pairs of
    ceil((A_l - A_r)/2) - 1 - (l - r) p_r, with A_r = 2 sum_{j<r} p_j + r."""
    Q = len(ps_used)
    A, s = [], 0
    for r in range(Q):
        A.append(2 * s + r)
        s += ps_used[r]
    best = 0
    for r in range(Q):
        for l in range(Q):
            if l != r:
                d = A[l] - A[r]
                ch = (d + 1) // 2 if d >= 0 else -((-d) // 2)
                best = max(best, ch - 1 - (l - r) * ps_used[r])
    return best


def mask_depth(mask: int, dirs, Q: int) -> int:
    """survivor_depth of the Q smallest surviving directions of an erasure mask."""
    used = sorted(p for i, p in enumerate(dirs) if not (mask >> i) & 1)[:Q]
    return survivor_depth(used)
