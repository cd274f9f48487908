"""Mojette transform oracle: a plain CPU implementation used to check the GPU path.

TEST INFRASTRUCTURE ONLY.  The product package never imports this module; only
the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
do.  The arithmetic lives in ``mojette_oracle.c`` (plain C, one loop per line of
the definitions); this file only builds it with gcc and marshals numpy arrays.

Paper: Pertin et al., arXiv 1504.07038.
  - ``proj_size``    Section 2.1, Eq. 2.
  - ``bin_min``      Section 2.1, Eq. 1 (smallest line position over the image).
  - ``katz``         Section 2.2, Eq. 3.
  - ``forward``      Section 2.1, Eq. 1, over a pluggable group ("any addition").
  - ``inverse``      Section 2.2, the peeling reconstruction.
  - ``encode_blocks`` / ``decode_blocks``  Section 2.3 and Section 3: the XOR
    erasure code with q_i = 1, one call per block.
  - ``encode_blocks_wide`` / ``decode_blocks_wide``  Section 3.1: the same code
    on 128-bit pixels and bins.
  - ``kept_bins`` / ``encode_blocks_kept`` / ``decode_blocks_kept``  Section 2.3:
    the code with the bins that reconstruction never uses left out.
  - ``encode_blocks_sys`` / ``decode_blocks_sys``  Section 2.3's systematic
    version: data lines stored as they are, parity projections beside them.

Group: ``kind=0`` XOR on uint64 words; ``kind=1`` integers modulo ``mod``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mojette_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK = 0
EINVAL = -1
ENOTRECON = -2
ENOMEM = -4
EINCONSISTENT = -5

XOR = 0
MODN = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build(force=False)
    lib = ctypes.CDLL(LIB)
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.orc_proj_size.argtypes = [i32, i32, i32, i32]
    lib.orc_proj_size.restype = i64
    lib.orc_bin_min.argtypes = [i32, i32, i32, i32]
    lib.orc_bin_min.restype = i64
    lib.orc_katz.argtypes = [i32, i32, vp, vp, i32]
    lib.orc_katz.restype = i32
    lib.orc_forward.argtypes = [i32, u64, vp, i32, i32, vp, vp, i32, vp, vp]
    lib.orc_forward.restype = i32
    lib.orc_forward_count.argtypes = [i32, u64, vp, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.orc_forward_count.restype = i32
    lib.orc_inverse.argtypes = [i32, u64, vp, vp, vp, vp, i32, i32, i32, vp, i32, vp]
    lib.orc_inverse.restype = i32
    lib.orc_inverse_kept.argtypes = [i32, u64, vp, vp, vp, vp, i32, i32, i32, vp, vp, vp, i32,
                                     vp]
    lib.orc_inverse_kept.restype = i32
    lib.orc_inverse_known.argtypes = [i32, u64, vp, vp, vp, vp, i32, i32, i32, vp, vp, i32, vp]
    lib.orc_inverse_known.restype = i32
    lib.orc_encode_blocks.argtypes = [vp, i64, i32, i32, vp, i32, vp]
    lib.orc_encode_blocks.restype = i32
    lib.orc_decode_blocks.argtypes = [vp, vp, i64, i32, i32, vp, i32, vp]
    lib.orc_decode_blocks.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def proj_size(p: int, q: int, P: int, Q: int) -> int:
    return int(_load().orc_proj_size(p, q, P, Q))


def bin_min(p: int, q: int, P: int, Q: int) -> int:
    return int(_load().orc_bin_min(p, q, P, Q))


def katz(P: int, Q: int, dirs) -> bool:
    p = np.ascontiguousarray([d[0] for d in dirs], dtype=np.int32)
    q = np.ascontiguousarray([d[1] for d in dirs], dtype=np.int32)
    return bool(_load().orc_katz(P, Q, _ptr(p), _ptr(q), len(dirs)))


def _dir_arrays(dirs):
    p = np.ascontiguousarray([int(d[0]) for d in dirs], dtype=np.int32)
    q = np.ascontiguousarray([int(d[1]) for d in dirs], dtype=np.int32)
    return p, q


def forward(image: np.ndarray, dirs, kind: int = XOR, mod: int = 0, return_ops: bool = False):
    """Eq. 1 for every direction (p, q) in ``dirs``; ``image`` is (Q, P) uint64.
    With ``return_ops`` also the number of group additions that combine two
    pixels (a bin's first pixel is a copy)."""
    img = np.ascontiguousarray(image, dtype=np.uint64)
    Q, P = img.shape
    p, q = _dir_arrays(dirs)
    sizes = [proj_size(int(a), int(b), P, Q) for a, b in zip(p, q)]
    off = np.zeros(len(sizes), dtype=np.int64)
    if sizes:
        off[1:] = np.cumsum(sizes)[:-1]
    flat = np.zeros(max(1, sum(sizes)), dtype=np.uint64)
    ops = ctypes.c_int64(0)
    rc = _load().orc_forward_count(kind, mod, _ptr(img), P, Q, _ptr(p), _ptr(q), len(sizes),
                                   _ptr(flat), _ptr(off), ctypes.addressof(ops))
    if rc != OK:
        raise ValueError(f"orc_forward failed: {rc}")
    out = [flat[o:o + s].copy() for o, s in zip(off, sizes)]
    return (out, int(ops.value)) if return_ops else out


def inverse(projs, dirs, P: int, Q: int, kind: int = XOR, mod: int = 0,
            verify: bool = False, return_ops: bool = False):
    """Peeling reconstruction (Section 2.2) from ``projs[i]`` along ``dirs[i]``.

    Returns ``(rc, image)`` (and the subtraction count when ``return_ops``);
    ``image`` is (Q, P) uint64 and meaningful only when ``rc == OK``.
    """
    p, q = _dir_arrays(dirs)
    sizes = [len(x) for x in projs]
    for a, b, s in zip(p, q, sizes):
        if s != proj_size(int(a), int(b), P, Q):
            raise ValueError("projection length does not match Eq. 2")
    off = np.zeros(len(sizes), dtype=np.int64)
    if sizes:
        off[1:] = np.cumsum(sizes)[:-1]
    flat = np.ascontiguousarray(np.concatenate(projs) if projs else np.zeros(1), dtype=np.uint64)
    img = np.zeros((Q, P), dtype=np.uint64)
    ops = ctypes.c_int64(0)
    rc = _load().orc_inverse(kind, mod, _ptr(flat), _ptr(off), _ptr(p), _ptr(q), len(sizes),
                             P, Q, _ptr(img), int(verify), ctypes.addressof(ops))
    if return_ops:
        return int(rc), img, int(ops.value)
    return int(rc), img


def block_stride(P: int, Q: int, p_list) -> int:
    return sum(proj_size(int(p), 1, P, Q) for p in p_list)


def encode_blocks(images: np.ndarray, P: int, Q: int, p_list) -> np.ndarray:
    """XOR code, q_i = 1: ``images`` (nblocks, Q, P) -> projections (nblocks, sum B_i)."""
    img = np.ascontiguousarray(images, dtype=np.uint64).reshape(-1, Q, P)
    p = np.ascontiguousarray(p_list, dtype=np.int32)
    out = np.zeros((img.shape[0], block_stride(P, Q, p_list)), dtype=np.uint64)
    rc = _load().orc_encode_blocks(_ptr(img), img.shape[0], P, Q, _ptr(p), len(p), _ptr(out))
    if rc != OK:
        raise ValueError(f"orc_encode_blocks failed: {rc}")
    return out


def decode_blocks(projs: np.ndarray, erased: np.ndarray, P: int, Q: int, p_list) -> np.ndarray:
    """Decode each block from its projections not flagged in ``erased`` (uint16 bit masks)."""
    pr = np.ascontiguousarray(projs, dtype=np.uint64)
    er = np.ascontiguousarray(erased, dtype=np.uint16).reshape(-1)
    p = np.ascontiguousarray(p_list, dtype=np.int32)
    out = np.zeros((er.shape[0], Q, P), dtype=np.uint64)
    rc = _load().orc_decode_blocks(_ptr(pr), _ptr(er), er.shape[0], P, Q, _ptr(p), len(p), _ptr(out))
    if rc != OK:
        raise ValueError(f"orc_decode_blocks failed: {rc}")
    return out


def encode_blocks_wide(images: np.ndarray, P: int, Q: int, p_list) -> np.ndarray:
    """The XOR code on 128-bit pixels and bins (Section 3.1).

    ``images`` is (nblocks, Q, P, 2) uint64: the two 64-bit words of each
    16-byte pixel in memory order.  XOR adds 128-bit values bit by bit, so
    word h of every bin is the XOR of word h of the pixels on its line: the
    transform is the 64-bit transform of the plane of first words beside that
    of the plane of second words.  Returns (nblocks, sum B_i, 2).
    """
    img = np.ascontiguousarray(images, dtype=np.uint64).reshape(-1, Q, P, 2)
    planes = [encode_blocks(np.ascontiguousarray(img[..., h]), P, Q, p_list) for h in (0, 1)]
    return np.stack(planes, axis=-1)


def decode_blocks_wide(projs: np.ndarray, erased: np.ndarray, P: int, Q: int,
                       p_list) -> np.ndarray:
    """Inverse of ``encode_blocks_wide``, word plane by word plane (Section 2.2
    peeling on each); ``projs`` is (nblocks, sum B_i, 2)."""
    pr = np.ascontiguousarray(projs, dtype=np.uint64).reshape(-1, block_stride(P, Q, p_list), 2)
    planes = [decode_blocks(np.ascontiguousarray(pr[..., h]), erased, P, Q, p_list)
              for h in (0, 1)]
    return np.stack(planes, axis=-1)


def kept_bins(p_list, P: int, Q: int) -> list[tuple[int, int]]:
    """The bins each projection of the XOR code (q_i = 1) must keep (Section
    2.3: bins that no reconstruction uses can be left out), for the
    reconstruction path of Section 2.2 as this project fixes it: of the
    surviving projections the Q with the smallest p are used and the r-th of
    them rebuilds image row r from its bins r*p - k, k = 0..P-1.

    Enumerates every erasure pattern that leaves at least Q projections and
    marks the bins the path reads.  Returns, per projection in the order of
    ``p_list``, (first kept index, count) with indices as in ``forward``
    (b - b_min); raises if a projection's kept bins are not contiguous.
    """
    n = len(p_list)
    order = sorted(range(n), key=lambda i: p_list[i])
    used = [np.zeros(proj_size(int(p), 1, P, Q), dtype=bool) for p in p_list]
    for mask in range(1 << n):
        alive = [i for i in order if not (mask >> i) & 1]
        if len(alive) < Q:
            continue
        for r, i in enumerate(alive[:Q]):
            p = int(p_list[i])
            b0 = bin_min(p, 1, P, Q)
            # bins r*p - k for k = 0..P-1, i.e. r*p - P + 1 .. r*p
            used[i][r * p - P + 1 - b0: r * p + 1 - b0] = True
    out = []
    for u in used:
        idx = np.flatnonzero(u)
        if len(idx) == 0:
            out.append((0, 0))
            continue
        if idx[-1] - idx[0] + 1 != len(idx):
            raise ValueError("kept bins are not contiguous")
        out.append((int(idx[0]), int(len(idx))))
    return out


def encode_blocks_kept(images: np.ndarray, P: int, Q: int, p_list) -> np.ndarray:
    """The XOR code storing only the kept bins of each projection, projections
    back to back in the order of ``p_list``: (nblocks, sum of kept counts)."""
    full = encode_blocks(images, P, Q, p_list)
    keep = kept_bins(p_list, P, Q)
    offs = np.concatenate([[0], np.cumsum([proj_size(int(p), 1, P, Q) for p in p_list])])
    parts = [full[:, offs[i] + lo: offs[i] + lo + cnt] for i, (lo, cnt) in enumerate(keep)]
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


def decode_blocks_kept(projs: np.ndarray, erased: np.ndarray, P: int, Q: int,
                       p_list) -> np.ndarray:
    """Peeling (Section 2.2) of each block from the kept bins of its
    projections not flagged in ``erased``; the missing bins are never used."""
    keep = kept_bins(p_list, P, Q)
    words = sum(c for _, c in keep)
    pr = np.ascontiguousarray(projs, dtype=np.uint64).reshape(-1, words)
    er = np.ascontiguousarray(erased, dtype=np.uint16).reshape(-1)
    offs = np.concatenate([[0], np.cumsum([c for _, c in keep])]).astype(np.int64)
    out = np.zeros((er.shape[0], Q, P), dtype=np.uint64)
    lib = _load()
    for b in range(er.shape[0]):
        alive = [i for i in range(len(p_list)) if not (int(er[b]) >> i) & 1]
        p = np.ascontiguousarray([int(p_list[i]) for i in alive], dtype=np.int32)
        q = np.ones(len(alive), dtype=np.int32)
        off = np.ascontiguousarray([offs[i] for i in alive], dtype=np.int64)
        lo = np.ascontiguousarray([keep[i][0] for i in alive], dtype=np.int64)
        cnt = np.ascontiguousarray([keep[i][1] for i in alive], dtype=np.int64)
        row = np.ascontiguousarray(pr[b])
        img = np.zeros((Q, P), dtype=np.uint64)
        rc = lib.orc_inverse_kept(XOR, 0, _ptr(row), _ptr(off), _ptr(p), _ptr(q), len(alive),
                                  P, Q, _ptr(lo), _ptr(cnt), _ptr(img), 0, None)
        if rc != OK:
            raise ValueError(f"orc_inverse_kept failed on block {b}: {rc}")
        out[b] = img
    return out


def encode_blocks_sys(images: np.ndarray, P: int, Q: int, parity_dirs) -> np.ndarray:
    """Systematic code (Section 2.3 mentions a systematic version without
    giving it; this is the construction used here): a block's Q data lines
    are stored as they are, and m parity projections along (p, 1) for p in
    ``parity_dirs`` are stored beside them.  Returns the parity pool
    (nblocks, sum B_i); the data lines are ``images`` themselves."""
    return encode_blocks(images, P, Q, parity_dirs)


def decode_blocks_sys(images: np.ndarray, parity: np.ndarray, erased: np.ndarray, P: int,
                      Q: int, parity_dirs, return_rc: bool = False):
    """Rebuild each block of the systematic code.  Packet i < Q is data line
    i, packet Q + j parity projection j; bit i of ``erased[b]`` set = packet i
    of block b lost (its contents are ignored).  The surviving lines are
    pixels known in advance; the peeling of Section 2.2 finds the others from
    the surviving parity projections.  Returns the images (and, with
    ``return_rc``, the per-block status: OK or ENOTRECON)."""
    img = np.ascontiguousarray(images, dtype=np.uint64).reshape(-1, Q, P)
    m = len(parity_dirs)
    words = block_stride(P, Q, parity_dirs)
    par = np.ascontiguousarray(parity, dtype=np.uint64).reshape(-1, words)
    er = np.ascontiguousarray(erased, dtype=np.uint16).reshape(-1)
    sizes = [proj_size(int(p), 1, P, Q) for p in parity_dirs]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    out = np.zeros_like(img)
    rcs = np.zeros(er.shape[0], dtype=np.int32)
    lib = _load()
    for b in range(er.shape[0]):
        mask = int(er[b])
        known = np.zeros((Q, P), dtype=np.uint8)
        cur = np.zeros((Q, P), dtype=np.uint64)
        for r in range(Q):
            if not (mask >> r) & 1:
                known[r] = 1
                cur[r] = img[b, r]
        alive = [j for j in range(m) if not (mask >> (Q + j)) & 1]
        p = np.ascontiguousarray([int(parity_dirs[j]) for j in alive], dtype=np.int32)
        q = np.ones(len(alive), dtype=np.int32)
        off = np.ascontiguousarray([offs[j] for j in alive], dtype=np.int64)
        row = np.ascontiguousarray(par[b])
        rc = lib.orc_inverse_known(XOR, 0, _ptr(row), _ptr(off), _ptr(p), _ptr(q), len(alive),
                                   P, Q, _ptr(known), _ptr(cur), 0, None)
        if rc not in (OK, ENOTRECON):
            raise ValueError(f"orc_inverse_known failed on block {b}: {rc}")
        rcs[b] = rc
        out[b] = cur
    return (out, rcs) if return_rc else out
