"""Host-only calls of the library built with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code (run by test_host_sanitized.py
in a process with the sanitizer runtime preloaded; no GPU is touched beyond
what a call does before its first device allocation).  ctypes only."""
import ctypes
import itertools
import sys

L = ctypes.CDLL(sys.argv[1])
i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


def arr(vals, t=ctypes.c_int32):
    return (t * max(1, len(vals)))(*vals)


def centered(n):
    return [i - n // 2 for i in range(n)]


L.mojette_block_words.restype = i64
L.mojette_trimmed_layout.restype = i64
L.mojette_chunk_matrix.restype = i64
L.mojette_decode_ring.restype = i32
L.mojette_decode_batch_launches.restype = i32
L.mojette_workspace_size.restype = i64
L.mojette_chunk_matrix.argtypes = [vp, i32, i32, vp, vp, i64]
L.mojette_decode_batch_launches.argtypes = [vp, i32, i32, i32, i64, i32, vp, vp, vp, i32]
L.mojette_trimmed_layout.argtypes = [vp, i32, i32, i32, vp, vp]
L.mojette_block_words.argtypes = [vp, i32, i32, i32]
L.mojette_decode_ring.argtypes = [vp, i32, i32, i32]

checked = 0
for n, Q in [(6, 4), (9, 6), (12, 8), (16, 12), (3, 2), (1, 1), (16, 16)]:
    d = arr(centered(n))
    for P in (1, 3, 64, 128, 1000, 1 << 20):
        assert L.mojette_block_words(d, n, P, Q) > 0
        first, count = arr([0] * n, ctypes.c_int64), arr([0] * n, ctypes.c_int64)
        assert L.mojette_trimmed_layout(d, n, P, Q, first, count) > 0
        R = L.mojette_decode_ring(d, n, P, Q)
        assert R >= 16
        ring, blocks, mode = arr([0] * 4), arr([0] * 4), arr([0] * 4)
        for nb in (1, 1000, 1 << 21):
            k = L.mojette_decode_batch_launches(d, n, P, Q, nb, 0, ring, blocks, mode, 4)
            assert k in (1, 2, -6), k
        checked += 1
    # transfer matrices of every survivor set of small codes (the host
    # symbolic sweep of the chunked decode)
    if n <= 9:
        for keep in itertools.combinations(range(n), Q):
            ps = arr(sorted(centered(n)[i] for i in keep))
            E = ctypes.c_int32(0)
            need = L.mojette_chunk_matrix(ps, Q, 128, ctypes.byref(E), None, 0)
            assert need >= 0 or need == -2, need     # -2: chunks that short cannot be interior
            if need <= 0:                            # 0: an empty state (one row)
                continue
            rows = (ctypes.c_uint64 * need)()
            assert L.mojette_chunk_matrix(ps, Q, 128, ctypes.byref(E), rows, need) == need
            checked += 1
# the chunk plan's threaded construction of every set's matrices runs on the
# host before its device upload (which fails without a GPU, or succeeds)
for n, Q, cols in [(6, 4, 256), (12, 8, 512), (9, 6, 128)]:
    h = ctypes.c_void_p(0)
    rc = L.mojette_chunk_plan_create(arr(centered(n)), n, Q, cols, ctypes.byref(h))
    assert rc in (0, -3), rc
    if rc == 0:
        L.mojette_chunk_plan_destroy(h)
    checked += 1
# the geometry plan's host checks and ring tables
class Geom(ctypes.Structure):
    _fields_ = [("Q", i32), ("n", i32), ("dirs", i32 * 16)]


geoms = (Geom * 4)()
for g, (k, m) in enumerate([(4, 2), (6, 3), (8, 4), (12, 4)]):
    geoms[g].Q, geoms[g].n = k, k + m
    for i, p in enumerate(centered(k + m)):
        geoms[g].dirs[i] = p
h = ctypes.c_void_p(0)
rc = L.mojette_plan_create(geoms, 4, None, ctypes.byref(h))
assert rc in (0, -3), rc
if rc == 0:
    assert L.mojette_workspace_size(h, 1000) > 0
    L.mojette_plan_destroy(h)
print(f"sanitized host calls: {checked} checks passed", flush=True)
