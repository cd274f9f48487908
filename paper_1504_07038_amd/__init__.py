"""Python binding of ``libmojette.so`` (Mojette erasure code on MI355X / gfx950).

Argument marshalling only: every step of encode and decode runs in the HIP
kernels behind the C ABI declared in ``include/mojette.h``.  PyTorch supplies
device memory (``torch.int64`` tensors carry the 64-bit pixel and bin words
bit for bit) and the current HIP stream.  If the library is not built, every
call raises: there is no CPU fallback.

Paper: Pertin, Feron, Van Kempen, Parrein, arXiv 1504.07038 -- Section 2.1
(forward transform, Eq. 1-2), Section 2.2 (inverse, Eq. 3), Section 2.3 (the
erasure code: k data lines, n projections with q_i = 1).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmojette.so")

MOJETTE_OK = 0
MOJETTE_EINVAL = -1
MOJETTE_ENOTRECON = -2
MOJETTE_EHIP = -3
MOJETTE_ENOMEM = -4
MOJETTE_EINCONSISTENT = -5
MOJETTE_ENOTSUP = -6
MOJETTE_ESCRATCH = -7
MOJETTE_SCRATCH_WORDS = 1 << 23
MOJETTE_VERIFY = 1
MOJETTE_TRIMMED_PATH = 1   # reconstruction path the trimmed layout is tied to
GEOM_WIDE = 1      # mojette_geom.flags: 128-bit pixels and bins
GEOM_TRIMMED = 2   # mojette_geom.flags: never-used bins left out
MAX_DIRS = 16
MAX_ROWS = 16


MAX_CLASSES = 16


class MojetteClass(ctypes.Structure):
    """``mojette_class``: nblocks blocks of one geometry in a mixed batch."""

    _fields_ = [("P", ctypes.c_int32), ("Q", ctypes.c_int32), ("n", ctypes.c_int32),
                ("dirs", ctypes.c_int32 * MAX_DIRS), ("nblocks", ctypes.c_int64)]


def make_classes(classes):
    """``classes``: iterable of (P, Q, dirs, nblocks) -> ctypes array."""
    classes = list(classes)
    arr = (MojetteClass * max(1, len(classes)))()
    for c, (P, Q, dirs, nb) in enumerate(classes):
        arr[c].P, arr[c].Q, arr[c].n, arr[c].nblocks = int(P), int(Q), len(dirs), int(nb)
        for i, p in enumerate(dirs):
            arr[c].dirs[i] = int(p)
    return arr, len(classes)


class MojetteJob(ctypes.Structure):
    """``mojette_job``: one geometry class with its own device buffers."""

    _fields_ = [("P", ctypes.c_int32), ("Q", ctypes.c_int32), ("n", ctypes.c_int32),
                ("dirs", ctypes.c_int32 * MAX_DIRS), ("nblocks", ctypes.c_int64),
                ("images", ctypes.c_void_p), ("projs", ctypes.c_void_p),
                ("slots", ctypes.c_void_p), ("erased", ctypes.c_void_p),
                ("plan", ctypes.c_void_p), ("workspace", ctypes.c_void_p)]


def make_jobs(jobs):
    """``jobs``: iterable of dicts with P, Q, dirs, nblocks, images, projs and
    optional slots (int64 device tensor), erased (int16 device tensor), plan
    (a ``ChunkPlan``) and workspace (int64 device tensor)."""
    jobs = list(jobs)
    arr = (MojetteJob * max(1, len(jobs)))()
    for c, j in enumerate(jobs):
        a = arr[c]
        a.P, a.Q, a.n, a.nblocks = int(j["P"]), int(j["Q"]), len(j["dirs"]), int(j["nblocks"])
        for i, p in enumerate(j["dirs"]):
            a.dirs[i] = int(p)
        a.images = _word_tensor(j["images"], "images")
        a.projs = _word_tensor(j["projs"], "projs")
        sl = j.get("slots")
        if sl is not None:
            import torch

            if sl.dtype != torch.int64:
                raise ValueError("slots must be int64")
        a.slots = _dev_ptr(sl, "slots")
        a.erased = _dev_ptr(j.get("erased"), "erased")
        plan = j.get("plan")
        a.plan = plan.handle if plan is not None else None
        ws = j.get("workspace")
        a.workspace = _word_tensor(ws, "workspace") if ws is not None else None
    return arr, len(jobs)


class MojetteGeom(ctypes.Structure):
    """``mojette_geom``: one code (Q rows, n directions) of a plan."""

    _fields_ = [("Q", ctypes.c_int32), ("n", ctypes.c_int32), ("dirs", ctypes.c_int32 * MAX_DIRS),
                ("flags", ctypes.c_uint32)]


class MojetteTune(ctypes.Structure):
    """``mojette_tune``: the schedule of one code (zero: the library's choice)."""

    _fields_ = [("decode_blocks_per_wave", ctypes.c_int32), ("decode_ring_split", ctypes.c_int32),
                ("encode_tile_cols", ctypes.c_int32),
                ("decode_two_corner_min_P", ctypes.c_int32)]


def block_dtype():
    """numpy dtype of ``mojette_block`` (24 bytes)."""
    import numpy as np

    return np.dtype([("image_off", "<u8"), ("proj_off", "<u8"), ("P", "<u4"),
                     ("geom_id", "<u2"), ("erasure_mask", "<u2")])


def make_blocks(image_off, proj_off, P, geom_id, erasure_mask=None):
    """Descriptors from per-block arrays -> a uint8 torch tensor on the device
    (nblocks x 24 bytes) ready for the batched calls."""
    import numpy as np
    import torch

    n = len(P)
    arr = np.zeros(n, dtype=block_dtype())
    arr["image_off"] = image_off
    arr["proj_off"] = proj_off
    arr["P"] = P
    arr["geom_id"] = geom_id
    if erasure_mask is not None:
        arr["erasure_mask"] = erasure_mask
    return torch.from_numpy(arr.view(np.uint8).copy()).to("cuda")


class MojetteError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = f"{where}: {strerror(status)} ({status})"
        if status == MOJETTE_EHIP:
            msg += f": {lib().mojette_last_hip_error().decode()}"
        super().__init__(msg)
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library, raising if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname as the system one.
    # Loading torch first makes the library's libamdhip64 dependency resolve
    # to that copy, so the process has ONE runtime and torch's streams and
    # allocations are valid handles for the library.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process: " + ", ".join(runtimes))
    i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "mojette_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "mojette_last_hip_error": ([], ctypes.c_char_p),
        "mojette_proj_size": ([i32, i32, i32], i64),
        "mojette_bin_offset": ([i32, i32, i32], i64),
        "mojette_block_words": ([vp, i32, i32, i32], i64),
        "mojette_decode_ring": ([vp, i32, i32, i32], i32),
        "mojette_encode": ([vp, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_decode": ([vp, vp, i32, vp, i32, i32, i32, vp, ctypes.c_uint32, vp], ctypes.c_int),
        "mojette_encode_wide": ([vp, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_decode_wide": ([vp, vp, i32, vp, i32, i32, i32, vp, ctypes.c_uint32, vp],
                                ctypes.c_int),
        "mojette_encode_trimmed": ([vp, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_decode_trimmed": ([vp, vp, i32, vp, i32, i32, i32, vp, ctypes.c_uint32, vp],
                                   ctypes.c_int),
        "mojette_encode_batch": ([vp, i64, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_decode_batch": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, vp], ctypes.c_int),
        "mojette_encode_batch_wide": ([vp, i64, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_verify_batch": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, vp], ctypes.c_int),
        "mojette_trimmed_layout": ([vp, i32, i32, i32, vp, vp], i64),
        "mojette_trimmed_path": ([], i32),
        "mojette_encode_batch_sys": ([vp, i64, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_sys_workspace": ([vp, i32, i32, i32, i64], i64),
        "mojette_decode_batch_sys": ([vp, vp, vp, i64, i32, i32, vp, i32, vp, vp, vp],
                                     ctypes.c_int),
        "mojette_encode_batch_trimmed": ([vp, i64, i32, i32, vp, i32, vp, vp], ctypes.c_int),
        "mojette_decode_batch_trimmed": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, vp],
                                         ctypes.c_int),
        "mojette_decode_batch_wide": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, vp],
                                      ctypes.c_int),
        "mojette_decode_batch_tuned": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, i32, vp],
                                       ctypes.c_int),
        "mojette_decode_batch_two_corner": ([vp, vp, i64, i32, i32, vp, i32, vp, vp, i32, vp],
                                            ctypes.c_int),
        "mojette_decode_max_blocks_per_wave": ([vp, i32, i32, i32], i32),
        "mojette_decode_default_blocks_per_wave": ([vp, i32, i32, i32], i32),
        "mojette_decode_batch_launches": ([vp, i32, i32, i32, i64, i32, vp, vp, vp, i32], i32),
        "mojette_classes_layout": ([vp, i32, vp, vp], ctypes.c_int),
        "mojette_encode_classes": ([vp, i32, vp, vp, vp], ctypes.c_int),
        "mojette_decode_classes": ([vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "mojette_encode_jobs": ([vp, i32, vp], ctypes.c_int),
        "mojette_decode_jobs": ([vp, i32, vp, vp], ctypes.c_int),
        "mojette_chunk_plan_create": ([vp, i32, i32, i32, vp], ctypes.c_int),
        "mojette_chunk_plan_destroy": ([vp], ctypes.c_int),
        "mojette_chunk_matrix": ([vp, i32, i32, vp, vp, i64], i64),
        "mojette_decode_chunked_workspace": ([vp, i32, i64], i64),
        "mojette_decode_batch_chunked": ([vp, vp, vp, i64, i32, vp, vp, vp, vp], ctypes.c_int),
        "mojette_decode_batch_chunked_trimmed": ([vp, vp, vp, i64, i32, vp, vp, vp, vp],
                                                 ctypes.c_int),
        "mojette_chunk_plan_create_wide": ([vp, i32, i32, i32, vp], ctypes.c_int),
        "mojette_plan_create": ([vp, i32, vp, vp], ctypes.c_int),
        "mojette_plan_destroy": ([vp], ctypes.c_int),
        "mojette_workspace_size": ([vp, i64], i64),
        "mojette_encode_batched": ([vp, vp, i64, vp, vp, vp, vp], ctypes.c_int),
        "mojette_decode_batched": ([vp, vp, i64, vp, vp, vp, vp], ctypes.c_int),
        "mojette_decode_batch_chunked_noalloc": ([vp, vp, vp, i64, i32, vp, vp, vp],
                                                 ctypes.c_int),
        "mojette_mlp_params": ([i32, i32], i32),
        "mojette_mlp_forward": ([vp, i32, i32, vp, i64, vp, vp], ctypes.c_int),
        "mojette_mlp_grad_workspace": ([i32, i32, i64], i64),
        "mojette_mlp_grad": ([vp, i32, i32, vp, vp, i64, vp, vp, vp], ctypes.c_int),
        "mojette_mlp_adam": ([vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, i32, vp], ctypes.c_int),
        "mojette_fill_splitmix64": ([vp, i64, u64, u64, vp], ctypes.c_int),
        "mojette_copy_words": ([vp, vp, i64, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _hip_runtimes_mapped() -> list[str]:
    """Distinct libamdhip64 files mapped into this process (Linux)."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1]
                if "libamdhip64.so" in os.path.basename(path):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return sorted(found)


def exported_symbols() -> list[str]:
    return [
        "mojette_strerror", "mojette_last_hip_error", "mojette_proj_size",
        "mojette_bin_offset", "mojette_block_words", "mojette_decode_ring", "mojette_encode",
        "mojette_decode", "mojette_encode_batch", "mojette_decode_batch",
        "mojette_encode_batch_wide", "mojette_decode_batch_wide", "mojette_encode_wide",
        "mojette_decode_wide", "mojette_encode_trimmed", "mojette_decode_trimmed",
        "mojette_verify_batch",
        "mojette_trimmed_layout", "mojette_trimmed_path", "mojette_encode_batch_trimmed",
        "mojette_decode_batch_trimmed",
        "mojette_encode_batch_sys", "mojette_sys_workspace", "mojette_decode_batch_sys",
        "mojette_decode_batch_tuned", "mojette_decode_batch_two_corner",
        "mojette_decode_max_blocks_per_wave",
        "mojette_decode_default_blocks_per_wave", "mojette_decode_batch_launches",
        "mojette_classes_layout", "mojette_encode_classes", "mojette_decode_classes",
        "mojette_encode_jobs", "mojette_decode_jobs", "mojette_chunk_plan_create",
        "mojette_chunk_plan_destroy", "mojette_chunk_matrix", "mojette_decode_chunked_workspace",
        "mojette_chunk_plan_create_wide",
        "mojette_decode_batch_chunked", "mojette_decode_batch_chunked_trimmed",
        "mojette_decode_batch_chunked_noalloc",
        "mojette_plan_create", "mojette_plan_destroy", "mojette_workspace_size",
        "mojette_encode_batched", "mojette_decode_batched",
        "mojette_mlp_params", "mojette_mlp_forward",
        "mojette_mlp_grad_workspace", "mojette_mlp_grad", "mojette_mlp_adam",
        "mojette_fill_splitmix64", "mojette_copy_words",
    ]


# ---- marshalling helpers -------------------------------------------------

def _i32_array(values):
    vals = [int(v) for v in values]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals), len(vals)


def _dev_ptr(t, name: str) -> int:
    if t is None:
        return 0
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _word_tensor(t, name: str) -> int:
    import torch

    if t.dtype not in (torch.int64, torch.uint64):
        raise ValueError(f"{name} must hold 64-bit words (torch.int64)")
    return _dev_ptr(t, name)


def _stream(stream) -> int:
    if stream is not None:
        return int(stream)
    import torch

    return torch.cuda.current_stream().cuda_stream


def _check(rc: int, where: str, check: bool) -> int:
    if check and rc != MOJETTE_OK:
        raise MojetteError(rc, where)
    return rc


# ---- the C ABI, name for name -------------------------------------------

def strerror(status: int) -> str:
    return lib().mojette_strerror(status).decode()


mojette_strerror = strerror


def mojette_proj_size(p: int, P: int, Q: int) -> int:
    return int(lib().mojette_proj_size(p, P, Q))


def mojette_bin_offset(p: int, P: int, Q: int) -> int:
    return int(lib().mojette_bin_offset(p, P, Q))


def mojette_block_words(dirs, P: int, Q: int) -> int:
    arr, n = _i32_array(dirs)
    return int(lib().mojette_block_words(arr, n, P, Q))


def mojette_decode_ring(dirs, P: int, Q: int) -> int:
    arr, n = _i32_array(dirs)
    return int(lib().mojette_decode_ring(arr, n, P, Q))


def mojette_encode(image, P: int, Q: int, dirs, proj_out, stream=None, check: bool = True) -> int:
    arr, n = _i32_array(dirs)
    ptrs = (ctypes.c_void_p * max(1, len(proj_out)))(
        *[_word_tensor(t, "proj_out") for t in proj_out])
    rc = lib().mojette_encode(_word_tensor(image, "image"), P, Q, arr, n, ptrs, _stream(stream))
    return _check(rc, "mojette_encode", check)


def mojette_decode(proj, proj_ids, dirs, P: int, Q: int, image_out, stream=None,
                   check: bool = True, verify: bool = False) -> int:
    """One block from m >= Q projections; verify=True sets MOJETTE_VERIFY (the
    call then checks every given projection against the decoded image and
    waits for the verdict)."""
    return _decode_one("mojette_decode", proj, proj_ids, dirs, P, Q, image_out, stream,
                       check, verify)


def mojette_encode_wide(image, P: int, Q: int, dirs, proj_out, stream=None,
                        check: bool = True) -> int:
    """mojette_encode for 16-byte pixels: image of Q*P pixels of two words,
    proj_out[i] of 2*B_i words."""
    return _encode_one("mojette_encode_wide", image, P, Q, dirs, proj_out, stream, check)


def mojette_encode_trimmed(image, P: int, Q: int, dirs, proj_out, stream=None,
                           check: bool = True) -> int:
    """mojette_encode storing the kept bins only: proj_out[i] of count[i]
    words (mojette_trimmed_layout)."""
    return _encode_one("mojette_encode_trimmed", image, P, Q, dirs, proj_out, stream, check)


def mojette_decode_trimmed(proj, proj_ids, dirs, P: int, Q: int, image_out, stream=None,
                           check: bool = True, verify: bool = False) -> int:
    """mojette_decode from projections in the trimmed layout."""
    return _decode_one("mojette_decode_trimmed", proj, proj_ids, dirs, P, Q, image_out, stream,
                       check, verify)


def _encode_one(name, image, P, Q, dirs, proj_out, stream, check):
    arr, n = _i32_array(dirs)
    ptrs = (ctypes.c_void_p * max(1, len(proj_out)))(
        *[_word_tensor(t, "proj_out") for t in proj_out])
    rc = getattr(lib(), name)(_word_tensor(image, "image"), P, Q, arr, n, ptrs, _stream(stream))
    return _check(rc, name, check)


def mojette_decode_wide(proj, proj_ids, dirs, P: int, Q: int, image_out, stream=None,
                        check: bool = True, verify: bool = False) -> int:
    """mojette_decode for 16-byte pixels (layouts as mojette_encode_wide)."""
    return _decode_one("mojette_decode_wide", proj, proj_ids, dirs, P, Q, image_out, stream,
                       check, verify)


def _decode_one(name, proj, proj_ids, dirs, P, Q, image_out, stream, check, verify):
    arr, n = _i32_array(dirs)
    ids, m = _i32_array(proj_ids)
    ptrs = (ctypes.c_void_p * max(1, len(proj)))(*[_word_tensor(t, "proj") for t in proj])
    rc = getattr(lib(), name)(ptrs, ids, m, arr, n, P, Q, _word_tensor(image_out, "image_out"),
                              MOJETTE_VERIFY if verify else 0, _stream(stream))
    return _check(rc, name, check)


def mojette_encode_batch(images, nblocks: int, P: int, Q: int, dirs, projs, stream=None,
                         check: bool = True) -> int:
    arr, n = _i32_array(dirs)
    rc = lib().mojette_encode_batch(_word_tensor(images, "images"), nblocks, P, Q, arr, n,
                                    _word_tensor(projs, "projs"), _stream(stream))
    return _check(rc, "mojette_encode_batch", check)


def _decode_masks(erased, status):
    import torch

    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    return _dev_ptr(erased, "erased"), _dev_ptr(status, "status")


def mojette_decode_batch(projs, erased, nblocks: int, P: int, Q: int, dirs, images,
                         status=None, stream=None, check: bool = True) -> int:
    arr, n = _i32_array(dirs)
    er, st = _decode_masks(erased, status)
    rc = lib().mojette_decode_batch(_word_tensor(projs, "projs"), er, nblocks, P, Q, arr, n,
                                    _word_tensor(images, "images"), st, _stream(stream))
    return _check(rc, "mojette_decode_batch", check)


def mojette_verify_batch(projs, erased, nblocks: int, P: int, Q: int, dirs, images, status,
                         stream=None, check: bool = True) -> int:
    """Compare every surviving projection with the projection of ``images``;
    a difference stores MOJETTE_EINCONSISTENT to ``status``."""
    arr, n = _i32_array(dirs)
    er, st = _decode_masks(erased, status)
    rc = lib().mojette_verify_batch(_word_tensor(projs, "projs"), er, nblocks, P, Q, arr, n,
                                    _word_tensor(images, "images"), st, _stream(stream))
    return _check(rc, "mojette_verify_batch", check)


def mojette_encode_batch_wide(images, nblocks: int, P: int, Q: int, dirs, projs, stream=None,
                              check: bool = True) -> int:
    """128-bit pixels: ``images`` holds nblocks x Q x P pixels of two words each."""
    arr, n = _i32_array(dirs)
    rc = lib().mojette_encode_batch_wide(_word_tensor(images, "images"), nblocks, P, Q, arr, n,
                                         _word_tensor(projs, "projs"), _stream(stream))
    return _check(rc, "mojette_encode_batch_wide", check)


def mojette_decode_batch_wide(projs, erased, nblocks: int, P: int, Q: int, dirs, images,
                              status=None, stream=None, check: bool = True) -> int:
    """128-bit pixels: projections of two-word bins, images of two-word pixels."""
    arr, n = _i32_array(dirs)
    er, st = _decode_masks(erased, status)
    rc = lib().mojette_decode_batch_wide(_word_tensor(projs, "projs"), er, nblocks, P, Q, arr,
                                         n, _word_tensor(images, "images"), st, _stream(stream))
    return _check(rc, "mojette_decode_batch_wide", check)


def mojette_trimmed_path() -> int:
    """Number of the reconstruction path the trimmed layout follows in this
    library (a pool written by the trimmed calls decodes only with a library
    that returns the same number)."""
    return int(lib().mojette_trimmed_path())


def mojette_trimmed_layout(dirs, P: int, Q: int):
    """(block words, [(first kept bin index, count) per projection]) of the
    layout without never-used bins; raises on bad arguments."""
    arr, n = _i32_array(dirs)
    first = (ctypes.c_int64 * max(1, n))()
    count = (ctypes.c_int64 * max(1, n))()
    words = lib().mojette_trimmed_layout(arr, n, P, Q, first, count)
    if words < 0:
        raise MojetteError(MOJETTE_EINVAL, "mojette_trimmed_layout")
    return int(words), [(int(first[i]), int(count[i])) for i in range(n)]


def mojette_encode_batch_trimmed(images, nblocks: int, P: int, Q: int, dirs, projs, stream=None,
                                 check: bool = True) -> int:
    """Batched encode storing only the bins some reconstruction reads."""
    arr, n = _i32_array(dirs)
    rc = lib().mojette_encode_batch_trimmed(_word_tensor(images, "images"), nblocks, P, Q, arr,
                                            n, _word_tensor(projs, "projs"), _stream(stream))
    return _check(rc, "mojette_encode_batch_trimmed", check)


def mojette_decode_batch_trimmed(projs, erased, nblocks: int, P: int, Q: int, dirs, images,
                                 status=None, stream=None, check: bool = True) -> int:
    """Batched decode from projections in the trimmed layout."""
    arr, n = _i32_array(dirs)
    er, st = _decode_masks(erased, status)
    rc = lib().mojette_decode_batch_trimmed(_word_tensor(projs, "projs"), er, nblocks, P, Q,
                                            arr, n, _word_tensor(images, "images"), st,
                                            _stream(stream))
    return _check(rc, "mojette_decode_batch_trimmed", check)


def mojette_encode_batch_sys(images, nblocks: int, P: int, Q: int, pdirs, parity, stream=None,
                             check: bool = True) -> int:
    """Systematic code: the parity projections of each block's data lines."""
    arr, m = _i32_array(pdirs)
    rc = lib().mojette_encode_batch_sys(_word_tensor(images, "images"), nblocks, P, Q, arr, m,
                                        _word_tensor(parity, "parity"), _stream(stream))
    return _check(rc, "mojette_encode_batch_sys", check)


def mojette_sys_workspace(pdirs, P: int, Q: int, nblocks: int) -> int:
    arr, m = _i32_array(pdirs)
    return int(lib().mojette_sys_workspace(arr, m, P, Q, nblocks))


def mojette_decode_batch_sys(images, parity, erased, nblocks: int, P: int, Q: int, pdirs,
                             workspace=None, status=None, stream=None, check: bool = True) -> int:
    """Systematic code: rebuild every lost data line in place in ``images``
    (``workspace`` is unused and may be None)."""
    arr, m = _i32_array(pdirs)
    er, st = _decode_masks(erased, status)
    ws = _word_tensor(workspace, "workspace") if workspace is not None else None
    rc = lib().mojette_decode_batch_sys(_word_tensor(images, "images"),
                                        _word_tensor(parity, "parity"), er, nblocks, P, Q, arr,
                                        m, ws, st, _stream(stream))
    return _check(rc, "mojette_decode_batch_sys", check)


def mojette_decode_batch_tuned(projs, erased, nblocks: int, P: int, Q: int, dirs, images,
                               blocks_per_wave: int, status=None, stream=None,
                               check: bool = True) -> int:
    import torch

    arr, n = _i32_array(dirs)
    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    rc = lib().mojette_decode_batch_tuned(_word_tensor(projs, "projs"),
                                          _dev_ptr(erased, "erased"), nblocks, P, Q, arr, n,
                                          _word_tensor(images, "images"),
                                          _dev_ptr(status, "status"), blocks_per_wave,
                                          _stream(stream))
    return _check(rc, "mojette_decode_batch_tuned", check)


def mojette_decode_batch_two_corner(projs, erased, nblocks: int, P: int, Q: int, dirs, images,
                                    status=None, blocks_per_wave: int = 0, stream=None,
                                    check: bool = True) -> int:
    """mojette_decode_batch swept from both ends of every block (half the
    dependency chain, the same words)."""
    import torch

    arr, n = _i32_array(dirs)
    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    rc = lib().mojette_decode_batch_two_corner(_word_tensor(projs, "projs"),
                                               _dev_ptr(erased, "erased"), nblocks, P, Q, arr, n,
                                               _word_tensor(images, "images"),
                                               _dev_ptr(status, "status"), blocks_per_wave,
                                               _stream(stream))
    return _check(rc, "mojette_decode_batch_two_corner", check)


def mojette_decode_max_blocks_per_wave(dirs, P: int, Q: int) -> int:
    arr, n = _i32_array(dirs)
    return int(lib().mojette_decode_max_blocks_per_wave(arr, n, P, Q))


def mojette_decode_batch_launches(dirs, P: int, Q: int, nblocks: int, blocks_per_wave: int = 0):
    """The launches a batched decode makes, as (ring words, blocks per
    wavefront, mode) per launch; raises on a negative status."""
    arr, n = _i32_array(dirs)
    ring, blocks, mode = (ctypes.c_int32 * 4)(), (ctypes.c_int32 * 4)(), (ctypes.c_int32 * 4)()
    k = int(lib().mojette_decode_batch_launches(arr, n, P, Q, nblocks, blocks_per_wave, ring,
                                                blocks, mode, 4))
    _check(k if k < 0 else 0, "mojette_decode_batch_launches", True)
    return [(ring[t], blocks[t], mode[t]) for t in range(k)]


def mojette_decode_default_blocks_per_wave(dirs, P: int, Q: int) -> int:
    arr, n = _i32_array(dirs)
    return int(lib().mojette_decode_default_blocks_per_wave(arr, n, P, Q))


def mojette_classes_layout(classes) -> tuple[int, int]:
    """(image words, projection words) of a mixed batch."""
    arr, n = make_classes(classes)
    iw, pw = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().mojette_classes_layout(arr, n, ctypes.addressof(iw), ctypes.addressof(pw))
    _check(rc, "mojette_classes_layout", True)
    return int(iw.value), int(pw.value)


def mojette_encode_classes(classes, images, projs, stream=None, check: bool = True) -> int:
    arr, n = make_classes(classes)
    rc = lib().mojette_encode_classes(arr, n, _word_tensor(images, "images"),
                                      _word_tensor(projs, "projs"), _stream(stream))
    return _check(rc, "mojette_encode_classes", check)


def mojette_decode_classes(classes, projs, erased, images, status=None, stream=None,
                           check: bool = True) -> int:
    import torch

    arr, n = make_classes(classes)
    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    rc = lib().mojette_decode_classes(arr, n, _word_tensor(projs, "projs"),
                                      _dev_ptr(erased, "erased"), _word_tensor(images, "images"),
                                      _dev_ptr(status, "status"), _stream(stream))
    return _check(rc, "mojette_decode_classes", check)


def mojette_encode_jobs(jobs, stream=None, check: bool = True) -> int:
    arr, n = make_jobs(jobs)
    rc = lib().mojette_encode_jobs(arr, n, _stream(stream))
    return _check(rc, "mojette_encode_jobs", check)


def mojette_decode_jobs(jobs, status=None, stream=None, check: bool = True) -> int:
    import torch

    arr, n = make_jobs(jobs)
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    rc = lib().mojette_decode_jobs(arr, n, _dev_ptr(status, "status"), _stream(stream))
    return _check(rc, "mojette_decode_jobs", check)


class ChunkPlan:
    """``mojette_chunk_plan``: transfer matrices of the chunked decode for one code
    (directions, Q) and one chunk length.  Creating it allocates device memory
    and synchronises; ``close()`` (or garbage collection) frees it."""

    def __init__(self, dirs, Q: int, chunk_cols: int, wide: bool = False):
        """wide=True: a plan for 128-bit pixels (mojette_chunk_plan_create_wide)."""
        arr, n = _i32_array(dirs)
        h = ctypes.c_void_p(0)
        name = "mojette_chunk_plan_create" + ("_wide" if wide else "")
        rc = getattr(lib(), name)(arr, n, Q, chunk_cols, ctypes.addressof(h))
        _check(rc, name, True)
        self.handle = h.value
        self.dirs, self.Q, self.chunk_cols = [int(p) for p in dirs], int(Q), int(chunk_cols)
        self.wide = bool(wide)

    def close(self) -> None:
        if self.handle:
            lib().mojette_chunk_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_words(self, P: int, nblocks: int) -> int:
        return int(lib().mojette_decode_chunked_workspace(self.handle, P, nblocks))


mojette_chunk_plan_create = ChunkPlan


def mojette_chunk_matrix(p_sorted, Q: int, chunk_cols: int):
    """(E, matrix rows as a (Q*E, ceil(Q*E/64)) uint64 array) of one survivor set."""
    import numpy as np

    arr, _ = _i32_array(p_sorted)
    E = ctypes.c_int32(0)
    need = int(lib().mojette_chunk_matrix(arr, Q, chunk_cols, ctypes.addressof(E), None, 0))
    if need < 0:
        raise MojetteError(MOJETTE_EINVAL if need == -1 else MOJETTE_ENOTSUP,
                           "mojette_chunk_matrix")
    rows = np.zeros(max(1, need), dtype=np.uint64)
    lib().mojette_chunk_matrix(arr, Q, chunk_cols, ctypes.addressof(E), rows.ctypes.data, need)
    d = Q * E.value
    rw = (d + 63) // 64
    return E.value, rows[:need].reshape(d, rw) if d else rows[:0].reshape(0, 0)


def mojette_decode_chunked_workspace(plan: ChunkPlan, P: int, nblocks: int) -> int:
    return plan.workspace_words(P, nblocks)


def mojette_decode_batch_chunked(plan: ChunkPlan, projs, erased, nblocks: int, P: int, images,
                                 workspace, status=None, stream=None, check: bool = True,
                                 trimmed: bool = False) -> int:
    """trimmed=True: projections in the layout without never-used bins
    (mojette_decode_batch_chunked_trimmed)."""
    import torch

    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    need = plan.workspace_words(P, nblocks)
    ws = 0
    if need > 0:
        if workspace is None or workspace.numel() < need:
            raise ValueError(f"workspace must hold {need} words")
        ws = _word_tensor(workspace, "workspace")
    name = "mojette_decode_batch_chunked" + ("_trimmed" if trimmed else "")
    rc = getattr(lib(), name)(plan.handle, _word_tensor(projs, "projs"),
                              _dev_ptr(erased, "erased"), nblocks, P,
                              _word_tensor(images, "images"), _dev_ptr(status, "status"), ws,
                              _stream(stream))
    return _check(rc, name, check)


def mojette_decode_batch_chunked_noalloc(plan: ChunkPlan, projs, erased, nblocks: int, P: int,
                                         images, status=None, stream=None,
                                         check: bool = True) -> int:
    """mojette_decode_batch_chunked with the library's fixed scratch memory
    as its workspace (no allocation; MOJETTE_ESCRATCH beyond
    MOJETTE_SCRATCH_WORDS words of workspace)."""
    import torch

    if erased is not None and erased.dtype not in (torch.int16, torch.uint16):
        raise ValueError("erased must be 16-bit masks")
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    rc = lib().mojette_decode_batch_chunked_noalloc(plan.handle, _word_tensor(projs, "projs"),
                                                    _dev_ptr(erased, "erased"), nblocks, P,
                                                    _word_tensor(images, "images"),
                                                    _dev_ptr(status, "status"), _stream(stream))
    return _check(rc, "mojette_decode_batch_chunked_noalloc", check)


class GeomPlan:
    """``mojette_plan``: the codes of the descriptor-driven batched calls and
    their schedules.  ``geoms``: list of (Q, dirs) or (Q, dirs, flags) with
    flags 0, GEOM_WIDE (128-bit pixels) or GEOM_TRIMMED (never-used bins
    left out); ``tune``: None or one dict per code with any of the
    ``mojette_tune`` fields.  Creating it allocates device memory and
    synchronises; ``close()`` (or garbage collection) frees it."""

    def __init__(self, geoms, tune=None):
        geoms = [tuple(g) if len(g) == 3 else (g[0], g[1], 0) for g in geoms]
        arr = (MojetteGeom * max(1, len(geoms)))()
        for g, (Q, dirs, flags) in enumerate(geoms):
            arr[g].Q, arr[g].n, arr[g].flags = int(Q), len(dirs), int(flags)
            for i, p in enumerate(dirs):
                arr[g].dirs[i] = int(p)
        tarr = None
        if tune is not None:
            tarr = (MojetteTune * max(1, len(geoms)))()
            for g, t in enumerate(tune):
                for k, v in (t or {}).items():
                    setattr(tarr[g], k, int(v))
        h = ctypes.c_void_p(0)
        rc = lib().mojette_plan_create(arr, len(geoms), tarr, ctypes.addressof(h))
        _check(rc, "mojette_plan_create", True)
        self.handle = h.value
        self.geoms = [(int(Q), [int(p) for p in dirs]) for Q, dirs, _ in geoms]
        self.flags = [int(f) for _, _, f in geoms]

    def close(self) -> None:
        if self.handle:
            lib().mojette_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, nblocks: int) -> int:
        return int(lib().mojette_workspace_size(self.handle, nblocks))

    def workspace(self, nblocks: int):
        import torch

        return torch.empty(max(1, self.workspace_bytes(nblocks)), dtype=torch.uint8, device="cuda")


mojette_plan_create = GeomPlan


def mojette_workspace_size(plan: GeomPlan, nblocks: int) -> int:
    return plan.workspace_bytes(nblocks)


def _desc_args(plan, blocks, nblocks, pool, workspace, status):
    import torch

    if blocks.dtype != torch.uint8 or blocks.numel() < 24 * nblocks:
        raise ValueError("blocks must be a uint8 tensor of nblocks descriptors (24 bytes each)")
    if workspace.dtype != torch.uint8 or workspace.numel() < plan.workspace_bytes(nblocks):
        raise ValueError(f"workspace must hold {plan.workspace_bytes(nblocks)} bytes")
    if status is not None and status.dtype != torch.int32:
        raise ValueError("status must be int32")
    return (plan.handle, _dev_ptr(blocks, "blocks"), nblocks, _word_tensor(pool, "pool"),
            _dev_ptr(workspace, "workspace"), _dev_ptr(status, "status"))


def mojette_encode_batched(plan: GeomPlan, blocks, nblocks: int, pool, workspace, status=None,
                           stream=None, check: bool = True) -> int:
    rc = lib().mojette_encode_batched(*_desc_args(plan, blocks, nblocks, pool, workspace, status),
                                      _stream(stream))
    return _check(rc, "mojette_encode_batched", check)


def mojette_decode_batched(plan: GeomPlan, blocks, nblocks: int, pool, workspace, status=None,
                           stream=None, check: bool = True) -> int:
    rc = lib().mojette_decode_batched(*_desc_args(plan, blocks, nblocks, pool, workspace, status),
                                      _stream(stream))
    return _check(rc, "mojette_decode_batched", check)


def _f32_tensor(t, name: str) -> int:
    import torch

    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    return _dev_ptr(t, name)


def mojette_mlp_params(d_in: int, hidden: int) -> int:
    return int(lib().mojette_mlp_params(d_in, hidden))


def mojette_mlp_forward(params, d_in: int, hidden: int, x, y, stream=None, check: bool = True):
    n = x.shape[0] if x.dim() > 1 else x.numel() // d_in
    rc = lib().mojette_mlp_forward(_f32_tensor(params, "params"), d_in, hidden,
                                   _f32_tensor(x, "x"), n, _f32_tensor(y, "y"), _stream(stream))
    return _check(rc, "mojette_mlp_forward", check)


def mojette_mlp_grad_workspace(d_in: int, hidden: int, n: int) -> int:
    return int(lib().mojette_mlp_grad_workspace(d_in, hidden, n))


def mojette_mlp_grad(params, d_in: int, hidden: int, x, t, grad, workspace, stream=None,
                     check: bool = True):
    n = t.numel()
    rc = lib().mojette_mlp_grad(_f32_tensor(params, "params"), d_in, hidden, _f32_tensor(x, "x"),
                                _f32_tensor(t, "t"), n, _f32_tensor(grad, "grad"),
                                _f32_tensor(workspace, "workspace"), _stream(stream))
    return _check(rc, "mojette_mlp_grad", check)


def mojette_mlp_adam(params, grad, m, v, lr: float, beta1: float, beta2: float, eps: float,
                     step: int, stream=None, check: bool = True):
    rc = lib().mojette_mlp_adam(_f32_tensor(params, "params"), _f32_tensor(grad, "grad"),
                                _f32_tensor(m, "m"), _f32_tensor(v, "v"), params.numel(), lr,
                                beta1, beta2, eps, step, _stream(stream))
    return _check(rc, "mojette_mlp_adam", check)


def mojette_fill_splitmix64(dst, nwords: int, seed: int, start: int = 0, stream=None,
                            check: bool = True) -> int:
    rc = lib().mojette_fill_splitmix64(_word_tensor(dst, "dst"), nwords,
                                       seed & 0xFFFFFFFFFFFFFFFF, start, _stream(stream))
    return _check(rc, "mojette_fill_splitmix64", check)


def mojette_copy_words(dst, src, nwords: int, stream=None, check: bool = True) -> int:
    rc = lib().mojette_copy_words(_word_tensor(dst, "dst"), _word_tensor(src, "src"), nwords,
                                  _stream(stream))
    return _check(rc, "mojette_copy_words", check)
