"""Build the gfx950 HIP library ``libmojette.so`` in-tree with hipcc.

Every source is compiled to an object in parallel, then the objects are
linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmojette.so")
SOURCES = ["api.hip", "chunk.hip", "encode.hip", "decode_single.hip", "decode_single_hi.hip",
           "decode_classes.hip", "decode_chunks.hip", "decode_sys.hip", "decode_sys_hi.hip",
           "decode_wide.hip", "mlp.hip", "synth.hip", "noalloc.hip", "batched.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # Packed FP32 arithmetic is kept out of generated code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


# Host code checked by AddressSanitizer and UndefinedBehaviorSanitizer (the
# device code is built as usual): a separate library for CPU-only checks,
# loaded with the sanitizer runtime preloaded.
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libmojette_san.so")
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    obj_dir, lib = (SAN_OBJ, SAN_LIB) if sanitize else (OBJ, LIB)
    flags = FLAGS + (SAN_FLAGS if sanitize else [])
    os.makedirs(obj_dir, exist_ok=True)
    objs = [os.path.join(obj_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC, *flags, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = lib + ".tmp"
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-shared-libsan"] if sanitize else []
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *link, *objs, "-o", tmp], verbose)
    os.replace(tmp, lib)
    return lib


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime the sanitized library links."""
    res = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                          "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        import glob

        cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        path = cands[-1] if cands else ""
    return path


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
