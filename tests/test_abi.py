"""C-ABI library checks that need no GPU: it loads, exports every declared
symbol, and its host-only geometry calls and argument checks behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(mojette_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not os.path.exists(mj.LIB_PATH):
        from paper_1504_07038_amd import build

        build.build()
    return mj


def test_every_declared_symbol_is_exported(mj):
    L = mj.lib()
    decl = declared_functions()
    assert len(decl) >= 11
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(mj.exported_symbols()) == decl


def test_proj_size_and_offset_match_eq2(mj):
    for P in (1, 3, 128, 256):
        for Q in (1, 4, 8, 12):
            for p in range(-8, 9):
                assert mj.mojette_proj_size(p, P, Q) == abs(p) * (Q - 1) + P
                assert mj.mojette_bin_offset(p, P, Q) == min(
                    -k + l * p for k in (0, P - 1) for l in (0, Q - 1))
    assert mj.mojette_block_words([-3, -2, -1, 0, 1, 2], 128, 4) == 795
    assert mj.mojette_block_words([-8 + i for i in range(16)], 128, 12) == 16 * 128 + 11 * 64


def test_decode_ring_is_power_of_two_and_covers_every_survivor_set(mj):
    for dirs, Q in [([-3, -2, -1, 0, 1, 2], 4), (list(range(-6, 6)), 8), (list(range(-4, 5)), 6),
                    (list(range(-8, 8)), 12), ([5, -1, 3], 2), ([0], 1)]:
        R = mj.mojette_decode_ring(dirs, 128, Q)
        assert R >= 16 and R & (R - 1) == 0


def test_argument_errors_before_any_launch(mj):
    """Bad arguments are rejected on the host, before any HIP call."""
    L = mj.lib()
    dirs = (ctypes.c_int32 * 3)(-1, 0, 1)
    dup = (ctypes.c_int32 * 3)(-1, 0, -1)
    fake = ctypes.c_void_p(0x1000)
    outs = (ctypes.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    assert L.mojette_encode(None, 8, 2, dirs, 3, outs, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode(fake, 0, 2, dirs, 3, outs, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode(fake, 8, 0, dirs, 3, outs, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode(fake, 8, 17, dirs, 3, outs, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode(fake, 8, 2, dup, 3, outs, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode(fake, 8, 2, dirs, 17, outs, None) == mj.MOJETTE_EINVAL
    ids = (ctypes.c_int32 * 2)(0, 0)
    projs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    assert L.mojette_decode(projs, ids, 2, dirs, 3, 8, 2, fake, 0, None) == mj.MOJETTE_EINVAL
    ids2 = (ctypes.c_int32 * 2)(0, 3)
    assert L.mojette_decode(projs, ids2, 2, dirs, 3, 8, 2, fake, 0, None) == mj.MOJETTE_EINVAL
    ids3 = (ctypes.c_int32 * 1)(1)
    assert L.mojette_decode(projs, ids3, 1, dirs, 3, 8, 2, fake, 0, None) == mj.MOJETTE_ENOTRECON
    ids4 = (ctypes.c_int32 * 2)(0, 1)
    assert L.mojette_decode(projs, ids4, 2, dirs, 3, 8, 2, fake, 2, None) == mj.MOJETTE_EINVAL  # unknown flag
    assert L.mojette_encode_batch(fake, -1, 8, 2, dirs, 3, fake, None) == mj.MOJETTE_EINVAL
    assert L.mojette_encode_batch(fake, 0, 8, 2, dirs, 3, fake, None) == mj.MOJETTE_OK
    assert L.mojette_decode_batch(fake, None, 0, 8, 2, dirs, 3, fake, None, None) == mj.MOJETTE_OK
    assert L.mojette_decode_batch(fake, None, 5, 8, 2, dup, 3, fake, None, None) == mj.MOJETTE_EINVAL
    assert L.mojette_fill_splitmix64(None, 5, 1, 0, None) == mj.MOJETTE_EINVAL
    assert mj.strerror(mj.MOJETTE_ENOTRECON).startswith("fewer than Q")


def test_binding_refuses_host_tensors(mj):
    import torch

    img = torch.zeros(8, dtype=torch.int64)
    with pytest.raises(ValueError):
        mj.mojette_encode(img, 4, 2, [-1, 0, 1], [img, img, img])


def test_package_does_not_import_the_oracle():
    """The product package has no route to the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1504_07038_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "mojette_oracle" not in text and "liboracle" not in text, fn


def test_classes_layout_and_argument_errors(mj):
    spec = [(128, 4, [-3, -2, -1, 0, 1, 2], 10), (256, 8, list(range(-6, 6)), 3)]
    iw, pw = mj.mojette_classes_layout(spec)
    assert iw == 10 * 512 + 3 * 2048
    assert pw == 10 * 795 + 3 * mj.mojette_block_words(list(range(-6, 6)), 256, 8)
    L = mj.lib()
    arr, n = mj.make_classes([(128, 4, [-3, -3, 0, 1], 5)])   # duplicate direction
    assert L.mojette_classes_layout(arr, n, None, None) == mj.MOJETTE_EINVAL
    arr, n = mj.make_classes([(128, 4, [-3, -2, 0, 1], -1)])  # negative count
    assert L.mojette_classes_layout(arr, n, None, None) == mj.MOJETTE_EINVAL
    arr, n = mj.make_classes([(128, 4, [40000, -2, 0, 1], 1)])  # |p| too large for a class
    assert L.mojette_encode_classes(arr, n, 0x1000, 0x2000, None) == mj.MOJETTE_EINVAL
    arr, n = mj.make_classes([(8, 2, [0, 1], 1)] * 17)          # too many classes
    assert L.mojette_classes_layout(arr, 17, None, None) == mj.MOJETTE_EINVAL


def test_mixed_classes_recipe():
    import synth

    cl = synth.mixed_classes(10000, 4)
    assert len(cl) == 16 and sum(c[3] for c in cl) == 10000
    for P, Q, dirs, nb, size in cl:
        assert len(dirs) - Q in (2, 3, 4) and P * Q * 8 >= size > (P - 1) * Q * 8
        assert 10000 / 16 * 0.8 < nb < 10000 / 16 * 1.2


def test_one_hip_runtime_even_when_the_library_loads_first():
    """The binding loads torch before the library, so the library's HIP
    dependency resolves to torch's copy: one runtime per process, whichever
    of the two the caller touches first."""
    import subprocess
    import sys

    code = ("import paper_1504_07038_amd as mj; mj.mojette_block_words([0, 1], 8, 2); "
            "import torch; torch.zeros(1); print(len(mj._hip_runtimes_mapped()))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_decode_launch_plan_split_and_32bit_slices(mj):
    """A large batch of the (12,8) code is decoded in two ring classes (a
    short-ring launch, then the deep blocks gathered from ranges of 256
    blocks); when blocks are so long that 256 of them pass 32-bit byte
    offsets, the batch stays in one launch, which still addresses its own
    few blocks with 32-bit offsets."""
    dirs = list(range(-6, 6))
    two = mj.mojette_decode_batch_launches(dirs, 128, 8, 1 << 19)
    assert [m for _, _, m in two] == [1, 2]
    assert two[0][0] < two[1][0]                     # short ring first
    assert mj.mojette_decode_batch_launches(dirs, 128, 8, 64)[0][2] == 0   # small batch: one
    # 12P + 252 words per block slice: 256 slices pass 2^31 bytes from P = 87,361 on
    P = 90000
    assert 256 * mj.mojette_block_words(dirs, P, 8) * 8 >= 1 << 31
    one = mj.mojette_decode_batch_launches(dirs, P, 8, 1 << 19)
    assert len(one) == 1 and one[0][2] == 0
    assert one[0][1] * mj.mojette_block_words(dirs, P, 8) * 8 < 1 << 31
    # a wave slice of even a few blocks beyond 32-bit offsets is refused
    with pytest.raises(mj.MojetteError):
        mj.mojette_decode_batch_launches([-1, 0, 1], 1 << 28, 2, 4, 2)


def test_geometry_plan_argument_errors(mj):
    """mojette_plan_create checks every code on the host before it touches a
    device; the batched calls check their arguments before any launch."""
    L = mj.lib()
    h = ctypes.c_void_p(0)

    def create(geoms, tune=None):
        arr = (mj.MojetteGeom * max(1, len(geoms)))()
        for g, geo in enumerate(geoms):
            Q, dirs = geo[0], geo[1]
            arr[g].Q, arr[g].n = Q, len(dirs)
            arr[g].flags = geo[2] if len(geo) > 2 else 0
            for i, p in enumerate(dirs):
                arr[g].dirs[i] = p
        t = None
        if tune is not None:
            t = (mj.MojetteTune * len(geoms))()
            for g, d in enumerate(tune):
                for k, v in d.items():
                    setattr(t[g], k, v)
        return L.mojette_plan_create(arr, len(geoms), t, ctypes.addressof(h))

    assert create([]) == mj.MOJETTE_EINVAL
    assert create([(4, [-1, 0, 0, 2, 3])]) == mj.MOJETTE_EINVAL        # duplicate direction
    assert create([(4, [-1, 0, 1])]) == mj.MOJETTE_EINVAL              # n < Q
    assert create([(17, list(range(16)))]) == mj.MOJETTE_EINVAL         # Q > 16
    assert create([(2, [0, 40000])]) == mj.MOJETTE_EINVAL              # |p| too large
    assert create([(4, [-3, -2, -1, 0, 1, 2])], [{"encode_tile_cols": 100}]) == mj.MOJETTE_EINVAL
    assert create([(4, [-3, -2, -1, 0, 1, 2])], [{"decode_blocks_per_wave": -2}]) == mj.MOJETTE_EINVAL
    six = [-3, -2, -1, 0, 1, 2]
    assert create([(4, six, mj.GEOM_WIDE | mj.GEOM_TRIMMED)]) == mj.MOJETTE_EINVAL   # combined
    assert create([(4, six, 4)]) == mj.MOJETTE_EINVAL                              # unknown flag
    assert create([(2, [0, 20000], mj.GEOM_WIDE)]) == mj.MOJETTE_EINVAL             # 2|p| too large
    assert create([(4, six, mj.GEOM_TRIMMED)],
                  [{"decode_two_corner_min_P": 512}]) == mj.MOJETTE_EINVAL          # trimmed, both ends
    assert h.value is None
    assert L.mojette_workspace_size(None, 10) == -1
    fake = ctypes.c_void_p(0x1000)
    assert L.mojette_encode_batched(None, fake, 1, fake, fake, None, None) == mj.MOJETTE_EINVAL
    assert L.mojette_decode_batched(None, fake, 1, fake, fake, None, None) == mj.MOJETTE_EINVAL
    assert ctypes.sizeof(mj.MojetteGeom) == 76 and mj.block_dtype().itemsize == 24


def test_trimmed_layout_names_its_reconstruction_path(mj):
    text = open(os.path.join(ROOT, "include", "mojette.h")).read()
    val = int(re.search(r"#define MOJETTE_TRIMMED_PATH (\d+)", text).group(1))
    assert mj.mojette_trimmed_path() == val == mj.MOJETTE_TRIMMED_PATH
