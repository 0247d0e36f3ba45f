"""Host-side checks of libdft3d.so that need no GPU: the library loads,
exports every function include/dft3d.h declares, validates arguments, and
plans schedules whose buffer chains are well formed."""
import ctypes
import os
import re

import pytest

from paper_1904_10119_amd import dft3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "dft3d.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dft3d_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = dft3d.lib()
    declared = header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(dft3d.EXPORTS) == declared


def test_status_strings():
    L = dft3d.lib()
    for st in range(0, -8, -1):
        s = L.dft3d_status_string(st)
        assert s and s != b"unknown status"
    assert L.dft3d_status_string(-99) == b"unknown status"


@pytest.mark.parametrize("shape", [(4, 0, 4), (8192, 2, 2), (4, 4, -2), (4097, 1, 1),
                                   (2, 5000, 3), (3, 3, 4099)])
def test_bad_sizes_rejected(shape):
    h = ctypes.c_void_p(1)
    st = dft3d.lib().dft3d_plan(*shape, 0, 0, ctypes.byref(h))
    assert st == dft3d.ERR_UNSUPPORTED_SIZE
    assert h.value is None
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe(shape)


def test_bad_enums_rejected():
    L = dft3d.lib()
    h = ctypes.c_void_p()
    assert L.dft3d_plan(8, 8, 8, 7, 0, ctypes.byref(h)) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_plan(8, 8, 8, 0, 5, ctypes.byref(h)) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_plan(8, 8, 8, 0, 0, None) == dft3d.ERR_INVALID_ARG
    # shuffled output is not offered by these schedules
    assert L.dft3d_plan_describe(8, 8, 8, 2, 1, None, None, 0, None, 0, None) == \
        dft3d.ERR_UNSUPPORTED_SCHEDULE
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((8, 8, 8), "slab", tile=3)


def test_null_handles_rejected():
    L = dft3d.lib()
    v = ctypes.c_int64()
    sz = ctypes.c_size_t()
    assert L.dft3d_plan_set_option(None, 1, 0) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_plan_get_option(None, 1, ctypes.byref(v)) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_workspace_size(None, ctypes.byref(sz)) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_execute(None, 1, 2, -1, None) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_execute_noalloc(None, 1, 2, -1, None) == dft3d.ERR_INVALID_ARG
    assert L.dft3d_destroy(None) == dft3d.OK
    assert L.dft3d_execute_batched(None, None, None, 0, -1, None) == dft3d.OK
    assert L.dft3d_execute_batched(None, None, None, 1, -1, None) == dft3d.ERR_INVALID_ARG


def test_no_device_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert dft3d.lib().dft3d_plan(64, 64, 64, 2, 0, ctypes.byref(h)) == \
        dft3d.ERR_NO_DEVICE
    assert h.value is None


SHAPES = [(1, 1, 1), (2, 4, 8), (64, 64, 64), (128, 64, 32), (1024, 1024, 1024),
          (2048, 1024, 512), (4096, 2, 16), (1, 4096, 1)]


def check_chain(d, shape):
    passes = d["passes"]
    assert passes, d
    n = shape[0] * shape[1] * shape[2]
    assert passes[0]["src"] == "in"
    assert passes[-1]["dst"] == "out"
    grouped = [p for p in passes if " group " in p["label"]]
    for axis in ("pencil2", "pencil1"):
        # grouped pencil passes: one block of planes each, together every point
        ps = [p for p in grouped if p["label"].startswith(axis)]
        assert not grouped or sum(p["pencils"] * p["n"] for p in ps) == n
    for i, p in enumerate(passes):
        assert p["dst"] != "in"
        if i and " group " in p["label"] and p["label"].startswith("pencil2"):
            assert p["src"] == "in"      # each group starts from the input
        elif i:
            assert p["src"] == passes[i - 1]["dst"]
        if p["src"] == p["dst"]:
            # only layout-preserving passes may run in place
            assert p["load"] == p["store"] and p["post_twiddle"] == 0
        assert p["threads"] <= 1024 and p["lds_bytes"] <= 160 * 1024
        # a fused plane pass covers plane_rows x n points per work item, a
        # fused two-axis volumetric pass n x n x tile points per workgroup
        if p["fused_axes"]:
            assert p["pencils"] * p["n"] * p["n"] * p["tile"] == n
        elif " group " not in p["label"]:
            assert p["pencils"] * p["n"] * max(1, p["plane_rows"]) == n
    uses_ws = any("ws" in (p["src"], p["dst"]) for p in passes)
    assert d["workspace_bytes"] == (8 * n if uses_ws else 0)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("schedule", ["auto", "slab", "pencil", "volumetric"])
def test_plan_chains_well_formed(shape, schedule):
    check_chain(dft3d.describe(shape, schedule), shape)


def test_pencil_is_three_rotating_passes():
    d = dft3d.describe((128, 64, 32), "pencil")
    assert [p["n"] for p in d["passes"]] == [32, 64, 128]
    assert all(p["load"] == "row" and p["store"] == "col" for p in d["passes"])


def test_slab_needs_no_workspace():
    d = dft3d.describe((1024, 1024, 1024), "slab")
    assert d["workspace_bytes"] == 0
    assert [p["n"] for p in d["passes"]] == [1024, 1024, 1024]


def test_volumetric_splits_every_axis():
    d = dft3d.describe((1024, 256, 64), "volumetric")
    ns = [p["n"] for p in d["passes"]]
    assert ns == [8, 8, 16, 16, 32, 32]
    assert [p["post_twiddle"] for p in d["passes"]] == [1, 0] * 3


def test_auto_splits_long_axes():
    # untuned auto splits only 4096-long axes; split_max lowers the bar
    # (unsplit, the 2048 array takes the cycled pencil order: axes 2, 0, 1)
    d = dft3d.describe((2048, 1024, 512), "auto")
    assert [p["n"] for p in d["passes"]] == [512, 2048, 1024]
    d = dft3d.describe((2048, 1024, 512), "auto", pencil_order=0)
    assert [p["n"] for p in d["passes"]] == [512, 1024, 2048]
    d = dft3d.describe((4096, 128, 64), "auto")
    assert [p["n"] for p in d["passes"]] == [64, 128, 64, 64]
    d = dft3d.describe((2048, 1024, 512), "auto", split_max=1024)
    assert [p["n"] for p in d["passes"]] == [512, 1024, 32, 64]


def test_auto_uses_slab_below_the_cache_size():
    # below 256 MiB: slab (planes up to 128 x 128 fused into one pass)
    d = dft3d.describe((64, 64, 64), "auto")
    assert d["schedule"] == "slab" and len(d["passes"]) == 2
    d = dft3d.describe((256, 256, 256), "auto")
    assert d["schedule"] == "slab" and len(d["passes"]) == 3
    d = dft3d.describe((4096, 8, 16), "auto")
    assert d["schedule"] == "slab"
    # from 256 MiB on: pencil
    assert dft3d.describe((512, 512, 128), "auto")["schedule"] == "pencil"
    assert dft3d.describe((1024, 1024, 1024), "auto")["schedule"] == "pencil"


def test_split_precision_uses_mfma_leaves_where_available():
    d = dft3d.describe((256, 256, 256), "pencil", precision="bf16x6")
    assert all(p["precision"] == dft3d.PRECISIONS["bf16x6"] for p in d["passes"])
    # lengths below 16 have no MFMA leaf and stay on FP32 butterflies (in
    # the rotation's pass order: axes 2, 1, 0)
    d = dft3d.describe((8, 256, 4), "pencil", precision="bf16x9", pencil_order=0)
    assert [p["precision"] for p in d["passes"]] == [0, dft3d.PRECISIONS["bf16x9"], 0]
    # four-step first halves (post twiddle) stay FP32
    d = dft3d.describe((2048, 1024, 512), "auto", precision="fp16x3", split_max=1024)
    assert [p["precision"] > 0 for p in d["passes"]] == [True, True, False, True]


def test_mfma_leaf_option():
    """DFT3D_OPT_MFMA_LEAF: 32 gives length-32 leaves where they are
    compiled (32^s r, r < 16), other lengths keep leaves of 16; FP32 plans
    ignore it; values other than 0, 16, 32 are rejected."""
    for n, want in ((32, [32]), (64, [32, 2]), (256, [32, 8]), (1024, [32, 32]),
                    (2048, [32, 32, 2]), (4096, [32, 32, 4])):
        d = dft3d.describe((4, 4, n), "pencil", precision="fp16x3", mfma_leaf=32)
        p = d["passes"][0]
        assert (p["n"], p["mfma_leaf"], p["radices"]) == (n, 32, want), p
    d = dft3d.describe((4, 4, 512), "pencil", precision="bf16x6", mfma_leaf=32)
    assert d["passes"][0]["mfma_leaf"] == 16 and d["passes"][0]["radices"] == [16, 16, 2]
    d = dft3d.describe((4, 4, 1024), "pencil", precision="bf16x6", mfma_leaf=16)
    assert d["passes"][0]["radices"] == [16, 16, 4]
    d = dft3d.describe((4, 4, 1024), "pencil", mfma_leaf=32)
    assert d["passes"][0]["mfma_leaf"] == 0
    for bad in (1, 8, 64, -1):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.describe((4, 4, 1024), "pencil", precision="bf16x6", mfma_leaf=bad)
