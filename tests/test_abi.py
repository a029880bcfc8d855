"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
and rejects bad arguments on the host before any device work (Section 7.1: non-power-
of-two axes are rejected rather than zero-padded)."""
import ctypes
import os
import re

import pytest

import paper_2609_28519_amd as dct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dct2d.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dct2d_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = dct.load()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), "missing export %s" % n
    assert set(names) == set(dct.EXPORTS)


def test_status_strings_and_version():
    assert dct.status_string(0) == "ok"
    assert "shape" in dct.status_string(-2)
    assert "gfx950" in dct.version()


@pytest.mark.parametrize("rows,cols,code", [(26, 32, -2), (32, 26, -2), (384, 384, -2), (512, 512, 0),
                                            (1024, 8, 0), (8, 1024, 0), (1024, 1024, 0), (2048, 8, -2),
                                            (8, 2048, -2), (4, 4, -2), (0, 8, -2), (8, 8, 0)])
def test_size_validation_on_host(rows, cols, code):
    lib = dct.load()
    # batch = 0 never touches the device: only validation runs
    assert lib.dct2d_forward(None, 0, rows, cols, rows * cols, None) == code


def test_argument_validation_on_host():
    lib = dct.load()
    assert lib.dct2d_forward(None, -1, 8, 8, 64, None) == -1          # negative batch
    assert lib.dct2d_forward(None, 0, 8, 8, 63, None) == -3           # stride < rows*cols
    assert lib.dct2d_transform_ex(5, None, None, 0, 8, 8, 64, 64, 0, None) == -1  # bad direction
    assert lib.dct2d_transform_ex(0, None, None, 0, 8, 8, 64, 64, 99, None) == -1  # bad precision
    assert lib.dct2d_forward(None, 3, 8, 8, 64, None) == -1           # null data with batch > 0
    assert lib.dct2d_forward(ctypes.c_void_p(0x1004), 3, 8, 8, 64, None) == -4   # misaligned
    assert lib.dct2d_forward(ctypes.c_void_p(0x1000), 3, 8, 8, 66, None) == -4   # stride % 4
    # in place (in == out) with different strides: array b would land on another array's input
    assert lib.dct2d_transform_ex(0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 3, 8, 8, 80, 64, 0,
                                  None) == -1
    # overlapping out-of-place buffers
    assert lib.dct2d_transform_ex(0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1100), 4, 8, 8, 64, 64, 0,
                                  None) == -1
    assert lib.dct2d_variant_count(26, 8, 0, 0) == 0
    # measurement helpers reject bad arguments before any launch
    assert lib.dct2d_fma_issue(None, 1, 1, None) == -1
    assert lib.dct2d_fma_issue(ctypes.c_void_p(0x1000), 0, 1, None) == -1
    assert lib.dct2d_fma_issue(ctypes.c_void_p(0x1002), 1, 1, None) == -4
    # axes of 512 and 1024: float32 path only; no variants, tuner or filter
    assert lib.dct2d_transform_ex(0, None, None, 0, 512, 512, 512 * 512, 512 * 512, 4, None) == -5
    assert lib.dct2d_transform_ex(1, None, None, 0, 1024, 64, 1024 * 64, 1024 * 64, 7, None) == 0
    assert lib.dct2d_variant_count(512, 512, 0, 0) == 0
    assert lib.dct2d_get_variant(1024, 8, 0, 0) == -2
    assert lib.dct2d_filter(None, None, 0, 512, 512, 512 * 512, 512 * 512, None, 0, None) == -2
    assert lib.dct2d_get_variant(26, 8, 0, 0) == -2
    assert lib.dct2d_set_variant(8, 8, 0, 0, 99) == -1


def test_image_transform_validation_on_host():
    """dct2d_image_transform(_noalloc) validate shapes and strides before any device work."""
    lib = dct.load()
    for fn in (lib.dct2d_image_transform, lib.dct2d_image_transform_noalloc):
        assert fn(0, None, None, 0, 600, 1000, 600000, 600000, None) == 0    # batch 0: no-op
        assert fn(0, None, None, 0, 384, 512, 384 * 512, 384 * 512, None) == 0
        assert fn(0, None, None, 0, 7, 8, 56, 56, None) == -2                # axis below 8
        assert fn(0, None, None, 0, 8, 1028, 8 * 1028, 8 * 1028, None) == -2  # axis above 1024
        assert fn(0, None, None, 0, 8, 10, 80, 80, None) == -2               # cols not a multiple of 4
        assert fn(0, None, None, 0, 600, 1000, 10, 10, None) == -3           # stride < rows*cols
        assert fn(3, None, None, 0, 8, 8, 64, 64, None) == -1                # direction
        assert fn(0, None, None, -1, 8, 8, 64, 64, None) == -1               # batch < 0
        assert fn(0, None, None, 2, 8, 8, 64, 64, None) == -1                # null with batch > 0
        a = ctypes.c_void_p(0x1000)
        assert fn(0, a, a, 3, 600, 1000, 600004, 600000, None) == -1          # in place, unequal strides
        assert fn(0, ctypes.c_void_p(0x1004), ctypes.c_void_p(0x900000), 2, 8, 8, 64, 64, None) == -4


def test_filter_validation_on_host():
    """dct2d_filter rejects bad arguments before any device work (fake device addresses)."""
    lib = dct.load()
    a = ctypes.c_void_p(0x100000)
    assert lib.dct2d_filter(None, None, 0, 8, 8, 64, 64, None, 0, None) == 0             # batch 0: no-op
    assert lib.dct2d_filter(None, None, 0, 26, 8, 208, 208, None, 0, None) == -2         # size
    assert lib.dct2d_filter(None, None, 0, 8, 8, 64, 64, None, -1, None) == -3           # lambda_stride < 0
    assert lib.dct2d_filter(None, None, 0, 8, 8, 64, 64, None, 10, None) == -3           # 0 < stride < 64
    assert lib.dct2d_filter(a, a, 3, 8, 8, 64, 64, None, 0, None) == -1                  # null lambda
    assert lib.dct2d_filter(a, a, 3, 8, 8, 64, 64, ctypes.c_void_p(0x200002), 0, None) == -4  # misaligned
    assert lib.dct2d_filter(a, a, 3, 8, 8, 64, 64, ctypes.c_void_p(0x100100), 0, None) == -1  # overlaps out
    assert lib.dct2d_filter(a, a, -1, 8, 8, 64, 64, ctypes.c_void_p(0x200000), 0, None) == -1  # batch < 0


def test_filter_policy_entry_on_host():
    """The filter's own policy entry (DCT2D_FILTER = 3): float32 only, starts as the round trip's."""
    lib = dct.load()
    fp32, bf16x6, auto = 0, 2, 7
    for n in (8, 64, 128, 256):
        assert lib.dct2d_variant_count(n, n, 3, fp32) == lib.dct2d_variant_count(n, n, 2, fp32) > 0
        assert lib.dct2d_variant_count(n, n, 3, bf16x6) == 0
        assert lib.dct2d_get_variant(n, n, 3, auto) == fp32
        assert lib.dct2d_get_variant(n, n, 3, fp32) == lib.dct2d_get_variant(n, n, 2, fp32)
    assert lib.dct2d_get_variant(8, 8, 3, bf16x6) == -5
    assert lib.dct2d_set_variant(8, 8, 3, bf16x6, 0) == -5
    assert lib.dct2d_set_variant(8, 8, 3, auto, bf16x6) == -5
    assert lib.dct2d_set_variant(8, 8, 3, auto, fp32) == 0
    keep = lib.dct2d_get_variant(8, 8, 3, fp32)
    assert lib.dct2d_set_variant(8, 8, 3, fp32, 5) == 0
    assert lib.dct2d_get_variant(8, 8, 3, fp32) == 5
    assert lib.dct2d_get_variant(8, 8, 2, fp32) != 5 or keep == 5  # the round trip's entry is separate
    assert lib.dct2d_set_variant(8, 8, 3, fp32, keep) == 0
    assert lib.dct2d_set_variant(8, 8, 3, fp32, 99) == -1
    assert lib.dct2d_tune(8, 8, 3, bf16x6, 64, None, None) == -5
    assert lib.dct2d_variant_count(8, 8, 4, fp32) == 0


def test_policy_save_and_load_round_trip(tmp_path):
    """The autotune cache (policy JSON) holds every direction, the filter's entry included,
    and loading it back reproduces it (host only)."""
    pol = dct.policy()
    assert "64x64/filter/fp32" in pol and pol["64x64/filter/auto"] == dct.FP32
    path = tmp_path / "pol.json"
    keep = dct.get_variant(32, 32, "filter", "fp32")
    try:
        dct.set_variant(32, 32, "filter", "fp32", (keep + 1) % dct.variant_count(32, 32, "filter", "fp32"))
        dct.save_policy(str(path))
        saved = dct.policy()
        dct.set_variant(32, 32, "filter", "fp32", keep)
        dct.load_policy(str(path))
        assert dct.policy() == saved
    finally:
        dct.set_variant(32, 32, "filter", "fp32", keep)
