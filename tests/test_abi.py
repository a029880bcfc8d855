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


@pytest.mark.parametrize("rows,cols,code", [(26, 32, -2), (32, 26, -2), (384, 384, -2), (512, 512, -2),
                                            (4, 4, -2), (0, 8, -2), (8, 8, 0)])
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
    # overlapping out-of-place buffers
    assert lib.dct2d_transform_ex(0, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1100), 4, 8, 8, 64, 64, 0,
                                  None) == -1
    assert lib.dct2d_variant_count(26, 8, 0, 0) == 0
    assert lib.dct2d_get_variant(26, 8, 0, 0) == -2
    assert lib.dct2d_set_variant(8, 8, 0, 0, 99) == -1


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
