"""CPU-only checks of the native library: it loads, exports every symbol that
include/mtp.h declares, and its basis enumeration (written separately from
the oracle's) gives the same basis in the same order."""
import ctypes
import os
import re

import pytest

from oracle import basis as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtp.h")


def _lib():
    from paper_2304_13144_amd import _lib
    try:
        return _lib.lib()
    except FileNotFoundError as e:
        pytest.fail(str(e))


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mtp_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_2304_13144_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_symbols()


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


@pytest.mark.parametrize("level", [2, 4, 6, 8, 12, 16])
def test_library_basis_equals_oracle_basis(level):
    from paper_2304_13144_amd import api
    lines = api.basis_describe(level)
    want = [str(b) for b in ob.basis(level)]
    assert lines == want


def test_describe_rejects_small_buffer():
    L = _lib()
    buf = ctypes.create_string_buffer(8)
    n = ctypes.c_int32()
    assert L.mtp_basis_describe(16, buf, len(buf), ctypes.byref(n)) == -1
    assert n.value == 92


def test_compiled_levels_cover_workloads():
    from paper_2304_13144_amd import api
    lv = api.compiled_levels()
    for L in (8, 16):
        assert L in lv


def test_row_stride_pads_to_the_grade_step():
    """The rows' column count the grade kernels read: m padded to a multiple
    of 32 (FP64 k chunks) or 64 (the int8 product's k step)."""
    from paper_2304_13144_amd import api
    assert [api.row_stride(m, "fp64") for m in (1, 32, 33, 212, 1114)] == [32, 32, 64, 224, 1120]
    assert [api.row_stride(m, "mixed") for m in (1, 64, 65, 212)] == [64, 64, 128, 256]
