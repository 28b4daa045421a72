"""CPU checks of the C-ABI library: it loads, and exports every declared symbol."""
import ctypes
import os
import re

import pytest

from paper_2403_09158_amd import ec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ec_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(ec.EXPORTS)


@pytest.mark.skipif(not os.path.exists(ec.LIB_PATH), reason="libec.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(ec.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    ec.load()  # argtypes bind without error


def test_defect_record_layout():
    from paper_2403_09158_amd.inputs import DEFECT_DTYPE

    assert DEFECT_DTYPE.itemsize == 104
    assert DEFECT_DTYPE.fields["c"][1] == 8
    assert DEFECT_DTYPE.fields["eig_v"][1] == 96
    assert ctypes.sizeof(ec.CProblem) == 120
    assert ec.CProblem.frame.offset == 48
    from paper_2403_09158_amd.inputs import LINE_DTYPE

    assert LINE_DTYPE.itemsize == 56
    assert LINE_DTYPE.fields["axis"][1] == 24 and LINE_DTYPE.fields["b"][1] == 32
