"""The C-ABI library: it loads without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aboria.h")
LIB = os.path.join(ROOT, "paper_1704_08907_amd", "libaboria_mi355x.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:aboria_status|const char\*|int32_t)\s+(aboria_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("aboria_build_cells", "aboria_pair_sum", "aboria_pair_sum_backward", "aboria_dense_sum"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1704_08907_amd import _native
    assert sorted(_native.EXPORTS) == declared()


def test_static_queries_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_1704_08907_amd import _native as N
    assert N.op_ny("spring", 3) == 3 and N.op_ny("soft_sphere", 3) == 1 and N.op_na("dem_spring") == 1
    assert N.lib().aboria_op_ny(99, 3) == -1 and N.lib().aboria_op_ny(1, 4) == -1
    assert N.variant_count() >= 1 and N.variant_name(0)
