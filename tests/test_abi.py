"""The C-ABI library loads and exports every entry point include/fe.h
declares (no GPU: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0905_2200_amd", "libfe.so")


def declared():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0905_2200_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("fe_create", "fe_destroy", "fe_sync", "fe_count", "fe_count_two_pass",
                 "fe_mine", "fe_result_free", "fe_last_error", "fe_validate"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_0905_2200_amd import fe
    assert set(fe.EXPORTS) <= set(declared())
