"""The C-ABI library loads on the CPU host and exports every symbol that
include/gedmg.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_03411_amd", "libgedmg.so")
HDR = os.path.join(ROOT, "include", "gedmg.h")


def declared():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(gedmg_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("gedmg_create", "gedmg_destroy", "gedmg_assemble", "gedmg_newton_step", "gedmg_csr"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_match_header():
    from paper_2604_03411_amd import gedmg
    assert set(declared()) <= set(gedmg.EXPORTED)
