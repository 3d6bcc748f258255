"""The C-ABI library loads and exports every function include/plds.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plds.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(plds_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("plds_create", "plds_batch_insert", "plds_batch_delete", "plds_update", "plds_coreness",
                 "plds_levels", "plds_destroy"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2106_03824_amd import plds
    if not os.path.exists(plds.LIB_PATH):
        pytest.fail("libplds.so not built")
    L = ctypes.CDLL(plds.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared()) == set(plds.EXPORTS)


def test_strerror_without_gpu():
    from paper_2106_03824_amd import plds
    assert plds.lib().plds_strerror(-2) == b"vertex id out of range"
