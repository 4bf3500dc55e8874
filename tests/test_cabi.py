"""The C-ABI library loads, exports every function include/ed.h declares, and
rejects invalid arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1004_3354_amd", "libedhip.so")
HDR = os.path.join(ROOT, "include", "ed.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ed_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libedhip.so not built")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_rejected(lib):
    lib.ed_last_error.restype = ctypes.c_char_p
    lib.ed_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ed_version()
    h = ctypes.c_void_p()
    for ns, a, b in [(0, 0, 0), (33, 1, 1), (8, 9, 0), (8, 0, -1)]:
        assert lib.ed_basis(ns, a, b, ctypes.byref(h)) == 1
        assert lib.ed_last_error()
    assert lib.ed_basis(4, 2, 2, None) == 1
    assert lib.ed_apply_H(None, None, None, None) == 1
    assert lib.ed_ham_create(None, None, 0, ctypes.byref(h)) == 1
    assert lib.ed_fill_random(None, 0, 1, 0, 0, None) == 0
    assert lib.ed_fill_random(None, 10, 1, 0, 0, None) == 1
    assert lib.ed_fill_random(None, 0, 1, 7, 0, None) == 1


def test_default_options(lib):
    from paper_1004_3354_amd import ed
    o = ed.options()
    # max_basis = 0: the basis is planned from the device memory (or the workspace)
    assert o.max_iter > 0 and o.max_basis == 0 and o.tol > 0 and o.reorth == 2
    assert ed.variant_count() >= 4
    assert all(ed.variant_name(v) for v in range(ed.variant_count()))
