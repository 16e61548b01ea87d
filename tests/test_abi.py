"""The C-ABI library loads without a GPU and exports every function that
include/ldgmg.h declares; the Python binding uses the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldgmg.h")
LIB = os.path.join(ROOT, "paper_2412_12506_amd", "libldgmg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ldgmg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("ldgmg_setup", "ldgmg_vcycle", "ldgmg_solve", "ldgmg_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libldgmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libldgmg.so not built")
def test_binding_covers_the_header():
    from paper_2412_12506_amd import ldgmg
    assert sorted(ldgmg.SYMBOLS) == declared()
    ldgmg.lib()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libldgmg.so not built")
def test_device_calls_without_upload_fail_cleanly():
    from paper_2412_12506_amd import ldgmg as L
    s = L.Solver(host_only=True, dim=2, n=4, p=1, smoother="jacobi")
    try:
        with pytest.raises(L.LdgmgError):
            L.ldgmg_vcycle(s.handle, 0, 0)
    finally:
        s.close()
