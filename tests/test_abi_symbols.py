"""The C-ABI library loads without a GPU and exports every function declared in include/ndtm.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ndtm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ndtm_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("ndtm_create", "ndtm_set_gauge", "ndtm_set_params", "ndtm_set_shifts", "ndtm_apply",
              "ndtm_mg_setup", "ndtm_solve", "ndtm_workspace_bytes", "ndtm_set_workspace"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_1805_09584_amd", "libndtm.so")
    if not os.path.exists(path):
        pytest.fail("libndtm.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
