"""The C-ABI library loads on a machine without a GPU and exports every entry point declared in
include/calib.h (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "calib.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:calib_status|void|const char\s*\*)\s*\*?\s*([a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("calib_init", "admm_local_step", "admm_consensus_update", "admm_solve", "calib_get",
              "calib_set_jones", "calib_destroy", "calib_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1502_00858_amd import build
    if not os.path.exists(build.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(build.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_lists_every_declared_symbol():
    from paper_1502_00858_amd import calib
    assert sorted(calib.EXPORTS) == sorted(n for n in _declared())
