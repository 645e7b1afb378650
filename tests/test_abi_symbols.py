"""The C-ABI library loads on a machine without a GPU and exports every
function that include/smrt.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smrt.h")
LIB = os.path.join(ROOT, "paper_2504_21784_amd", "libsmrt.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smrt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("smrt_create", "smrt_destroy", "smrt_sweep", "smrt_compute_closures", "smrt_lo_solve", "smrt_step",
              "smrt_set_state", "smrt_get_state", "smrt_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsmrt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsmrt.so not built")
def test_binding_signatures_cover_header():
    from paper_2504_21784_amd import smrt
    assert set(declared_functions()) <= set(smrt._SIGS), set(declared_functions()) - set(smrt._SIGS)
    smrt.load()
