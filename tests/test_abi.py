"""The C ABI library loads on a machine without a GPU and exports every
function include/rel.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rel.h")
LIB = os.path.join(ROOT, "paper_2608_13696_amd", "librel.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:rel_status|const char\*)\s+(rel_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_operator_calls():
    names = declared_functions()
    for required in ("rel_filter_compact", "rel_join_build", "rel_join_probe", "rel_groupby_agg",
                     "rel_filter_join_agg", "rel_batch_create", "rel_batch_run"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librel.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librel.so not built")
def test_status_strings_without_a_device():
    lib = ctypes.CDLL(LIB)
    lib.rel_status_string.restype = ctypes.c_char_p
    assert lib.rel_status_string(0) == b"ok"
    assert lib.rel_status_string(3) == b"duplicate build key"
