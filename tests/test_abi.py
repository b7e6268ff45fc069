"""CPU-side checks of the C ABI: the library loads, exports every entry point
include/ttr.h declares, and status strings work without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttr.h")
LIB = os.path.join(ROOT, "paper_2011_06532_amd", "libttr.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ttr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    syms = declared_symbols()
    for name in ["ttr_add", "ttr_hadamard", "ttr_dot", "ttr_norm", "ttr_orthogonalize", "ttr_round"]:
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libttr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libttr.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.ttr_status_string.restype = ctypes.c_char_p
    assert lib.ttr_status_string(0) == b"ok"
    assert lib.ttr_status_string(3) == b"output capacity too small"
    assert lib.ttr_status_string(99) == b"unknown status"


def test_binding_lists_header_symbols():
    from paper_2011_06532_amd import ttr
    assert sorted(ttr.SYMBOLS) == declared_symbols()
