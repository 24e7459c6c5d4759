"""CPU-side checks of the C ABI: the library loads and exports every function
include/aln.h declares, and the binding's structs match the header's sizes.
No compute call is made (there may be no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2607_06225_amd import aln

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "aln.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aln_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert header_functions() == sorted(aln.EXPORTS)


@pytest.mark.skipif(not os.path.exists(aln.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(aln.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    lib.aln_abi_version.restype = ctypes.c_int32
    assert lib.aln_abi_version() == 1


def test_struct_layouts():
    assert aln.RESULT_DTYPE.itemsize == 48
    assert ctypes.sizeof(aln._Params) == 24
    assert ctypes.sizeof(aln._Footprint) == 32
    assert ctypes.sizeof(aln._Batch) == 56
    assert ctypes.sizeof(aln._Scoring) == 24


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(aln.AlnError):
        _load_missing(tmp_path)


def _load_missing(tmp_path):
    saved = aln._lib
    try:
        aln._lib = None
        aln.load_library(str(tmp_path / "nope.so"))
    finally:
        aln._lib = saved
