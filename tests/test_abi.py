"""CPU-side checks of the C ABI: the library loads and exports every function
include/aln.h declares, and the binding's structs match the header's sizes.
No compute call is made (there may be no GPU)."""
import ctypes
import os
import re
import subprocess

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
    assert ctypes.sizeof(aln._ServerCfg) == 32
    assert ctypes.sizeof(aln._Request) == 72
    assert ctypes.sizeof(aln._ServerStats) == 64
    assert aln.COMPLETION_DTYPE.itemsize == 104


STRUCTS = {
    "aln_scoring": aln._Scoring, "aln_params": aln._Params, "aln_batch": aln._Batch,
    "aln_footprint": aln._Footprint, "aln_server_cfg": aln._ServerCfg,
    "aln_request": aln._Request, "aln_server_stats": aln._ServerStats,
    "aln_tuning": aln._Tuning, "aln_fold_params": aln._FoldParams,
    "aln_fold_batch": aln._FoldBatch, "aln_launch_info": aln._LaunchInfo,
}
NUMPY_STRUCTS = {"aln_result": aln.RESULT_DTYPE, "aln_completion": aln.COMPLETION_DTYPE,
                 "aln_fold_result": aln.FOLD_RESULT_DTYPE, "aln_task_info": aln.TASK_INFO_DTYPE}


def test_header_layouts_match_the_binding(tmp_path):
    """Compile a probe against include/aln.h with the host C compiler and
    compare every struct's size and field offsets with the binding's."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aln.h"', "int main(void) {"]
    expect = {}
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        expect[cname] = ctypes.sizeof(cls)
        for fname, _ in cls._fields_:
            key = f"{cname}.{fname}"
            lines.append(f'printf("{key} %zu\\n", offsetof({cname}, {fname}));')
            expect[key] = getattr(cls, fname).offset
    for cname, dt in NUMPY_STRUCTS.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        expect[cname] = dt.itemsize
        for fname in dt.names:
            if cname == "aln_completion" and fname in aln.RESULT_DTYPE.names:
                key = f"{cname}.result.{fname}"
                expr = f"offsetof(aln_completion, result) + offsetof(aln_result, {fname})"
            else:
                key = f"{cname}.{fname}"
                expr = f"offsetof({cname}, {fname})"
            lines.append(f'printf("{key} %zu\\n", (size_t)({expr}));')
            expect[key] = dt.fields[fname][1]
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {k: int(v) for k, v in (ln.split() for ln in out.strip().splitlines())}
    assert got == expect


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
