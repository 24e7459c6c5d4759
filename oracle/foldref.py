"""ctypes front end of the folding oracle (foldref.c): Nussinov base-pair
maximisation, unpruned or with X-drop pruning transferred from alignment.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import ctypes
import os

import numpy as np

from .alnref import load, _ptr, _u8

# codes A, C, G, U = 0..3
A, C, G, U = 0, 1, 2, 3
NO_XDROP = -1


class FoldrefOut(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int64), ("i", ctypes.c_int32), ("j", ctypes.c_int32),
                ("cells", ctypes.c_int64), ("terms", ctypes.c_int64), ("full", ctypes.c_int32),
                ("status", ctypes.c_int32)]


FOLD_DTYPE = np.dtype([("score", np.int64), ("i", np.int32), ("j", np.int32),
                       ("cells", np.int64), ("terms", np.int64), ("full", np.int32),
                       ("status", np.int32)])
assert FOLD_DTYPE.itemsize == ctypes.sizeof(FoldrefOut)


def _pair(pair):
    p = np.ascontiguousarray(np.asarray(pair, dtype=np.int32).reshape(16))
    return p


def fold(pair, x, min_loop=0, xdrop=NO_XDROP, warmup=15):
    """Fold one sequence; returns a dict (score, i, j, cells, terms, full, status)."""
    lib = load()
    p = _pair(pair)
    xa = _u8(x)
    out = FoldrefOut()
    lib.foldref_fold(_ptr(p), int(min_loop), int(xdrop), int(warmup),
                     _ptr(xa) if xa.size else None, int(xa.size), ctypes.byref(out))
    return dict(score=int(out.score), i=int(out.i), j=int(out.j), cells=int(out.cells),
                terms=int(out.terms), full=int(out.full), status=int(out.status))


def fold_batch(pair, x, off, length, min_loop=0, xdrop=NO_XDROP, warmup=15, nthreads=None):
    """Fold n concatenated sequences on host threads; returns a structured array."""
    lib = load()
    p = _pair(pair)
    x = np.ascontiguousarray(x, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    length = np.ascontiguousarray(length, dtype=np.int32)
    n = int(length.size)
    out = (FoldrefOut * max(n, 1))()
    rc = lib.foldref_fold_batch(_ptr(p), int(min_loop), int(xdrop), int(warmup), n, _ptr(x),
                                _ptr(off), _ptr(length), ctypes.cast(out, ctypes.c_void_p),
                                int(nthreads or os.cpu_count() or 1))
    if rc != 0:
        raise RuntimeError(f"foldref_fold_batch failed: {rc}")
    return np.frombuffer(out, dtype=FOLD_DTYPE, count=n).copy()
