"""ctypes front end of the C oracle (alnref.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  ``build()`` compiles the
shared library with gcc; ``align`` / ``align_batch`` marshal NumPy arrays into
the C calls and return plain Python values.
"""
import ctypes
import os
import subprocess

import numpy as np

GLOBAL, LOCAL, EXTEND = 0, 1, 2
FULL, BAND, XDROP, ZDROP = 0, 1, 2, 3
OK, UNREACHABLE, CIGAR_CAP, BAD_SYMBOL = 0, 1, 2, 3
OP_I, OP_D, OP_EQ, OP_X = 1, 2, 7, 8

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alnref.c")
_SRC_FOLD = os.path.join(_HERE, "foldref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class AlnrefOut(ctypes.Structure):
    _fields_ = [
        ("score", ctypes.c_int64),
        ("q_end", ctypes.c_int32),
        ("r_end", ctypes.c_int32),
        ("q_begin", ctypes.c_int32),
        ("r_begin", ctypes.c_int32),
        ("cells", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("cigar_len", ctypes.c_int32),
        ("span", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def build(force=True):
    """Compile liboracle.so (alignment and folding oracles) with gcc (plain
    -O2, no intrinsics)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.run(
        ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
         "-o", tmp, _SRC, _SRC_FOLD, "-lpthread"],
        check=True,
    )
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.alnref_align.argtypes = [P, i32, i32, i32, i32, i32, i32, i32,
                                 P, i32, P, i32, P, i32,
                                 ctypes.POINTER(AlnrefOut)]
    lib.alnref_align.restype = ctypes.c_int
    lib.alnref_align_batch.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32,
                                       P, P, P, P, P, P, P, P, P, P, i32]
    lib.alnref_align_batch.restype = ctypes.c_int
    lib.foldref_fold.argtypes = [P, i32, i32, i32, P, i32, P]
    lib.foldref_fold.restype = ctypes.c_int
    lib.foldref_fold_batch.argtypes = [P, i32, i32, i32, i32, P, P, P, P, i32]
    lib.foldref_fold_batch.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _u8(x):
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint8))


def decode_cigar(words):
    """CIGAR words (len << 4 | op) -> list of (op_char, len)."""
    ch = {OP_I: "I", OP_D: "D", OP_EQ: "=", OP_X: "X"}
    return [(ch[int(w) & 15], int(w) >> 4) for w in words]


def align(matrix, gap_open, gap_extend, q, r, mode=GLOBAL, prune=FULL,
          band_w=0, xdrop=0, want_cigar=False, cigar_cap=None):
    """Align one pair. Returns a dict with score, end/begin cells, cells,
    status and (if requested) the CIGAR words as a NumPy uint32 array."""
    lib = load()
    mat = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    alphabet = int(round(mat.size ** 0.5))
    assert alphabet * alphabet == mat.size
    qa, ra = _u8(q), _u8(r)
    M, N = int(qa.size), int(ra.size)
    cig = None
    cap = 0
    if want_cigar:
        cap = int(cigar_cap) if cigar_cap is not None else M + N + 1
        cig = np.zeros(max(cap, 1), dtype=np.uint32)
    out = AlnrefOut()
    lib.alnref_align(_ptr(mat), alphabet, int(gap_open), int(gap_extend),
                     int(mode), int(prune), int(band_w), int(xdrop),
                     _ptr(qa) if M else None, M, _ptr(ra) if N else None, N,
                     _ptr(cig), cap, ctypes.byref(out))
    res = dict(score=int(out.score), q_end=int(out.q_end), r_end=int(out.r_end),
               q_begin=int(out.q_begin), r_begin=int(out.r_begin),
               cells=int(out.cells), status=int(out.status), span=int(out.span))
    if want_cigar:
        res["cigar"] = cig[: out.cigar_len].copy()
    return res


def align_batch(matrix, gap_open, gap_extend, q, q_off, q_len, r, r_off, r_len,
                mode=GLOBAL, prune=FULL, band_w=0, xdrop=0, want_cigar=False,
                nthreads=None):
    """Align n pairs from concatenated code arrays on ``nthreads`` host threads.
    Returns a dict of NumPy arrays (score, q_end, r_end, q_begin, r_begin,
    cells, status, cigar_len) plus ``cigar`` / ``cigar_off`` when requested."""
    lib = load()
    mat = np.ascontiguousarray(np.asarray(matrix, dtype=np.int32))
    alphabet = int(round(mat.size ** 0.5))
    q = np.ascontiguousarray(q, dtype=np.uint8)
    r = np.ascontiguousarray(r, dtype=np.uint8)
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(r_off, dtype=np.int64)
    q_len = np.ascontiguousarray(q_len, dtype=np.int32)
    r_len = np.ascontiguousarray(r_len, dtype=np.int32)
    n = int(q_len.size)
    out = (AlnrefOut * max(n, 1))()
    cig = cig_off = cig_cap = None
    if want_cigar:
        cig_cap = (q_len.astype(np.int64) + r_len + 1).astype(np.int32)
        cig_off = np.zeros(n, dtype=np.int64)
        if n > 1:
            cig_off[1:] = np.cumsum(cig_cap[:-1], dtype=np.int64)
        cig = np.zeros(max(int(cig_cap.sum()), 1), dtype=np.uint32)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    rc = lib.alnref_align_batch(
        _ptr(mat), alphabet, int(gap_open), int(gap_extend), int(mode),
        int(prune), int(band_w), int(xdrop), n, _ptr(q), _ptr(q_off),
        _ptr(q_len), _ptr(r), _ptr(r_off), _ptr(r_len), _ptr(cig),
        _ptr(cig_off), _ptr(cig_cap), ctypes.cast(out, ctypes.c_void_p),
        int(nthreads))
    if rc != 0:
        raise RuntimeError(f"alnref_align_batch failed: {rc}")
    arr = np.frombuffer(out, dtype=np.dtype([
        ("score", np.int64), ("q_end", np.int32), ("r_end", np.int32),
        ("q_begin", np.int32), ("r_begin", np.int32), ("cells", np.int64),
        ("status", np.int32), ("cigar_len", np.int32), ("span", np.int32),
        ("reserved", np.int32)]), count=n)
    res = {k: np.array(arr[k]) for k in arr.dtype.names}
    if want_cigar:
        res["cigar"] = cig
        res["cigar_off"] = cig_off
    return res
