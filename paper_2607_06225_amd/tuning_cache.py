"""Persisted autotuning results (a JSON file of tile choices).

An entry is keyed by what the choice depends on: the device (name and
architecture), the kernels (a hash of the loaded library's bytes, so that a
rebuilt library never reuses an old choice), the scoring scheme, the
alignment parameters and the batch's shape (pair count and length
quantiles rounded to two significant figures).  The stored value is the
context's tuning as ``Context.tuning()`` returns it.
"""
import hashlib
import json
import os
import tempfile

import numpy as np

_lib_hash = {}


def library_hash(path):
    """sha256 of the library file (hex, first 16 digits), cached per path."""
    if path not in _lib_hash:
        h = hashlib.sha256()
        with open(path, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _lib_hash[path] = h.hexdigest()[:16]
    return _lib_hash[path]


def _sig2(x):
    """x rounded to two significant figures (0 stays 0)."""
    x = float(x)
    if x == 0:
        return 0.0
    return float(f"{x:.2g}")


def shape_signature(q_len, r_len):
    q = np.asarray(q_len, dtype=np.int64)
    r = np.asarray(r_len, dtype=np.int64)
    out = [int(q.size)]
    for a in (q, r):
        if a.size:
            out += [_sig2(np.min(a)), _sig2(np.median(a)), _sig2(np.max(a))]
        else:
            out += [0.0, 0.0, 0.0]
    return out


def make_key(lib_path, device, matrix, gap_open, gap_extend, mode, prune, band_w, xdrop, width,
             want_cigar, q_len, r_len):
    sc = hashlib.sha256(np.ascontiguousarray(matrix, dtype=np.int32).tobytes())
    sc.update(f"{int(gap_open)},{int(gap_extend)}".encode())
    fields = dict(device=str(device), lib=library_hash(lib_path), scoring=sc.hexdigest()[:16],
                  params=[int(mode), int(prune), int(band_w), int(xdrop), int(width),
                          int(bool(want_cigar))],
                  shape=shape_signature(q_len, r_len))
    return json.dumps(fields, sort_keys=True)


def load(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def lookup(path, key):
    return load(path).get(key)


def store(path, key, tuning):
    """Add (or replace) one entry; the file is rewritten atomically."""
    data = load(path)
    data[key] = tuning
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning-", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, sort_keys=True, indent=1)
    os.replace(tmp, path)
