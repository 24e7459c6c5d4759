"""The persisted tuning cache (host logic only): keys change with every input
a tile choice depends on, and entries survive a rewrite of the file."""
import json

import numpy as np

from paper_2607_06225_amd import tuning_cache as TC


def key(tmp_path, lib=b"lib-a", **over):
    libf = tmp_path / f"lib-{hash(lib) & 0xffff}.so"
    libf.write_bytes(lib)
    kw = dict(device="MI355X/gfx950", matrix=np.eye(4, dtype=np.int32) * 3 - 1, gap_open=-4,
              gap_extend=-2, mode=0, prune=0, band_w=0, xdrop=0, width=0, want_cigar=True,
              q_len=np.array([1000, 1010, 990]), r_len=np.array([1000, 1000, 1003]))
    kw.update(over)
    return TC.make_key(str(libf), **kw)


def test_key_depends_on_every_input(tmp_path):
    k0 = key(tmp_path)
    assert key(tmp_path) == k0
    assert key(tmp_path, lib=b"lib-b") != k0                      # rebuilt library
    assert key(tmp_path, device="other") != k0
    assert key(tmp_path, gap_open=-5) != k0
    assert key(tmp_path, matrix=np.eye(4, dtype=np.int32) * 2 - 1) != k0
    for f in ("mode", "prune", "band_w", "xdrop", "width"):
        assert key(tmp_path, **{f: 1}) != k0, f
    assert key(tmp_path, want_cigar=False) != k0
    assert key(tmp_path, q_len=np.array([1000, 1010, 990, 1000])) != k0  # pair count
    assert key(tmp_path, r_len=np.array([5000, 5000, 5000])) != k0
    # lengths within two significant figures share an entry
    assert key(tmp_path, q_len=np.array([1001, 1011, 991])) == k0


def test_store_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert TC.lookup(path, "k") is None
    TC.store(path, "k1", {"sw16_rows": 8})
    TC.store(path, "k2", {"sw16_rows": 12})
    TC.store(path, "k1", {"sw16_rows": 4})
    assert TC.lookup(path, "k1") == {"sw16_rows": 4}
    assert TC.lookup(path, "k2") == {"sw16_rows": 12}
    assert set(json.load(open(path))) == {"k1", "k2"}


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert TC.lookup(str(p), "k") is None
    TC.store(str(p), "k", {"x": 1})
    assert TC.lookup(str(p), "k") == {"x": 1}
