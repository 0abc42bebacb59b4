"""Autotune cache handling (host only)."""
import json

from paper_2504_17954_amd import autotune as A


def test_corrupt_cache_falls_back(tmp_path):
    p = tmp_path / "cache.json"
    p.write_text("{not json")
    assert A.load_cache(str(p)) == {}
    p.write_text(json.dumps([1, 2, 3]))
    assert A.load_cache(str(p)) == {}


def test_store_and_validate(tmp_path):
    p = str(tmp_path / "c.json")
    A.store("k", dict(A.DEFAULT), p)
    assert A.load_cache(p)["k"] == A.DEFAULT
    assert A.valid(A.DEFAULT)
    for bad in ({**A.DEFAULT, "fwd_px": 3}, {**A.DEFAULT, "sort_chunk": -1}, {"fwd_px": 1}):
        assert not A.valid(bad)
    assert all(A.valid(c) for c in A.CANDIDATES)
