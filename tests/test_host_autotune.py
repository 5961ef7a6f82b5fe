"""Host side of the batch-shape autotuner (no GPU): the batch signature and
the JSON cache."""
import json

import pytest

autotune = pytest.importorskip("paper_1611_06115_amd.autotune")


def test_signature_buckets():
    a = autotune.signature([16, 20, 2000, 2040], [0, 8, 3, 4], 256_000_000)
    b = autotune.signature([17, 21, 1999, 2040], [0, 9, 4, 5], 257_000_000)
    assert a == b  # same buckets
    c = autotune.signature([16, 20, 2000, 2040], [0, 8, 3, 40], 256_000_000)
    assert a != c  # k bucket changed
    d = autotune.signature([16] * 8, [0] * 8, 256_000_000)
    assert d.startswith("c3,n27,") and "m4k0:1" in d


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = autotune.Cache(path)
    assert c.get("gfx950|hip", "sig") is None
    c.put("gfx950|hip", "sig", {"group_size": 8, "sub_ranges": 0, "lane_words": 4, "ms": 1.5})
    c2 = autotune.Cache(path)
    assert c2.get("gfx950|hip", "sig")["group_size"] == 8
    with open(path) as f:
        assert json.load(f)["gfx950|hip"]["sig"]["lane_words"] == 4


def test_cache_ignores_corrupt_file(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.Cache(str(path)).data == {}


def test_candidates_are_valid_shapes():
    for g, s, r in autotune.DEFAULT_CANDIDATES:
        assert 1 <= g <= 16 and 0 <= s <= 1000 and r in (4, 6)
