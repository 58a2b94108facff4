"""The JSON tuning cache (host logic only, no GPU)."""
import json

from paper_1702_00496_amd import tuning


def test_store_lookup_roundtrip_and_overwrite(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    k1 = tuning.make_key("gfx950", 256, 3, (32, 32, 32), 4, 0, "time", "f32", "ab2", "advdiff", "rng")
    k2 = tuning.make_key("gfx950", 256, 3, (32, 32, 32), 4, 0, "time", "f64", "ab2", "advdiff", "rng")
    assert k1 != k2
    assert tuning.lookup(path, k1) is None
    tuning.store(path, k1, 2, {1: 0.08, 2: 0.07})
    tuning.store(path, k2, 4, {4: 0.15})
    assert tuning.lookup(path, k1) == {"variant": 2, "ms": {"1": 0.08, "2": 0.07}}
    tuning.store(path, k1, 9, {9: 0.06})
    assert tuning.lookup(path, k1)["variant"] == 9
    assert tuning.lookup(path, k2)["variant"] == 4
    assert sorted(json.load(open(path))) == sorted([k1, k2])


def test_unreadable_or_foreign_cache_is_a_miss(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text("not json")
    assert tuning.lookup(str(path), "k") is None
    path.write_text(json.dumps({"k": {"variant": "two"}}))
    assert tuning.lookup(str(path), "k") is None
    tuning.store(str(path), "k", 1, {})
    assert tuning.lookup(str(path), "k") == {"variant": 1, "ms": {}}
