"""The on-disk cache of tuned launch shapes (host logic only)."""
import json

from paper_2504_21784_amd.tune_cache import TuneCache, problem_key

ENTRY = {"waves_per_band": 1, "bands_per_group": 16, "pairs_per_lane": 1, "workgroups_per_cu": 0, "ms": 0.55}


def test_key_names_device_precision_fixup_and_every_problem():
    k = problem_key("batch", "AMD Instinct MI355X gfx950 256 CUs", 1, [(256, 256, 16, 40), (64, 96, 4, 12)], fixup=1)
    assert k == "batch|AMD Instinct MI355X gfx950 256 CUs|p1|f1|256x256g16a40;64x96g4a12"
    assert problem_key("single", "d", 0, [(8, 8, 4, 12)]) != problem_key("single", "d", 1, [(8, 8, 4, 12)])
    assert problem_key("single", "d", 0, [(8, 8, 4, 12)]) != problem_key("batch", "d", 0, [(8, 8, 4, 12)])


def test_roundtrip_and_update(tmp_path):
    c = TuneCache(str(tmp_path / "sub" / "shapes.json"))
    assert c.get("k") is None
    c.put("k", ENTRY)
    assert c.get("k") == ENTRY
    c.put("other", dict(ENTRY, ms=1.0))
    c.put("k", dict(ENTRY, bands_per_group=8))
    c2 = TuneCache(c.path)
    assert c2.get("k")["bands_per_group"] == 8 and c2.get("other")["ms"] == 1.0
    assert not [p for p in (tmp_path / "sub").iterdir() if p.name.endswith(".tmp")]


def test_unreadable_or_incomplete_entries_count_as_missing(tmp_path):
    path = tmp_path / "shapes.json"
    path.write_text("{not json")
    c = TuneCache(str(path))
    assert c.get("k") is None
    c.put("k", ENTRY)                    # a torn file is replaced
    assert c.get("k") == ENTRY
    path.write_text(json.dumps({"k": {"waves_per_band": 1}, "l": 3}))
    assert c.get("k") is None and c.get("l") is None


def test_environment_names_the_file(tmp_path, monkeypatch):
    monkeypatch.setenv("SMRT_TUNE_CACHE", str(tmp_path / "env.json"))
    assert TuneCache().path == str(tmp_path / "env.json")
