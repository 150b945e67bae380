"""CPU-only checks of the tuning cache file: entries written by wrs_tune_save
load back, malformed files are rejected, and entries for other device kinds
are kept (they are never used on this one)."""
import json
import os

import pytest


@pytest.fixture(scope="module")
def wrs():
    import paper_1903_00227_amd as w
    if not os.path.exists(w.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    w.lib()
    return w


def test_entries_for_another_device_round_trip(wrs, tmp_path):
    src = tmp_path / "in.json"
    src.write_text(json.dumps({"format": "wrs-tuning-1", "entries": [
        {"arch": "gfx000", "cus": 1, "op": "build", "log2": 12, "value": 8, "us": 5.5},
        {"arch": "gfx000", "cus": 1, "op": "sample", "log2": 20, "value": 2, "us": 7.0}]}))
    wrs.tune_load(str(src))
    out = tmp_path / "out.json"
    wrs.tune_save(str(out))
    doc = json.load(open(out))
    got = {(e["arch"], e["cus"], e["op"], e["log2"]): (e["value"], e["us"]) for e in doc["entries"]}
    assert got[("gfx000", 1, "build", 12)] == (8, 5.5)
    assert got[("gfx000", 1, "sample", 20)] == (2, 7.0)


@pytest.mark.parametrize("text", [
    "",
    "{}",
    '{"entries": [ {"arch": "gfx000", "cus": 1, "op": "build", "log2": 12, "value": 12} ]}',
    '{"entries": [ {"arch": "gfx000", "cus": 1, "op": "gather", "log2": 12, "value": 8} ]}',
    '{"entries": [ {"arch": "gfx000", "op": "build", "log2": 12, "value": 8} ]}',
    '{"entries": [ {"arch": "gfx000", "cus": 1, "op": "build", "log2": 12, "value": 8} '])
def test_malformed_files_are_rejected(wrs, tmp_path, text):
    p = tmp_path / "bad.json"
    p.write_text(text)
    with pytest.raises(wrs.WrsError) as e:
        wrs.tune_load(str(p))
    assert e.value.code == wrs.EINVAL


def test_missing_file(wrs, tmp_path):
    with pytest.raises(wrs.WrsError) as e:
        wrs.tune_load(str(tmp_path / "none.json"))
    assert e.value.code == wrs.EINVAL
