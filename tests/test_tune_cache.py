"""The autotuner's JSON cache (host-only entry points; no GPU needed)."""
import json
import os

import pytest

from paper_1202_6168_amd import ditr


def test_missing_file_is_not_found(tmp_path):
    assert ditr.tune_cache_get(str(tmp_path / "none.json"), 1) is None


def test_round_trip_and_replace(tmp_path):
    path = str(tmp_path / "tune.json")
    o = ditr.opts_default(alpha=1.35, refresh_at=1e-6, part_type=ditr.PART_CB, part_nodes=2048,
                          sweeps_per_claim=3)
    ditr.tune_cache_put(path, 0xDEADBEEF12345678, o, 0.01, 0.012)
    ditr.tune_cache_put(path, 7, ditr.opts_default(alpha=2.0), 0.5, 0.6)
    got = ditr.tune_cache_get(path, 0xDEADBEEF12345678)
    assert got is not None
    assert (got.alpha, got.refresh_at, got.part_type, got.part_nodes, got.sweeps_per_claim) == \
        (1.35, 1e-6, ditr.PART_CB, 2048, 3)
    # fields that are not tuned come from the base options
    base = ditr.opts_default(max_rounds=5, mode=ditr.MODE_SWEEP)
    got = ditr.tune_cache_get(path, 7, base)
    assert got.alpha == 2.0 and got.max_rounds == 5 and got.mode == ditr.MODE_SWEEP
    # replacing a key keeps one entry for it
    ditr.tune_cache_put(path, 7, ditr.opts_default(alpha=1.2))
    doc = json.load(open(path))
    assert doc["format"] == "ditr-tune-cache" and doc["version"] == 1
    keys = [e["key"] for e in doc["entries"]]
    assert sorted(keys) == sorted(["deadbeef12345678", "0000000000000007"])
    assert ditr.tune_cache_get(path, 7).alpha == 1.2
    assert ditr.tune_cache_get(path, 8) is None
    assert not [f for f in os.listdir(tmp_path) if ".tmp." in f]


@pytest.mark.parametrize("text", ["", "{", "[1, 2]", '{"format": "other", "entries": []}',
                                  '{"format": "ditr-tune-cache", "entries": {}}',
                                  "\x00\x01garbage", '{"format": "ditr-tune-cache", "entries": [' * 40])
def test_unreadable_cache_counts_as_empty_and_is_repaired(tmp_path, text):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as fp:
        fp.write(text)
    assert ditr.tune_cache_get(path, 1) is None
    ditr.tune_cache_put(path, 1, ditr.opts_default(alpha=1.75))
    assert ditr.tune_cache_get(path, 1).alpha == 1.75
    json.load(open(path))


def test_bad_entries_are_skipped(tmp_path):
    path = str(tmp_path / "tune.json")
    doc = {"format": "ditr-tune-cache", "version": 1, "entries": [
        {"key": "0000000000000001", "alpha": 0.5},              # alpha <= 1
        {"key": "0000000000000002", "part_type": 9},            # unknown partition type
        {"key": "12", "alpha": 1.3},                            # malformed key
        {"key": "0000000000000003", "alpha": 1.3, "extra": [1, {"a": None}], "ok": True},
    ]}
    json.dump(doc, open(path, "w"))
    assert ditr.tune_cache_get(path, 1) is None
    assert ditr.tune_cache_get(path, 2) is None
    assert ditr.tune_cache_get(path, 3).alpha == 1.3


def test_put_rejects_out_of_range_and_unwritable(tmp_path):
    with pytest.raises(ditr.DitrError) as e:
        ditr.tune_cache_put(str(tmp_path / "t.json"), 1, ditr.opts_default(alpha=1.0))
    assert e.value.status == ditr.EINVAL
    with pytest.raises(ditr.DitrError) as e:
        ditr.tune_cache_put(str(tmp_path / "no" / "dir" / "t.json"), 1, ditr.opts_default())
    assert e.value.status == ditr.EINVAL
