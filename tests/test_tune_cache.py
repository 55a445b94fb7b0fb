"""tune.py's JSON cache on the CPU: path selection, atomic writes, corrupt
or unreadable files ignored."""
import json
import os

from paper_1702_05487_amd import tune


def test_cache_path_precedence(monkeypatch, tmp_path):
    monkeypatch.setenv("RKL_TUNE_CACHE", str(tmp_path / "env.json"))
    assert tune.cache_path(str(tmp_path / "arg.json")) == str(tmp_path / "arg.json")
    assert tune.cache_path() == str(tmp_path / "env.json")
    monkeypatch.delenv("RKL_TUNE_CACHE")
    assert tune.cache_path().endswith(os.path.join(".cache", "rkl", "tune.json"))


def test_save_load_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    d = {"k": {"variant": 3, "ms": 1.5, "tile": [32, 8, 64, 1]}}
    tune._save(path, d)
    assert tune._load(path) == d
    assert [f for f in os.listdir(tmp_path / "sub") if f != "tune.json"] == []   # no temp file left


def test_corrupt_or_missing_cache_is_ignored(tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert tune._load(str(bad)) == {}
    lst = tmp_path / "list.json"
    lst.write_text(json.dumps([1, 2]))
    assert tune._load(str(lst)) == {}
    assert tune._load(str(tmp_path / "missing.json")) == {}


def test_malformed_entries_are_ignored():
    from paper_1702_05487_amd import rkl
    n = rkl.rkl_variant_count()
    d = {"num": 3, "none": {"ms": 1.0}, "str": {"variant": "2"}, "bool": {"variant": True},
         "neg": {"variant": -1}, "big": {"variant": n}, "ok": {"variant": n - 1}}
    for k in ("num", "none", "str", "bool", "neg", "big", "missing"):
        assert tune._cached_variant(d, k) is None, k
    assert tune._cached_variant(d, "ok") == n - 1


def test_failed_write_leaves_no_temp_file(tmp_path):
    path = str(tmp_path / "tune.json")
    try:
        tune._save(path, {"k": object()})        # not JSON-serialisable
    except TypeError:
        pass
    assert os.listdir(tmp_path) == []
