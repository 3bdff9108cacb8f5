"""Host side of autotuning: the cache file and the tuning-table marshalling
(fl_default_tuning is a host function, so it runs without a GPU)."""
import json
import os

import pytest

from paper_2403_03504_amd import tuning_cache as tc


def test_key_separates_device_version_bound_and_sizes():
    dev = {"name": "X", "arch": "gfx950", "cus": 256}
    k = tc.make_key(dev, "1.0", 1e-3, [1024, 4096])
    assert k != tc.make_key(dict(dev, cus=128), "1.0", 1e-3, [1024, 4096])
    assert k != tc.make_key(dev, "1.1", 1e-3, [1024, 4096])
    assert k != tc.make_key(dev, "1.0", 1e-4, [1024, 4096])
    assert k != tc.make_key(dev, "1.0", 1e-3, [1024, 8192])
    assert k == tc.make_key(dict(dev), "1.0", 1e-3, (1024, 4096))


def test_store_and_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "t.json")
    table = {"fmm_min_nodes": 3000, "bucket_max": [5000, 2 ** 31 - 1], "p": [4, 8], "leaf_size": [32, 64],
             "max_rel_err": 1e-3}
    assert tc.lookup("a", path) is None
    tc.store("a", {"tuning": table, "samples": []}, path)
    tc.store("b", {"tuning": dict(table, fmm_min_nodes=1)}, path)
    assert tc.lookup("a", path)["tuning"] == table
    assert tc.lookup("b", path)["tuning"]["fmm_min_nodes"] == 1
    assert not [f for f in os.listdir(os.path.dirname(path)) if f.endswith(".tmp")]


def test_malformed_cache_is_ignored(tmp_path):
    path = str(tmp_path / "t.json")
    open(path, "w").write("{not json")
    assert tc.lookup("a", path) is None
    json.dump({"a": {"tuning": {"p": [8]}}}, open(path, "w"))
    assert tc.lookup("a", path) is None  # incomplete table
    tc.store("c", {"tuning": {"fmm_min_nodes": 1, "bucket_max": [1], "p": [8], "leaf_size": [64]}}, path)
    assert tc.lookup("c", path) is not None


def test_env_var_selects_the_file(monkeypatch, tmp_path):
    monkeypatch.setenv(tc.ENV, str(tmp_path / "x.json"))
    assert tc.cache_path() == str(tmp_path / "x.json")


def test_default_table_and_struct_roundtrip():
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_03504_amd",
                       "libfa2lay.so")
    if not os.path.exists(lib):
        pytest.fail("libfa2lay.so is not built")
    from paper_2403_03504_amd import fa2lay as fl
    d = fl.default_tuning()
    assert d == {"fmm_min_nodes": 4096, "bucket_max": [2 ** 31 - 1], "p": [8], "leaf_size": [64],
                 "list_lanes": [0], "max_rel_err": 0.0}
    t = {"fmm_min_nodes": 100, "bucket_max": [10, 20, 30], "p": [4, 6, 16], "leaf_size": [1, 2, 3],
         "list_lanes": [1, 8, 0], "max_rel_err": 0.5}
    assert fl.Tuning.from_dict(t).to_dict() == t
    with pytest.raises(ValueError):
        fl.Tuning.from_dict(dict(t, p=[4]))
