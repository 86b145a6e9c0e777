"""Host logic of the autotuner's table (no GPU): keys and lookups."""

import json

import pytest


@pytest.fixture()
def tune(tmp_path, monkeypatch):
    from paper_1402_6964_amd import tune as t
    monkeypatch.setattr(t, "TUNED", str(tmp_path / "tuned.json"))
    return t


def test_key_buckets_by_log2_rows(tune):
    assert tune.key("f32", "row", 25, 10_000_000) == "f32:row:25:23"
    assert tune.key("f32", "row", 25, 2 ** 23) == tune.key("f32", "row", 25, 2 ** 24 - 1)
    assert tune.key("f64", "col", 64, 1) == "f64:col:64:0"


def test_lookup_missing_and_present(tune):
    assert tune.lookup("f32", "row", 25, 10_000_000) is None
    with open(tune.TUNED, "w") as f:
        json.dump({"f32:row:25:23": {"leaf_rows": 4883, "tree_arity": 16, "ms": 0.4}}, f)
    cfg = tune.lookup("f32", "row", 25, 10_000_000)
    assert (cfg.leaf_rows, cfg.tree_arity, cfg.rows_per_lane) == (4883, 16, 0)
    with open(tune.TUNED, "w") as f:
        json.dump({"f32:row:25:23": {"leaf_rows": 1000, "ms": 0.4}}, f)   # entries without an arity
    assert tune.lookup("f32", "row", 25, 10_000_000).tree_arity == 0


def test_unreadable_table_is_empty(tune):
    with open(tune.TUNED, "w") as f:
        f.write("not json")
    assert tune.load() == {}
